// rounds.hip -- per-query bookkeeping of the batched LO-RANSAC rounds (ImLoc
// Sec. 3.3: batches of minimal sets; stop after the sample cap or once the
// probability of having missed the best model is small), plus small utility
// kernels.  One thread per query unless noted.
#include "imloc_device.h"
#include "imloc_kernels.h"

namespace imloc {

__global__ void fill_i32_kernel(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

__global__ void fill_u8_kernel(uint8_t* p, int64_t n, uint8_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u8_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

// Scoring-set gather: S_j = point floor(j * n / m), j < m.
__global__ void gather_subset_kernel(const float* __restrict__ U, const float* __restrict__ V,
                                     const float* __restrict__ X, const float* __restrict__ Y,
                                     const float* __restrict__ Z, const float* __restrict__ W, int64_t n, int64_t m,
                                     float* __restrict__ dst) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const int64_t i = (int64_t)(((uint64_t)j * (uint64_t)n) / (uint64_t)m);  // n < 2^31: no overflow
  dst[j] = U[i];
  dst[m + j] = V[i];
  dst[2 * m + j] = X[i];
  dst[3 * m + j] = Y[i];
  dst[4 * m + j] = Z[i];
  dst[5 * m + j] = W ? W[i] : 1.0f;
}

// Batched gather: grid (blocks, queries); queries whose scoring set is not
// their full set read from the table where to gather from and to.
__global__ void gather_subsets_kernel(const QueryDesc* __restrict__ qd) {
  const QueryDesc& d = qd[blockIdx.y];
  if (!d.fresh || d.S.u == d.full.u) return;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d.m) return;
  const int64_t i = (int64_t)(((uint64_t)j * (uint64_t)d.n) / (uint64_t)d.m);  // n < 2^31: no overflow
  float* dst = const_cast<float*>(d.S.u);
  const int64_t m = d.m;
  dst[j] = d.full.u[i];
  dst[m + j] = d.full.v[i];
  dst[2 * m + j] = d.full.X[i];
  dst[3 * m + j] = d.full.Y[i];
  dst[4 * m + j] = d.full.Z[i];
  dst[5 * m + j] = d.full.w ? d.full.w[i] : 1.0f;
}

hipError_t launch_gather_subsets(const QueryDesc* qd, int nq, int64_t max_m, hipStream_t s) {
  if (nq <= 0 || max_m <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_subsets_kernel, dim3((unsigned)((max_m + 255) / 256), nq), dim3(256), 0, s, qd);
  return hipGetLastError();
}

hipError_t launch_gather_subset(const CorrF32& c, int64_t n, int64_t m, float* dst, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_subset_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, c.u, c.v, c.X, c.Y,
                     c.Z, c.w, n, m, dst);
  return hipGetLastError();
}

// Samples of the coming round: the rest of the budget, at most one batch;
// none once the query stopped.
__device__ inline int64_t round_samples(const QueryDesc& d, const BestState& b) {
  if (!b.active) return 0;
  const int64_t left = d.total - b.drawn;
  return left < d.batch ? left : d.batch;
}

// One workgroup of 1024 threads per query: reset the state and sum the
// scoring-set weights in float64 (thread t adds elements t + 1024 (16 k + u)
// into sixteen partial sums, u = 0..15, so that sixteen loads are in flight;
// the partials, the waves and the workgroup are combined in a fixed order).
// With `begin`, also set up the first round (samples, candidate counter).
constexpr int kInitThreads = 1024;

__global__ __launch_bounds__(kInitThreads) void init_queries_kernel(QueryDesc* __restrict__ qd,
                                                                    BestState* __restrict__ st,
                                                                    int32_t* __restrict__ n_cand, int begin) {
  const int q = blockIdx.x;
  QueryDesc& d = qd[q];
  if (!d.fresh) return;
  double p[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) p[u] = 0.0;
  const float* __restrict__ w = d.S.w;
  const int64_t m = d.m;
  if (w) {
    for (int64_t i0 = threadIdx.x; i0 < m; i0 += 16 * kInitThreads) {
      float x[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int64_t i = i0 + (int64_t)kInitThreads * u;
        x[u] = i < m ? w[i] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u) p[u] += (double)x[u];
    }
  } else {
    for (int64_t i0 = threadIdx.x; i0 < m; i0 += 16 * kInitThreads) {
#pragma unroll
      for (int u = 0; u < 16; ++u) p[u] += i0 + (int64_t)kInitThreads * u < m ? 1.0 : 0.0;
    }
  }
#pragma unroll
  for (int h = 8; h >= 1; h >>= 1) {
#pragma unroll
    for (int u = 0; u < h; ++u) p[u] += p[u + h];
  }
  const double s = wave_sum(p[0]);
  __shared__ double sw[kInitThreads / kWave];
  if ((threadIdx.x & (kWave - 1)) == 0) sw[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    for (int k = 0; k < kInitThreads / kWave; ++k) tot += sw[k];
    BestState& b = st[q];
    for (int e = 0; e < 12; ++e) b.pose[e] = (e == 0 || e == 4 || e == 8) ? 1.0 : 0.0;
    b.cost = __builtin_inf();
    b.count = 0;
    b.h = -1;
    b.j = -1;
    b.have = 0;
    b.lo_runs = 0;
    b.candidates = 0;
    b.inlier_residuals = 0;
    b.weight_sum = tot;
    b.final_cost = 0.0;
    b.full_count = 0;
    b.drawn = 0;
    b.batches = 0;
    const bool can = d.m >= 3 && d.total > 0;
    b.active = can ? 1 : 0;
    b.finished = can ? 0 : 1;
    if (begin) {
      d.B = round_samples(d, b);
      n_cand[q] = 0;
    }
  }
}

hipError_t launch_init_queries(QueryDesc* qd, BestState* st, int32_t* n_cand, int nq, bool begin, hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  hipLaunchKernelGGL(init_queries_kernel, dim3(nq), dim3(kInitThreads), 0, s, qd, st, n_cand, begin ? 1 : 0);
  return hipGetLastError();
}

__global__ void retire_kernel(BestState* __restrict__ st, int nq) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < nq && st[q].finished == 1) st[q].finished = 2;
}

hipError_t launch_retire(BestState* st, int nq, hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  hipLaunchKernelGGL(retire_kernel, dim3((nq + 255) / 256), dim3(256), 0, s, st, nq);
  return hipGetLastError();
}

__global__ void begin_round_kernel(QueryDesc* __restrict__ qd, const BestState* __restrict__ st, int32_t* n_cand,
                                   int nq) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  qd[q].B = round_samples(qd[q], st[q]);
  n_cand[q] = 0;
}

hipError_t launch_begin_round(QueryDesc* qd, const BestState* st, CandBuf cb, int nq, hipStream_t s) {
  hipLaunchKernelGGL(begin_round_kernel, dim3((nq + 255) / 256), dim3(256), 0, s, qd, st, cb.n, nq);
  return hipGetLastError();
}

// Stopping rule: samples needed for inlier ratio eps with minimal sets of 3.
__device__ inline int64_t required_samples(double eps, double conf, int64_t cap) {
  if (!(eps > 0.0)) return cap;
  if (eps >= 1.0) return 0;
  const double denom = log1p(-eps * eps * eps);
  if (!(denom < 0.0)) return cap;
  const double k = ceil(log(1.0 - conf) / denom);
  if (!(k < (double)cap)) return cap;
  if (k < 0.0) return 0;
  return (int64_t)k;
}

// The end of a round for every query, in one workgroup: the round's local
// optimisations update the running best (in selection order, a strictly
// lower refined cost replaces it), the sample count advances, the stopping
// rule runs, and with `begin_next` the next round is set up (samples,
// candidate counter).  The number of queries still sampling is summed in the
// workgroup and written to *active_count (nothing to clear beforehand).
__global__ __launch_bounds__(1024) void round_end_kernel(QueryDesc* __restrict__ qd, CandBuf cb,
                                                         const int32_t* __restrict__ sel,
                                                         const int32_t* __restrict__ n_sel,
                                                         const double* __restrict__ lo_pose,
                                                         const double* __restrict__ lo_cost,
                                                         const int64_t* __restrict__ lo_count, int nq, int kmax,
                                                         BestState* __restrict__ st, int32_t* __restrict__ active_count,
                                                         int begin_next) {
  long long act = 0;
  for (int q = threadIdx.x; q < nq; q += blockDim.x) {
    QueryDesc& d = qd[q];
    BestState& b = st[q];
    if (d.B > 0) {
      const int ns = n_sel[q];
      for (int slot = 0; slot < ns; ++slot) {
        const int p = q * kmax + slot;
        if (lo_cost[p] < b.cost) {
          b.cost = lo_cost[p];
          b.count = lo_count[p];
          for (int e = 0; e < 12; ++e) b.pose[e] = lo_pose[12 * (int64_t)p + e];
          const int64_t o = d.cand_off + sel[q * kMaxTopK + slot];
          b.h = cb.h[o];
          b.j = cb.j[o];
          b.have = 1;
        }
      }
      b.lo_runs += ns;
      b.drawn += d.B;
      b.batches += 1;
      bool more;
      if (d.fixed) {
        more = b.drawn < d.total;
      } else {
        int64_t need = required_samples((double)b.count / (double)d.m, d.confidence, d.total);
        if (need < d.min_iters) need = d.min_iters;
        if (need > d.total) need = d.total;
        more = b.drawn < need;
      }
      if (!more) {
        b.active = 0;
        b.finished = 1;
      }
    }
    act += b.active;
    if (begin_next) {
      d.B = round_samples(d, b);
      cb.n[q] = 0;
    }
  }
  act = wave_sum(act);
  __shared__ long long s_act[1024 / kWave];
  if ((threadIdx.x & (kWave - 1)) == 0) s_act[threadIdx.x / kWave] = act;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long t = 0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) t += s_act[w];
    *active_count = (int32_t)t;
  }
}

hipError_t launch_round_end(QueryDesc* qd, CandBuf cb, const int32_t* sel, const int32_t* n_sel,
                            const double* lo_pose, const double* lo_cost, const int64_t* lo_count, int nq, int kmax,
                            BestState* st, int32_t* active_count, bool begin_next, hipStream_t s) {
  hipLaunchKernelGGL(round_end_kernel, dim3(1), dim3(1024), 0, s, qd, cb, sel, n_sel, lo_pose, lo_cost, lo_count, nq,
                     kmax, st, active_count, begin_next ? 1 : 0);
  return hipGetLastError();
}

}  // namespace imloc
