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

// One workgroup per query: reset the state and sum the scoring-set weights
// (float64, fixed order).
__global__ __launch_bounds__(256) void init_queries_kernel(const QueryDesc* __restrict__ qd, BestState* __restrict__ st) {
  const int q = blockIdx.x;
  const QueryDesc& d = qd[q];
  if (!d.fresh) return;
  double s = 0.0;
  if (d.S.w) {
    for (int64_t i = threadIdx.x; i < d.m; i += 256) s += d.S.w[i];
  } else {
    for (int64_t i = threadIdx.x; i < d.m; i += 256) s += 1.0;
  }
  s = wave_sum(s);
  __shared__ double sw[4];
  if ((threadIdx.x & 63) == 0) sw[threadIdx.x / 64] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
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
    b.weight_sum = ((sw[0] + sw[1]) + sw[2]) + sw[3];
    b.final_cost = 0.0;
    b.full_count = 0;
    b.drawn = 0;
    b.batches = 0;
    const bool can = d.m >= 3 && d.total > 0;
    b.active = can ? 1 : 0;
    b.finished = can ? 0 : 1;
  }
}

hipError_t launch_init_queries(const QueryDesc* qd, BestState* st, int nq, hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  hipLaunchKernelGGL(init_queries_kernel, dim3(nq), dim3(256), 0, s, qd, st);
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
  int64_t B = 0;
  if (st[q].active) {
    const int64_t left = qd[q].total - st[q].drawn;
    B = left < qd[q].batch ? left : qd[q].batch;
  }
  qd[q].B = B;
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

__global__ void end_round_kernel(const QueryDesc* __restrict__ qd, BestState* __restrict__ st, int nq,
                                 int32_t* active_count) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  int act = 0;
  if (q < nq) {
    const QueryDesc& d = qd[q];
    BestState& b = st[q];
    if (d.B > 0) {
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
    act = b.active;
  }
  const long long tot = wave_sum((long long)act);
  if ((threadIdx.x & 63) == 0 && tot) atomicAdd(active_count, (int32_t)tot);
}

hipError_t launch_end_round(const QueryDesc* qd, BestState* st, int nq, int32_t* active_count, hipStream_t s) {
  hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(64), 0, s, active_count, (int64_t)1, 0);
  hipLaunchKernelGGL(end_round_kernel, dim3((nq + 255) / 256), dim3(256), 0, s, qd, st, nq, active_count);
  return hipGetLastError();
}

}  // namespace imloc
