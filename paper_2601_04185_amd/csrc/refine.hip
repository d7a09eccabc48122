// refine.hip -- float64 Gauss-Newton of LO-RANSAC (ImLoc Sec. 3.3):
//   local optimisation: non-linear refinement of the truncated squared
//     reprojection error of a new best hypothesis on the scoring set, the
//     inlier set re-evaluated at every iterate;
//   final refinement: robust Cauchy loss, weighted by the confidences, over
//     all inliers of the full set at the best pose (held fixed).
// Each Gauss-Newton iteration is one launch over (point chunk x problem)
// workgroups for every problem of a batch of queries.  A workgroup
// accumulates the 6x6 normal equations (upper triangle), the gradient, the
// cost and the inlier count in float64 with a fixed thread-to-point map and
// reduction tree; partial sums are combined in chunk order, so the result is
// deterministic.  Residual r = pi(R X + t) - x; left update on SO(3).
#include "imloc_device.h"
#include "imloc_kernels.h"

namespace imloc {

constexpr int kAcc = 29;  // 21 (H upper) + 6 (g) + cost + count
constexpr int kGNThreads = 256;
constexpr int kGNWaves = kGNThreads / kWave;
constexpr int kGNPPT = 8;                       // points per thread per chunk
constexpr int kGNChunk = kGNThreads * kGNPPT;   // points per workgroup

__device__ inline void acc_point(double* a, const Cam& K, double x, double y, double z, double du, double dv,
                                 double wt) {
  const double iz = 1.0 / z;
  const double a00 = K.fx * iz, a02 = -K.fx * x * iz * iz;
  const double a11 = K.fy * iz, a12 = -K.fy * y * iz * iz;
  // d x_c / d(dw, dt) rows: (0, z, -y, 1, 0, 0), (-z, 0, x, 0, 1, 0), (y, -x, 0, 0, 0, 1)
  const double J0[6] = {a02 * y, a00 * z - a02 * x, -a00 * y, a00, 0.0, a02};
  const double J1[6] = {-a11 * z + a12 * y, -a12 * x, a11 * x, 0.0, a11, a12};
  int k = 0;
#pragma unroll
  for (int r = 0; r < 6; ++r) {
#pragma unroll
    for (int c = r; c < 6; ++c) { a[k] = fma(wt, J0[r] * J0[c] + J1[r] * J1[c], a[k]); ++k; }
  }
#pragma unroll
  for (int r = 0; r < 6; ++r) a[21 + r] = fma(wt, J0[r] * du + J1[r] * dv, a[21 + r]);
}

// The same for a rig camera: x_c = R_c x_r + t_c with the rig-frame point x_r
// moving under the left update of the rig pose, so the rows of d(pixel)/dx_c
// are carried through R_c: J = [x_r x r, r] for each row r of d(pixel)/dx_c R_c.
__device__ inline void acc_point_rig(double* a, const Cam& K, const double xr[3], double x, double y, double z,
                                     const double* Rc, double du, double dv, double wt) {
  const double iz = 1.0 / z;
  const double p0[3] = {K.fx * iz, 0.0, -K.fx * x * iz * iz};
  const double p1[3] = {0.0, K.fy * iz, -K.fy * y * iz * iz};
  double r0[3], r1[3];
  for (int c = 0; c < 3; ++c) {
    r0[c] = p0[0] * Rc[c] + p0[1] * Rc[3 + c] + p0[2] * Rc[6 + c];
    r1[c] = p1[0] * Rc[c] + p1[1] * Rc[3 + c] + p1[2] * Rc[6 + c];
  }
  double w0[3], w1[3];
  cross3(xr, r0, w0);
  cross3(xr, r1, w1);
  const double J0[6] = {w0[0], w0[1], w0[2], r0[0], r0[1], r0[2]};
  const double J1[6] = {w1[0], w1[1], w1[2], r1[0], r1[1], r1[2]};
  int k = 0;
#pragma unroll
  for (int r = 0; r < 6; ++r) {
#pragma unroll
    for (int c = r; c < 6; ++c) { a[k] = fma(wt, J0[r] * J0[c] + J1[r] * J1[c], a[k]); ++k; }
  }
#pragma unroll
  for (int r = 0; r < 6; ++r) a[21 + r] = fma(wt, J0[r] * du + J1[r] * dv, a[21 + r]);
}

// Per-problem Gauss-Newton state, double-buffered across launches.
struct GNState {
  double cur[12];      // accepted pose
  double eval[12];     // pose evaluated by the launch that wrote this state
  double cur_cost;
  double cur_count;
  int32_t done;
  int32_t accepted;
};

__host__ __device__ inline int chunks_for(int64_t n) {
  const int64_t c = (n + kGNChunk - 1) / kGNChunk;
  return c > 0 ? (int)c : 1;
}

int gn_chunks(int64_t n) { return chunks_for(n); }

size_t gn_scratch_bytes(int nprob, int chunks_max) {
  if (nprob < 1) nprob = 1;
  if (chunks_max < 1) chunks_max = 1;
  return (((size_t)2 * nprob * sizeof(GNState) + 255) & ~size_t(255)) +
         (size_t)2 * nprob * chunks_max * kAcc * sizeof(double) + 256;
}

// Packed row-wise index of (r, c), r <= c, in the 21-entry upper triangle.
__host__ __device__ constexpr int upk(int r, int c) { return r * 6 - (r * (r - 1)) / 2 + (c - r); }

// Solve from the reduced sums (LDS); thread 0 only.  Cholesky H = U^T U in
// place on the packed upper triangle (pivot reciprocals computed once), then
// U^T y = -g, U d = y, and the left update.  Every loop has constant bounds and is unrolled, so the factor, the
// vectors and the rotation stay in registers (about 100 VGPRs, below what the
// accumulation path needs).  Returns false if H is not positive definite.
__device__ __forceinline__ bool gn_solve_step(const double* tot, const double* cur, double* next) {
  double h[21], inv[6];
#pragma unroll
  for (int e = 0; e < 21; ++e) h[e] = tot[e];
  bool ok = true;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double dsum = h[upk(i, i)];
#pragma unroll
    for (int m = 0; m < i; ++m) dsum -= h[upk(m, i)] * h[upk(m, i)];
    ok = ok && dsum > 0.0;
    const double uii = sqrt(fmax(dsum, 0.0));
    inv[i] = 1.0 / uii;
    h[upk(i, i)] = uii;
#pragma unroll
    for (int j = i + 1; j < 6; ++j) {
      double sum = h[upk(i, j)];
#pragma unroll
      for (int m = 0; m < i; ++m) sum -= h[upk(m, i)] * h[upk(m, j)];
      h[upk(i, j)] = sum * inv[i];
    }
  }
  if (!ok) return false;
  double y[6], d[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double sum = -tot[21 + i];
#pragma unroll
    for (int m = 0; m < i; ++m) sum -= h[upk(m, i)] * y[m];
    y[i] = sum * inv[i];
  }
#pragma unroll
  for (int i = 5; i >= 0; --i) {
    double sum = y[i];
#pragma unroll
    for (int m = i + 1; m < 6; ++m) sum -= h[upk(i, m)] * d[m];
    d[i] = sum * inv[i];
  }
  // left update: R' = Exp(dw) R, t' = Exp(dw) t + dt
  double E[9];
  so3_exp(d, E);
#pragma unroll
  for (int r = 0; r < 3; ++r) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
      next[3 * r + c] = E[3 * r] * cur[c] + E[3 * r + 1] * cur[3 + c] + E[3 * r + 2] * cur[6 + c];
    next[9 + r] = E[3 * r] * cur[9] + E[3 * r + 1] * cur[10] + E[3 * r + 2] * cur[11] + d[3 + r];
  }
  return true;
}

// One launch of a batched multi-workgroup Gauss-Newton run.  Launch k of a
// problem:
//   k = 0: evaluate the start pose;
//   k >= 1: reduce the partial sums of launch k-1 (every workgroup of the
//     problem, in chunk order, so all take the same decision), accept the
//     evaluated pose if its cost did not rise (at k = 1 it is the start),
//     solve the normal equations of the accepted pose for the next pose
//     (unless the iteration budget is spent), and evaluate that.
// MODE 0 (local optimisation): truncated cost over the scoring set.
// MODE 1 (final refinement): Cauchy cost over the in-set, which launch 0
// marks as the inliers (tau) of the start pose.
template <int MODE, bool RIG>
__global__ __launch_bounds__(kGNThreads) void gn_kernel(
    const QueryDesc* __restrict__ qd, CandBuf cb, const int32_t* __restrict__ sel, const int32_t* __restrict__ n_sel,
    const double* __restrict__ start_direct, BestState* __restrict__ bst, int kmax, int k, GNState* __restrict__ gst,
    double* __restrict__ part, int chunks_max, int nprob, uint8_t* __restrict__ in_set_all,
    double* __restrict__ out_pose, double* __restrict__ out_cost, int64_t* __restrict__ out_count) {
  const int p = blockIdx.y;
  const int chunk = blockIdx.x;
  int q;
  const double* start;
  if (MODE == 0) {
    q = start_direct ? 0 : p / kmax;
    const int slot = p - q * kmax;
    if (!start_direct && slot >= n_sel[q]) return;
    start = start_direct ? start_direct + 12 * (int64_t)p
                         : cb.pose + 12 * (qd[q].cand_off + sel[q * kMaxTopK + slot]);
  } else {
    q = p;
    if (!start_direct && !(bst[q].finished == 1 && bst[q].have)) return;
    start = start_direct ? start_direct + 12 * (int64_t)q : bst[q].pose;
  }
  const QueryDesc& d = qd[q];
  const CorrF32 c = MODE == 0 ? d.S : d.full;
  const int64_t n = MODE == 0 ? d.m : d.n;
  const int iters = MODE == 0 ? d.lo_iters : d.final_iters;
  const double tau2 = d.tau * d.tau, s2 = d.cauchy_s * d.cauchy_s;
  const Cam K{d.fx, d.fy, d.cx, d.cy};
  const int chunks = chunks_for(n);
  if (chunk >= chunks) return;
  uint8_t* in_set = MODE == 1 ? in_set_all + d.in_set_off : nullptr;
  GNState* prev = gst + (int64_t)((k + 1) & 1) * nprob + p;
  GNState* next = gst + (int64_t)(k & 1) * nprob + p;
  const double* part_prev = part + ((int64_t)((k + 1) & 1) * nprob + p) * chunks_max * kAcc;
  double* part_next = part + ((int64_t)(k & 1) * nprob + p) * chunks_max * kAcc;
  const bool prev_done = k > 0 && prev->done != 0;

  const int64_t base = (int64_t)chunk * kGNChunk + threadIdx.x;
  // the chunk's points of a live problem are loaded first: one memory latency
  // per launch, overlapping the reduction of the previous partial sums and
  // the solve
  float pX[kGNPPT], pY[kGNPPT], pZ[kGNPPT], pu[kGNPPT], pv[kGNPPT], pw[kGNPPT];
  bool use[kGNPPT];
#pragma unroll
  for (int t = 0; t < kGNPPT; ++t) {
    const int64_t i = base + (int64_t)t * kGNThreads;
    use[t] = !prev_done && i < n;
    pX[t] = pY[t] = pZ[t] = pu[t] = pv[t] = 0.0f;
    pw[t] = 1.0f;
    if (MODE == 1 && k > 0 && use[t]) use[t] = in_set[i] != 0;
    if (use[t]) {
      pX[t] = gmem(c.X)[i];
      pY[t] = gmem(c.Y)[i];
      pZ[t] = gmem(c.Z)[i];
      pu[t] = gmem(c.u)[i];
      pv[t] = gmem(c.v)[i];
      if (c.w) pw[t] = gmem(c.w)[i];
    }
  }


  __shared__ double s_rig[RIG ? kMaxCams * 16 : 1];
  const bool rig = RIG && d.ncam > 0;  // the RIG = false variant runs batches without rig queries
  const int64_t* seg = MODE == 0 ? d.segS : d.segF;
  if (rig)
    for (int e = threadIdx.x; e < 16 * d.ncam; e += kGNThreads) s_rig[e] = d.rig[e];
  __shared__ double s_grp[8][kAcc];
  __shared__ double s_tot[kAcc];
  __shared__ double s_cur[12], s_eval[12];
  __shared__ double s_cost, s_count;
  __shared__ int s_done, s_accepted;
  if (k == 0) {
    if (threadIdx.x < 12) {
      s_cur[threadIdx.x] = start[threadIdx.x];
      s_eval[threadIdx.x] = start[threadIdx.x];
    }
    if (threadIdx.x == 0) {
      s_cost = __builtin_inf();
      s_count = 0.0;
      s_done = 0;
      s_accepted = 0;
    }
    __syncthreads();
  } else {
    // partial sums of launch k-1 in chunk order: thread (v, g) sums chunks g, g+8, ...
    const int v = threadIdx.x % kAcc, g = threadIdx.x / kAcc;
    if (!prev_done && g < 8) {
      // chunks g, g + 8, ...: loaded four at a time, summed in chunk order
      double sum = 0.0;
      for (int ch0 = g; ch0 < chunks; ch0 += 32) {
        double t[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int ch = ch0 + 8 * u;
          t[u] = ch < chunks ? part_prev[(int64_t)ch * kAcc + v] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (ch0 + 8 * u < chunks) sum += t[u];
      }
      s_grp[g][v] = sum;
    }
    if (threadIdx.x < 12) {
      s_cur[threadIdx.x] = prev->cur[threadIdx.x];
      s_eval[threadIdx.x] = prev->eval[threadIdx.x];
    }
    __syncthreads();
    if ((int)threadIdx.x < kAcc && !prev_done) {
      double t = 0.0;
      for (int gg = 0; gg < 8; ++gg) t += s_grp[gg][threadIdx.x];
      s_tot[threadIdx.x] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      s_cost = prev->cur_cost;
      s_count = prev->cur_count;
      s_done = prev->done;
      s_accepted = prev->accepted;
      if (!s_done) {
        // the evaluated pose becomes the accepted one if its cost did not rise
        if (k == 1 || s_tot[27] <= s_cost) {
          for (int e = 0; e < 12; ++e) s_cur[e] = s_eval[e];
          s_cost = s_tot[27];
          s_count = s_tot[28];
          if (k > 1) s_accepted += 1;
          if (k - 1 >= iters || !gn_solve_step(s_tot, s_cur, s_eval)) s_done = 1;
        } else {
          s_done = 1;  // the step raised the cost: keep the accepted pose
        }
      }
    }
    __syncthreads();
  }
  // workgroup (0, p) records the state for the next launch and the outputs
  if (chunk == 0) {
    if (threadIdx.x < 12) {
      next->cur[threadIdx.x] = s_cur[threadIdx.x];
      next->eval[threadIdx.x] = s_eval[threadIdx.x];
      if (s_done && out_pose) out_pose[12 * (int64_t)p + threadIdx.x] = s_cur[threadIdx.x];
    }
    if (threadIdx.x == 0) {
      next->cur_cost = s_cost;
      next->cur_count = s_count;
      next->done = s_done;
      next->accepted = s_accepted;
      if (s_done) {
        if (out_cost) out_cost[p] = s_cost;
        if (out_count) out_count[p] = (int64_t)s_count;
      }
    }
  }
  if (s_done) return;

  // accumulate this chunk at the evaluated pose
  double P[12];
  for (int e = 0; e < 12; ++e) P[e] = s_eval[e];
  double a[kAcc];
#pragma unroll
  for (int e = 0; e < kAcc; ++e) a[e] = 0.0;
#pragma unroll
  for (int t = 0; t < kGNPPT; ++t) {
    if (!use[t]) continue;
    const int64_t i = base + (int64_t)t * kGNThreads;
    const double X = pX[t], Y = pY[t], Z = pZ[t];
    const double w = pw[t];
    double x = P[0] * X + P[1] * Y + P[2] * Z + P[9];
    double y = P[3] * X + P[4] * Y + P[5] * Z + P[10];
    double z = P[6] * X + P[7] * Y + P[8] * Z + P[11];
    Cam Kp = K;
    const double* Rc = nullptr;
    const double xr[3] = {x, y, z};
    if (rig) {  // through the point's camera: x_c = R_c x_r + t_c
      const double* rc = s_rig + 16 * cam_of(seg, d.ncam, i);
      Kp = Cam{rc[0], rc[1], rc[2], rc[3]};
      Rc = rc + 4;
      x = Rc[0] * xr[0] + Rc[1] * xr[1] + Rc[2] * xr[2] + rc[13];
      y = Rc[3] * xr[0] + Rc[4] * xr[1] + Rc[5] * xr[2] + rc[14];
      z = Rc[6] * xr[0] + Rc[7] * xr[1] + Rc[8] * xr[2] + rc[15];
    }
    double du = 0.0, dv = 0.0, r2 = 0.0;
    const bool front = z > 0.0;
    if (front) {
      du = Kp.fx * x / z + Kp.cx - (double)pu[t];
      dv = Kp.fy * y / z + Kp.cy - (double)pv[t];
      r2 = du * du + dv * dv;
    }
    if (MODE == 0) {
      if (front && r2 < tau2) {
        a[27] += w * r2;
        a[28] += 1.0;
        if (rig) acc_point_rig(a, Kp, xr, x, y, z, Rc, du, dv, w);
        else acc_point(a, K, x, y, z, du, dv, w);
      } else {
        a[27] += w * tau2;
      }
    } else {
      if (k == 0) {
        const bool in = front && r2 < tau2;
        in_set[i] = in ? 1 : 0;
        if (!in) continue;
      }
      a[28] += 1.0;
      if (!front) {
        a[27] += w * s2 * log1p(tau2 / s2);
        continue;
      }
      a[27] += w * s2 * log1p(r2 / s2);
      if (rig) acc_point_rig(a, Kp, xr, x, y, z, Rc, du, dv, w / (1.0 + r2 / s2));
      else acc_point(a, K, x, y, z, du, dv, w / (1.0 + r2 / s2));
    }
  }
  __shared__ double s_part[kGNWaves][kAcc];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
  for (int e = 0; e < kAcc; ++e) {
    const double v = wave_sum(a[e]);
    if (lane == 0) s_part[wave][e] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < kAcc) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kGNWaves; ++w) t += s_part[w][threadIdx.x];
    part_next[(int64_t)chunk * kAcc + threadIdx.x] = t;
  }
}

static void split_scratch(void* scratch, int nprob, GNState** st, double** part) {
  *st = reinterpret_cast<GNState*>(scratch);
  *part = reinterpret_cast<double*>(reinterpret_cast<char*>(scratch) +
                                    (((size_t)2 * nprob * sizeof(GNState) + 255) & ~size_t(255)));
}

hipError_t launch_lo(const QueryDesc* qd, CandBuf cb, const int32_t* sel, const int32_t* n_sel,
                     const double* start_direct, int nprob, int kmax, int chunks_max, int iters_max, void* scratch,
                     double* out_pose, double* out_cost, int64_t* out_count, bool any_rig, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  GNState* st;
  double* part;
  split_scratch(scratch, nprob, &st, &part);
  auto kern = any_rig ? gn_kernel<0, true> : gn_kernel<0, false>;
  for (int k = 0; k <= iters_max + 1; ++k)
    hipLaunchKernelGGL(kern, dim3(chunks_max, nprob), dim3(kGNThreads), 0, s, qd, cb, sel, n_sel,
                       start_direct, (BestState*)nullptr, kmax, k, st, part, chunks_max, nprob, (uint8_t*)nullptr,
                       out_pose, out_cost, out_count);
  return hipGetLastError();
}

hipError_t launch_refine(const QueryDesc* qd, BestState* bst, const double* start_direct, int nq, int chunks_max,
                         int iters_max, uint8_t* in_set, void* scratch, double* out_pose, double* out_cost,
                         bool any_rig, hipStream_t s) {
  if (nq <= 0) return hipSuccess;
  GNState* st;
  double* part;
  split_scratch(scratch, nq, &st, &part);
  CandBuf none{};
  auto kern = any_rig ? gn_kernel<1, true> : gn_kernel<1, false>;
  for (int k = 0; k <= iters_max + 1; ++k)
    hipLaunchKernelGGL(kern, dim3(chunks_max, nq), dim3(kGNThreads), 0, s, qd, none,
                       (const int32_t*)nullptr, (const int32_t*)nullptr, start_direct, bst, 1, k, st, part, chunks_max,
                       nq, in_set, out_pose, out_cost, (int64_t*)nullptr);
  return hipGetLastError();
}

// Running best after a round's local optimisations: in selection order, a
// strictly lower refined cost replaces the best.  One thread per query.
__global__ void update_best_kernel(const QueryDesc* __restrict__ qd, CandBuf cb, const int32_t* __restrict__ sel,
                                   const int32_t* __restrict__ n_sel, const double* __restrict__ lo_pose,
                                   const double* __restrict__ lo_cost, const int64_t* __restrict__ lo_count, int nq,
                                   int kmax, BestState* __restrict__ st) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq || qd[q].B <= 0) return;
  BestState& b = st[q];
  const int ns = n_sel[q];
  for (int slot = 0; slot < ns; ++slot) {
    const int p = q * kmax + slot;
    if (lo_cost[p] < b.cost) {
      b.cost = lo_cost[p];
      b.count = lo_count[p];
      for (int e = 0; e < 12; ++e) b.pose[e] = lo_pose[12 * (int64_t)p + e];
      const int64_t o = qd[q].cand_off + sel[q * kMaxTopK + slot];
      b.h = cb.h[o];
      b.j = cb.j[o];
      b.have = 1;
    }
  }
  b.lo_runs += ns;
}

hipError_t launch_update_best(const QueryDesc* qd, CandBuf cb, const int32_t* sel, const int32_t* n_sel,
                              const double* lo_pose, const double* lo_cost, const int64_t* lo_count, int nq,
                              int kmax, BestState* st, hipStream_t s) {
  hipLaunchKernelGGL(update_best_kernel, dim3((nq + 255) / 256), dim3(256), 0, s, qd, cb, sel, n_sel, lo_pose,
                     lo_cost, lo_count, nq, kmax, st);
  return hipGetLastError();
}

// Inlier mask over all points of every query that just finished, at its final
// pose (float64), and its count; a query without a pose gets a zero mask.
__global__ void mask_kernel(const QueryDesc* __restrict__ qd, BestState* __restrict__ st,
                            const double* __restrict__ fin_pose, int all) {
  const int q = blockIdx.y;
  if (!all && st[q].finished != 1) return;
  const QueryDesc& d = qd[q];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if ((int64_t)blockIdx.x * blockDim.x >= d.n) return;
  const bool have = all || st[q].have != 0;
  const double* pose = fin_pose + 12 * (int64_t)q;
  long long in = 0;
  if (i < d.n && have) {
    const double X = gmem(d.full.X)[i], Y = gmem(d.full.Y)[i], Z = gmem(d.full.Z)[i];
    double x = pose[0] * X + pose[1] * Y + pose[2] * Z + pose[9];
    double y = pose[3] * X + pose[4] * Y + pose[5] * Z + pose[10];
    double z = pose[6] * X + pose[7] * Y + pose[8] * Z + pose[11];
    double fx = d.fx, fy = d.fy, cx = d.cx, cy = d.cy;
    if (d.ncam > 0) {  // through the point's rig camera
      const double* rc = d.rig + 16 * cam_of(d.segF, d.ncam, i);
      const double* Rc = rc + 4;
      const double xr[3] = {x, y, z};
      x = Rc[0] * xr[0] + Rc[1] * xr[1] + Rc[2] * xr[2] + rc[13];
      y = Rc[3] * xr[0] + Rc[4] * xr[1] + Rc[5] * xr[2] + rc[14];
      z = Rc[6] * xr[0] + Rc[7] * xr[1] + Rc[8] * xr[2] + rc[15];
      fx = rc[0]; fy = rc[1]; cx = rc[2]; cy = rc[3];
    }
    if (z > 0.0) {
      const double du = fx * x / z + cx - (double)gmem(d.full.u)[i];
      const double dv = fy * y / z + cy - (double)gmem(d.full.v)[i];
      in = (du * du + dv * dv < d.tau * d.tau) ? 1 : 0;
    }
  }
  if (i < d.n && d.mask) d.mask[i] = (uint8_t)in;
  const long long tot = wave_sum(in);
  if ((threadIdx.x & (kWave - 1)) == 0 && tot)
    atomicAdd((unsigned long long*)&st[q].full_count, (unsigned long long)tot);
}

hipError_t launch_mask(const QueryDesc* qd, BestState* st, const double* fin_pose, int nq, int64_t max_n, int all,
                       hipStream_t s) {
  if (nq <= 0 || max_n <= 0) return hipSuccess;
  hipLaunchKernelGGL(mask_kernel, dim3((unsigned)((max_n + 255) / 256), nq), dim3(256), 0, s, qd, st, fin_pose, all);
  return hipGetLastError();
}

}  // namespace imloc
