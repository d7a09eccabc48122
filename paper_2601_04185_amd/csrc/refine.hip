// refine.hip -- float64 Gauss-Newton passes of LO-RANSAC (ImLoc Sec. 3.3):
//   local optimisation: non-linear refinement of the truncated squared
//     reprojection error of a new best hypothesis on the scoring set, the
//     inlier set re-evaluated at every iterate;
//   final refinement: robust Cauchy loss, weighted by the confidences, over
//     all inliers of the full set at the best pose (held fixed).
// One workgroup per problem; every pass accumulates the 6x6 normal equations
// (upper triangle), the gradient, the cost and the inlier count in float64
// with a fixed thread-to-point map and a fixed reduction tree, so the result
// is deterministic.  Residual r = pi(R X + t) - x; left update on SO(3).
#include "imloc_device.h"
#include "imloc_kernels.h"

namespace imloc {

constexpr int kGNBlock = 1024;
constexpr int kGNWaves = kGNBlock / kWave;
constexpr int kAcc = 29;  // 21 (H upper) + 6 (g) + cost + count

struct Acc {
  double v[kAcc];
};

__device__ inline void acc_point(Acc& a, const Cam& K, double x, double y, double z, double du, double dv, double wt) {
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
    for (int c = r; c < 6; ++c) { a.v[k] = fma(wt, J0[r] * J0[c] + J1[r] * J1[c], a.v[k]); ++k; }
  }
#pragma unroll
  for (int r = 0; r < 6; ++r) a.v[21 + r] = fma(wt, J0[r] * du + J1[r] * dv, a.v[21 + r]);
}

// MODE 0: truncated cost over all m points.  MODE 1: Cauchy over the set
// marked in in_set (built at the first pass when build is true).
template <int MODE>
__device__ void gn_pass(const CorrF32& c, int64_t m, const Cam& K, const Pose& P, double tau2, double s2,
                        uint8_t* in_set, bool build, double* s_tot) {
  Acc a;
#pragma unroll
  for (int e = 0; e < kAcc; ++e) a.v[e] = 0.0;
  for (int64_t i = threadIdx.x; i < m; i += kGNBlock) {
    const double X = c.X[i], Y = c.Y[i], Z = c.Z[i];
    const double w = c.w ? (double)c.w[i] : 1.0;
    const double x = P.R[0] * X + P.R[1] * Y + P.R[2] * Z + P.t[0];
    const double y = P.R[3] * X + P.R[4] * Y + P.R[5] * Z + P.t[1];
    const double z = P.R[6] * X + P.R[7] * Y + P.R[8] * Z + P.t[2];
    double du = 0.0, dv = 0.0, r2 = 0.0;
    const bool front = z > 0.0;
    if (front) {
      du = K.fx * x / z + K.cx - (double)c.u[i];
      dv = K.fy * y / z + K.cy - (double)c.v[i];
      r2 = du * du + dv * dv;
    }
    if (MODE == 0) {
      if (front && r2 < tau2) {
        a.v[27] += w * r2;
        a.v[28] += 1.0;
        acc_point(a, K, x, y, z, du, dv, w);
      } else {
        a.v[27] += w * tau2;
      }
    } else {
      if (build) in_set[i] = (front && r2 < tau2) ? 1 : 0;
      if (!in_set[i]) continue;
      a.v[28] += 1.0;
      if (!front) {
        a.v[27] += w * s2 * log1p(tau2 / s2);
        continue;
      }
      a.v[27] += w * s2 * log1p(r2 / s2);
      acc_point(a, K, x, y, z, du, dv, w / (1.0 + r2 / s2));
    }
  }
  __shared__ double s_part[kGNWaves][kAcc];
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
#pragma unroll
  for (int e = 0; e < kAcc; ++e) {
    const double v = wave_sum(a.v[e]);
    if (lane == 0) s_part[wave][e] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < kAcc) {
    double t = 0.0;
    for (int w = 0; w < kGNWaves; ++w) t += s_part[w][threadIdx.x];
    s_tot[threadIdx.x] = t;
  }
  __syncthreads();
}

template <int MODE>
__device__ void gn_run(const CorrF32& c, int64_t m, const Cam& K, const double* start, double tau2, double s2,
                       int iters, uint8_t* in_set, double* out_pose, double* out_cost, int64_t* out_count) {
  __shared__ double s_tot[kAcc];
  __shared__ double s_cur[12], s_cand[12];
  __shared__ double s_H[21], s_g[6];
  __shared__ int s_ok;
  if ((int)threadIdx.x < 12) s_cur[threadIdx.x] = start[threadIdx.x];
  __syncthreads();
  Pose P;
  for (int e = 0; e < 9; ++e) P.R[e] = s_cur[e];
  for (int e = 0; e < 3; ++e) P.t[e] = s_cur[9 + e];
  gn_pass<MODE>(c, m, K, P, tau2, s2, in_set, true, s_tot);
  double cur_cost = s_tot[27];
  double cur_cnt = s_tot[28];
  if ((int)threadIdx.x < 21) s_H[threadIdx.x] = s_tot[threadIdx.x];
  if ((int)threadIdx.x < 6) s_g[threadIdx.x] = s_tot[21 + threadIdx.x];
  __syncthreads();
  for (int it = 0; it < iters; ++it) {
    if (threadIdx.x == 0) {
      double b[6], d[6];
      for (int r = 0; r < 6; ++r) b[r] = -s_g[r];
      s_ok = chol6_solve_packed(s_H, b, d) ? 1 : 0;
      if (s_ok) {
        Pose Q;
        for (int e = 0; e < 9; ++e) Q.R[e] = s_cur[e];
        for (int e = 0; e < 3; ++e) Q.t[e] = s_cur[9 + e];
        Pose O;
        pose_left_update(Q, d, O);
        for (int e = 0; e < 9; ++e) s_cand[e] = O.R[e];
        for (int e = 0; e < 3; ++e) s_cand[9 + e] = O.t[e];
      }
    }
    __syncthreads();
    if (!s_ok) break;
    Pose Q;
    for (int e = 0; e < 9; ++e) Q.R[e] = s_cand[e];
    for (int e = 0; e < 3; ++e) Q.t[e] = s_cand[9 + e];
    gn_pass<MODE>(c, m, K, Q, tau2, s2, in_set, false, s_tot);
    const double new_cost = s_tot[27];
    if (!(new_cost <= cur_cost)) break;
    cur_cost = new_cost;
    cur_cnt = s_tot[28];
    if ((int)threadIdx.x < 12) s_cur[threadIdx.x] = s_cand[threadIdx.x];
    if ((int)threadIdx.x < 21) s_H[threadIdx.x] = s_tot[threadIdx.x];
    if ((int)threadIdx.x < 6) s_g[threadIdx.x] = s_tot[21 + threadIdx.x];
    __syncthreads();
  }
  if ((int)threadIdx.x < 12) out_pose[threadIdx.x] = s_cur[threadIdx.x];
  if (threadIdx.x == 0) {
    *out_cost = cur_cost;
    if (out_count) *out_count = (int64_t)cur_cnt;
  }
}

__global__ __launch_bounds__(kGNBlock) void lo_kernel(CorrF32 c, int64_t m, Cam K, double tau2, int iters,
                                                      const double* __restrict__ cand_pose,
                                                      const int32_t* __restrict__ sel,
                                                      const int32_t* __restrict__ n_sel, double* __restrict__ out_pose,
                                                      double* __restrict__ out_cost, int64_t* __restrict__ out_count) {
  const int q = blockIdx.x;
  if (n_sel && q >= *n_sel) return;
  const int src = sel ? sel[q] : q;
  gn_run<0>(c, m, K, cand_pose + 12 * (int64_t)src, tau2, 0.0, iters, nullptr, out_pose + 12 * q, out_cost + q,
            out_count ? out_count + q : nullptr);
}

hipError_t launch_lo(const CorrF32& c, int64_t m, CamH Kh, double tau, int32_t iters, const double* cand_pose,
                     const int32_t* sel, const int32_t* n_sel, int32_t k, double* out_pose, double* out_cost,
                     int64_t* out_count, hipStream_t s) {
  if (k <= 0) return hipSuccess;
  Cam K{Kh.fx, Kh.fy, Kh.cx, Kh.cy};
  hipLaunchKernelGGL(lo_kernel, dim3(k), dim3(kGNBlock), 0, s, c, m, K, tau * tau, iters, cand_pose, sel, n_sel,
                     out_pose, out_cost, out_count);
  return hipGetLastError();
}

__global__ __launch_bounds__(kGNBlock) void refine_kernel(CorrF32 c, int64_t n, Cam K, double tau2, double s2,
                                                          int iters, const double* __restrict__ start,
                                                          uint8_t* __restrict__ in_set, double* __restrict__ out_pose,
                                                          double* __restrict__ out_cost) {
  gn_run<1>(c, n, K, start, tau2, s2, iters, in_set, out_pose, out_cost, nullptr);
}

hipError_t launch_refine(const CorrF32& c, int64_t n, CamH Kh, double tau, double scale, int32_t iters,
                         const double* start, uint8_t* in_set, double* out_pose, double* out_cost, hipStream_t s) {
  Cam K{Kh.fx, Kh.fy, Kh.cx, Kh.cy};
  hipLaunchKernelGGL(refine_kernel, dim3(1), dim3(kGNBlock), 0, s, c, n, K, tau * tau, scale * scale, iters, start,
                     in_set, out_pose, out_cost);
  return hipGetLastError();
}

// Inlier mask over all points at a pose (float64), and its count.
__global__ void mask_kernel(CorrF32 c, int64_t n, Cam K, double tau2, const double* __restrict__ pose,
                            uint8_t* __restrict__ mask, int64_t* __restrict__ count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  long long in = 0;
  if (i < n) {
    const double X = c.X[i], Y = c.Y[i], Z = c.Z[i];
    const double x = pose[0] * X + pose[1] * Y + pose[2] * Z + pose[9];
    const double y = pose[3] * X + pose[4] * Y + pose[5] * Z + pose[10];
    const double z = pose[6] * X + pose[7] * Y + pose[8] * Z + pose[11];
    if (z > 0.0) {
      const double du = K.fx * x / z + K.cx - (double)c.u[i];
      const double dv = K.fy * y / z + K.cy - (double)c.v[i];
      in = (du * du + dv * dv < tau2) ? 1 : 0;
    }
    if (mask) mask[i] = (uint8_t)in;
  }
  const long long tot = wave_sum(in);
  if ((threadIdx.x & (kWave - 1)) == 0 && tot && count) atomicAdd((unsigned long long*)count, (unsigned long long)tot);
}

hipError_t launch_mask(const CorrF32& c, int64_t n, CamH Kh, double tau, const double* pose, uint8_t* mask,
                       int64_t* count, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  Cam K{Kh.fx, Kh.fy, Kh.cx, Kh.cy};
  hipLaunchKernelGGL(mask_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, c, n, K, tau * tau, pose, mask,
                     count);
  return hipGetLastError();
}

// Running best after a batch's local optimisations: in selection order, a
// strictly lower refined cost replaces the best.
__global__ void update_best_kernel(const int64_t* __restrict__ ch, const int32_t* __restrict__ cj,
                                   const int32_t* __restrict__ sel, const int32_t* __restrict__ n_sel,
                                   const double* __restrict__ lo_pose, const double* __restrict__ lo_cost,
                                   const int64_t* __restrict__ lo_count, BestState* st) {
  if (threadIdx.x != 0) return;
  const int ns = *n_sel;
  for (int q = 0; q < ns; ++q) {
    if (lo_cost[q] < st->cost) {
      st->cost = lo_cost[q];
      st->count = lo_count[q];
      for (int e = 0; e < 12; ++e) st->pose[e] = lo_pose[12 * q + e];
      st->h = ch[sel[q]];
      st->j = cj[sel[q]];
      st->have = 1;
    }
  }
  st->lo_runs += ns;
}

hipError_t launch_update_best(const CandBuf& cb, const int32_t* sel, const int32_t* n_sel, const double* lo_pose,
                              const double* lo_cost, const int64_t* lo_count, BestState* st, hipStream_t s) {
  hipLaunchKernelGGL(update_best_kernel, dim3(1), dim3(64), 0, s, cb.h, cb.j, sel, n_sel, lo_pose, lo_cost, lo_count,
                     st);
  return hipGetLastError();
}

__global__ void init_state_kernel(BestState* st) {
  if (threadIdx.x != 0) return;
  for (int e = 0; e < 12; ++e) st->pose[e] = (e == 0 || e == 4 || e == 8) ? 1.0 : 0.0;
  st->cost = __builtin_inf();
  st->count = 0;
  st->h = -1;
  st->j = -1;
  st->have = 0;
  st->lo_runs = 0;
  st->candidates = 0;
  st->inlier_residuals = 0;
  st->weight_sum = 0.0;
  st->final_cost = 0.0;
  st->full_count = 0;
}

hipError_t launch_init_state(BestState* st, hipStream_t s) {
  hipLaunchKernelGGL(init_state_kernel, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

}  // namespace imloc
