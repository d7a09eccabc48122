// score.hip -- hypothesis scoring, the hot loop of LO-RANSAC (ImLoc Sec. 3.3:
// every pose hypothesis is scored against every scored correspondence by a
// confidence-weighted truncated squared reprojection error).
//
// Layout: one lane per correspondence (PPL correspondences per lane kept in
// registers, coalesced structure-of-arrays loads), candidates wave-uniform so
// their projection rows live in scalar registers.  The rows are K [R | t] with
// the first two divided by tau, and the observations enter divided by tau, so
// per residual:
//   (a', b', w) = P' [X, 1]              9 FMA
//   du' = a' - u' w, dv' = b' - v' w     2 FMA
//   e' = du'^2 + dv'^2                   MUL + FMA    (= e / tau^2)
//   inlier iff e' < w |w|                MUL + CMP    (division-free; rejects w <= 0)
// The inlier count is a wave ballot + popcount (scalar unit).  The truncated
// cost is accumulated as MSAC = tau^2 (sum_i w_i - sum_in w_i (1 - e'/(w |w|))),
// so only inlier lanes of a wave with at least one inlier pay a reciprocal.
// Partial sums are written per (candidate, point chunk) and reduced in chunk
// order, so results do not depend on scheduling.
#include "imloc_device.h"
#include "imloc_kernels.h"

namespace imloc {

constexpr int kScoreBlock = 256;
constexpr int kScoreWaves = kScoreBlock / kWave;

// Copy a wave-uniform value into a vector register once, so that FMAs taking
// two uniform operands do not re-materialise it for every residual.
__device__ inline float to_vgpr(float x) {
  float r;
  asm("v_mov_b32 %0, %1" : "=v"(r) : "s"(x));
  return r;
}

// Projection rows are stored pre-divided by tau in their first two rows
// (a' = a / tau, b' = b / tau), and the observations enter as u / tau, v / tau:
// then e' = du'^2 + dv'^2 = e / tau^2 and the inlier test is e' < w |w|.
template <int PPL, int CT>
__global__ __launch_bounds__(kScoreBlock) void score_f32_kernel(
    const float* __restrict__ U, const float* __restrict__ V, const float* __restrict__ X,
    const float* __restrict__ Y, const float* __restrict__ Z, const float* __restrict__ W, int64_t m,
    const float* __restrict__ P, const int32_t* __restrict__ n_cand, float inv_tau, int64_t cap,
    uint32_t* __restrict__ part_cnt, float* __restrict__ part_gain) {
  const int ncand = *n_cand;
  const int tile0 = blockIdx.y * CT;
  if (tile0 >= ncand) return;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int64_t base = (int64_t)blockIdx.x * (kScoreBlock * PPL) + wave * (kWave * PPL) + lane;
  float pu[PPL], pv[PPL], px[PPL], py[PPL], pz[PPL], pw[PPL];
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const int64_t i = base + (int64_t)k * kWave;
    if (i < m) {
      pu[k] = U[i] * inv_tau; pv[k] = V[i] * inv_tau; px[k] = X[i]; py[k] = Y[i]; pz[k] = Z[i];
      pw[k] = W ? W[i] : 1.0f;
    } else {  // a NaN residual is never an inlier
      pu[k] = __builtin_nanf(""); pv[k] = 0.f; px[k] = 0.f; py[k] = 0.f; pz[k] = 0.f; pw[k] = 0.f;
    }
  }
  __shared__ uint32_t s_cnt[CT][kScoreWaves];
  __shared__ float s_gain[CT][kScoreWaves];
  const int cend = min(CT, ncand - tile0);
  const float4* pc = reinterpret_cast<const float4*>(P + 16 * (int64_t)tile0);
  float4 n0 = pc[0], n1 = pc[1], n2 = pc[2];
  for (int c = 0; c < cend; ++c) {
    const float4 r0 = n0, r1 = n1, r2 = n2;
    if (c + 1 < cend) {  // prefetch the next candidate's rows
      n0 = pc[4 * (c + 1)]; n1 = pc[4 * (c + 1) + 1]; n2 = pc[4 * (c + 1) + 2];
    }
    const float o0 = to_vgpr(r0.w), o1 = to_vgpr(r1.w), o2 = to_vgpr(r2.w);
    uint32_t cnt = 0;
    uint64_t any = 0;
    float e[PPL], t[PPL];
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      const float a = fmaf(r0.z, pz[k], fmaf(r0.y, py[k], fmaf(r0.x, px[k], o0)));
      const float b = fmaf(r1.z, pz[k], fmaf(r1.y, py[k], fmaf(r1.x, px[k], o1)));
      const float w = fmaf(r2.z, pz[k], fmaf(r2.y, py[k], fmaf(r2.x, px[k], o2)));
      const float du = fmaf(-pu[k], w, a), dv = fmaf(-pv[k], w, b);
      e[k] = fmaf(dv, dv, du * du);
      t[k] = w * fabsf(w);
      const uint64_t bal = __ballot(e[k] < t[k]);
      cnt += (uint32_t)__popcll(bal);
      any |= bal;
    }
    float gain = 0.f;
    if (any) {
#pragma unroll
      for (int k = 0; k < PPL; ++k)
        if (e[k] < t[k]) gain = fmaf(pw[k], fmaf(-e[k], __builtin_amdgcn_rcpf(t[k]), 1.0f), gain);
      gain = wave_sum(gain);
    }
    if (lane == 0) {
      s_cnt[c][wave] = cnt;
      s_gain[c][wave] = gain;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < cend) {
    const int c = threadIdx.x;
    uint32_t cnt = 0;
    float gain = 0.f;
#pragma unroll
    for (int w = 0; w < kScoreWaves; ++w) { cnt += s_cnt[c][w]; gain += s_gain[c][w]; }
    part_cnt[(int64_t)blockIdx.x * cap + tile0 + c] = cnt;
    part_gain[(int64_t)blockIdx.x * cap + tile0 + c] = gain;
  }
}

// Float64 scoring (every step in double; the projection rows are formed from
// the float64 pose per candidate).
template <int PPL, int CT>
__global__ __launch_bounds__(kScoreBlock) void score_f64_kernel(
    const float* __restrict__ U, const float* __restrict__ V, const float* __restrict__ X,
    const float* __restrict__ Y, const float* __restrict__ Z, const float* __restrict__ W, int64_t m,
    const double* __restrict__ poses, const int32_t* __restrict__ n_cand, Cam K, double tau2, int64_t cap,
    uint32_t* __restrict__ part_cnt, double* __restrict__ part_gain) {
  const int ncand = *n_cand;
  const int tile0 = blockIdx.y * CT;
  if (tile0 >= ncand) return;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int64_t base = (int64_t)blockIdx.x * (kScoreBlock * PPL) + wave * (kWave * PPL) + lane;
  double pu[PPL], pv[PPL], px[PPL], py[PPL], pz[PPL], pw[PPL];
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const int64_t i = base + (int64_t)k * kWave;
    if (i < m) {
      pu[k] = U[i]; pv[k] = V[i]; px[k] = X[i]; py[k] = Y[i]; pz[k] = Z[i];
      pw[k] = W ? W[i] : 1.0;
    } else {
      pu[k] = __builtin_nan(""); pv[k] = 0.0; px[k] = 0.0; py[k] = 0.0; pz[k] = 0.0; pw[k] = 0.0;
    }
  }
  __shared__ uint32_t s_cnt[CT][kScoreWaves];
  __shared__ double s_gain[CT][kScoreWaves];
  const int cend = min(CT, ncand - tile0);
  for (int c = 0; c < cend; ++c) {
    const double* q = poses + 12 * (int64_t)(tile0 + c);
    Pose Pp;
    for (int e = 0; e < 9; ++e) Pp.R[e] = q[e];
    for (int e = 0; e < 3; ++e) Pp.t[e] = q[9 + e];
    double M[12];
    projection_rows(Pp, K, M);
    uint32_t cnt = 0;
    double gain = 0.0;
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      const double a = fma(M[2], pz[k], fma(M[1], py[k], fma(M[0], px[k], M[3])));
      const double b = fma(M[6], pz[k], fma(M[5], py[k], fma(M[4], px[k], M[7])));
      const double w = fma(M[10], pz[k], fma(M[9], py[k], fma(M[8], px[k], M[11])));
      const double du = fma(-pu[k], w, a), dv = fma(-pv[k], w, b);
      const double e = fma(dv, dv, du * du);
      const double t = (tau2 * w) * fabs(w);
      const bool in = e < t;
      const uint64_t bal = __ballot(in);
      if (bal) {
        cnt += (uint32_t)__popcll(bal);
        if (in) gain += pw[k] * (1.0 - e / t);
      }
    }
    if (cnt) gain = wave_sum(gain);
    if (lane == 0) {
      s_cnt[c][wave] = cnt;
      s_gain[c][wave] = gain;
    }
  }
  __syncthreads();
  if ((int)threadIdx.x < cend) {
    const int c = threadIdx.x;
    uint32_t cnt = 0;
    double gain = 0.0;
#pragma unroll
    for (int w = 0; w < kScoreWaves; ++w) { cnt += s_cnt[c][w]; gain += s_gain[c][w]; }
    part_cnt[(int64_t)blockIdx.x * cap + tile0 + c] = cnt;
    part_gain[(int64_t)blockIdx.x * cap + tile0 + c] = gain;
  }
}

ScorePlan plan_score(int64_t m, int64_t cand_cap, int precision) {
  ScorePlan p;
  if (precision == 0) {
    p.ppl = m > 65536 ? 8 : m > 16384 ? 4 : m > 4096 ? 2 : 1;
  } else {
    p.ppl = m > 65536 ? 4 : m > 8192 ? 2 : 1;
  }
  p.ct = 32;
  const int64_t per_block = (int64_t)kScoreBlock * p.ppl;
  p.chunks = (int)((m + per_block - 1) / per_block);
  if (p.chunks < 1) p.chunks = 1;
  p.tiles = (int)((cand_cap + p.ct - 1) / p.ct);
  if (p.tiles < 1) p.tiles = 1;
  p.cap = cand_cap;
  return p;
}

size_t score_partial_bytes(const ScorePlan& p) {
  return (size_t)p.chunks * (size_t)p.cap * (sizeof(uint32_t) + sizeof(double));
}

template <int PPL>
static void launch_f32(const CorrF32& c, int64_t m, float inv_tau, const ScorePlan& pl, const CandBuf& cb,
                       uint32_t* pc, float* pg, hipStream_t s) {
  hipLaunchKernelGGL((score_f32_kernel<PPL, 32>), dim3(pl.chunks, pl.tiles), dim3(kScoreBlock), 0, s, c.u, c.v, c.X,
                     c.Y, c.Z, c.w, m, cb.proj, cb.n, inv_tau, pl.cap, pc, pg);
}
template <int PPL>
static void launch_f64(const CorrF32& c, int64_t m, Cam K, double tau2, const ScorePlan& pl, const CandBuf& cb,
                       uint32_t* pc, double* pg, hipStream_t s) {
  hipLaunchKernelGGL((score_f64_kernel<PPL, 32>), dim3(pl.chunks, pl.tiles), dim3(kScoreBlock), 0, s, c.u, c.v, c.X,
                     c.Y, c.Z, c.w, m, cb.pose, cb.n, K, tau2, pl.cap, pc, pg);
}

hipError_t launch_score(const CorrF32& c, int64_t m, CamH Kh, double tau, int precision, const ScorePlan& pl,
                        const CandBuf& cb, uint32_t* part_cnt, float* part_gain, double* part_gain64,
                        hipStream_t s) {
  if (precision == 0) {
    const float inv_tau = (float)(1.0 / tau);
    switch (pl.ppl) {
      case 1: launch_f32<1>(c, m, inv_tau, pl, cb, part_cnt, part_gain, s); break;
      case 2: launch_f32<2>(c, m, inv_tau, pl, cb, part_cnt, part_gain, s); break;
      case 4: launch_f32<4>(c, m, inv_tau, pl, cb, part_cnt, part_gain, s); break;
      default: launch_f32<8>(c, m, inv_tau, pl, cb, part_cnt, part_gain, s); break;
    }
  } else {
    Cam K{Kh.fx, Kh.fy, Kh.cx, Kh.cy};
    const double tau2 = tau * tau;
    switch (pl.ppl) {
      case 1: launch_f64<1>(c, m, K, tau2, pl, cb, part_cnt, part_gain64, s); break;
      case 2: launch_f64<2>(c, m, K, tau2, pl, cb, part_cnt, part_gain64, s); break;
      default: launch_f64<4>(c, m, K, tau2, pl, cb, part_cnt, part_gain64, s); break;
    }
  }
  return hipGetLastError();
}

// One thread per candidate: partials summed in chunk order (float64).
__global__ void reduce_scores_kernel(const int32_t* __restrict__ n_cand, int chunks, int64_t cap,
                                     const uint32_t* __restrict__ part_cnt, const float* __restrict__ part_gain,
                                     const double* __restrict__ part_gain64, double tau2, BestState* st,
                                     int32_t* __restrict__ count, double* __restrict__ msac) {
  const int nc = *n_cand;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  long long cnt = 0;
  if (c < nc) {
    double g = 0.0;
    for (int ch = 0; ch < chunks; ++ch) {
      cnt += part_cnt[(int64_t)ch * cap + c];
      g += part_gain64 ? part_gain64[(int64_t)ch * cap + c] : (double)part_gain[(int64_t)ch * cap + c];
    }
    count[c] = (int32_t)cnt;
    msac[c] = tau2 * (st->weight_sum - g);
  }
  const long long tot = wave_sum(cnt);
  if ((threadIdx.x & (kWave - 1)) == 0 && tot) atomicAdd((unsigned long long*)&st->inlier_residuals, (unsigned long long)tot);
  if (c == 0) atomicAdd((unsigned long long*)&st->candidates, (unsigned long long)nc);
}

hipError_t launch_reduce_scores(const ScorePlan& pl, const CandBuf& cb, double tau, const uint32_t* part_cnt,
                                const float* part_gain, const double* part_gain64, int precision, BestState* st,
                                hipStream_t s) {
  const int64_t n = pl.cap;
  hipLaunchKernelGGL(reduce_scores_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, cb.n, pl.chunks,
                     pl.cap, part_cnt, part_gain, precision == 0 ? nullptr : part_gain64, tau * tau, st, cb.count,
                     cb.msac);
  return hipGetLastError();
}

// Sum of weights over the scoring set, float64, fixed order (one workgroup).
__global__ __launch_bounds__(1024) void weight_sum_kernel(const float* __restrict__ W, int64_t m, BestState* st) {
  double s = 0.0;
  if (W) {
    for (int64_t i = threadIdx.x; i < m; i += 1024) s += W[i];
  } else {
    for (int64_t i = threadIdx.x; i < m; i += 1024) s += 1.0;
  }
  s = wave_sum(s);
  __shared__ double sw[16];
  if ((threadIdx.x & 63) == 0) sw[threadIdx.x / 64] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += sw[w];
    st->weight_sum = t;
  }
}

hipError_t launch_weight_sum(const CorrF32& c, int64_t m, BestState* st, hipStream_t s) {
  hipLaunchKernelGGL(weight_sum_kernel, dim3(1), dim3(1024), 0, s, c.w, m, st);
  return hipGetLastError();
}

// Top-k of the batch by (msac asc, count desc, h asc, j asc) among candidates
// whose truncated cost beats the running best; k rounds of a workgroup argmin.
__device__ inline bool cand_less(int a, int b, const int32_t* cnt, const double* ms, const int64_t* h, const int32_t* j) {
  if (ms[a] != ms[b]) return ms[a] < ms[b];
  if (cnt[a] != cnt[b]) return cnt[a] > cnt[b];
  if (h[a] != h[b]) return h[a] < h[b];
  return j[a] < j[b];
}

constexpr int kSelBlock = 256;
constexpr int kMaxTopK = 32;

__global__ __launch_bounds__(kSelBlock) void select_kernel(const int32_t* __restrict__ n_cand,
                                                           const int32_t* __restrict__ cnt,
                                                           const double* __restrict__ ms,
                                                           const int64_t* __restrict__ ch,
                                                           const int32_t* __restrict__ cj, int k, const BestState* st,
                                                           int32_t* __restrict__ sel, int32_t* __restrict__ n_sel) {
  const int nc = *n_cand;
  const double gate = st->cost;
  __shared__ int s_sel[kMaxTopK];
  __shared__ int s_red[kSelBlock];
  int r = 0;
  for (; r < k; ++r) {
    int bi = -1;
    for (int c = threadIdx.x; c < nc; c += kSelBlock) {
      if (!(ms[c] < gate)) continue;
      bool taken = false;
      for (int q = 0; q < r; ++q) taken |= (s_sel[q] == c);
      if (taken) continue;
      if (bi < 0 || cand_less(c, bi, cnt, ms, ch, cj)) bi = c;
    }
    s_red[threadIdx.x] = bi;
    __syncthreads();
    for (int off = kSelBlock / 2; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) {
        const int a = s_red[threadIdx.x], b = s_red[threadIdx.x + off];
        if (a < 0 || (b >= 0 && cand_less(b, a, cnt, ms, ch, cj))) s_red[threadIdx.x] = b;
      }
      __syncthreads();
    }
    const int win = s_red[0];
    __syncthreads();
    if (win < 0) break;
    if (threadIdx.x == 0) { s_sel[r] = win; sel[r] = win; }
    __syncthreads();
  }
  if (threadIdx.x == 0) *n_sel = r;
}

hipError_t launch_select(const CandBuf& cb, int32_t k, const BestState* st, int32_t* sel, int32_t* n_sel,
                         hipStream_t s) {
  if (k > kMaxTopK) k = kMaxTopK;
  hipLaunchKernelGGL(select_kernel, dim3(1), dim3(kSelBlock), 0, s, cb.n, cb.count, cb.msac, cb.h, cb.j, k, st, sel,
                     n_sel);
  return hipGetLastError();
}

}  // namespace imloc
