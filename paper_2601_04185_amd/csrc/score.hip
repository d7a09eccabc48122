// score.hip -- hypothesis scoring, the hot loop of LO-RANSAC (ImLoc Sec. 3.3:
// every pose hypothesis is scored against every scored correspondence by a
// confidence-weighted truncated squared reprojection error), and the
// per-query top-k selection of the candidates to refine.
//
// Work decomposition: a work item is (query, tile of CT candidates, chunk of
// 256 * PPL correspondences); persistent workgroups walk a device-side work
// list, so one launch covers any mix of queries.
//
// Layout: one lane per correspondence (PPL correspondences per lane kept in
// registers, coalesced structure-of-arrays loads).  A work item first stages
// its tile's projection rows in LDS; each wave then reads a candidate's rows
// with broadcast LDS loads into vector registers, so that every multiply-add
// of the loop has vector operands only (on gfx950 a multiply-add with a
// scalar-register operand issues about 1.7 times slower, one with a neg or
// abs modifier about 1.5 times).  The rows are K [R | t] with the first two
// divided by tau, and the observations enter divided by tau and negated, so
// per residual:
//   (a', b', w) = P' [X, 1]              9 FMA
//   du' = a' + (-u') w, dv' likewise     2 FMA
//   e' = du'^2 + dv'^2                   MUL + FMA    (= e / tau^2)
//   inlier iff e' - w |w| < 0            FMA + CMP    (one rounding; rejects w <= 0 and NaN)
// The inlier count is a wave ballot + popcount (scalar unit).  The truncated
// cost is MSAC = tau^2 (sum_i w_i - G), G = sum_in w_i (w |w| - e')/(w |w|),
// computed only in point slots whose ballot is not empty (a wave-uniform
// branch), so most candidates pay no reciprocal at all.
//
// Accumulation: each wave's partial G (a float sum over its fixed set of
// 64 * PPL correspondences) is converted once to fixed point (2^-32) and all
// partials are added with integer atomics, as are the counts.  Integer sums
// do not depend on the order, so a candidate's score is the same for any
// tiling, grid size or mix of queries.  The per-(candidate, wave) table in
// LDS starts at zero and only a wave block with inliers writes its entry (its
// count and float partial); the conversion to fixed point happens in the
// item's final reduction, off the candidate loop.
#include "imloc_device.h"
#include "imloc_kernels.h"
#include "query_device.h"

namespace imloc {

constexpr int kScoreBlock = 256;
constexpr int kScoreWaves = kScoreBlock / kWave;
constexpr int kScoreMaxRounds = kScoreMaxPoints / (kScoreWaves * kScoreWaveBlock);  // wave blocks per wave and item
static_assert(kScoreMaxRounds == 2, "a work item of 4,096 correspondences gives each wave two blocks");

// Sum over the 64 lanes of a full wave with DPP lane moves (pairs, quads,
// rows of 16 by shifts, then the row broadcasts 15 and 31); lane 63 ends with
// the total.  Every lane must be active.
template <int CTRL>
__device__ inline float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
__device__ inline float wave_scan_dpp(float x) {
  x += dpp_move<0xb1>(x);   // quad_perm [1, 0, 3, 2]
  x += dpp_move<0x4e>(x);   // quad_perm [2, 3, 0, 1]
  x += dpp_move<0x114>(x);  // row_shr:4
  x += dpp_move<0x118>(x);  // row_shr:8
  x += dpp_move<0x142>(x);  // row_bcast:15
  x += dpp_move<0x143>(x);  // row_bcast:31
  return x;  // lane 63 holds the total
}

// Correspondences per work item: `pts` in float32 scoring (a multiple of the
// 512-correspondence wave block), 256 * kScorePPL64 in float64 scoring.
__device__ inline int64_t chunk_pts(const QueryDesc& d, int pts) {
  return d.precision ? (int64_t)kScoreBlock * kScorePPL64 : (int64_t)pts;
}
__device__ inline int64_t chunks_of(const QueryDesc& d, int pts) {
  const int64_t per = chunk_pts(d, pts);
  int64_t c = 0;
  if (d.ncam == 0) {
    c = (d.m + per - 1) / per;
  } else {  // a rig: every camera's segment is chunked on its own
    for (int k = 0; k < d.ncam; ++k) c += (d.segS[k + 1] - d.segS[k] + per - 1) / per;
  }
  return c > 0 ? c : 1;
}

// Points [begin, end) and camera of chunk `chunk` of the scoring set.
struct ChunkRange {
  int64_t begin, end;
  int cam;
};
__device__ inline ChunkRange chunk_range(const QueryDesc& d, int64_t chunk, int pts) {
  const int64_t per = chunk_pts(d, pts);
  if (d.ncam == 0) return ChunkRange{chunk * per, d.m, 0};
  for (int k = 0; k < d.ncam; ++k) {
    const int64_t nch = (d.segS[k + 1] - d.segS[k] + per - 1) / per;
    if (chunk < nch) return ChunkRange{d.segS[k] + chunk * per, d.segS[k + 1], k};
    chunk -= nch;
  }
  return ChunkRange{0, 0, 0};
}


// Work list: items_q = tiles_q * chunks_q for queries sampling this round;
// item_off = exclusive prefix, item_off[nq] = total (one workgroup).  Also
// zeroes the round's selection counters (the selection follows the scoring).
__global__ __launch_bounds__(1024) void worklist_kernel(const QueryDesc* __restrict__ qd,
                                                        const int32_t* __restrict__ n_cand, int nq, int ct, int pts,
                                                        int64_t* __restrict__ item_off, int32_t* __restrict__ sel_done) {
  __shared__ long long s[1024];
  const int seg = (nq + 1023) / 1024;
  const int q0 = threadIdx.x * seg, q1 = min(nq, q0 + seg);
  long long sum = 0;
  for (int q = q0; q < q1; ++q) {
    const QueryDesc& d = qd[q];
    if (d.B > 0) sum += (long long)((n_cand[q] + ct - 1) / ct) * chunks_of(d, pts);
  }
  s[threadIdx.x] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const long long v = (int)threadIdx.x >= off ? s[threadIdx.x - off] : 0;
    __syncthreads();
    s[threadIdx.x] += v;
    __syncthreads();
  }
  long long run = s[threadIdx.x] - sum;
  for (int q = q0; q < q1; ++q) {
    item_off[q] = run;
    sel_done[q] = 0;
    const QueryDesc& d = qd[q];
    if (d.B > 0) run += (long long)((n_cand[q] + ct - 1) / ct) * chunks_of(d, pts);
  }
  if (threadIdx.x == 1023) item_off[nq] = s[1023];
}

hipError_t launch_worklist(const QueryDesc* qd, CandBuf cb, int nq, ScoreTune tune, int64_t* item_off,
                           hipStream_t s) {
  hipLaunchKernelGGL(worklist_kernel, dim3(1), dim3(1024), 0, s, qd, cb.n, nq, tune.ct, tune.pts, item_off,
                     cb.sel_done);
  return hipGetLastError();
}

// One float32 work item: CT candidates against pts correspondences.  The
// correspondences come in wave blocks of 512 (lane l, slot k: block start +
// 64 k + l); every (candidate, wave block) pair is scored by exactly one wave,
// whose count and gain partial (a float sum over that block, converted once
// to fixed point) are then added as integers, so the results do not depend on
// pts.  pts >= 2048: each wave takes blocks w, w + 4, ... for every
// candidate; pts < 2048: the waves split into 2048 / pts candidate groups,
// each of pts / 512 waves (one block each).  MULTI: pts > 2048, compiled
// apart (the loop over a wave's blocks costs registers the one-block form
// does not need).
template <int CT, bool MULTI>
__device__ __forceinline__ void score_item_f32(const QueryDesc& d, const float* __restrict__ proj,
                                               uint32_t* __restrict__ ccnt, unsigned long long* __restrict__ cgain,
                                               BestState* st, int64_t tile, int64_t chunk, int ncand, int pts,
                                               uint32_t (*s_cnt)[kScoreWaves],
                                               float (*s_part)[kScoreMaxRounds * kScoreWaves], uint32_t* s_item,
                                               float4 (*s_rows)[3]) {
  constexpr int PPL = kScorePPL32;
  // the wave index in a scalar register: the candidate range and the block
  // derived from it are wave-uniform, so the candidate loop stays scalar
  const int lane = threadIdx.x & (kWave - 1), wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const float inv_tau = (float)(1.0 / d.tau);
  const ChunkRange rg = chunk_range(d, chunk, pts);
  const int c0 = (int)(tile * CT);
  const int cend = min(CT, ncand - c0);
  const int nblk = pts / kScoreWaveBlock;  // wave blocks of the item
  const int groups = nblk >= kScoreWaves ? 1 : kScoreWaves / nblk;
  const int wpg = kScoreWaves / groups;    // waves per candidate group
  const int grp = wave / wpg, gsz = CT / groups;
  const int cg0 = grp * gsz, cg1 = min(cend, cg0 + gsz);
  const int rounds = MULTI ? nblk / kScoreWaves : 1;
  // the tile's projection rows into LDS: every wave then reads a candidate's
  // 12 values as three broadcast 16-byte LDS loads into vector registers
  // (a multiply-add with a scalar-register operand issues about 1.7 times
  // slower than one with vector operands only on this chip)
  {
    const int rows = rows_per_slot(d);
    const float4* __restrict__ pc =
        reinterpret_cast<const float4*>(proj + d.proj_off + 16 * ((int64_t)rows * c0 + rg.cam));
    for (int e = threadIdx.x; e < 3 * cend; e += kScoreBlock) {
      const int c = e / 3, r = e - 3 * c;
      s_rows[c][r] = pc[(int64_t)4 * rows * c + r];
    }
  }
  const auto U = gmem(d.S.u);
  const auto V = gmem(d.S.v);
  const auto X = gmem(d.S.X);
  const auto Y = gmem(d.S.Y);
  const auto Z = gmem(d.S.Z);
  const auto W = gmem(d.S.w);
  uint32_t item_cnt = 0;
  for (int r = 0; r < rounds; ++r) {
    const int blk = nblk >= kScoreWaves ? wave + r * kScoreWaves : wave % wpg;
    const int64_t base = rg.begin + (int64_t)blk * kScoreWaveBlock + lane;
    float pu[PPL], pv[PPL], px[PPL], py[PPL], pz[PPL], pw[PPL];
#pragma unroll
    for (int k = 0; k < PPL; ++k) {
      const int64_t i = base + (int64_t)k * kWave;
      if (i < rg.end) {
        // observations negated, so that du' = a' + pu w is a multiply-add without modifiers
        pu[k] = -(U[i] * inv_tau); pv[k] = -(V[i] * inv_tau); px[k] = X[i]; py[k] = Y[i]; pz[k] = Z[i];
        pw[k] = W ? W[i] : 1.0f;
      } else {  // a NaN residual is never an inlier
        pu[k] = __builtin_nanf(""); pv[k] = 0.f; px[k] = 0.f; py[k] = 0.f; pz[k] = 0.f; pw[k] = 0.f;
      }
    }
    if (r == 0) __syncthreads();  // the rows are staged
    for (int c = cg0; c < cg1; ++c) {
      // (the other waves of the SIMD cover the LDS latency)
      const float4 r0 = s_rows[c][0], r1 = s_rows[c][1], r2 = s_rows[c][2];
      uint32_t cnt = 0;
      uint64_t bal[PPL];
      float dd[PPL], ww[PPL];
#pragma unroll
      for (int k = 0; k < PPL; ++k) {
        const float a = fmaf(r0.z, pz[k], fmaf(r0.y, py[k], fmaf(r0.x, px[k], r0.w)));
        const float b = fmaf(r1.z, pz[k], fmaf(r1.y, py[k], fmaf(r1.x, px[k], r1.w)));
        const float w = fmaf(r2.z, pz[k], fmaf(r2.y, py[k], fmaf(r2.x, px[k], r2.w)));
        const float du = fmaf(pu[k], w, a), dv = fmaf(pv[k], w, b);
        // inlier iff e' < w |w|: the sign of e' - w |w| rounded once (rejects w <= 0 and NaN)
        dd[k] = fmaf(-w, fabsf(w), fmaf(dv, dv, du * du));
        ww[k] = w;
        bal[k] = __ballot(dd[k] < 0.f);
        cnt += (uint32_t)__popcll(bal[k]);
      }
      if (cnt) {  // G += w_i (w|w| - e') / (w|w|) over the inliers, point slots with no inlier skipped
        // (the empty volatile statements keep these wave-uniform branches as
        // branches: most candidates have no inlier in most slots)
        asm volatile("");
        float gain = 0.f;
#pragma unroll
        for (int k = 0; k < PPL; ++k) {
          if (bal[k]) {
            asm volatile("");
            const float t = ww[k] * fabsf(ww[k]);
            if (dd[k] < 0.f) gain = fmaf(-pw[k] * dd[k], __builtin_amdgcn_rcpf(t), gain);
          }
        }
        gain = wave_scan_dpp(gain);  // the block's total in lane 63
        if (lane == kWave - 1) {
          s_cnt[c][wave] = MULTI ? s_cnt[c][wave] + cnt : cnt;
          s_part[c][wave * kScoreMaxRounds + r] = gain;
        }
      }
      item_cnt += cnt;
    }
  }
  if (lane == 0) s_item[wave] = item_cnt;
  __syncthreads();
  if ((int)threadIdx.x < cend) {  // the waves of the candidate's group
    const int c = threadIdx.x, w0 = (c / gsz) * wpg;
    uint32_t cnt = 0;
    unsigned long long g = 0;
    for (int w = w0; w < w0 + wpg; ++w) {
      cnt += s_cnt[c][w];
      s_cnt[c][w] = 0;  // the table is empty again for the next item
      for (int r = 0; r < rounds; ++r) {  // each wave block's float partial to fixed point once
        const float p = s_part[c][w * kScoreMaxRounds + r];
        if (p != 0.f) g += (unsigned long long)((double)p * kGainScale);
        s_part[c][w * kScoreMaxRounds + r] = 0.f;
      }
    }
    const int64_t slot = d.cand_off + c0 + c;
    if (cnt) atomicAdd(&ccnt[slot], cnt);
    if (g) atomicAdd(&cgain[slot], g);
  }
  if (threadIdx.x == 0) {  // one add per item to the query's counter (same-address atomics serialise)
    unsigned long long tot = 0;
#pragma unroll
    for (int w = 0; w < kScoreWaves; ++w) tot += s_item[w];
    if (tot) atomicAdd((unsigned long long*)&st->inlier_residuals, tot);
  }
  __syncthreads();
}

// Float64 scoring (every step in double; the projection rows are formed from
// the float64 pose per candidate).
template <int CT>
__device__ __forceinline__ void score_item_f64(const QueryDesc& d, const double* __restrict__ pose,
                                               uint32_t* __restrict__ ccnt, unsigned long long* __restrict__ cgain,
                                               BestState* st, int64_t tile, int64_t chunk, int ncand,
                                               uint32_t (*s_cnt)[kScoreWaves],
                                               unsigned long long (*s_gain)[kScoreWaves], uint32_t* s_item) {
  constexpr int PPL = kScorePPL64;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const ChunkRange rg = chunk_range(d, chunk, 0);
  const int64_t base = rg.begin + wave * (kWave * PPL) + lane;
  const double tau2 = d.tau * d.tau;
  double pu[PPL], pv[PPL], px[PPL], py[PPL], pz[PPL], pw[PPL];
#pragma unroll
  for (int k = 0; k < PPL; ++k) {
    const int64_t i = base + (int64_t)k * kWave;
    if (i < rg.end) {
      pu[k] = gmem(d.S.u)[i]; pv[k] = gmem(d.S.v)[i]; px[k] = gmem(d.S.X)[i]; py[k] = gmem(d.S.Y)[i];
      pz[k] = gmem(d.S.Z)[i];
      pw[k] = d.S.w ? gmem(d.S.w)[i] : 1.0;
    } else {
      pu[k] = __builtin_nan(""); pv[k] = 0.0; px[k] = 0.0; py[k] = 0.0; pz[k] = 0.0; pw[k] = 0.0;
    }
  }
  const int c0 = (int)(tile * CT);
  const int cend = min(CT, ncand - c0);
  uint32_t item_cnt = 0;
  for (int c = 0; c < cend; ++c) {
    const double* q = pose + 12 * (d.cand_off + c0 + c);
    Pose Pp, Pc;
    for (int e = 0; e < 9; ++e) Pp.R[e] = q[e];
    for (int e = 0; e < 3; ++e) Pp.t[e] = q[9 + e];
    Cam K;
    camera_pose(d, rg.cam, Pp, Pc, K);
    double M[12];
    projection_rows(Pc, K, M);
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
    unsigned long long gfx = 0;
    if (cnt) {
      gain = wave_sum(gain);
      gfx = (unsigned long long)(gain * kGainScale);
    }
    item_cnt += cnt;
    if (lane == 0) {
      s_cnt[c][wave] = cnt;
      s_gain[c][wave] = gfx;
    }
  }
  if (lane == 0) s_item[wave] = item_cnt;
  __syncthreads();
  if ((int)threadIdx.x < cend) {
    const int c = threadIdx.x;
    uint32_t cnt = 0;
    unsigned long long g = 0;
#pragma unroll
    for (int w = 0; w < kScoreWaves; ++w) { cnt += s_cnt[c][w]; g += s_gain[c][w]; }
    const int64_t slot = d.cand_off + c0 + c;
    if (cnt) atomicAdd(&ccnt[slot], cnt);
    if (g) atomicAdd(&cgain[slot], g);
  }
  if (threadIdx.x == 0) {  // one add per item to the query's counter (same-address atomics serialise)
    unsigned long long tot = 0;
#pragma unroll
    for (int w = 0; w < kScoreWaves; ++w) tot += s_item[w];
    if (tot) atomicAdd((unsigned long long*)&st->inlier_residuals, tot);
  }
  __syncthreads();
}

// Persistent workgroups over the work list; every workgroup exits once the
// item index passes the device-side total.
template <int CT, bool MULTI>
__global__ __launch_bounds__(kScoreBlock) void score_kernel(const QueryDesc* __restrict__ qd,
                                                            const float* __restrict__ proj,
                                                            const double* __restrict__ pose,
                                                            const int32_t* __restrict__ ncand,
                                                            uint32_t* __restrict__ ccnt,
                                                            unsigned long long* __restrict__ cgain,
                                                            BestState* __restrict__ st, int nq, int pts,
                                                            const int64_t* __restrict__ item_off) {
  __shared__ uint32_t s_cnt[CT][kScoreWaves];    // float32 items
  __shared__ float s_part[CT][kScoreMaxRounds * kScoreWaves];
  __shared__ uint32_t s_cnt64[CT][kScoreWaves];  // float64 items
  __shared__ unsigned long long s_gain[CT][kScoreWaves];
  __shared__ uint32_t s_item[kScoreWaves];
  __shared__ float4 s_rows[CT][3];
  // the float32 (candidate, wave) table starts empty, and every item's final
  // reduction empties what it read: a wave block writes its entry only when it
  // holds inliers
  for (int e = threadIdx.x; e < CT * kScoreWaves; e += kScoreBlock) {
    (&s_cnt[0][0])[e] = 0;
#pragma unroll
    for (int r = 0; r < kScoreMaxRounds; ++r) (&s_part[0][0])[e * kScoreMaxRounds + r] = 0.f;
  }
  __syncthreads();
  const int64_t total = item_off[nq];
  for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
    int lo = 0, hi = nq - 1;  // the query owning item w: last q with item_off[q] <= w
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (item_off[mid] <= w) lo = mid; else hi = mid - 1;
    }
    const QueryDesc& d = qd[lo];
    const int64_t chunks = chunks_of(d, pts);
    const int64_t local = w - item_off[lo];
    const int64_t tile = local / chunks, chunk = local - tile * chunks;
    const int nc = ncand[lo];
    if (d.precision == 0)
      score_item_f32<CT, MULTI>(d, proj, ccnt, cgain, st + lo, tile, chunk, nc, pts, s_cnt, s_part, s_item,
                                s_rows);
    else
      score_item_f64<CT>(d, pose, ccnt, cgain, st + lo, tile, chunk, nc, s_cnt64, s_gain, s_item);
  }
}

hipError_t launch_score(const QueryDesc* qd, CandBuf cb, BestState* st, int nq, const int64_t* item_off,
                        ScoreTune tune, int precision, hipStream_t s) {
  (void)precision;
  const dim3 grid(tune.blocks > 0 ? tune.blocks : 2048), block(kScoreBlock);
  unsigned long long* g = reinterpret_cast<unsigned long long*>(cb.gain);
  const int pts = tune.pts;
  const bool multi = pts > kScoreBlock * kScorePPL32;
#define IMLOC_SCORE_LAUNCH(CT)                                                                                 \
  if (multi)                                                                                                   \
    hipLaunchKernelGGL((score_kernel<CT, true>), grid, block, 0, s, qd, cb.proj, cb.pose, cb.n, cb.cnt, g, st, nq, \
                       pts, item_off);                                                                         \
  else                                                                                                         \
    hipLaunchKernelGGL((score_kernel<CT, false>), grid, block, 0, s, qd, cb.proj, cb.pose, cb.n, cb.cnt, g, st,    \
                       nq, pts, item_off);
  switch (tune.ct) {
    case 128:
      IMLOC_SCORE_LAUNCH(128)
      break;
    case 64:
      IMLOC_SCORE_LAUNCH(64)
      break;
    default:
      IMLOC_SCORE_LAUNCH(32)
      break;
  }
#undef IMLOC_SCORE_LAUNCH
  return hipGetLastError();
}

__device__ inline double cand_msac(const QueryDesc& d, const BestState& b, uint64_t gain) {
  return d.tau * d.tau * (b.weight_sum - (double)gain * (1.0 / kGainScale));
}

__global__ void candidate_costs_kernel(const QueryDesc* __restrict__ qd, const BestState* __restrict__ st, CandBuf cb,
                                       int64_t np, int32_t* __restrict__ count, double* __restrict__ msac) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const int64_t o = qd[0].cand_off + i;
  count[i] = (int32_t)cb.cnt[o];
  msac[i] = cand_msac(qd[0], st[0], cb.gain[o]);
}

hipError_t launch_candidate_costs(const QueryDesc* qd, const BestState* st, CandBuf cb, int64_t np, int32_t* count,
                                  double* msac, hipStream_t s) {
  if (np <= 0) return hipSuccess;
  hipLaunchKernelGGL(candidate_costs_kernel, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, qd, st, cb, np,
                     count, msac);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Top-k of a query's batch by (msac asc, count desc, h asc, j asc) among the
// candidates whose truncated cost beats the running best.  One workgroup per
// query.
// ---------------------------------------------------------------------------
struct Key {
  double ms;
  long long hj;   // sample index * 4 + solution index
  int cnt, idx;
};

__device__ inline bool key_less(const Key& a, const Key& b) {
  if (a.ms != b.ms) return a.ms < b.ms;
  if (a.cnt != b.cnt) return a.cnt > b.cnt;
  return a.hj < b.hj;
}

__device__ inline Key key_none() { return Key{__builtin_inf(), 0x7fffffffffffffffll, -1, -1}; }

__device__ inline Key shfl_key(const Key& k, int lane_xor) {
  Key o;
  o.ms = __shfl_xor(k.ms, lane_xor, kWave);
  o.hj = __shfl_xor(k.hj, lane_xor, kWave);
  o.cnt = __shfl_xor(k.cnt, lane_xor, kWave);
  o.idx = __shfl_xor(k.idx, lane_xor, kWave);
  return o;
}

constexpr int kSelList = 8;      // per-thread list of the fast path (k <= 8)
constexpr int kSelUnroll = 4;    // candidates loaded together per thread
constexpr int kSelThreads = 256;
constexpr int kSelWaves = kSelThreads / kWave;
constexpr int kSelGroups = 16;   // phase-1 workgroups per query, at most
constexpr int kSelPerThread = 4; // phase-1 candidates per thread, about

__device__ inline Key load_key(const QueryDesc& d, const BestState& b, const CandBuf& cb, int c) {
  const int64_t o = d.cand_off + c;
  return Key{cand_msac(d, b, cb.gain[o]), (long long)cb.h[o] * 4 + cb.j[o], (int)cb.cnt[o], c};
}

// Order-preserving 64-bit image of a double (total order of the non-NaN
// values): equal images <=> equal values.
__device__ inline unsigned long long ms_order(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// 64-bit unsigned minimum over the wave, received by every lane.  Partners:
// lane ^ 32 and lane ^ 16 (swap instructions), lane ^ 8 (row_ror 8), lane ^ 7
// (row_half_mirror), lane ^ 2 and lane ^ 1 (quad_perm); together they cover
// the 64 lanes.  Every lane of the wave must be active.
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, 0xf, 0xf, false);
  return ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo;
}

__device__ __forceinline__ unsigned long long umin64(unsigned long long a, unsigned long long b) {
  return a < b ? a : b;
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
  {
    const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)v, (unsigned)v, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(v >> 32), (unsigned)(v >> 32), false, false);
    v = umin64(((unsigned long long)hi[0] << 32) | lo[0], ((unsigned long long)hi[1] << 32) | lo[1]);
  }
  {
    const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)v, (unsigned)v, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(v >> 32), (unsigned)(v >> 32), false, false);
    v = umin64(((unsigned long long)hi[0] << 32) | lo[0], ((unsigned long long)hi[1] << 32) | lo[1]);
  }
  v = umin64(v, dpp_u64<0x128>(v));
  v = umin64(v, dpp_u64<0x141>(v));
  v = umin64(v, dpp_u64<0x4e>(v));
  v = umin64(v, dpp_u64<0xb1>(v));
  return v;
}

// k rounds of "pop the smallest list head of the wave" over per-lane sorted
// lists of L keys; round r writes its key to out[r] (LDS, visible to the wave
// after a wave barrier).  A round takes the wave minimum of the 64-bit image
// of msac; only when several lanes hold that same msac do the full keys
// decide.  Returns the number of keys popped (< k when the lists run dry).
// Every lane of the wave must be active.
template <int L>
__device__ int wave_pop_k(Key (&list)[L], int k, Key* out) {
  const int lane = threadIdx.x & (kWave - 1);
  int r = 0;
  for (; r < k; ++r) {
    const Key head = list[0];
    const bool valid = head.idx >= 0;
    const unsigned long long pr = valid ? ms_order(head.ms) : ~0ull;
    const unsigned long long m = wave_min_u64(pr);
    const unsigned long long tie = __ballot(valid && pr == m);
    if (tie == 0) break;  // uniform: the lists ran dry
    int wl;
    if (__popcll(tie) == 1) {
      wl = __ffsll((long long)tie) - 1;
    } else {
      // several lanes share the smallest msac: full-key argmin among them
      Key bk = ((tie >> lane) & 1ull) ? head : key_none();
      int bl = ((tie >> lane) & 1ull) ? lane : -1;
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) {
        const Key o = shfl_key(bk, off);
        const int ol = __shfl_xor(bl, off, kWave);
        if (ol >= 0 && (bl < 0 || key_less(o, bk))) { bk = o; bl = ol; }
      }
      wl = __builtin_amdgcn_readfirstlane(bl);
    }
    if (lane == wl) {
      out[r] = head;
#pragma unroll
      for (int e = 0; e + 1 < L; ++e) list[e] = list[e + 1];
      list[L - 1] = key_none();
    }
  }
  __syncwarp();
  return r;
}

__device__ inline void list_insert(Key (&list)[kSelList], Key x) {
  if (!key_less(x, list[kSelList - 1])) return;
  // sorted insertion as a compare-and-swap pass (static register indices)
#pragma unroll
  for (int e = 0; e < kSelList; ++e) {
    if (key_less(x, list[e])) {
      const Key t = list[e];
      list[e] = x;
      x = t;
    }
  }
}

__host__ __device__ inline int select_groups(int64_t n_cand) {
  const int64_t g = (n_cand + kSelThreads * kSelPerThread - 1) / (kSelThreads * kSelPerThread);
  return g < 1 ? 1 : (g > kSelGroups ? kSelGroups : (int)g);
}

// Top k (k <= 8) in one launch: workgroup b of a query scans candidates
// b * 256 + t + j * G * 256, every thread keeps its best kSelList in
// registers, each wave pops its k smallest, wave 0 pops the workgroup's k
// smallest from the waves' lists and writes them to part[q][b][0..k)
// (key_none() past the end).  The last of the query's G workgroups to finish
// (counted in cb.sel_done) merges the G lists into the query's top k.
__global__ __launch_bounds__(kSelThreads) void select_kernel(const QueryDesc* __restrict__ qd,
                                                             BestState* __restrict__ st, CandBuf cb,
                                                             Key* __restrict__ part, int32_t* __restrict__ sel,
                                                             int32_t* __restrict__ n_sel) {
  const int q = blockIdx.y, b = blockIdx.x;
  const QueryDesc& d = qd[q];
  if (d.B <= 0) {
    if (b == 0 && threadIdx.x == 0) n_sel[q] = 0;
    return;
  }
  const int nc = cb.n[q];
  const int G = select_groups(d.cap);
  if (b >= G) return;
  const int k = d.k;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const BestState& bs = st[q];
  const double gate = bs.cost;
  Key list[kSelList];
#pragma unroll
  for (int e = 0; e < kSelList; ++e) list[e] = key_none();
  const int stride = G * kSelThreads;
  for (int c0 = b * kSelThreads + threadIdx.x; c0 < nc; c0 += kSelUnroll * stride) {
    Key xs[kSelUnroll];
#pragma unroll
    for (int u = 0; u < kSelUnroll; ++u) {
      const int c = c0 + u * stride;
      xs[u] = c < nc ? load_key(d, bs, cb, c) : key_none();
    }
#pragma unroll
    for (int u = 0; u < kSelUnroll; ++u)
      if (xs[u].idx >= 0 && xs[u].ms < gate) list_insert(list, xs[u]);
  }
  __shared__ Key s_wave[kSelWaves][kSelList];
  __shared__ int s_got[kSelWaves];
  __shared__ Key s_out[kSelList];
  const int got = wave_pop_k<kSelList>(list, k, s_wave[wave]);
  if (lane == 0) s_got[wave] = got;
  __syncthreads();
  if (wave != 0) return;
  // wave 0: the workgroup's k smallest from the waves' lists (one key per lane)
  Key one[1];
  one[0] = (lane < kSelWaves * k && lane % k < s_got[lane / k]) ? s_wave[lane / k][lane % k] : key_none();
  const int got_b = wave_pop_k<1>(one, k, s_out);
  Key* mine = part + ((int64_t)q * kSelGroups + b) * kSelList;
  if (lane < k) mine[lane] = lane < got_b ? s_out[lane] : key_none();
  // publish, then count this workgroup; the last one merges
  __threadfence();
  int last = 0;
  if (lane == 0) last = atomicAdd(&cb.sel_done[q], 1) == G - 1;
  if (!__builtin_amdgcn_readfirstlane(last)) return;
  __threadfence();
  // G * k <= 128 keys, two per lane, each pair sorted
  const Key* all = part + (int64_t)q * kSelGroups * kSelList;
  Key two[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int e = lane + u * kWave;
    two[u] = e < G * k ? all[(e / k) * kSelList + e % k] : key_none();
  }
  if (two[1].idx >= 0 && (two[0].idx < 0 || key_less(two[1], two[0]))) {
    const Key t = two[0];
    two[0] = two[1];
    two[1] = t;
  }
  const int got_q = wave_pop_k<2>(two, k, s_out);
  if (lane < got_q) sel[q * kMaxTopK + lane] = s_out[lane].idx;
  if (lane == 0) {
    n_sel[q] = got_q;
    st[q].candidates += nc;
  }
}

size_t select_scratch_bytes(int nq) {
  return (size_t)(nq > 0 ? nq : 1) * kSelGroups * kSelList * sizeof(Key);
}

// General path (k up to 32): k rounds of a workgroup argmin over all
// candidates not yet taken.
__global__ __launch_bounds__(256) void select_rounds_kernel(const QueryDesc* __restrict__ qd,
                                                            BestState* __restrict__ st, CandBuf cb,
                                                            int32_t* __restrict__ sel, int32_t* __restrict__ n_sel) {
  const int q = blockIdx.x;
  const QueryDesc& d = qd[q];
  if (d.B <= 0) {
    if (threadIdx.x == 0) n_sel[q] = 0;
    return;
  }
  const int nc = cb.n[q];
  const int k = d.k;
  const BestState& b = st[q];
  const double gate = b.cost;
  __shared__ int s_sel[kMaxTopK];
  __shared__ Key s_red[256];
  int r = 0;
  for (; r < k; ++r) {
    Key bi = key_none();
    for (int c = threadIdx.x; c < nc; c += 256) {
      const Key x = load_key(d, b, cb, c);
      if (!(x.ms < gate)) continue;
      bool taken = false;
      for (int t = 0; t < r; ++t) taken |= (s_sel[t] == c);
      if (taken) continue;
      if (bi.idx < 0 || key_less(x, bi)) bi = x;
    }
    s_red[threadIdx.x] = bi;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
      if ((int)threadIdx.x < off) {
        const Key a = s_red[threadIdx.x], bb = s_red[threadIdx.x + off];
        if (a.idx < 0 || (bb.idx >= 0 && key_less(bb, a))) s_red[threadIdx.x] = bb;
      }
      __syncthreads();
    }
    const int win = s_red[0].idx;
    __syncthreads();
    if (win < 0) break;
    if (threadIdx.x == 0) { s_sel[r] = win; sel[q * kMaxTopK + r] = win; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    n_sel[q] = r;
    st[q].candidates += nc;
  }
}

hipError_t launch_select(const QueryDesc* qd, const BestState* st, CandBuf cb, int nq, int kmax, int64_t max_cap,
                         void* scratch, int32_t* sel, int32_t* n_sel, hipStream_t s) {
  BestState* stw = const_cast<BestState*>(st);
  if (kmax <= kSelList) {
    Key* part = reinterpret_cast<Key*>(scratch);
    hipLaunchKernelGGL(select_kernel, dim3(select_groups(max_cap), nq), dim3(kSelThreads), 0, s, qd, stw, cb, part,
                       sel, n_sel);
  } else {
    hipLaunchKernelGGL(select_rounds_kernel, dim3(nq), dim3(256), 0, s, qd, stw, cb, sel, n_sel);
  }
  return hipGetLastError();
}

}  // namespace imloc
