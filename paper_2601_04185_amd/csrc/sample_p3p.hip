// sample_p3p.hip -- minimal sampling (Philox4x64-10) and float64 P3P, four
// lanes per sample (generalised P3P of rig queries: eight lanes per sample),
// candidates compacted per workgroup (ImLoc Sec. 3.3, "Pose Estimation":
// batches of minimal sets, P3P hypotheses).
#include "gp3p_device.h"
#include "imloc_device.h"
#include "imloc_kernels.h"
#include "query_device.h"

namespace imloc {


// P3P: four lanes per sample (a workgroup of four waves holds 64 samples).
// The four lanes of a sample draw the same minimal set and build the same
// conics; lanes 0 and 2 search det(D1 + g D2) for degenerate members, lanes
// 1 and 3 det(e D1 + D2), and the pair's better member (the first search's
// on ties) is exchanged through LDS; lane j then cuts slot j (line j / 2,
// intersection j % 2), and a scan over the four slots removes duplicates and
// gives the canonical order.
constexpr int kP3PLanes = 4;
constexpr int kP3PThreads = 256;  // four waves, 64 samples: one slot reservation per 64 samples
constexpr int kP3PSamples = kP3PThreads / kP3PLanes;

// grid (sample blocks, queries): the lanes 4 g .. 4 g + 3 of block b of query
// q work on sample drawn_q + 64 b + g.
__global__ __launch_bounds__(kP3PThreads) void sample_p3p_kernel(const QueryDesc* __restrict__ qd,
                                                               const BestState* __restrict__ st, CandBuf cb,
                                                               int32_t* __restrict__ triples) {
  const int q = blockIdx.y;
  const QueryDesc& d = qd[q];
  if (d.ncam > 0) return;  // rig queries: sample_gp3p_kernel
  const int64_t count = d.B;
  const int64_t s0 = (int64_t)blockIdx.x * kP3PSamples;
  if (s0 >= count) return;
  const int grp = threadIdx.x / kP3PLanes, j = threadIdx.x % kP3PLanes;
  const int64_t s = s0 + grp;
  const int64_t h0 = st[q].drawn;
  const Cam K{d.fx, d.fy, d.cx, d.cy};
  __shared__ double s_q[kP3PThreads], s_root[kP3PThreads];
  __shared__ int s_ok[kP3PThreads];
  __shared__ double s_l[5][kP3PThreads];
  const int g0 = kP3PLanes * grp;
  double y[3][3], x[3][3];
  double l[3] = {0.0, 0.0, 0.0};
  bool keep = false;
  int rank = 0;
  if (s < count) {  // uniform over the four lanes of a sample from here on
    const uint64_t h = (uint64_t)(h0 + s);
    int idx[3] = {-1, -1, -1};
    const bool ok = d.exhaustive ? unrank_triple(h, (uint64_t)d.m, idx)
                                 : sample_triple(d.seed, d.qid, h, (uint64_t)d.m, idx);
    if (triples && j < 3) triples[3 * s + j] = ok ? idx[j] : -1;
    P3PSetup su;
    if (ok) {
      for (int k = 0; k < 3; ++k) {
        const int i = idx[k];
        const double bx = ((double)d.S.u[i] - K.cx) / K.fx, by = ((double)d.S.v[i] - K.cy) / K.fy;
        const double inv = 1.0 / sqrt(bx * bx + by * by + 1.0);
        y[k][0] = bx * inv; y[k][1] = by * inv; y[k][2] = inv;
        x[k][0] = d.S.X[i]; x[k][1] = d.S.Y[i]; x[k][2] = d.S.Z[i];
      }
    }
    if (ok && p3p_setup(y, x, su)) {
      // the best degenerate member of this lane's search, then of the pair
      double root = 0.0;
      const double mq = p3p_best_member(su, (j & 1) == 0, root);
      s_q[threadIdx.x] = mq;
      s_root[threadIdx.x] = root;
      __syncwarp();
      const double q1 = s_q[g0], q2 = s_q[g0 + 1];
      const bool from_f = !(q2 > q1);
      const double best_root = from_f ? s_root[g0] : s_root[g0 + 1];
      __syncwarp();
      int okj = 0;
      double k0 = __builtin_inf(), k1 = __builtin_inf();
      if (q1 > 0.0 || q2 > 0.0) {
        double D0[9], T = 0.0, S = 0.0;
        p3p_member(su, best_root, from_f, D0, T, S);
        okj = p3p_slot(su, D0, T, S, from_f, j, l) ? 1 : 0;
        if (okj) {
          k0 = l[0] * y[0][2];
          k1 = l[1] * y[1][2];
        }
      }
      s_ok[threadIdx.x] = okj;
      s_l[0][threadIdx.x] = l[0];
      s_l[1][threadIdx.x] = l[1];
      s_l[2][threadIdx.x] = l[2];
      s_l[3][threadIdx.x] = k0;
      s_l[4][threadIdx.x] = k1;
      __syncwarp();
      keep = p3p_keep_rank(s_ok + g0, s_l[0] + g0, s_l[1] + g0, s_l[2] + g0, s_l[3] + g0, s_l[4] + g0, j, rank);
    }
  }
  // candidate slots: one per kept solution of the workgroup, in lane order
  // (workgroups append in completion order -- the order of the candidates
  // never enters a result)
  constexpr int kWaves = kP3PThreads / kWave;
  __shared__ int s_wcnt[kWaves], s_base;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const uint64_t kept = __ballot(keep);
  if (lane == 0) s_wcnt[wave] = __popcll(kept);
  __syncthreads();
  if (threadIdx.x == 0) {
    int total = 0;
    for (int w = 0; w < kWaves; ++w) total += s_wcnt[w];
    s_base = total > 0 ? atomicAdd(&cb.n[q], total) : 0;
  }
  __syncthreads();
  if (!keep) return;
  int before = 0;
  for (int w = 0; w < wave; ++w) before += s_wcnt[w];
  const int64_t local = s_base + before + __popcll(kept & ((1ull << lane) - 1ull));
  const int64_t o = d.cand_off + local;
  double Xi[9];
  p3p_frame_inverse(x, Xi);
  Pose P;
  p3p_pose(l, y, x, Xi, P);
  for (int e = 0; e < 9; ++e) cb.pose[12 * o + e] = P.R[e];
  for (int e = 0; e < 3; ++e) cb.pose[12 * o + 9 + e] = P.t[e];
  write_candidate_rows(d, cb.proj, local, P);
  cb.h[o] = h0 + s;
  cb.j[o] = rank;
  cb.cnt[o] = 0;
  cb.gain[o] = 0;
}

// Generalised P3P for rig queries: eight lanes per sample (a one-wave
// workgroup holds eight samples).  The eight lanes of a sample draw the same
// minimal set and build the same resultant; lane j refines the root of piece j
// at every level of the derivative splitting, lifts final root j to depths,
// and writes solution j, the per-level results being exchanged through LDS
// within the wave.
constexpr int kGP3PLanes = 8;
// One wave (eight samples) per workgroup: a round of 2,048 samples is 256
// waves, and one per CU runs faster than four per CU on a quarter of the CUs.
constexpr int kGP3PThreads = 64;
constexpr int kGP3PSamples = kGP3PThreads / kGP3PLanes;

// Levels DEG..D of the derivative splitting of the degree-D resultant c on
// lane j; kind/root: the sample's eight LDS slots.
template <int D, int DEG>
__device__ inline void gp3p_levels(const double* c, int j, int* kind, double* root, double& a, double& b,
                                   bool& counted, double& r) {
  double p[DEG + 1], dp[DEG];
  deriv_coeffs<D, D - DEG>(c, p);
  deriv_coeffs<D, D - DEG + 1>(c, dp);
  double x = 0.0;
  const int k = j < DEG ? piece_root<DEG>(p, dp, a, b, j == DEG - 1, x) : 0;
  kind[j] = k;
  root[j] = x;
  __syncwarp();
  level_scan<DEG>(kind, root, j, a, b, counted);
  r = x;
  __syncwarp();
  if constexpr (DEG < D) gp3p_levels<D, DEG + 1>(c, j, kind, root, a, b, counted, r);
}

template <int D>
__device__ inline bool gp3p_root(const double* c, int j, int* kind, double* root, double& r) {
  double a = -1.0, b = 1.0;
  bool counted = false;
  gp3p_levels<D, 1>(c, j, kind, root, a, b, counted, r);
  return j < D && counted;
}

// grid (sample blocks, queries): the lanes 8 g .. 8 g + 7 of block b of query
// q work on sample drawn_q + 8 b + g.
__global__ __launch_bounds__(kGP3PThreads) void sample_gp3p_kernel(const QueryDesc* __restrict__ qd,
                                                                const BestState* __restrict__ st, CandBuf cb,
                                                                int32_t* __restrict__ triples) {
  const int q = blockIdx.y;
  const QueryDesc& d = qd[q];
  if (d.ncam == 0) return;
  const int64_t count = d.B;
  const int64_t s0 = (int64_t)blockIdx.x * kGP3PSamples;
  if (s0 >= count) return;
  const int grp = threadIdx.x / kGP3PLanes, j = threadIdx.x % kGP3PLanes;
  const int64_t s = s0 + grp;
  const int64_t h0 = st[q].drawn;
  __shared__ int s_kind[kGP3PThreads];
  __shared__ double s_val[3][kGP3PThreads];
  int* kind = s_kind + kGP3PLanes * grp;
  double* v0 = s_val[0] + kGP3PLanes * grp;
  double* v1 = s_val[1] + kGP3PLanes * grp;
  double* v2 = s_val[2] + kGP3PLanes * grp;
  GP3PIn g;
  double X[3][3];
  double l[3] = {0.0, 0.0, 0.0};
  bool keep = false;
  int rank = 0;
  if (s < count) {  // uniform over the eight lanes of a sample from here on
    const uint64_t h = (uint64_t)(h0 + s);
    int idx[3] = {-1, -1, -1};
    const bool ok = d.exhaustive ? unrank_triple(h, (uint64_t)d.m, idx)
                                 : sample_triple(d.seed, d.qid, h, (uint64_t)d.m, idx);
    if (triples && j < 3) triples[3 * s + j] = ok ? idx[j] : -1;
    if (ok) {
      for (int k = 0; k < 3; ++k) {
        const int i = idx[k];
        const double* rc = d.rig + 16 * cam_of(d.segS, d.ncam, i);
        const double* Rc = rc + 4;
        const double* tc = rc + 13;
        const double bx = ((double)d.S.u[i] - rc[2]) / rc[0], by = ((double)d.S.v[i] - rc[3]) / rc[1];
        double f[3];
        for (int c = 0; c < 3; ++c) {
          g.o[k][c] = -(Rc[c] * tc[0] + Rc[3 + c] * tc[1] + Rc[6 + c] * tc[2]);
          f[c] = Rc[c] * bx + Rc[3 + c] * by + Rc[6 + c];
        }
        const double inv = 1.0 / sqrt(dot3(f, f));
        for (int c = 0; c < 3; ++c) g.f[k][c] = f[c] * inv;
        X[k][0] = d.S.X[i]; X[k][1] = d.S.Y[i]; X[k][2] = d.S.Z[i];
      }
      const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
      for (int e = 0; e < 3; ++e) {
        double v[3];
        for (int c = 0; c < 3; ++c) v[c] = X[pa[e]][c] - X[pb[e]][c];
        g.d2[e] = dot3(v, v);
      }
      GP3PPoly y;
      const int deg = gp3p_poly(g, y);
      double r = 0.0;
      bool valid = false;
      switch (deg) {  // almost always 8; lower when leading coefficients vanish
        case 8: valid = gp3p_root<8>(y.oct, j, kind, v0, r); break;
        case 7: valid = gp3p_root<7>(y.oct, j, kind, v0, r); break;
        case 6: valid = gp3p_root<6>(y.oct, j, kind, v0, r); break;
        case 5: valid = gp3p_root<5>(y.oct, j, kind, v0, r); break;
        case 4: valid = gp3p_root<4>(y.oct, j, kind, v0, r); break;
        case 3: valid = gp3p_root<3>(y.oct, j, kind, v0, r); break;
        case 2: valid = gp3p_root<2>(y.oct, j, kind, v0, r); break;
        case 1: valid = gp3p_root<1>(y.oct, j, kind, v0, r); break;
        default: break;
      }
      const bool lifted = valid && gp3p_lift(g, y, r, l);
      kind[j] = lifted ? 1 : 0;
      v0[j] = l[0];
      v1[j] = l[1];
      v2[j] = l[2];
      __syncwarp();
      keep = gp3p_keep_rank<kGP3PLanes>(kind, v0, v1, v2, j, rank);
    }
  }
  // candidate slots: one per kept solution of the workgroup, in lane order
  constexpr int kWaves = kGP3PThreads / kWave;
  __shared__ int s_wcnt[kWaves], s_base;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const uint64_t kept = __ballot(keep);
  if (lane == 0) s_wcnt[wave] = __popcll(kept);
  __syncthreads();
  if (threadIdx.x == 0) {
    int total = 0;
    for (int w = 0; w < kWaves; ++w) total += s_wcnt[w];
    s_base = total > 0 ? atomicAdd(&cb.n[q], total) : 0;
  }
  __syncthreads();
  if (!keep) return;
  int before = 0;
  for (int w = 0; w < wave; ++w) before += s_wcnt[w];
  const int64_t local = s_base + before + __popcll(kept & ((1ull << lane) - 1ull));
  const int64_t o = d.cand_off + local;
  double P[3][3];
  for (int i = 0; i < 3; ++i)
    for (int c = 0; c < 3; ++c) P[i][c] = g.o[i][c] + l[i] * g.f[i][c];
  Pose pose;
  if (!gp3p_pose(P, X, pose)) {  // degenerate triangle: an identity placeholder never wins a score
    for (int e = 0; e < 9; ++e) pose.R[e] = (e % 4 == 0) ? 1.0 : 0.0;
    pose.t[0] = pose.t[1] = 0.0;
    pose.t[2] = -1e30;
  }
  for (int e = 0; e < 9; ++e) cb.pose[12 * o + e] = pose.R[e];
  for (int e = 0; e < 3; ++e) cb.pose[12 * o + 9 + e] = pose.t[e];
  write_candidate_rows(d, cb.proj, local, pose);
  cb.h[o] = h0 + s;
  cb.j[o] = rank;
  cb.cnt[o] = 0;
  cb.gain[o] = 0;
}

hipError_t launch_sample_p3p(const QueryDesc* qd, const BestState* st, CandBuf cb, int nq, int64_t max_b,
                             int32_t* triples, hipStream_t s) {
  if (nq <= 0 || max_b <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((max_b + kP3PSamples - 1) / kP3PSamples);
  hipLaunchKernelGGL(sample_p3p_kernel, dim3(blocks, nq), dim3(kP3PThreads), 0, s, qd, st, cb, triples);
  return hipGetLastError();
}

hipError_t launch_sample_gp3p(const QueryDesc* qd, const BestState* st, CandBuf cb, int nq, int64_t max_b,
                              int32_t* triples, hipStream_t s) {
  if (nq <= 0 || max_b <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((max_b + kGP3PSamples - 1) / kGP3PSamples);
  hipLaunchKernelGGL(sample_gp3p_kernel, dim3(blocks, nq), dim3(kGP3PThreads), 0, s, qd, st, cb, triples);
  return hipGetLastError();
}

// Candidates from given float64 poses (query 0).
__global__ void set_candidates_kernel(const QueryDesc* __restrict__ qd, const double* __restrict__ poses, int64_t np,
                                      CandBuf cb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) cb.n[0] = (int32_t)np;
  if (i >= np) return;
  const QueryDesc& d = qd[0];
  const int64_t o = d.cand_off + i;
  Pose P;
  for (int e = 0; e < 9; ++e) P.R[e] = poses[12 * i + e];
  for (int e = 0; e < 3; ++e) P.t[e] = poses[12 * i + 9 + e];
  for (int e = 0; e < 12; ++e) cb.pose[12 * o + e] = poses[12 * i + e];
  write_candidate_rows(d, cb.proj, i, P);
  cb.h[o] = i;
  cb.j[o] = 0;
  cb.cnt[o] = 0;
  cb.gain[o] = 0;
}

hipError_t launch_set_candidates(const QueryDesc* qd, const double* poses, int64_t np, CandBuf cb, hipStream_t s) {
  const int64_t n = np > 0 ? np : 1;
  hipLaunchKernelGGL(set_candidates_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, qd, poses, np, cb);
  return hipGetLastError();
}

}  // namespace imloc
