// refine.hip -- float64 Gauss-Newton of LO-RANSAC (ImLoc Sec. 3.3, "Pose
// Estimation"):
//   local optimisation: Gauss-Newton on the truncated cost over the scoring
//     set, started from a candidate that beats the running best; the inlier
//     set is taken again at every iterate;
//   final refinement: IRLS on the Cauchy loss, each point weighted by its
//     confidence, over the inliers of the full set at the best pose (that set
//     stays fixed).
// Each Gauss-Newton iteration is one launch over (point chunk x problem)
// workgroups for every problem of a batch of queries (or, for large batches,
// an evaluation launch and a decision launch).  A workgroup accumulates the
// 6x6 normal equations (upper triangle), the gradient, the cost and the
// inlier count of a 512-point chunk in float64 with a fixed thread-to-point
// map and reduction tree; partial sums are combined in chunk order, so the
// result depends on the problem alone, not on the batch around it or the
// launch form.  The final refinement's first evaluation also compacts each
// chunk's in-set; its later evaluations take only those points (thread t:
// the chunk's t-th and (t + 256)-th in-set points).  Residual
// r = pi(R X + t) - x; left update on SO(3).
#include "imloc_device.h"
#include "imloc_kernels.h"

namespace imloc {

constexpr int kAcc = 29;  // 21 (H upper) + 6 (g) + cost + count
constexpr double kStepTol2 = 1e-20;  // squared length of a step that ends a run
constexpr int kGNThreads = 256;
constexpr int kGNWaves = kGNThreads / kWave;
constexpr int kGNPPT = 2;                       // points per thread per chunk
constexpr int kGNChunk = kGNThreads * kGNPPT;   // points per chunk (fixed: the summation order depends on n only)

// 1 / z for the per-point work of an evaluation (z > 0 and finite): the
// hardware reciprocal and two Newton steps, within about an ulp of the
// rounded quotient, in 5 instructions where a rounded division takes about
// 10.  Every launch form uses it, so they still agree bit for bit.
__device__ __forceinline__ double recip_pos(double z) {
  double r = __builtin_amdgcn_rcp(z);
  r = fma(r, fma(-z, r, 1.0), r);
  return fma(r, fma(-z, r, 1.0), r);
}

// Normal equations of one point, given iz = 1 / z of its camera coordinates.
// The rows of d(pixel)/d(dw, dt) are J0 = (a02 y, a00 z - a02 x, -a00 y, a00,
// 0, a02) and J1 = (a12 y - a11 z, -a12 x, a11 x, 0, a11, a12); the products
// with their structural zeros are left out (H[3][4] gets nothing).  W false:
// every weight is 1 (the local optimisation of queries without confidences),
// whose weighted rows are the rows themselves -- the same bits without the
// ten multiplications.
template <bool W>
__device__ inline void acc_point(double* a, const Cam& K, double x, double y, double z, double iz, double du,
                                 double dv, double wt) {
  const double a00 = K.fx * iz, a02 = -K.fx * x * iz * iz;
  const double a11 = K.fy * iz, a12 = -K.fy * y * iz * iz;
  const double J0[6] = {a02 * y, a00 * z - a02 * x, -a00 * y, a00, 0.0, a02};
  const double J1[6] = {-a11 * z + a12 * y, -a12 * x, a11 * x, 0.0, a11, a12};
  double W0[6], W1[6];
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    W0[r] = W ? wt * J0[r] : J0[r];
    W1[r] = W ? wt * J1[r] : J1[r];
  }
  int k = 0;
#pragma unroll
  for (int r = 0; r < 6; ++r) {
#pragma unroll
    for (int c = r; c < 6; ++c) {
      const bool z0 = r == 4 || c == 4, z1 = r == 3 || c == 3;
      if (!z0 && !z1) a[k] = fma(W0[r], J0[c], fma(W1[r], J1[c], a[k]));
      else if (!z0) a[k] = fma(W0[r], J0[c], a[k]);
      else if (!z1) a[k] = fma(W1[r], J1[c], a[k]);
      ++k;
    }
  }
#pragma unroll
  for (int r = 0; r < 6; ++r) {
    if (r == 4) a[21 + r] = fma(W1[r], dv, a[21 + r]);
    else if (r == 3) a[21 + r] = fma(W0[r], du, a[21 + r]);
    else a[21 + r] = fma(W0[r], du, fma(W1[r], dv, a[21 + r]));
  }
}

// The same for a rig camera: x_c = R_c x_r + t_c with the rig-frame point x_r
// moving under the left update of the rig pose, so the rows of d(pixel)/dx_c
// are carried through R_c: J = [x_r x r, r] for each row r of d(pixel)/dx_c R_c.
__device__ inline void acc_point_rig(double* a, const Cam& K, const double xr[3], double x, double y, double iz,
                                     const double* Rc, double du, double dv, double wt) {
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

// Per-problem Gauss-Newton state after a decision, double-buffered.
struct GNState {
  double cur[12];      // accepted pose
  double eval[12];     // pose the next evaluation runs at
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

// The final refinement's in-set, compacted per chunk by its first evaluation
// (the set stays fixed): a count per chunk (uint16, padded to 256 bytes), then
// per chunk the offsets in the chunk of its in-set points, in point order
// (uint16 x kGNChunk).  Later evaluations read only those points.
__host__ __device__ inline int64_t inset_head_bytes(int64_t C) { return (2 * C + 255) & ~int64_t(255); }
__host__ __device__ inline int64_t inset_bytes_for(int64_t n) {
  const int64_t C = chunks_for(n);
  return inset_head_bytes(C) + (int64_t)2 * kGNChunk * C;
}
int64_t gn_inset_bytes(int64_t n) { return inset_bytes_for(n); }

size_t gn_scratch_bytes(int nprob, int chunks_max) {
  if (nprob < 1) nprob = 1;
  if (chunks_max < 1) chunks_max = 1;
  return (((size_t)2 * nprob * sizeof(GNState) + 255) & ~size_t(255)) +
         (size_t)2 * nprob * chunks_max * kAcc * sizeof(double) + 256;
}

// Packed row-wise index of (r, c), r <= c, in the 21-entry upper triangle.
__host__ __device__ constexpr int upk(int r, int c) { return r * 6 - (r * (r - 1)) / 2 + (c - r); }

// A double moved across lanes by a DPP control (both 32-bit halves).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Exchange of lanes 32..63 of x with lanes 0..31 of y (swap16: odd 16-lane
// rows of x with even rows of y); then x + y holds, in a lane with that lane
// bit clear, the pair sum of x, and with it set, the pair sum of y.
__device__ __forceinline__ void swap32_f64(double& x, double& y) {
  const long long bx = __double_as_longlong(x), by = __double_as_longlong(y);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)bx, (unsigned)by, false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap((unsigned)(bx >> 32), (unsigned)(by >> 32), false, false);
  x = __longlong_as_double(((long long)hi[0] << 32) | (unsigned)lo[0]);
  y = __longlong_as_double(((long long)hi[1] << 32) | (unsigned)lo[1]);
}

__device__ __forceinline__ void swap16_f64(double& x, double& y) {
  const long long bx = __double_as_longlong(x), by = __double_as_longlong(y);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)bx, (unsigned)by, false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap((unsigned)(bx >> 32), (unsigned)(by >> 32), false, false);
  x = __longlong_as_double(((long long)hi[0] << 32) | (unsigned)lo[0]);
  y = __longlong_as_double(((long long)hi[1] << 32) | (unsigned)lo[1]);
}

// One halving level on lane bit B with the partner given by a DPP control:
// a lane keeps the lower half of the list if its bit is clear, the upper
// half if set, and adds what the partner (bit flipped) did not keep.
template <int CTRL, int H>
__device__ __forceinline__ void halve_dpp(double* v, bool upper) {
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const double send = upper ? v[i] : v[i + H];
    const double keep = upper ? v[i + H] : v[i];
    v[i] = keep + dpp_f64<CTRL>(send);
  }
}

// Wave sums of the 29 accumulators by recursive halving (about 125
// instructions instead of 29 separate reductions): after the six levels, lane
// l holds the wave total of entry l >> 1 (entries 29..31 are zero padding).
// Partners: lane ^ 32 and lane ^ 16 by the swap instructions, lane ^ 8
// (row_ror 8), lane ^ 7 (row_half_mirror: bit 2 flips, and the lanes already
// merged on bits 0..1 are all covered after the last two levels), lane ^ 2,
// lane ^ 1 (quad_perm).  The order of additions depends on the lane only.
__device__ __forceinline__ double wave_sum29(const double* a) {
  double v[32];
#pragma unroll
  for (int e = 0; e < 32; ++e) v[e] = e < kAcc ? a[e] : 0.0;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    double x = v[i], y = v[i + 16];
    swap32_f64(x, y);
    v[i] = x + y;
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    double x = v[i], y = v[i + 8];
    swap16_f64(x, y);
    v[i] = x + y;
  }
  const int lane = threadIdx.x & (kWave - 1);
  halve_dpp<0x128, 4>(v, (lane & 8) != 0);   // row_ror 8: lane ^ 8
  halve_dpp<0x141, 2>(v, (lane & 4) != 0);   // row_half_mirror: lane ^ 7
  halve_dpp<0x4e, 1>(v, (lane & 2) != 0);    // quad_perm [2, 3, 0, 1]: lane ^ 2
  return v[0] + dpp_f64<0xb1>(v[0]);         // quad_perm [1, 0, 3, 2]: lane ^ 1
}

// Inlier test of point i of the full set at a final pose (float64, through
// the point's rig camera for a rig query): depth > 0 and squared pixel
// residual below tau^2.  Shared by the mask kernel and the fused final
// refinement, so both give the same mask.
__device__ __forceinline__ bool mask_test(const QueryDesc& d, const double* pose, double X, double Y, double Z,
                                          double u, double v, int64_t i) {
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
  if (!(z > 0.0)) return false;
  const double du = fx * x / z + cx - u;
  const double dv = fy * y / z + cy - v;
  return du * du + dv * dv < d.tau * d.tau;
}

struct GNArgs {
  const QueryDesc* qd;
  CandBuf cb;
  const int32_t* sel;
  const int32_t* n_sel;
  const double* start_direct;
  BestState* bst;
  GNState* gst;
  double* part;
  uint8_t* in_set_all;
  double* out_pose;
  double* out_cost;
  int64_t* out_count;
  int kmax, cmax, nprob;
  int fuse_mask;  // final refinement: the launch that ends a run writes the mask of its chunk
};

// Problem p's query.  LO (MODE 0): problem p = q * kmax + slot starts from
// the slot-th selected candidate of query q; refinement (MODE 1): problem q
// starts from the query's best pose once it has finished sampling.
template <int MODE>
__device__ __forceinline__ int gn_query(const GNArgs& g, int p) {
  return MODE == 0 ? (g.start_direct ? 0 : p / g.kmax) : p;
}

// Whether problem p has work this round.
template <int MODE>
__device__ __forceinline__ bool gn_live(const GNArgs& g, int p, int q) {
  if (g.start_direct) return true;
  if (MODE == 0) return p - q * g.kmax < g.n_sel[q];
  return (g.bst[q].finished == 1) & (g.bst[q].have != 0);
}

// Start pose of a live problem.
template <int MODE>
__device__ __forceinline__ const double* gn_start(const GNArgs& g, int p, int q) {
  if (MODE == 0)
    return g.start_direct ? g.start_direct + 12 * (int64_t)p
                          : g.cb.pose + 12 * (g.qd[q].cand_off + g.sel[q * kMaxTopK + (p - q * g.kmax)]);
  return g.start_direct ? g.start_direct + 12 * (int64_t)q : g.bst[q].pose;
}

__device__ __forceinline__ const double* gn_part(const GNArgs& g, int buf, int p) {
  return g.part + ((int64_t)buf * g.nprob + p) * g.cmax * kAcc;
}

// The C chunk partial sums of one problem in a fixed order: thread (v, grp)
// adds chunks grp, grp + 8, ... of entry v in chunk order, then the eight
// group sums are added in group order.  The first 16 chunks of every thread
// (128 of the problem) are loaded at kernel entry by gn_part_issue, whose
// addresses need only the problem index, so their latency overlaps the
// descriptor loads; gn_part_sum adds them and loads any further ones.
struct GNPart {
  double x[16];
};

__device__ __forceinline__ void gn_part_issue(const double* part, int cmax, GNPart& r) {
  const int v = threadIdx.x % kAcc, grp = threadIdx.x / kAcc;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int c = grp + 8 * u;
    r.x[u] = (grp < 8 && c < cmax) ? part[(int64_t)c * kAcc + v] : 0.0;
  }
}

// Every thread calls it.
__device__ void gn_part_sum(const double* part, int C, const GNPart& r, double (*s_grp)[kAcc], double* s_tot) {
  const int v = threadIdx.x % kAcc, grp = threadIdx.x / kAcc;
  if (grp < 8) {
    double sum = 0.0;
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (grp + 8 * u < C) sum += r.x[u];
    for (int c0 = grp + 128; c0 < C; c0 += 128) {
      double x[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int c = c0 + 8 * u;
        x[u] = c < C ? part[(int64_t)c * kAcc + v] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (c0 + 8 * u < C) sum += x[u];
    }
    s_grp[grp][v] = sum;
  }
  __syncthreads();
  if ((int)threadIdx.x < kAcc) {
    double t = 0.0;
#pragma unroll
    for (int gg = 0; gg < 8; ++gg) t += s_grp[gg][threadIdx.x];
    s_tot[threadIdx.x] = t;
  }
  __syncthreads();
}

// Decision j of a run, on the sums of evaluation j at s.eval: the evaluated
// pose becomes the accepted one if its cost did not rise (at j = 0 it is the
// start); unless the iteration budget is spent, the normal equations at the
// accepted pose give the pose of evaluation j + 1.  A cost-raising step, or a
// system that is not positive definite, ends the run with the accepted pose.
// Run by the 64 lanes of wave 0 (every lane takes the same branches): every
// lane solves the 6 x 6 system itself (solve6_schur), and lane e < 12 forms
// element e of the next pose.  Returns true when this decision ends the run.
struct GNShared {
  double cur[12], eval[12];
  double cost, count;
  int done, accepted;
};

// H d = -g for the 6x6 normal equations given by tot (upper triangle of H,
// packed by rows, then g), through the Schur complement of the rotation
// block: H = [A B; B^T C], d_t = S^-1 (b_t - B^T A^-1 b_r) with S = C - B^T
// A^-1 B, d_r = A^-1 b_r - A^-1 B d_t; the 3x3 inverses by adjugates.  H is
// positive definite exactly when A and S are (leading minors checked); false
// otherwise.  Every lane solves it in its own registers: no lane exchanges,
// two divisions on the dependency chain.
__device__ __forceinline__ bool solve6_schur(const double* t, double x[6]) {
  const double h00 = t[0], h01 = t[1], h02 = t[2], h03 = t[3], h04 = t[4], h05 = t[5];
  const double h11 = t[6], h12 = t[7], h13 = t[8], h14 = t[9], h15 = t[10];
  const double h22 = t[11], h23 = t[12], h24 = t[13], h25 = t[14];
  const double h33 = t[15], h34 = t[16], h35 = t[17], h44 = t[18], h45 = t[19], h55 = t[20];
  const double br[3] = {-t[21], -t[22], -t[23]}, bt[3] = {-t[24], -t[25], -t[26]};
  // A^-1 by its adjugate
  const double c00 = fma(h11, h22, -h12 * h12), c01 = fma(h02, h12, -h01 * h22), c02 = fma(h01, h12, -h02 * h11);
  const double c11 = fma(h00, h22, -h02 * h02), c12 = fma(h01, h02, -h00 * h12), c22 = fma(h00, h11, -h01 * h01);
  const double detA = fma(h00, c00, fma(h01, c01, h02 * c02));
  const bool okA = h00 > 0.0 && c22 > 0.0 && detA > 0.0;
  const double ia = 1.0 / detA;
  const double I[3][3] = {{c00 * ia, c01 * ia, c02 * ia}, {c01 * ia, c11 * ia, c12 * ia}, {c02 * ia, c12 * ia, c22 * ia}};
  const double B[3][3] = {{h03, h04, h05}, {h13, h14, h15}, {h23, h24, h25}};
  const double C[3][3] = {{h33, h34, h35}, {h34, h44, h45}, {h35, h45, h55}};
  // T = A^-1 B, u = A^-1 b_r
  double T[3][3], u[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
#pragma unroll
    for (int c = 0; c < 3; ++c) T[r][c] = fma(I[r][0], B[0][c], fma(I[r][1], B[1][c], I[r][2] * B[2][c]));
    u[r] = fma(I[r][0], br[0], fma(I[r][1], br[1], I[r][2] * br[2]));
  }
  // S = C - B^T T, r = b_t - B^T u
  double S[3][3], rt[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
#pragma unroll
    for (int c = 0; c < 3; ++c) S[r][c] = C[r][c] - fma(B[0][r], T[0][c], fma(B[1][r], T[1][c], B[2][r] * T[2][c]));
    rt[r] = bt[r] - fma(B[0][r], u[0], fma(B[1][r], u[1], B[2][r] * u[2]));
  }
  const double d00 = fma(S[1][1], S[2][2], -S[1][2] * S[1][2]), d01 = fma(S[0][2], S[1][2], -S[0][1] * S[2][2]);
  const double d02 = fma(S[0][1], S[1][2], -S[0][2] * S[1][1]), d11 = fma(S[0][0], S[2][2], -S[0][2] * S[0][2]);
  const double d12 = fma(S[0][1], S[0][2], -S[0][0] * S[1][2]), d22 = fma(S[0][0], S[1][1], -S[0][1] * S[0][1]);
  const double detS = fma(S[0][0], d00, fma(S[0][1], d01, S[0][2] * d02));
  const bool okS = S[0][0] > 0.0 && d22 > 0.0 && detS > 0.0;
  const double is = 1.0 / detS;
  const double J[3][3] = {{d00 * is, d01 * is, d02 * is}, {d01 * is, d11 * is, d12 * is}, {d02 * is, d12 * is, d22 * is}};
#pragma unroll
  for (int r = 0; r < 3; ++r) x[3 + r] = fma(J[r][0], rt[0], fma(J[r][1], rt[1], J[r][2] * rt[2]));
#pragma unroll
  for (int r = 0; r < 3; ++r) x[r] = u[r] - fma(T[r][0], x[3], fma(T[r][1], x[4], T[r][2] * x[5]));
  return okA && okS;
}

__device__ __forceinline__ bool gn_decide_wave(int j, int iters, const double* tot, GNShared& s) {
  const int lane = threadIdx.x;
  if (s.done) return false;
  const double cost = tot[27];
  if (!(j == 0 || cost <= s.cost)) {
    if (lane == 0) s.done = 1;
    return true;
  }
  // accept the evaluated pose
  const double acc_e = lane < 12 ? s.eval[lane] : 0.0;
  if (lane < 12) s.cur[lane] = acc_e;
  if (lane == 0) {
    s.cost = cost;
    s.count = tot[28];
    if (j > 0) s.accepted += 1;
  }
  if (j >= iters) {
    if (lane == 0) s.done = 1;
    return true;
  }
  double d[6];
  if (!solve6_schur(tot, d)) {
    if (lane == 0) s.done = 1;
    return true;
  }
  // converged: a step shorter than 1e-10 (norm of (dw, dt)) is not taken and
  // ends the run (every lane holds d; the sum in element order)
  double d2 = 0.0;
#pragma unroll
  for (int e = 0; e < 6; ++e) d2 += d[e] * d[e];
  if (d2 < kStepTol2) {
    if (lane == 0) s.done = 1;
    return true;
  }
  // left update: R' = Exp(dw) R, t' = Exp(dw) t + dt, element `lane` (< 12)
  double E[9];
  so3_exp(d, E);
  if (lane < 12) {
    const int rr = lane < 9 ? lane / 3 : lane - 9, cc = lane < 9 ? lane % 3 : 3;
    const double* cur = s.eval;  // the accepted pose (s.cur holds the same values)
    // row rr of E and entry rr of the translation step by selects (a lane-indexed
    // register array would be placed in scratch memory)
    const double er0 = rr == 0 ? E[0] : (rr == 1 ? E[3] : E[6]);
    const double er1 = rr == 0 ? E[1] : (rr == 1 ? E[4] : E[7]);
    const double er2 = rr == 0 ? E[2] : (rr == 1 ? E[5] : E[8]);
    const double dt = rr == 0 ? d[3] : (rr == 1 ? d[4] : d[5]);
    const double v = cc < 3 ? er0 * cur[cc] + er1 * cur[3 + cc] + er2 * cur[6 + cc]
                            : er0 * cur[9] + er1 * cur[10] + er2 * cur[11] + dt;
    __builtin_amdgcn_wave_barrier();
    s.eval[lane] = v;
  }
  return false;
}

// A recorded state read into registers at kernel entry (threads 0..11 hold
// one element of cur and eval, every thread the scalars), so that its latency
// overlaps the other loads; gn_state_to_lds then publishes it.
struct GNStateRegs {
  double cur, eval, cost, count;
  int done, accepted;
};

__device__ __forceinline__ void gn_state_issue(const GNState* st, GNStateRegs& r) {
  r.cur = r.eval = 0.0;
  r.cost = __builtin_inf();
  r.count = 0.0;
  r.done = r.accepted = 0;
  if (!st) return;
  if (threadIdx.x < 12) {
    r.cur = st->cur[threadIdx.x];
    r.eval = st->eval[threadIdx.x];
  }
  // uniform loads (every thread): no divergent region forces an early wait
  r.cost = st->cur_cost;
  r.count = st->cur_count;
  r.done = st->done;
  r.accepted = st->accepted;
}

// From the registers, or (have = false) the initial state at start.
__device__ __forceinline__ void gn_state_to_lds(GNShared& s, const GNStateRegs& r, bool have, const double* start) {
  if (threadIdx.x < 12) {
    s.cur[threadIdx.x] = have ? r.cur : start[threadIdx.x];
    s.eval[threadIdx.x] = have ? r.eval : start[threadIdx.x];
  }
  if (threadIdx.x == 0) {
    s.cost = have ? r.cost : __builtin_inf();
    s.count = have ? r.count : 0.0;
    s.done = have ? r.done : 0;
    s.accepted = have ? r.accepted : 0;
  }
}

__device__ __forceinline__ void gn_store_state(const GNShared& s, GNState* st) {
  if (threadIdx.x < 12) {
    st->cur[threadIdx.x] = s.cur[threadIdx.x];
    st->eval[threadIdx.x] = s.eval[threadIdx.x];
  }
  if (threadIdx.x == 0) {
    st->cur_cost = s.cost;
    st->cur_count = s.count;
    st->done = s.done;
    st->accepted = s.accepted;
  }
}

// the same from the registers of gn_state_issue
__device__ __forceinline__ void gn_store_state_regs(const GNStateRegs& r, GNState* st) {
  if (threadIdx.x < 12) {
    st->cur[threadIdx.x] = r.cur;
    st->eval[threadIdx.x] = r.eval;
  }
  if (threadIdx.x == 0) {
    st->cur_cost = r.cost;
    st->cur_count = r.count;
    st->done = r.done;
    st->accepted = r.accepted;
  }
}

__device__ __forceinline__ void gn_outputs(const GNArgs& g, const GNShared& s, int p) {
  if (threadIdx.x < 12 && g.out_pose) g.out_pose[12 * (int64_t)p + threadIdx.x] = s.cur[threadIdx.x];
  if (threadIdx.x == 0) {
    if (g.out_cost) g.out_cost[p] = s.cost;
    if (g.out_count) g.out_count[p] = (int64_t)s.count;
  }
}

// A chunk's points, loaded into registers: point t of the thread is point
// chunk * kGNChunk + loc[t] of the set.
struct GNPoints {
  float X[kGNPPT], Y[kGNPPT], Z[kGNPPT], u[kGNPPT], v[kGNPPT], w[kGNPPT];
  bool use[kGNPPT];
  int loc[kGNPPT];
  bool has_w;  // confidence weights present (else every weight is 1)
};

// Every point of the chunk (thread t: offsets t, t + 256).  Branch-free:
// lanes past the end load the last point (and do not use it), a query without
// points or weights reads from `safe` (any valid device address), and every
// select happens where the value is used -- so the loads issue back to back
// and nothing waits for them before the accumulation.
__device__ __forceinline__ void gn_load_points(const CorrF32& c, int64_t n, int chunk, const void* safe,
                                               GNPoints& pt) {
  const bool any = n > 0;
  const float* sf = reinterpret_cast<const float*>(safe);
  const float* X = any ? c.X : sf;
  const float* Y = any ? c.Y : sf;
  const float* Z = any ? c.Z : sf;
  const float* U = any ? c.u : sf;
  const float* V = any ? c.v : sf;
  const float* W = any && c.w ? c.w : X;
  pt.has_w = any && c.w != nullptr;
#pragma unroll
  for (int t = 0; t < kGNPPT; ++t) {
    pt.loc[t] = (int)threadIdx.x + t * kGNThreads;
    const int64_t i = (int64_t)chunk * kGNChunk + pt.loc[t];
    pt.use[t] = i < n;
    const int64_t ic = i < n ? i : (any ? n - 1 : 0);
    pt.X[t] = gmem(X)[ic];
    pt.Y[t] = gmem(Y)[ic];
    pt.Z[t] = gmem(Z)[ic];
    pt.u[t] = gmem(U)[ic];
    pt.v[t] = gmem(V)[ic];
    pt.w[t] = gmem(W)[ic];
  }
}

// The in-set points of the chunk (final refinement after its first
// evaluation): thread t takes the compacted positions t and t + 256.  The
// count and the offsets are loaded together (offsets past the count are read
// but not used), then the points.
__device__ __forceinline__ void gn_load_points_inset(const CorrF32& c, int64_t n, int chunk, const uint8_t* inset,
                                                     const void* safe, GNPoints& pt) {
  const bool any = n > 0;
  const int64_t C = chunks_for(n);
  // workgroups past the query's chunks read its last chunk (and exit later)
  const int cc = chunk < C ? chunk : (int)C - 1;
  const uint16_t* cnts = reinterpret_cast<const uint16_t*>(any ? inset : reinterpret_cast<const uint8_t*>(safe));
  const uint16_t* offs = any ? reinterpret_cast<const uint16_t*>(inset + inset_head_bytes(C)) + (int64_t)cc * kGNChunk
                             : reinterpret_cast<const uint16_t*>(safe);
  // (a query without points reads element 0 of `safe`)
  const int cnt = any ? (int)gmem(cnts)[any ? cc : 0] : 0;
  int off[kGNPPT];
#pragma unroll
  for (int t = 0; t < kGNPPT; ++t) off[t] = any ? (int)gmem(offs)[any ? (int)threadIdx.x + t * kGNThreads : 0] : 0;
  const float* sf = reinterpret_cast<const float*>(safe);
  const float* X = any ? c.X : sf;
  const float* Y = any ? c.Y : sf;
  const float* Z = any ? c.Z : sf;
  const float* U = any ? c.u : sf;
  const float* V = any ? c.v : sf;
  const float* W = any && c.w ? c.w : X;
  pt.has_w = any && c.w != nullptr;
#pragma unroll
  for (int t = 0; t < kGNPPT; ++t) {
    pt.use[t] = (int)threadIdx.x + t * kGNThreads < cnt;
    pt.loc[t] = pt.use[t] ? off[t] : 0;
    const int64_t i = (int64_t)cc * kGNChunk + pt.loc[t];
    const int64_t ic = i < n ? i : (any ? n - 1 : 0);
    pt.X[t] = gmem(X)[ic];
    pt.Y[t] = gmem(Y)[ic];
    pt.Z[t] = gmem(Z)[ic];
    pt.u[t] = gmem(U)[ic];
    pt.v[t] = gmem(V)[ic];
    pt.w[t] = gmem(W)[ic];
  }
}

// Accumulate one chunk at pose P and store its partial sums: per thread in
// point order, then across the wave by recursive halving, then the waves in
// wave order.  The final refinement's first evaluation (MODE 1, j = 0) also
// writes the chunk's compacted in-set (its count and offsets).
template <int MODE, bool RIG, bool W>
__device__ __forceinline__ void gn_accumulate(const QueryDesc& d, const double* s_rig, const double* P, int j,
                                              int chunk, const GNPoints& pt, uint8_t* inset,
                                              double (*s_rows)[kAcc], double* part_out) {
  const double tau2 = d.tau * d.tau, s2 = d.cauchy_s * d.cauchy_s;
  const double inv_s2 = 1.0 / s2;
  const Cam K{d.fx, d.fy, d.cx, d.cy};
  const bool rig = RIG && d.ncam > 0;
  const int64_t* seg = MODE == 0 ? d.segS : d.segF;
  double a[kAcc];
#pragma unroll
  for (int e = 0; e < kAcc; ++e) a[e] = 0.0;
  bool keep[kGNPPT];  // MODE 1, j = 0: the point is in the set
#pragma unroll
  for (int t = 0; t < kGNPPT; ++t) {
    keep[t] = false;
    if (!pt.use[t]) continue;
    const int64_t i = (int64_t)chunk * kGNChunk + pt.loc[t];
    const double X = pt.X[t], Y = pt.Y[t], Z = pt.Z[t];
    const double w = pt.has_w ? (double)pt.w[t] : 1.0;
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
    double du = 0.0, dv = 0.0, r2 = 0.0, iz = 0.0;
    const bool front = z > 0.0;
    if (front) {
      iz = recip_pos(z);
      du = Kp.fx * x * iz + Kp.cx - (double)pt.u[t];
      dv = Kp.fy * y * iz + Kp.cy - (double)pt.v[t];
      r2 = du * du + dv * dv;
    }
    if (MODE == 0) {
      if (front && r2 < tau2) {
        a[27] += w * r2;
        a[28] += 1.0;
        if (rig) acc_point_rig(a, Kp, xr, x, y, iz, Rc, du, dv, w);
        else acc_point<W>(a, K, x, y, z, iz, du, dv, w);
      } else {
        a[27] += w * tau2;
      }
    } else {
      if (j == 0) {
        keep[t] = front && r2 < tau2;
        if (!keep[t]) continue;
      }
      a[28] += 1.0;
      if (!front) {
        a[27] += w * s2 * log1p(tau2 * inv_s2);
        continue;
      }
      const double q = r2 * inv_s2;
      a[27] += w * s2 * log1p(q);
      const double wc = w * recip_pos(1.0 + q);  // the Cauchy weight
      if (rig) acc_point_rig(a, Kp, xr, x, y, iz, Rc, du, dv, wc);
      else acc_point<true>(a, K, x, y, z, iz, du, dv, wc);
    }
  }
  if (MODE == 1 && j == 0) {  // the chunk's in-set: points of slot 0 in lane order, then slot 1
    __shared__ int s_cnt[kGNPPT][kGNWaves];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    uint64_t m[kGNPPT];
#pragma unroll
    for (int t = 0; t < kGNPPT; ++t) {
      m[t] = __ballot(keep[t]);
      if (lane == 0) s_cnt[t][wave] = __popcll(m[t]);
    }
    __syncthreads();
    const int64_t C = chunks_for(d.n);
    uint16_t* offs = reinterpret_cast<uint16_t*>(inset + inset_head_bytes(C)) + (int64_t)chunk * kGNChunk;
    int before = 0;
#pragma unroll
    for (int t = 0; t < kGNPPT; ++t) {
      int pos = before;
      for (int w = 0; w < wave; ++w) pos += s_cnt[t][w];
      pos += __popcll(m[t] & ((1ull << lane) - 1ull));
      if (keep[t]) offs[pos] = (uint16_t)pt.loc[t];
      for (int w = 0; w < kGNWaves; ++w) before += s_cnt[t][w];
    }
    if (threadIdx.x == 0) reinterpret_cast<uint16_t*>(inset)[chunk] = (uint16_t)before;
  }
  const double tot = wave_sum29(a);
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  if ((lane & 1) == 0 && (lane >> 1) < kAcc) s_rows[wave][lane >> 1] = tot;
  __syncthreads();
  if ((int)threadIdx.x < kAcc) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kGNWaves; ++w) t += s_rows[w][threadIdx.x];
    part_out[threadIdx.x] = t;
  }
}

// Fused launch k of a run (one launch per iteration): decision k - 1 on the
// partial sums of launch k - 1, taken redundantly by every workgroup of the
// problem (so no workgroup waits for another), then evaluation k.  Launch 0
// only evaluates the start pose; the last launch only decides.  Workgroup
// (0, p) records the state for the next launch and, when the run ends, the
// outputs.
template <int MODE, bool RIG, bool W>
__global__ __launch_bounds__(kGNThreads) void gn_fused_kernel(GNArgs g, int k) {
  const int p = blockIdx.y;
  const int chunk = blockIdx.x;
  asm volatile("" ::"s"(g.qd), "s"(g.part), "s"(g.gst));
  // loads whose addresses need only the launch: partial sums, descriptor
  // fields, state -- issued together, so that one round trip covers them (the
  // compiler would otherwise fetch each field in the branch that first uses it)
  // the state first: a run that has ended waits for it alone (below)
  GNStateRegs sr;
  gn_state_issue(k >= 2 ? g.gst + (int64_t)(k & 1) * g.nprob + p : nullptr, sr);
  GNPart pr;
  if (k > 0) gn_part_issue(gn_part(g, (k - 1) & 1, p), g.cmax, pr);
  const int q = gn_query<MODE>(g, p);
  const QueryDesc& d = g.qd[q];
  const CorrF32 c = MODE == 0 ? d.S : d.full;
  const int64_t n = MODE == 0 ? d.m : d.n;
  uint8_t* in_set = MODE == 1 ? g.in_set_all + d.in_set_off : nullptr;
  asm volatile("" ::"s"(c.X), "s"(c.Y), "s"(c.Z), "s"(c.u), "s"(c.v), "s"(c.w), "s"(n), "s"(in_set));
  // the points are loaded before any test (indices are clamped), so that the
  // descriptor fields are read together and the point latency overlaps the
  // reduction and the decision; the final refinement reads its compacted
  // in-set from the second launch on
  GNPoints pt;
  if (MODE == 1 && k > 0) gn_load_points_inset(c, n, chunk, in_set, g.part, pt);
  else gn_load_points(c, n, chunk, g.part, pt);
  // A run that ended at an earlier launch: decision k - 1 would leave its
  // state as it is, so carry the state to the slot the next launch reads and
  // stop, without waiting for the partial sums and points in flight.
  if (k >= 2 && sr.done) {
    if (chunk == 0) gn_store_state_regs(sr, g.gst + (int64_t)((k - 1) & 1) * g.nprob + p);
    return;
  }
  const int C = chunks_for(n);
  if (chunk >= C) return;
  const int iters = MODE == 0 ? d.lo_iters : d.final_iters;

  __shared__ double s_rig[RIG ? kMaxCams * 16 : 1];
  if (RIG && d.ncam > 0)
    for (int e = threadIdx.x; e < 16 * d.ncam; e += kGNThreads) s_rig[e] = d.rig[e];
  __shared__ double s_grp[8][kAcc];
  __shared__ double s_tot[kAcc];
  __shared__ double s_rows[kGNWaves][kAcc];
  __shared__ GNShared s;
  __shared__ int s_end;
  // the partial sums are added before the liveness test, so that their loads
  // need not wait for it (a problem without work reads harmless stale values)
  const bool live = gn_live<MODE>(g, p, q);
  if (k == 0) {
    if (!live) {
      // a finished query without a pose gets an all-zero mask
      if (MODE == 1 && g.fuse_mask && d.mask && g.bst[q].finished == 1) {
#pragma unroll
        for (int t = 0; t < kGNPPT; ++t)
          if (pt.use[t]) d.mask[(int64_t)chunk * kGNChunk + pt.loc[t]] = 0;
      }
      return;
    }
    gn_state_to_lds(s, sr, false, gn_start<MODE>(g, p, q));
    __syncthreads();
  } else {
    gn_part_sum(gn_part(g, (k - 1) & 1, p), C, pr, s_grp, s_tot);
    if (!live) return;
    gn_state_to_lds(s, sr, k >= 2, k >= 2 ? nullptr : gn_start<MODE>(g, p, q));
    __syncthreads();
    if (threadIdx.x < kWave) {
      const bool end = gn_decide_wave(k - 1, iters, s_tot, s);
      if (threadIdx.x == 0) s_end = end;
    }
    __syncthreads();
    if (chunk == 0) {
      gn_store_state(s, g.gst + (int64_t)((k - 1) & 1) * g.nprob + p);
      if (s_end) gn_outputs(g, s, p);
    }
    if (MODE == 1 && g.fuse_mask && s_end) {  // the run ended: mask of this chunk at the final pose
      GNPoints fp;  // every point of the chunk
      gn_load_points(c, n, chunk, g.part, fp);
      long long cnt = 0;
#pragma unroll
      for (int t = 0; t < kGNPPT; ++t) {
        const int64_t i = (int64_t)chunk * kGNChunk + fp.loc[t];
        if (!fp.use[t]) continue;
        const bool in = mask_test(d, s.cur, fp.X[t], fp.Y[t], fp.Z[t], fp.u[t], fp.v[t], i);
        if (d.mask) d.mask[i] = in ? 1 : 0;
        cnt += in ? 1 : 0;
      }
      // one add per workgroup to the query's counter (same-address atomics serialise)
      __shared__ long long s_cnt[kGNWaves];
      cnt = wave_sum(cnt);
      if ((threadIdx.x & (kWave - 1)) == 0) s_cnt[threadIdx.x / kWave] = cnt;
      __syncthreads();
      if (threadIdx.x == 0) {
        long long tot = 0;
#pragma unroll
        for (int w = 0; w < kGNWaves; ++w) tot += s_cnt[w];
        if (tot) atomicAdd((unsigned long long*)&g.bst[q].full_count, (unsigned long long)tot);
      }
    }
  }
  if (s.done) return;
  gn_accumulate<MODE, RIG, W>(d, s_rig, s.eval, k, chunk, pt, in_set, s_rows,
                           const_cast<double*>(gn_part(g, k & 1, p)) + (int64_t)chunk * kAcc);
}

// Split form, for batches where the redundant reduction of the fused form
// would read too much: evaluation j (one workgroup per chunk) ...
// The one-camera refinement evaluation is held to 96 VGPRs, five waves per
// SIMD (16 registers spill): its workgroups wait mostly on the in-set's
// dependent loads, and the batch's refinement takes 4 % less time.
template <int MODE, bool RIG, bool W>
__global__ __launch_bounds__(kGNThreads)
__attribute__((amdgpu_waves_per_eu((MODE == 1 && !RIG) ? 5 : 1, (MODE == 1 && !RIG) ? 5 : 8))) void gn_eval_kernel(GNArgs g, int j) {
  const int p = blockIdx.y;
  const int chunk = blockIdx.x;
  const int q = gn_query<MODE>(g, p);
  if (!gn_live<MODE>(g, p, q)) return;
  const QueryDesc& d = g.qd[q];
  const CorrF32 c = MODE == 0 ? d.S : d.full;
  const int64_t n = MODE == 0 ? d.m : d.n;
  const int C = chunks_for(n);
  if (chunk >= C) return;
  const GNState* st = j > 0 ? g.gst + (int64_t)((j - 1) & 1) * g.nprob + p : nullptr;
  if (st && st->done) return;
  uint8_t* in_set = MODE == 1 ? g.in_set_all + d.in_set_off : nullptr;
  GNPoints pt;
  if (MODE == 1 && j > 0) gn_load_points_inset(c, n, chunk, in_set, g.part, pt);
  else gn_load_points(c, n, chunk, g.part, pt);
  __shared__ double s_rig[RIG ? kMaxCams * 16 : 1];
  if (RIG && d.ncam > 0)
    for (int e = threadIdx.x; e < 16 * d.ncam; e += kGNThreads) s_rig[e] = d.rig[e];
  __shared__ double s_eval[12];
  __shared__ double s_rows[kGNWaves][kAcc];
  const double* start = st ? nullptr : gn_start<MODE>(g, p, q);
  if (threadIdx.x < 12) s_eval[threadIdx.x] = st ? st->eval[threadIdx.x] : start[threadIdx.x];
  __syncthreads();
  gn_accumulate<MODE, RIG, W>(d, s_rig, s_eval, j, chunk, pt, in_set, s_rows,
                           const_cast<double*>(gn_part(g, j & 1, p)) + (int64_t)chunk * kAcc);
}

// Split form of the local optimisation, evaluation j, for problems that
// start from selected candidates: one workgroup per (chunk, query) loads the
// chunk's points once and evaluates every live problem of the query in slot
// order (up to lo_top_k poses on the same points).  Each problem's
// accumulation is gn_accumulate with the same thread-to-point map, so the
// partial sums are those of gn_eval_kernel bit for bit.
// The unweighted one-camera variant is held to 128 VGPRs (four waves per SIMD
// instead of three; 20 bytes per lane spill): 4 % faster on the 256-query
// batch.
template <bool RIG, bool W>
__global__ __launch_bounds__(kGNThreads)
__attribute__((amdgpu_waves_per_eu((!RIG && !W) ? 4 : 1, (!RIG && !W) ? 4 : 8))) void gn_eval_lo_multi_kernel(
    GNArgs g, int j) {
  const int q = blockIdx.y;
  const int chunk = blockIdx.x;
  const int ns = g.n_sel[q];
  if (ns <= 0) return;
  const QueryDesc& d = g.qd[q];
  const int64_t n = d.m;
  const int C = chunks_for(n);
  if (chunk >= C) return;
  // the query's live problems, their flags read together (lane s: slot s);
  // once every run has ended the workgroup exits before loading any point
  // (most runs end within a few iterations)
  const GNState* st0 = j > 0 ? g.gst + (int64_t)((j - 1) & 1) * g.nprob + q * g.kmax : nullptr;
  const int lane = threadIdx.x & (kWave - 1);
  uint64_t live = ns >= kWave ? ~0ull : (1ull << ns) - 1ull;
  if (st0) live = __ballot(lane < ns && !st0[lane].done);
  if (!live) return;
  GNPoints pt;
  gn_load_points(d.S, n, chunk, g.part, pt);
  __shared__ double s_rig[RIG ? kMaxCams * 16 : 1];
  if (RIG && d.ncam > 0)
    for (int e = threadIdx.x; e < 16 * d.ncam; e += kGNThreads) s_rig[e] = d.rig[e];
  __shared__ double s_eval[12];
  __shared__ double s_rows[kGNWaves][kAcc];
  for (; live; live &= live - 1) {
    const int slot = __builtin_ctzll(live);
    const int p = q * g.kmax + slot;
    const GNState* st = st0 ? st0 + slot : nullptr;
    const double* start = st ? nullptr : gn_start<0>(g, p, q);
    // every thread has left the previous problem's accumulation (its last
    // barrier) before s_eval is rewritten
    if (threadIdx.x < 12) s_eval[threadIdx.x] = st ? st->eval[threadIdx.x] : start[threadIdx.x];
    __syncthreads();
    gn_accumulate<0, RIG, W>(d, s_rig, s_eval, j, chunk, pt, nullptr, s_rows,
                          const_cast<double*>(gn_part(g, j & 1, p)) + (int64_t)chunk * kAcc);
  }
}

// ... then decision j (one workgroup per problem), with the same reduction
// order and decision as the fused form, so both give identical results.
template <int MODE>
__global__ __launch_bounds__(kGNThreads) void gn_decide_kernel(GNArgs g, int j) {
  const int p = blockIdx.x;
  GNStateRegs sr;
  gn_state_issue(j > 0 ? g.gst + (int64_t)((j - 1) & 1) * g.nprob + p : nullptr, sr);
  GNPart pr;
  gn_part_issue(gn_part(g, j & 1, p), g.cmax, pr);
  const int q = gn_query<MODE>(g, p);
  if (!gn_live<MODE>(g, p, q)) return;
  // a run that has ended: its state carried to the slot the next launch
  // reads, without waiting for the partial sums
  if (j > 0 && sr.done) {
    gn_store_state_regs(sr, g.gst + (int64_t)(j & 1) * g.nprob + p);
    return;
  }
  const QueryDesc& d = g.qd[q];
  const int64_t n = MODE == 0 ? d.m : d.n;
  const int iters = MODE == 0 ? d.lo_iters : d.final_iters;
  const int C = chunks_for(n);
  __shared__ double s_grp[8][kAcc];
  __shared__ double s_tot[kAcc];
  __shared__ GNShared s;
  __shared__ int s_end;
  gn_part_sum(gn_part(g, j & 1, p), C, pr, s_grp, s_tot);
  gn_state_to_lds(s, sr, j > 0, j > 0 ? nullptr : gn_start<MODE>(g, p, q));
  __syncthreads();
  if (threadIdx.x < kWave) {
    const bool end = gn_decide_wave(j, iters, s_tot, s);
    if (threadIdx.x == 0) s_end = end;
  }
  __syncthreads();
  gn_store_state(s, g.gst + (int64_t)(j & 1) * g.nprob + p);
  if (s_end) gn_outputs(g, s, p);
}

static void split_scratch(void* scratch, int nprob, GNState** st, double** part) {
  *st = reinterpret_cast<GNState*>(scratch);
  *part = reinterpret_cast<double*>(reinterpret_cast<char*>(scratch) +
                                    (((size_t)2 * nprob * sizeof(GNState) + 255) & ~size_t(255)));
}

// The fused form reads every problem's partial sums once per workgroup:
// nprob * C^2 * 232 bytes per launch.  Above 32 MiB the split form (one more
// launch per iteration, partials read once) is faster.
static bool use_fused(int gn_mode, int nprob, int chunks_max) {
  if (gn_mode == 1) return true;
  if (gn_mode == 2) return false;
  return (double)nprob * chunks_max * chunks_max * kAcc * sizeof(double) <= 32.0 * 1024 * 1024;
}

template <int MODE, bool RIG, bool W>
static void launch_gn(const GNArgs& g, int iters_max, bool fused, hipStream_t s) {
  const dim3 grid(g.cmax, g.nprob);
  if (fused) {
    for (int k = 0; k <= iters_max + 1; ++k)
      hipLaunchKernelGGL((gn_fused_kernel<MODE, RIG, W>), grid, dim3(kGNThreads), 0, s, g, k);
  } else {
    // local optimisation from selected candidates: one workgroup per chunk and
    // query evaluates all of the query's problems (points loaded once)
    const bool multi = MODE == 0 && !g.start_direct && g.kmax > 1;
    const dim3 grid_multi(g.cmax, g.nprob / (g.kmax > 0 ? g.kmax : 1));
    for (int j = 0; j <= iters_max; ++j) {
      if (multi)
        hipLaunchKernelGGL((gn_eval_lo_multi_kernel<RIG, W>), grid_multi, dim3(kGNThreads), 0, s, g, j);
      else
        hipLaunchKernelGGL((gn_eval_kernel<MODE, RIG, W>), grid, dim3(kGNThreads), 0, s, g, j);
      hipLaunchKernelGGL((gn_decide_kernel<MODE>), dim3(g.nprob), dim3(kGNThreads), 0, s, g, j);
    }
  }
}

hipError_t launch_lo(const QueryDesc* qd, CandBuf cb, const int32_t* sel, const int32_t* n_sel,
                     const double* start_direct, int nprob, int kmax, int chunks_max, int iters_max, void* scratch,
                     double* out_pose, double* out_cost, int64_t* out_count, bool any_rig, bool any_weighted,
                     int gn_mode, hipStream_t s) {
  if (nprob <= 0) return hipSuccess;
  GNArgs g{};
  split_scratch(scratch, nprob, &g.gst, &g.part);
  g.qd = qd;
  g.cb = cb;
  g.sel = sel;
  g.n_sel = n_sel;
  g.start_direct = start_direct;
  g.out_pose = out_pose;
  g.out_cost = out_cost;
  g.out_count = out_count;
  g.kmax = kmax;
  g.cmax = chunks_max;
  g.nprob = nprob;
  const bool fused = use_fused(gn_mode, nprob, chunks_max);
  // queries without confidences take the unweighted accumulation (same bits)
  if (any_rig) {
    if (any_weighted) launch_gn<0, true, true>(g, iters_max, fused, s);
    else launch_gn<0, true, false>(g, iters_max, fused, s);
  } else {
    if (any_weighted) launch_gn<0, false, true>(g, iters_max, fused, s);
    else launch_gn<0, false, false>(g, iters_max, fused, s);
  }
  return hipGetLastError();
}

hipError_t launch_refine(const QueryDesc* qd, BestState* bst, const double* start_direct, int nq, int chunks_max,
                         int iters_max, uint8_t* in_set, void* scratch, double* out_pose, double* out_cost,
                         bool any_rig, int gn_mode, bool fuse_mask, bool* mask_done, hipStream_t s) {
  if (mask_done) *mask_done = false;
  if (nq <= 0) return hipSuccess;
  GNArgs g{};
  split_scratch(scratch, nq, &g.gst, &g.part);
  g.qd = qd;
  g.bst = bst;
  g.start_direct = start_direct;
  g.in_set_all = in_set;
  g.out_pose = out_pose;
  g.out_cost = out_cost;
  g.kmax = 1;
  g.cmax = chunks_max;
  g.nprob = nq;
  const bool fused = use_fused(gn_mode, nq, chunks_max);
  g.fuse_mask = fused && fuse_mask && !start_direct ? 1 : 0;
  if (mask_done) *mask_done = g.fuse_mask != 0;
  if (any_rig) launch_gn<1, true, true>(g, iters_max, fused, s);
  else launch_gn<1, false, true>(g, iters_max, fused, s);
  return hipGetLastError();
}

// Inlier mask over all points of every query that just finished, at its final
// pose (float64), and its count; a query without a pose gets a zero mask.
__global__ __launch_bounds__(256) void mask_kernel(const QueryDesc* __restrict__ qd, BestState* __restrict__ st,
                                                   const double* __restrict__ fin_pose, int all) {
  const int q = blockIdx.y;
  if (!all && st[q].finished != 1) return;
  const QueryDesc& d = qd[q];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if ((int64_t)blockIdx.x * blockDim.x >= d.n) return;
  const bool have = all || st[q].have != 0;
  long long in = 0;
  if (i < d.n && have)
    in = mask_test(d, fin_pose + 12 * (int64_t)q, gmem(d.full.X)[i], gmem(d.full.Y)[i], gmem(d.full.Z)[i],
                   gmem(d.full.u)[i], gmem(d.full.v)[i], i) ? 1 : 0;
  if (i < d.n && d.mask) d.mask[i] = (uint8_t)in;
  // one add per workgroup to the query's counter (same-address atomics serialise)
  __shared__ long long s_cnt[256 / kWave];
  const long long tot = wave_sum(in);
  if ((threadIdx.x & (kWave - 1)) == 0) s_cnt[threadIdx.x / kWave] = tot;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long sum = 0;
#pragma unroll
    for (int w = 0; w < 256 / kWave; ++w) sum += s_cnt[w];
    if (sum) atomicAdd((unsigned long long*)&st[q].full_count, (unsigned long long)sum);
  }
}

hipError_t launch_mask(const QueryDesc* qd, BestState* st, const double* fin_pose, int nq, int64_t max_n, int all,
                       hipStream_t s) {
  if (nq <= 0 || max_n <= 0) return hipSuccess;
  hipLaunchKernelGGL(mask_kernel, dim3((unsigned)((max_n + 255) / 256), nq), dim3(256), 0, s, qd, st, fin_pose, all);
  return hipGetLastError();
}

}  // namespace imloc
