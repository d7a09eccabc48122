// triangulate.hip -- mapping-time depth of every pixel of a mapping image by
// 1-DoF triangulation of dense matches (ImLoc Sec. 3.3 "Depth Estimation by
// Dense Matching").
//
// Poses are known, so the point of pixel (row i, col j) lies on its ray
// X(l) = C0 + l r0, r0 = R0^T K0^-1 [j + 0.5, i + 0.5, 1]^T (l is the z-depth).
// Each match of the pixel in covisible view k (confidence >= 0.05) is a unit
// ray rk from the view's centre Ck; the angular error of depth l for it is the
// angle between X(l) - Ck and rk.  Per pixel:
//   1. every match gives one depth hypothesis: the depth minimising its own
//      angular error, in closed form (the cosine's derivative along the ray
//      vanishes at one depth); it counts if that is a minimum at l > 0;
//   2. each hypothesis counts the matches within 2 degrees; the most inliers
//      win, ties going to the lowest view;
//   3. the depth is refined on that inlier set by minimising the
//      confidence-weighted sum of squared angular errors (1-D Newton on the
//      derivative, its own derivative by a central difference, step halving
//      while the cost rises, to a step below 1e-12 l);
//   4. it is kept if the inlier set has at least min_inliers (4) members.
//
// Two launches, one thread per pixel, one wave per workgroup, float64
// throughout (on MI355X the float64 vector rate equals the non-packed float32
// rate):
//   - triangulate_kernel: steps 1, 2 and 4 for every pixel; a pixel whose
//     depth needs refinement is appended to a queue (one atomic per wave);
//   - tri_refine_kernel: step 3, a quad of lanes per queued pixel.
// Refinement is most of the arithmetic, but only the pixels with enough
// inliers (about half of a mapping image) need it, and each runs its own
// number of Newton steps; run in place, every wave would pay for its slowest
// lane while its other lanes idle.  Compacted, the waves of the second launch
// are full.  The per-view constants sit in LDS (broadcast reads), and so do
// the pixels' unit match rays (first launch: [view][lane], 24 B per view and
// lane; second: [slot][lane] with the weights, 28 B per slot and lane), which
// keeps the loops over views compact; the LDS is sized by the actual view
// count at launch.  Match arrays are [view][H][W], so the loads of the first
// launch are coalesced; the second recomputes the rays of its pixel's inliers
// with the same arithmetic.
#include "imloc_device.h"
#include "imloc_kernels.h"

namespace imloc {

struct TriViewDev {
  double fx, fy, cx, cy;
  double Rt[9];   // R^T row-major: world direction = Rt * K^-1 [u, v, 1]^T
  double b[3];    // C0 - Ck
  double pad;
};

__device__ inline void tri_ray(const TriViewDev& v, double u, double w, double r[3]) {
  const double dx = (u - v.cx) / v.fx, dy = (w - v.cy) / v.fy;
  for (int c = 0; c < 3; ++c) r[c] = v.Rt[3 * c] * dx + v.Rt[3 * c + 1] * dy + v.Rt[3 * c + 2];
}

// unit ray of a match (u, w) in a view
__device__ inline void tri_unit_ray(const TriViewDev& v, float u, float w, double r[3]) {
  tri_ray(v, u, w, r);
  const double inv = 1.0 / sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  r[0] *= inv;
  r[1] *= inv;
  r[2] *= inv;
}

// angle between a = b + l r0 and the unit ray r
__device__ inline double tri_angle(const double b[3], const double r0[3], double l, const double r[3]) {
  const double a0 = b[0] + l * r0[0], a1 = b[1] + l * r0[1], a2 = b[2] + l * r0[2];
  const double x0 = a1 * r[2] - a2 * r[1], x1 = a2 * r[0] - a0 * r[2], x2 = a0 * r[1] - a1 * r[0];
  const double S = sqrt(x0 * x0 + x1 * x1 + x2 * x2);
  const double s = a0 * r[0] + a1 * r[1] + a2 * r[2];
  return atan2(S, s);
}

// the same angle and, on request, d(angle)/dl
__device__ inline double tri_angle_d(const double b[3], const double r0[3], double l, const double r[3],
                                     double* dth) {
  const double a0 = b[0] + l * r0[0], a1 = b[1] + l * r0[1], a2 = b[2] + l * r0[2];
  const double x0 = a1 * r[2] - a2 * r[1], x1 = a2 * r[0] - a0 * r[2], x2 = a0 * r[1] - a1 * r[0];
  const double S2 = x0 * x0 + x1 * x1 + x2 * x2;
  const double S = sqrt(S2);
  const double s = a0 * r[0] + a1 * r[1] + a2 * r[2];
  const double th = atan2(S, s);
  if (dth) {
    const double q = a0 * a0 + a1 * a1 + a2 * a2;
    const double y0 = r0[1] * r[2] - r0[2] * r[1], y1 = r0[2] * r[0] - r0[0] * r[2], y2 = r0[0] * r[1] - r0[1] * r[0];
    const double be = r0[0] * r[0] + r0[1] * r[1] + r0[2] * r[2];
    if (S2 > 1e-24 * q) {
      // (s dS/dl - S be) / q with dS/dl = (x . y) / S, over one division
      *dth = (s * (x0 * y0 + x1 * y1 + x2 * y2) - S2 * be) / (S * q);
    } else {
      *dth = s * sqrt(y0 * y0 + y1 * y1 + y2 * y2) / q;  // the limit where the angle vanishes
    }
  }
  return th;
}

// Dynamic LDS of one workgroup: per-view constants [V + 1] (entry 0: the
// mapping camera), then the unit match rays x, y, z, each [rows][kWave], and
// for the refinement the weights [rows][kWave] (rows = V for the hypotheses;
// for the refinement, where a lane holds every fourth view, rows = ceil(V / 4)).
size_t tri_lds_bytes(int V, int rows, bool weights) {
  return (size_t)(V + 1) * sizeof(TriViewDev) +
         (size_t)rows * kWave * (3 * sizeof(double) + (weights ? sizeof(float) : 0));
}

struct TriLds {
  TriViewDev* view;
  double *rx, *ry, *rz;
  float* w;
};

// carve the dynamic LDS and load the per-view constants (every lane of the
// workgroup takes part)
__device__ inline TriLds tri_lds_setup(const TriArgs& a, int rows, bool weights) {
  extern __shared__ double s_dyn[];
  TriLds L;
  L.view = reinterpret_cast<TriViewDev*>(s_dyn);
  L.rx = s_dyn + (size_t)(a.V + 1) * (sizeof(TriViewDev) / sizeof(double));
  L.ry = L.rx + rows * kWave;
  L.rz = L.ry + rows * kWave;
  L.w = weights ? reinterpret_cast<float*>(L.rz + rows * kWave) : nullptr;
  for (int e = threadIdx.x; e <= a.V; e += kWave) {
    const double* src = a.views + 16 * e;
    TriViewDev v;
    v.fx = src[0]; v.fy = src[1]; v.cx = src[2]; v.cy = src[3];
    for (int c = 0; c < 9; ++c) v.Rt[c] = src[4 + c];
    for (int c = 0; c < 3; ++c) v.b[c] = src[13 + c];
    v.pad = 0.0;
    L.view[e] = v;
  }
  __syncthreads();
  return L;
}

// The refinement runs on a quad of lanes per pixel: lane j of the quad takes
// the views k = j, j + 4, ... of the inlier set, and the sums are added over
// the quad by DPP.  The butterfly gives every lane of the quad the same bits
// ((x0 + x1) + (x2 + x3) up to commutation), so the four lanes take the same
// decisions.  A pixel's Newton chain is a quarter as long, and four times as
// many waves hide each other's latency.
constexpr int kTriQuad = 4;
constexpr int kTriLoadGroup = 8;  // match loads issued together

__host__ __device__ inline int tri_quad_rows(int V) { return (V + kTriQuad - 1) / kTriQuad; }

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const unsigned long long v = (unsigned long long)__double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}

__device__ __forceinline__ double quad_sum(double x) {
  x += dpp_f64<0xb1>(x);  // quad_perm [1, 0, 3, 2]
  x += dpp_f64<0x4e>(x);  // quad_perm [2, 3, 0, 1]
  return x;
}

// Lane j of a quad holds the views k = j + 4 s in slots s < KQ (KQ =
// ceil(V / 4), a template bound, so the slot loops unroll); a slot without an
// inlier holds the ray (0, 0, 1) with weight 0 and contributes an exact 0.

// Cost e = sum w th^2 at depth l over the quad's share of the inlier set
// (rays read from LDS), summed over the quad.  Branch-free over the slots, so
// that their angle computations interleave.
template <int KQ>
__device__ inline double tri_cost(const TriLds& L, int V, int lane, uint32_t set, const double r0[3], double l) {
  const int sub = lane & (kTriQuad - 1);
  double c[KQ];
#pragma unroll
  for (int j = 0; j < KQ; ++j) {
    const int k = sub + kTriQuad * j;
    const bool in = k < V && ((set >> k) & 1u);
    const int o = j * kWave + lane;
    const double r[3] = {L.rx[o], L.ry[o], L.rz[o]};
    const double th = tri_angle(L.view[in ? k + 1 : 1].b, r0, l, r);
    c[j] = in ? (double)L.w[o] * th * th : 0.0;
  }
  double e = 0.0;
#pragma unroll
  for (int j = 0; j < KQ; ++j) e += c[j];
  return quad_sum(e);
}

// g = sum w th dth/dl at the depths l[0..3) (three independent chains) and
// the Gauss-Newton curvature hgn = sum w (dth/dl)^2 at l[0], summed over the
// quad.
struct TriGrad {
  double g[3], hgn;
};

template <int KQ>
__device__ inline TriGrad tri_grad3(const TriLds& L, int V, int lane, uint32_t set, const double r0[3],
                                    const double l[3]) {
  const int sub = lane & (kTriQuad - 1);
  TriGrad out{};
#pragma unroll
  for (int j = 0; j < KQ; ++j) {
    const int k = sub + kTriQuad * j;
    if (!(k < V && ((set >> k) & 1u))) continue;
    const int o = j * kWave + lane;
    const double r[3] = {L.rx[o], L.ry[o], L.rz[o]};
    const double w = L.w[o];
    const double* b = L.view[k + 1].b;
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      double J;
      const double th = tri_angle_d(b, r0, l[t], r, &J);
      out.g[t] += w * th * J;
      if (t == 0) out.hgn += w * J * J;
    }
  }
#pragma unroll
  for (int t = 0; t < 3; ++t) out.g[t] = quad_sum(out.g[t]);
  out.hgn = quad_sum(out.hgn);
  return out;
}

// the ray of pixel p of the mapping image (unnormalised: its z-component in
// the camera is 1, so that l is the z-depth)
__device__ inline void tri_pixel_ray(const TriArgs& a, const TriViewDev& v0, int64_t p, double r0[3]) {
  const int i = (int)(p / a.W), j = (int)(p - (int64_t)i * a.W);
  tri_ray(v0, (double)j + 0.5, (double)i + 0.5, r0);
}

// Steps 1, 2 and 4: one wave per workgroup; each lane's match rays live in
// LDS ([view][lane], so the lanes of a wave hit distinct banks).  The loops
// over hypotheses and views run over all views with the same view in every
// lane (a lane skips the views it has no match in), so the view constants are
// uniform and come from scalar loads.  A pixel to refine is queued with its
// hypothesis and inlier set.
__global__ __launch_bounds__(kWave) void triangulate_kernel(TriArgs a) {
  const TriLds L = tri_lds_setup(a, a.V, false);
  TriViewDev* s_view = L.view;
  double *s_rx = L.rx, *s_ry = L.ry, *s_rz = L.rz;
  const int lane = threadIdx.x;
  const int64_t HW = (int64_t)a.H * a.W;
  const int64_t p = (int64_t)blockIdx.x * kWave + lane;
  const bool pix = p < HW;  // the lanes past the image take part in the queue's ballot only
  double r0[3];
  tri_pixel_ray(a, s_view[0], pix ? p : 0, r0);
  const double ep = r0[0] * r0[0] + r0[1] * r0[1] + r0[2] * r0[2];

  // the pixel's matches: unit rays.  The loads of a group of views are issued
  // together, so that the group waits for one memory latency, not one per view.
  uint32_t ok = 0;
  for (int k0 = 0; pix && k0 < a.V; k0 += kTriLoadGroup) {
    float mu[kTriLoadGroup], mv[kTriLoadGroup], cf[kTriLoadGroup];
#pragma unroll
    for (int j = 0; j < kTriLoadGroup; ++j) {
      const int64_t o = (int64_t)min(k0 + j, a.V - 1) * HW + p;
      mu[j] = a.mu[o]; mv[j] = a.mv[o]; cf[j] = a.conf[o];
    }
#pragma unroll
    for (int j = 0; j < kTriLoadGroup; ++j) {
      const int k = k0 + j;
      if (k < a.V && cf[j] >= a.min_conf && isfinite(mu[j]) && isfinite(mv[j])) {
        double r[3];
        tri_unit_ray(s_view[k + 1], mu[j], mv[j], r);
        s_rx[k * kWave + lane] = r[0];
        s_ry[k * kWave + lane] = r[1];
        s_rz[k * kWave + lane] = r[2];
        ok |= 1u << k;
      }
    }
  }

  // hypotheses, in view order
  int best_n = 0;
  double best_l = 0.0;
  uint32_t best_set = 0;
  for (int h = 0; h < a.V; ++h) {
    if (!((ok >> h) & 1u)) continue;
    const double* b = a.views + 16 * (h + 1) + 13;  // C0 - C_h
    const int oh = h * kWave + lane;
    const double rh[3] = {s_rx[oh], s_ry[oh], s_rz[oh]};
    const double al = b[0] * rh[0] + b[1] * rh[1] + b[2] * rh[2];
    const double be = r0[0] * rh[0] + r0[1] * rh[1] + r0[2] * rh[2];
    const double ga = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    const double de = b[0] * r0[0] + b[1] * r0[1] + b[2] * r0[2];
    const double den = be * de - al * ep;
    if (den == 0.0) continue;
    const double l = (al * de - be * ga) / den;
    if (!(l > 0.0) || !isfinite(l)) continue;
    const double cosl = (al + l * be) / sqrt(ga + 2.0 * l * de + l * l * ep);
    if (!(cosl > fabs(be) / sqrt(ep))) continue;
    // inliers: angle < thr  <=>  a.r > 0 and (a.r)^2 > cos^2(thr) |a|^2
    uint32_t set = 0;
    for (int k = 0; k < a.V; ++k) {
      if (!((ok >> k) & 1u)) continue;
      const double* bk = a.views + 16 * (k + 1) + 13;
      const double a0 = bk[0] + l * r0[0], a1 = bk[1] + l * r0[1], a2 = bk[2] + l * r0[2];
      const int ok_ = k * kWave + lane;
      const double s = a0 * s_rx[ok_] + a1 * s_ry[ok_] + a2 * s_rz[ok_];
      const double q = a0 * a0 + a1 * a1 + a2 * a2;
      if (s > 0.0 && s * s > a.cos2_thr * q) set |= 1u << k;
    }
    const int cnt = __popc(set);
    if (cnt > best_n) {
      best_n = cnt;
      best_l = l;
      best_set = set;
    }
  }

  const bool refine = pix && best_n > 0 && best_n >= a.min_inliers;
  // queue the pixels to refine: one counter add per wave, slots in lane order
  const uint64_t bal = __ballot(refine);
  if (bal) {
    int base = 0;
    if (lane == __ffsll((unsigned long long)bal) - 1) base = atomicAdd(a.n_tasks, __popcll(bal));
    base = __shfl(base, __ffsll((unsigned long long)bal) - 1);
    if (refine) {
      const int slot = base + __popcll(bal & ((1ull << lane) - 1));
      a.tasks[slot] = TriTask{best_l, (int32_t)p, best_set};
    }
  }
  if (!pix) return;
  if (a.inliers) a.inliers[p] = best_n;
  if (!refine) {
    if (a.depth) a.depth[p] = 0.0f;
    if (a.codes) a.codes[p] = 0;
  }
}

// Step 3 for the queued pixels, a quad of lanes each: Newton's method on the
// derivative of the confidence-weighted sum of squared angular errors over
// the inlier set (its own derivative by a central difference, the
// Gauss-Newton curvature where that is not positive), a step that raises the
// cost halved up to 30 times, until the step is below 1e-12 l or max_iters
// steps.  A step below 1e-12 l is not tried while being halved either: near
// the minimum the cost's rounding noise exceeds such a step's decrease, and a
// wave would otherwise halve on towards one ulp for its unluckiest lane.  Launched over the largest possible queue; waves past its length
// return at once.
template <int KQ>
__global__ __launch_bounds__(kWave) void tri_refine_kernel(TriArgs a) {
  constexpr int kPerWave = kWave / kTriQuad;  // pixels per wave
  const int n = *a.n_tasks;
  if ((int64_t)blockIdx.x * kPerWave >= n) return;
  const TriLds L = tri_lds_setup(a, tri_quad_rows(a.V), true);
  const int lane = threadIdx.x;
  const int64_t t = (int64_t)blockIdx.x * kPerWave + lane / kTriQuad;
  if (t >= n) return;  // the whole quad
  const TriTask task = a.tasks[t];
  const int64_t HW = (int64_t)a.H * a.W;
  const int64_t p = task.p;
  const uint32_t set = task.set;
  double r0[3];
  tri_pixel_ray(a, L.view[0], p, r0);
  // this lane's share of the rays (slot j: view sub + 4 j), loads issued together
  const int sub = lane & (kTriQuad - 1);
  float mu[KQ], mv[KQ], cf[KQ];
#pragma unroll
  for (int j = 0; j < KQ; ++j) {
    const int k = sub + kTriQuad * j;
    const int64_t o = (int64_t)(k < a.V ? k : 0) * HW + p;  // view 0 always exists
    mu[j] = a.mu[o]; mv[j] = a.mv[o]; cf[j] = a.conf[o];
  }
#pragma unroll
  for (int j = 0; j < KQ; ++j) {
    const int k = sub + kTriQuad * j;
    double r[3] = {0.0, 0.0, 1.0};
    float w = 0.0f;
    if (k < a.V && ((set >> k) & 1u)) {
      tri_unit_ray(L.view[k + 1], mu[j], mv[j], r);
      w = cf[j];
    }
    const int row = j * kWave + lane;
    L.rx[row] = r[0];
    L.ry[row] = r[1];
    L.rz[row] = r[2];
    L.w[row] = w;
  }
  double l = task.l;
  double e = tri_cost<KQ>(L, a.V, lane, set, r0, l);
  for (int it = 0; it < a.max_iters; ++it) {
    const double dl = 1e-6 * l;
    const double pts[3] = {l, l + dl, l - dl};
    const TriGrad ev = tri_grad3<KQ>(L, a.V, lane, set, r0, pts);
    const double g = ev.g[0];
    if (g == 0.0) break;
    const double gp = (ev.g[1] - ev.g[2]) / (2.0 * dl);
    const double curv = gp > 0.0 ? gp : ev.hgn;
    if (!(curv > 0.0)) break;
    double step = -g / curv;
    bool moved = false;
    for (int half = 0; half < 30; ++half) {
      if (fabs(step) <= 1e-12 * l) break;  // converged: not tried
      const double ln = l + step;
      if (ln > 0.0) {
        const double en = tri_cost<KQ>(L, a.V, lane, set, r0, ln);
        if (en <= e) {
          moved = ln != l;
          l = ln;
          e = en;
          break;
        }
      }
      step *= 0.5;
    }
    if (!moved || fabs(step) <= 1e-12 * l) break;
  }
  const double depth = l > 0.0 ? l : 0.0;
  const float d32 = (float)depth;
  if ((lane & (kTriQuad - 1)) == 0) {
    if (a.depth) a.depth[p] = d32;
    if (a.codes) a.codes[p] = depth > 0.0 ? log8_code(d32) : (uint8_t)0;
  }
}

hipError_t launch_triangulate(const TriArgs& a, hipStream_t s) {
  const int64_t HW = (int64_t)a.H * a.W;
  if (HW <= 0) return hipSuccess;
  const dim3 grid((unsigned)((HW + kWave - 1) / kWave));
  const hipError_t e = launch_fill_i32(a.n_tasks, 1, 0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(triangulate_kernel, grid, dim3(kWave), tri_lds_bytes(a.V, a.V, false), s, a);
  const dim3 grid_refine((unsigned)((HW * kTriQuad + kWave - 1) / kWave));
  const size_t lds = tri_lds_bytes(a.V, tri_quad_rows(a.V), true);
  switch (tri_quad_rows(a.V)) {  // slots per lane, 1..8 for 1..32 views
    case 1: hipLaunchKernelGGL(tri_refine_kernel<1>, grid_refine, dim3(kWave), lds, s, a); break;
    case 2: hipLaunchKernelGGL(tri_refine_kernel<2>, grid_refine, dim3(kWave), lds, s, a); break;
    case 3: hipLaunchKernelGGL(tri_refine_kernel<3>, grid_refine, dim3(kWave), lds, s, a); break;
    case 4: hipLaunchKernelGGL(tri_refine_kernel<4>, grid_refine, dim3(kWave), lds, s, a); break;
    case 5: hipLaunchKernelGGL(tri_refine_kernel<5>, grid_refine, dim3(kWave), lds, s, a); break;
    case 6: hipLaunchKernelGGL(tri_refine_kernel<6>, grid_refine, dim3(kWave), lds, s, a); break;
    case 7: hipLaunchKernelGGL(tri_refine_kernel<7>, grid_refine, dim3(kWave), lds, s, a); break;
    default: hipLaunchKernelGGL(tri_refine_kernel<8>, grid_refine, dim3(kWave), lds, s, a); break;
  }
  return hipGetLastError();
}

}  // namespace imloc
