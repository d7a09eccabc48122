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
// One thread per pixel, one wave per workgroup, float64 throughout (on MI355X
// the float64 vector rate equals the non-packed float32 rate).  The per-view
// constants sit in LDS (broadcast reads), and so do the pixel's unit match
// rays and weights ([view][lane], sized by the template bound on the view
// count), which keeps the loops over views compact.  Match arrays are
// [view][H][W], so the loads of a wave are coalesced.
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

// angle between a = b + l r0 and the unit ray r, and, on request, d(angle)/dl
__device__ inline double tri_angle_d(const double b[3], const double r0[3], double l, const double r[3],
                                     double* dth) {
  const double a0 = b[0] + l * r0[0], a1 = b[1] + l * r0[1], a2 = b[2] + l * r0[2];
  const double x0 = a1 * r[2] - a2 * r[1], x1 = a2 * r[0] - a0 * r[2], x2 = a0 * r[1] - a1 * r[0];
  const double S = sqrt(x0 * x0 + x1 * x1 + x2 * x2);
  const double s = a0 * r[0] + a1 * r[1] + a2 * r[2];
  const double th = atan2(S, s);
  if (dth) {
    const double q = a0 * a0 + a1 * a1 + a2 * a2;
    const double y0 = r0[1] * r[2] - r0[2] * r[1], y1 = r0[2] * r[0] - r0[0] * r[2], y2 = r0[0] * r[1] - r0[1] * r[0];
    const double be = r0[0] * r[0] + r0[1] * r[1] + r0[2] * r[2];
    if (S > 1e-12 * sqrt(q)) {
      const double dS = (x0 * y0 + x1 * y1 + x2 * y2) / S;
      *dth = (s * dS - S * be) / q;
    } else {
      *dth = s * sqrt(y0 * y0 + y1 * y1 + y2 * y2) / q;  // the limit where the angle vanishes
    }
  }
  return th;
}

// Cost terms at up to three depths l[0..np): g = sum w th dth/dl, e = sum w
// th^2 and the Gauss-Newton curvature hgn = sum w (dth/dl)^2 (at l[0]) over
// the views in `set`, rays read from LDS.
struct TriEval {
  double g[3], e[3], hgn;
};

template <int VMAX>
__device__ inline TriEval tri_eval(const TriViewDev* views, const double (*rx)[kWave], const double (*ry)[kWave],
                                   const double (*rz)[kWave], const float (*wk)[kWave], int lane, uint32_t set,
                                   const double r0[3], const double* l, int np) {
  TriEval out{};
  for (uint32_t m = set; m != 0; m &= m - 1) {
    const int k = __ffs(m) - 1;
    const double r[3] = {rx[k][lane], ry[k][lane], rz[k][lane]};
    const double w = wk[k][lane];
    for (int t = 0; t < np; ++t) {
      double J;
      const double th = tri_angle_d(views[k + 1].b, r0, l[t], r, &J);
      out.g[t] += w * th * J;
      out.e[t] += w * th * th;
      if (t == 0) out.hgn += w * J * J;
    }
  }
  return out;
}

// One wave per workgroup; each lane's match rays and weights live in LDS
// ([view][lane], so the lanes of a wave hit distinct banks).
template <int VMAX>
__global__ __launch_bounds__(kWave) void triangulate_kernel(TriArgs a) {
  __shared__ TriViewDev s_view[VMAX + 1];  // [0]: the mapping camera (b unused)
  __shared__ double s_rx[VMAX][kWave], s_ry[VMAX][kWave], s_rz[VMAX][kWave];
  __shared__ float s_w[VMAX][kWave];
  const int lane = threadIdx.x;
  for (int e = lane; e <= a.V; e += kWave) {
    const double* src = a.views + 16 * e;
    TriViewDev v;
    v.fx = src[0]; v.fy = src[1]; v.cx = src[2]; v.cy = src[3];
    for (int c = 0; c < 9; ++c) v.Rt[c] = src[4 + c];
    for (int c = 0; c < 3; ++c) v.b[c] = src[13 + c];
    v.pad = 0.0;
    s_view[e] = v;
  }
  __syncthreads();
  const int64_t HW = (int64_t)a.H * a.W;
  const int64_t p = (int64_t)blockIdx.x * kWave + lane;
  if (p >= HW) return;
  const int i = (int)(p / a.W), j = (int)(p - (int64_t)i * a.W);
  double r0[3];
  tri_ray(s_view[0], (double)j + 0.5, (double)i + 0.5, r0);
  const double ep = r0[0] * r0[0] + r0[1] * r0[1] + r0[2] * r0[2];

  // the pixel's matches: unit rays and weights
  uint32_t ok = 0;
  for (int k = 0; k < a.V; ++k) {
    const int64_t o = (int64_t)k * HW + p;
    const float mu = a.mu[o], mv = a.mv[o], cf = a.conf[o];
    if (cf >= a.min_conf && isfinite(mu) && isfinite(mv)) {
      double r[3];
      tri_ray(s_view[k + 1], mu, mv, r);
      const double inv = 1.0 / sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
      s_rx[k][lane] = r[0] * inv;
      s_ry[k][lane] = r[1] * inv;
      s_rz[k][lane] = r[2] * inv;
      s_w[k][lane] = cf;
      ok |= 1u << k;
    }
  }

  // hypotheses, in view order
  int best_n = 0;
  double best_l = 0.0;
  uint32_t best_set = 0;
  for (uint32_t mh = ok; mh != 0; mh &= mh - 1) {
    const int h = __ffs(mh) - 1;
    const double* b = s_view[h + 1].b;
    const double rh[3] = {s_rx[h][lane], s_ry[h][lane], s_rz[h][lane]};
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
    for (uint32_t mk = ok; mk != 0; mk &= mk - 1) {
      const int k = __ffs(mk) - 1;
      const double* bk = s_view[k + 1].b;
      const double a0 = bk[0] + l * r0[0], a1 = bk[1] + l * r0[1], a2 = bk[2] + l * r0[2];
      const double s = a0 * s_rx[k][lane] + a1 * s_ry[k][lane] + a2 * s_rz[k][lane];
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

  double depth = 0.0;
  if (best_n > 0 && best_n >= a.min_inliers) {
    double l = best_l;
    double pts[3] = {l, 0.0, 0.0};
    double e = tri_eval<VMAX>(s_view, s_rx, s_ry, s_rz, s_w, lane, best_set, r0, pts, 1).e[0];
    for (int it = 0; it < a.max_iters; ++it) {
      const double dl = 1e-6 * l;
      pts[0] = l; pts[1] = l + dl; pts[2] = l - dl;
      const TriEval ev = tri_eval<VMAX>(s_view, s_rx, s_ry, s_rz, s_w, lane, best_set, r0, pts, 3);
      const double g = ev.g[0];
      if (g == 0.0) break;
      const double gp = (ev.g[1] - ev.g[2]) / (2.0 * dl);
      const double curv = gp > 0.0 ? gp : ev.hgn;
      if (!(curv > 0.0)) break;
      double step = -g / curv;
      bool moved = false;
      for (int half = 0; half < 30; ++half) {
        const double ln = l + step;
        if (ln > 0.0) {
          pts[0] = ln;
          const double en = tri_eval<VMAX>(s_view, s_rx, s_ry, s_rz, s_w, lane, best_set, r0, pts, 1).e[0];
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
    depth = l > 0.0 ? l : 0.0;
  }
  const float d32 = (float)depth;
  if (a.depth) a.depth[p] = d32;
  if (a.inliers) a.inliers[p] = best_n;
  if (a.codes) a.codes[p] = depth > 0.0 ? log8_code(d32) : (uint8_t)0;
}

int tri_vmax(int V) { return V <= 8 ? 8 : (V <= 16 ? 16 : 32); }

hipError_t launch_triangulate(const TriArgs& a, hipStream_t s) {
  const int64_t HW = (int64_t)a.H * a.W;
  if (HW <= 0) return hipSuccess;
  const dim3 grid((unsigned)((HW + kWave - 1) / kWave));
  switch (tri_vmax(a.V)) {
    case 8: hipLaunchKernelGGL(triangulate_kernel<8>, grid, dim3(kWave), 0, s, a); break;
    case 16: hipLaunchKernelGGL(triangulate_kernel<16>, grid, dim3(kWave), 0, s, a); break;
    default: hipLaunchKernelGGL(triangulate_kernel<32>, grid, dim3(kWave), 0, s, a); break;
  }
  return hipGetLastError();
}

}  // namespace imloc
