/*
 * triangulate.c -- FP64 CPU oracle of ImLoc's mapping-time depth estimation
 * by dense matching (Sec. 3.3 "Depth Estimation by Dense Matching").
 *
 * TEST INFRASTRUCTURE ONLY (see imloc_oracle.h).  One pixel at a time, plain
 * loops, FP64.
 *
 * For a pixel of the mapping image, whose pose is known, the world point is
 * X(l) = C0 + l r0 with r0 = R0^T K0^-1 [u, v, 1]^T, so l is the z-depth.  Each
 * match (a pixel of a covisible image k with confidence >= 0.05) observes the
 * point along the unit ray rk = R_k^T K_k^-1 [u_k, v_k, 1]^T / |.| from C_k.  The
 * angular error of depth l for match k is the angle between X(l) - C_k and rk.
 *
 * Readings taken where the paper is silent:
 *   - pixel (row i, col j) has centre (j + 0.5, i + 0.5);
 *   - the depth hypothesis of a match is the depth that minimises its own
 *     angular error; it exists iff that minimum is attained at a finite l > 0;
 *   - a match is an inlier of a depth iff its angular error is strictly below
 *     the threshold (2 degrees);
 *   - the hypothesis with the most inliers wins, ties going to the lowest
 *     view index;
 *   - the refinement minimises the confidence-weighted sum of squared angular
 *     errors over the inliers of the winning hypothesis (a fixed set), by a
 *     safeguarded 1-D Newton iteration, to convergence;
 *   - the depth is kept iff that inlier set has more than 3 members
 *     (min_inliers = 4); otherwise the output depth is 0.
 */
#include "imloc_oracle.h"

#include <math.h>
#include <stdlib.h>

typedef struct {
  double C0[3], r0[3];
} tri_pixel;

static double dot3d(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void cross3d(const double *a, const double *b, double *o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

/* camera centre -R^T t and world direction R^T K^-1 [u, v, 1]^T */
static void centre_of(const orc_pose *T, double C[3]) {
  for (int r = 0; r < 3; ++r) C[r] = -(T->R[r] * T->t[0] + T->R[3 + r] * T->t[1] + T->R[6 + r] * T->t[2]);
}

static void ray_of(const orc_camera *K, const orc_pose *T, double u, double v, double r[3]) {
  const double d[3] = {(u - K->cx) / K->fx, (v - K->cy) / K->fy, 1.0};
  for (int c = 0; c < 3; ++c) r[c] = T->R[c] * d[0] + T->R[3 + c] * d[1] + T->R[6 + c] * d[2];
}

/* Angular error (radians) of depth l for the observation (Ck, unit rk). */
double orc_tri_angle(const double C0[3], const double r0[3], double l, const double Ck[3], const double rk[3]) {
  double a[3], x[3];
  for (int c = 0; c < 3; ++c) a[c] = C0[c] + l * r0[c] - Ck[c];
  cross3d(a, rk, x);
  return atan2(sqrt(dot3d(x, x)), dot3d(a, rk));
}

/* Depth minimising the angular error of one observation.  With b = C0 - Ck,
 * the cosine of the angle is (al + l be) / sqrt(ga + 2 l de + l^2 ep) where
 * al = b.rk, be = r0.rk, ga = b.b, de = b.r0, ep = r0.r0; its derivative
 * vanishes where (be ga - al de) + l (be de - al ep) = 0, one root.  That root
 * is the angle's minimum iff the cosine there exceeds its limits +-be/sqrt(ep)
 * at l -> +-inf.  Returns 0 if there is no minimum at a finite l > 0. */
int orc_tri_hypothesis(const double C0[3], const double r0[3], const double Ck[3], const double rk[3], double *l) {
  double b[3];
  for (int c = 0; c < 3; ++c) b[c] = C0[c] - Ck[c];
  const double al = dot3d(b, rk), be = dot3d(r0, rk), ga = dot3d(b, b), de = dot3d(b, r0), ep = dot3d(r0, r0);
  const double den = be * de - al * ep;
  if (den == 0.0) return 0;
  const double x = (al * de - be * ga) / den;
  if (!(x > 0.0) || !isfinite(x)) return 0;
  const double cosx = (al + x * be) / sqrt(ga + 2.0 * x * de + x * x * ep);
  if (!(cosx > fabs(be) / sqrt(ep))) return 0;
  *l = x;
  return 1;
}

/* Weighted sum of squared angular errors over the observations in use. */
static double tri_cost(const tri_pixel *px, double l, int n, const double (*Ck)[3], const double (*rk)[3],
                       const double *w) {
  double e = 0.0;
  for (int k = 0; k < n; ++k) {
    const double th = orc_tri_angle(px->C0, px->r0, l, Ck[k], rk[k]);
    e += w[k] * th * th;
  }
  return e;
}

/* d(angle)/dl of one observation (the limit where the angle vanishes). */
static double tri_dangle(const tri_pixel *px, double l, const double Ck[3], const double rk[3]) {
  double a[3], x[3], y[3];
  for (int c = 0; c < 3; ++c) a[c] = px->C0[c] + l * px->r0[c] - Ck[c];
  cross3d(a, rk, x);
  cross3d(px->r0, rk, y);
  const double S = sqrt(dot3d(x, x)), s = dot3d(a, rk), q = dot3d(a, a);
  const double be = dot3d(px->r0, rk);
  if (S > 1e-12 * sqrt(q)) {
    const double dS = dot3d(x, y) / S;
    return (s * dS - S * be) / q;
  }
  return s * sqrt(dot3d(y, y)) / q;
}

/* Half the derivative of the cost: sum_k w_k angle_k d(angle_k)/dl; and the
 * Gauss-Newton curvature sum_k w_k (d angle_k / dl)^2. */
static double tri_grad(const tri_pixel *px, double l, int n, const double (*Ck)[3], const double (*rk)[3],
                       const double *w, double *gn) {
  double g = 0.0, h = 0.0;
  for (int k = 0; k < n; ++k) {
    const double th = orc_tri_angle(px->C0, px->r0, l, Ck[k], rk[k]);
    const double J = tri_dangle(px, l, Ck[k], rk[k]);
    g += w[k] * th * J;
    h += w[k] * J * J;
  }
  if (gn) *gn = h;
  return g;
}

/* Newton's method on the cost's derivative (its own derivative by a central
 * difference, the Gauss-Newton curvature where that is not positive), a step
 * that raises the cost halved up to 30 times, until the step is below 1e-12 l
 * or max_iters steps.  A step below 1e-12 l counts as convergence also while
 * it is being halved: it is not tried (near the minimum the cost's rounding
 * noise exceeds the decrease of such a step, and trying it would only halve
 * it on towards one ulp). */
static double tri_refine_full(const double C0[3], const double r0[3], double l0, int n, const double (*Ck)[3],
                              const double (*rk)[3], const double *w, int max_iters, double *cost_out,
                              double *curv_out);

double orc_tri_refine(const double C0[3], const double r0[3], double l0, int n, const double (*Ck)[3],
                      const double (*rk)[3], const double *w, int max_iters) {
  return tri_refine_full(C0, r0, l0, n, Ck, rk, w, max_iters, NULL, NULL);
}

/* The refinement, and the cost and its second derivative at the result (the
 * derivative of the cost's derivative by the same central difference). */
static double tri_refine_full(const double C0[3], const double r0[3], double l0, int n, const double (*Ck)[3],
                              const double (*rk)[3], const double *w, int max_iters, double *cost_out,
                              double *curv_out) {
  tri_pixel px;
  for (int c = 0; c < 3; ++c) { px.C0[c] = C0[c]; px.r0[c] = r0[c]; }
  double l = l0, e = tri_cost(&px, l, n, Ck, rk, w);
  for (int it = 0; it < max_iters; ++it) {
    double h;
    const double g = tri_grad(&px, l, n, Ck, rk, w, &h);
    if (g == 0.0) break;
    const double dl = 1e-6 * l;
    const double gp = (tri_grad(&px, l + dl, n, Ck, rk, w, NULL) - tri_grad(&px, l - dl, n, Ck, rk, w, NULL)) / (2.0 * dl);
    const double curv = gp > 0.0 ? gp : h;
    if (!(curv > 0.0)) break;
    double step = -g / curv;
    int moved = 0;
    for (int half = 0; half < 30; ++half) {
      if (fabs(step) <= 1e-12 * l) break;
      const double ln = l + step;
      if (ln > 0.0) {
        const double en = tri_cost(&px, ln, n, Ck, rk, w);
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
  if (cost_out) *cost_out = e;
  if (curv_out) {
    const double dl = 1e-6 * l;
    /* d(cost)/dl = 2 g, so d2(cost)/dl2 = 2 dg/dl */
    *curv_out = 2.0 * (tri_grad(&px, l + dl, n, Ck, rk, w, NULL) - tri_grad(&px, l - dl, n, Ck, rk, w, NULL)) / (2.0 * dl);
  }
  return l;
}

void orc_triangulate(int32_t H, int32_t W, const orc_camera *K0, const orc_pose *T0, int32_t V,
                     const orc_camera *Kv, const orc_pose *Tv, const float *mu, const float *mv, const float *conf,
                     const orc_tri_params *p, double *depth, int32_t *inliers, int32_t *best_view,
                     uint8_t *ambiguous, double *cost, double *curv) {
  const double thr = p->angle_deg * (M_PI / 180.0);
  const float min_conf = (float)p->min_conf;
  double (*Cv)[3] = malloc(sizeof(double[3]) * (V > 0 ? V : 1));
  double (*rk)[3] = malloc(sizeof(double[3]) * (V > 0 ? V : 1));
  double (*Cs)[3] = malloc(sizeof(double[3]) * (V > 0 ? V : 1));
  double (*rs)[3] = malloc(sizeof(double[3]) * (V > 0 ? V : 1));
  double *ws = malloc(sizeof(double) * (V > 0 ? V : 1));
  int *ok = malloc(sizeof(int) * (V > 0 ? V : 1));
  double *wk = malloc(sizeof(double) * (V > 0 ? V : 1));
  for (int k = 0; k < V; ++k) centre_of(&Tv[k], Cv[k]);
  tri_pixel px;
  centre_of(T0, px.C0);
  for (int64_t i = 0; i < H; ++i) {
    for (int64_t j = 0; j < W; ++j) {
      const int64_t pix = i * W + j;
      ray_of(K0, T0, (double)j + 0.5, (double)i + 0.5, px.r0);
      for (int k = 0; k < V; ++k) {
        const int64_t o = (int64_t)k * H * W + pix;
        ok[k] = conf[o] >= min_conf && isfinite(mu[o]) && isfinite(mv[o]);
        if (!ok[k]) continue;
        ray_of(&Kv[k], &Tv[k], mu[o], mv[o], rk[k]);
        const double nr = sqrt(dot3d(rk[k], rk[k]));
        for (int c = 0; c < 3; ++c) rk[k][c] /= nr;
        wk[k] = conf[o];
      }
      int best = -1, best_n = 0;
      double best_l = 0.0, margin = INFINITY;
      for (int h = 0; h < V; ++h) {
        double l;
        if (!ok[h] || !orc_tri_hypothesis(px.C0, px.r0, Cv[h], rk[h], &l)) continue;
        int cnt = 0;
        for (int k = 0; k < V; ++k) {
          if (!ok[k]) continue;
          const double th = orc_tri_angle(px.C0, px.r0, l, Cv[k], rk[k]);
          if (th < thr) ++cnt;
          if (fabs(th - thr) < margin) margin = fabs(th - thr);
        }
        if (cnt > best_n) { best = h; best_n = cnt; best_l = l; }
      }
      depth[pix] = 0.0;
      inliers[pix] = best_n;
      if (cost) cost[pix] = 0.0;
      if (curv) curv[pix] = 0.0;
      if (best_view) best_view[pix] = best;
      if (ambiguous) ambiguous[pix] = margin < 1e-9;
      if (best < 0 || best_n < p->min_inliers) continue;
      int n = 0;
      for (int k = 0; k < V; ++k) {
        if (!ok[k] || !(orc_tri_angle(px.C0, px.r0, best_l, Cv[k], rk[k]) < thr)) continue;
        for (int c = 0; c < 3; ++c) { Cs[n][c] = Cv[k][c]; rs[n][c] = rk[k][c]; }
        ws[n++] = wk[k];
      }
      double ce = 0.0, cc = 0.0;
      const double l = tri_refine_full(px.C0, px.r0, best_l, n, (const double (*)[3])Cs, (const double (*)[3])rs, ws,
                                       p->max_refine_iters, &ce, &cc);
      if (cost) cost[pix] = ce;
      if (curv) curv[pix] = cc;
      depth[pix] = l > 0.0 ? l : 0.0;
    }
  }
  free(Cv); free(rk); free(Cs); free(rs); free(ws); free(ok); free(wk);
}
