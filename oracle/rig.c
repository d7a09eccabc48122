/*
 * rig.c -- FP64 CPU oracle of LO-RANSAC for a multi-camera rig (generalized
 * absolute pose; ImLoc Appendix "LaMAR Hololens Results": a GPU generalized
 * absolute pose estimator for rig queries, with the LO-RANSAC of Sec. 3.3
 * "Pose Estimation").
 *
 * TEST INFRASTRUCTURE ONLY (see imloc_oracle.h).  Plain loops, FP64.
 *
 * Model: the query is a rig of C cameras with intrinsics K_c and known
 * cam_from_rig (R_c, t_c); the unknown is rig_from_world (R, t).  A world
 * point X seen by camera c projects through x_c = R_c (R X + t) + t_c.
 *
 * Minimal solver (generalised P3P): three rays in the rig frame, origin o_i =
 * -R_c^T t_c and unit direction f_i = R_c^T K_c^-1 [u, v, 1]^T / |.|, and three
 * world points.  The rig-frame points o_i + l_i f_i must keep the world
 * distances d_ij, three quadrics in (l1, l2, l3).  Here they are solved as a
 * definition: for l1 on the interval where both l2 (from the (1,2) distance)
 * and l3 (from the (1,3) distance) are real, each of the 4 sign branches gives
 * l2(l1), l3(l1) in closed form, and the (2,3) distance residual is scanned
 * for sign changes, bisected and Newton-polished on all three quadrics.  The
 * pose aligns the rig-frame triangle with the world triangle.
 *
 * Everything else follows the single-camera oracle with camera-aware
 * residuals: MSAC scoring, top-k LO (Gauss-Newton on the truncated cost, left
 * update of the rig pose), stopping rule, Cauchy refinement over the inliers
 * of the full set, inlier mask.
 */
#include "imloc_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static double rdot(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static void rcross(const double *a, const double *b, double *o) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}

/* 3x3 determinant and adjugate (row-major) */
static double rdet3(const double *M) {
  return M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) + M[2] * (M[3] * M[7] - M[4] * M[6]);
}

static void radj3(const double *M, double *A) {
  A[0] = M[4] * M[8] - M[5] * M[7]; A[1] = M[2] * M[7] - M[1] * M[8]; A[2] = M[1] * M[5] - M[2] * M[4];
  A[3] = M[5] * M[6] - M[3] * M[8]; A[4] = M[0] * M[8] - M[2] * M[6]; A[5] = M[2] * M[3] - M[0] * M[5];
  A[6] = M[3] * M[7] - M[4] * M[6]; A[7] = M[1] * M[6] - M[0] * M[7]; A[8] = M[0] * M[4] - M[1] * M[3];
}

/* ------------------------------------------------------------------------- */
/* Generalised P3P.                                                            */
/* ------------------------------------------------------------------------- */
typedef struct {
  double o[3][3], f[3][3], d2[3];  /* d2: |X1-X2|^2, |X1-X3|^2, |X2-X3|^2 */
} gp3p_in;

/* the three distance residuals at (l1, l2, l3) */
static void gp3p_res(const gp3p_in *g, const double l[3], double r[3]) {
  const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
  for (int e = 0; e < 3; ++e) {
    const int a = pa[e], b = pb[e];
    double v[3];
    for (int c = 0; c < 3; ++c) v[c] = g->o[a][c] + l[a] * g->f[a][c] - g->o[b][c] - l[b] * g->f[b][c];
    r[e] = rdot(v, v) - g->d2[e];
  }
}

/* l_k of the (1,k) distance for given l1 on branch s (+1/-1); 0 if not real */
static int gp3p_branch(const gp3p_in *g, int k, double l1, int s, double *lk) {
  double D[3];
  for (int c = 0; c < 3; ++c) D[c] = g->o[0][c] - g->o[k][c];
  const double ck = rdot(g->f[0], g->f[k]), ek = rdot(D, g->f[k]), g1 = rdot(D, g->f[0]);
  const double kk = rdot(D, D) - g->d2[k - 1];
  /* |D + l1 f1 - lk fk|^2 = d^2:  lk^2 - 2 lk (l1 ck + ek) + l1^2 + 2 l1 g1 + kk = 0 */
  const double mid = l1 * ck + ek;
  const double disc = mid * mid - (l1 * l1 + 2.0 * l1 * g1 + kk);
  if (disc < 0.0) return 0;
  *lk = mid + s * sqrt(disc);
  return 1;
}

/* interval of l1 where the (1,k) distance has a real lk */
static int gp3p_interval(const gp3p_in *g, int k, double *lo, double *hi) {
  double D[3];
  for (int c = 0; c < 3; ++c) D[c] = g->o[0][c] - g->o[k][c];
  const double ck = rdot(g->f[0], g->f[k]), ek = rdot(D, g->f[k]), g1 = rdot(D, g->f[0]);
  const double kk = rdot(D, D) - g->d2[k - 1];
  /* disc(l1) = (ck^2 - 1) l1^2 + 2 (ck ek - g1) l1 + (ek^2 - kk) >= 0 */
  const double A = ck * ck - 1.0, B = 2.0 * (ck * ek - g1), Cc = ek * ek - kk;
  if (!(A < 0.0)) return 0;  /* parallel rays */
  const double dq = B * B - 4.0 * A * Cc;
  if (dq < 0.0) return 0;
  const double r1 = (-B + sqrt(dq)) / (2.0 * A), r2 = (-B - sqrt(dq)) / (2.0 * A);
  *lo = r1 < r2 ? r1 : r2;
  *hi = r1 < r2 ? r2 : r1;
  return 1;
}

static double gp3p_f(const gp3p_in *g, double l1, int s2, int s3, int *ok) {
  double l[3] = {l1, 0.0, 0.0}, r[3];
  *ok = gp3p_branch(g, 1, l1, s2, &l[1]) && gp3p_branch(g, 2, l1, s3, &l[2]);
  if (!*ok) return 0.0;
  gp3p_res(g, l, r);
  return r[2];
}

/* Newton on the three quadrics (3x3 Jacobian), while the residual drops. */
static void gp3p_polish(const gp3p_in *g, double l[3]) {
  for (int it = 0; it < 8; ++it) {
    double r[3];
    gp3p_res(g, l, r);
    const double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    /* d/dl of |o_a + l_a f_a - o_b - l_b f_b|^2: 2 v.f_a, -2 v.f_b */
    double J[9] = {0};
    const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
    for (int e = 0; e < 3; ++e) {
      double v[3];
      for (int c = 0; c < 3; ++c) v[c] = g->o[pa[e]][c] + l[pa[e]] * g->f[pa[e]][c] - g->o[pb[e]][c] - l[pb[e]] * g->f[pb[e]][c];
      J[3 * e + pa[e]] = 2.0 * rdot(v, g->f[pa[e]]);
      J[3 * e + pb[e]] = -2.0 * rdot(v, g->f[pb[e]]);
    }
    const double det = rdet3(J);
    if (!(fabs(det) > 0.0)) return;
    double A[9], n[3], r2[3];
    radj3(J, A);
    for (int k = 0; k < 3; ++k) n[k] = l[k] - (A[3 * k] * r[0] + A[3 * k + 1] * r[1] + A[3 * k + 2] * r[2]) / det;
    gp3p_res(g, n, r2);
    if (!(r2[0] * r2[0] + r2[1] * r2[1] + r2[2] * r2[2] < rr)) return;
    l[0] = n[0]; l[1] = n[1]; l[2] = n[2];
  }
}

/* R, t with P_i = R X_i + t from the two triangle frames. */
static int rig_pose_from_triangles(const double P[3][3], const double X[3][3], orc_pose *o) {
  double a[3], b[3], c[3], A[3], B[3], Cx[3];
  for (int k = 0; k < 3; ++k) {
    a[k] = X[0][k] - X[1][k]; b[k] = X[0][k] - X[2][k];
    A[k] = P[0][k] - P[1][k]; B[k] = P[0][k] - P[2][k];
  }
  rcross(a, b, c);
  rcross(A, B, Cx);
  double Mx[9], My[9], adj[9];
  for (int r = 0; r < 3; ++r) {
    Mx[3 * r] = a[r]; Mx[3 * r + 1] = b[r]; Mx[3 * r + 2] = c[r];
    My[3 * r] = A[r]; My[3 * r + 1] = B[r]; My[3 * r + 2] = Cx[r];
  }
  const double det = rdet3(Mx);
  if (!(fabs(det) > 0.0)) return 0;
  radj3(Mx, adj);
  double R[9];
  for (int r = 0; r < 3; ++r)
    for (int cc = 0; cc < 3; ++cc)
      R[3 * r + cc] = (My[3 * r] * adj[cc] + My[3 * r + 1] * adj[3 + cc] + My[3 * r + 2] * adj[6 + cc]) / det;
  /* two Newton-Schulz steps towards the nearest rotation */
  for (int it = 0; it < 2; ++it) {
    double RtR[9], Rn[9];
    for (int r = 0; r < 3; ++r)
      for (int cc = 0; cc < 3; ++cc) RtR[3 * r + cc] = R[r] * R[cc] + R[3 + r] * R[3 + cc] + R[6 + r] * R[6 + cc];
    for (int r = 0; r < 3; ++r)
      for (int cc = 0; cc < 3; ++cc) {
        double s = 0.0;
        for (int m = 0; m < 3; ++m) s += R[3 * r + m] * ((m == cc ? 3.0 : 0.0) - RtR[3 * m + cc]);
        Rn[3 * r + cc] = 0.5 * s;
      }
    memcpy(R, Rn, sizeof(R));
  }
  memcpy(o->R, R, sizeof(R));
  for (int r = 0; r < 3; ++r) o->t[r] = P[0][r] - (R[3 * r] * X[0][0] + R[3 * r + 1] * X[0][1] + R[3 * r + 2] * X[0][2]);
  return 1;
}

int orc_gp3p(const double o[9], const double f[9], const double Xw[9], orc_pose out[8], double depths[24],
             int32_t *ill) {
  gp3p_in g;
  *ill = 0;
  for (int i = 0; i < 3; ++i) {
    const double nf = sqrt(f[3 * i] * f[3 * i] + f[3 * i + 1] * f[3 * i + 1] + f[3 * i + 2] * f[3 * i + 2]);
    for (int c = 0; c < 3; ++c) { g.o[i][c] = o[3 * i + c]; g.f[i][c] = f[3 * i + c] / nf; }
  }
  const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
  double dsum = 0.0;
  for (int e = 0; e < 3; ++e) {
    double v[3];
    for (int c = 0; c < 3; ++c) v[c] = Xw[3 * pa[e] + c] - Xw[3 * pb[e] + c];
    g.d2[e] = rdot(v, v);
    dsum += g.d2[e];
  }
  double lo2, hi2, lo3, hi3;
  if (!gp3p_interval(&g, 1, &lo2, &hi2) || !gp3p_interval(&g, 2, &lo3, &hi3)) return 0;
  double lo = fmax(0.0, fmax(lo2, lo3)), hi = fmin(hi2, hi3);
  if (!(hi > lo)) return 0;
  const int N = 8192;
  const double mid = 0.5 * (lo + hi), half = 0.5 * (hi - lo);
  double sols[32][3];
  int ns = 0;
  for (int s2 = -1; s2 <= 1; s2 += 2) {
    for (int s3 = -1; s3 <= 1; s3 += 2) {
      double tp = 0.0, fp = 0.0;
      int okp = 0;
      double fm1 = 0.0, fm2 = 0.0;  /* previous two |F| for the tangency test */
      for (int it = 0; it <= N; ++it) {
        const double th = M_PI * (double)it / N;
        const double l1 = mid - half * cos(th);
        int ok;
        const double fv = gp3p_f(&g, l1, s2, s3, &ok);
        if (ok && okp && ((fv < 0.0) != (fp < 0.0) || fv == 0.0)) {
          /* bisect in theta */
          double a = tp, b = th, fa = fp;
          for (int k = 0; k < 200; ++k) {
            const double m = 0.5 * (a + b);
            if (m <= a || m >= b) break;
            int okm;
            const double fmv = gp3p_f(&g, mid - half * cos(m), s2, s3, &okm);
            if (!okm) break;
            if (fmv == 0.0) { a = b = m; break; }
            if ((fmv < 0.0) == (fa < 0.0)) { a = m; fa = fmv; } else { b = m; }
          }
          const double l1r = mid - half * cos(0.5 * (a + b));
          double l[3] = {l1r, 0.0, 0.0};
          if (gp3p_branch(&g, 1, l1r, s2, &l[1]) && gp3p_branch(&g, 2, l1r, s3, &l[2]) && ns < 32) {
            sols[ns][0] = l[0]; sols[ns][1] = l[1]; sols[ns][2] = l[2];
            ++ns;
          }
        }
        if (ok && it >= 2 && okp) {
          /* a local minimum of |F| near zero without a sign change: near-double root */
          const double av = fabs(fv);
          if (fm1 < fm2 && fm1 < av && fm1 < 1e-6 * dsum && (fv < 0.0) == (fp < 0.0)) *ill = 1;
        }
        fm2 = fm1;
        fm1 = ok ? fabs(fv) : INFINITY;
        tp = th;
        fp = fv;
        okp = ok;
      }
    }
  }
  /* positive depths, polished, consistent, deduplicated */
  double keep[8][3];
  int nk = 0;
  for (int s = 0; s < ns; ++s) {
    double l[3] = {sols[s][0], sols[s][1], sols[s][2]};
    if (!(l[0] > 0.0 && l[1] > 0.0 && l[2] > 0.0)) continue;
    gp3p_polish(&g, l);
    if (!(l[0] > 0.0 && l[1] > 0.0 && l[2] > 0.0)) continue;
    double r[3];
    gp3p_res(&g, l, r);
    if (!(fabs(r[0]) + fabs(r[1]) + fabs(r[2]) < 1e-6 * dsum)) continue;
    int dup = 0;
    for (int e = 0; e < nk; ++e)
      if (fabs(keep[e][0] - l[0]) + fabs(keep[e][1] - l[1]) + fabs(keep[e][2] - l[2]) <= 1e-9 * (l[0] + l[1] + l[2]))
        dup = 1;
    if (dup || nk >= 8) continue;
    if (fmin(l[0], fmin(l[1], l[2])) < 1e-6 * sqrt(dsum)) *ill = 1;
    keep[nk][0] = l[0]; keep[nk][1] = l[1]; keep[nk][2] = l[2];
    ++nk;
  }
  /* canonical order: l1, then l2 */
  for (int a = 1; a < nk; ++a)
    for (int b = a; b > 0 && (keep[b][0] < keep[b - 1][0] || (keep[b][0] == keep[b - 1][0] && keep[b][1] < keep[b - 1][1])); --b)
      for (int c = 0; c < 3; ++c) { const double t = keep[b][c]; keep[b][c] = keep[b - 1][c]; keep[b - 1][c] = t; }
  int nout = 0;
  for (int s = 0; s < nk; ++s) {
    double P[3][3], X[3][3];
    for (int i = 0; i < 3; ++i)
      for (int c = 0; c < 3; ++c) { P[i][c] = g.o[i][c] + keep[s][i] * g.f[i][c]; X[i][c] = Xw[3 * i + c]; }
    if (!rig_pose_from_triangles(P, X, &out[nout])) continue;
    if (depths) for (int i = 0; i < 3; ++i) depths[3 * nout + i] = keep[s][i];
    ++nout;
  }
  return nout;
}

/* ------------------------------------------------------------------------- */
/* Camera-aware residuals.                                                     */
/* ------------------------------------------------------------------------- */
static double rig_w(const orc_rig_corr *c, int64_t i) { return c->w ? (double)c->w[i] : 1.0; }

/* x_c = R_c (R X + t) + t_c of correspondence i; also the rig-frame point */
static void rig_point(const orc_pose *P, const orc_rig_camera *cam, const orc_rig_corr *c, int64_t i, double xr[3],
                      double xc[3]) {
  const double X[3] = {c->X[i], c->Y[i], c->Z[i]};
  for (int r = 0; r < 3; ++r) xr[r] = P->R[3 * r] * X[0] + P->R[3 * r + 1] * X[1] + P->R[3 * r + 2] * X[2] + P->t[r];
  const orc_rig_camera *k = &cam[c->cam[i]];
  for (int r = 0; r < 3; ++r) xc[r] = k->R[3 * r] * xr[0] + k->R[3 * r + 1] * xr[1] + k->R[3 * r + 2] * xr[2] + k->t[r];
}

void orc_rig_score(const orc_pose *poses, int64_t np, const orc_rig_corr *c, const orc_rig_camera *cams,
                   double tau, int32_t *count, double *msac) {
  const double tau2 = tau * tau;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t p = 0; p < np; ++p) {
    int32_t cnt = 0;
    double m = 0.0;
    for (int64_t i = 0; i < c->n; ++i) {
      double xr[3], xc[3];
      rig_point(&poses[p], cams, c, i, xr, xc);
      const double w = rig_w(c, i);
      if (!(xc[2] > 0.0)) { m += w * tau2; continue; }
      const orc_camera *K = &cams[c->cam[i]].K;
      const double du = K->fx * xc[0] / xc[2] + K->cx - (double)c->u[i];
      const double dv = K->fy * xc[1] / xc[2] + K->cy - (double)c->v[i];
      const double r2 = du * du + dv * dv;
      if (r2 < tau2) { ++cnt; m += w * r2; } else { m += w * tau2; }
    }
    count[p] = cnt;
    msac[p] = m;
  }
}

/* normal equations of one residual: pixel(x_c) with x_c = R_c P + t_c and the
 * left update P' = Exp(dw) P + dt of the rig-frame point P */
static void rig_accumulate(const orc_camera *K, const double Rc[9], const double xr[3], const double xc[3], double du,
                           double dv, double wgt, double H[36], double g[6]) {
  const double iz = 1.0 / xc[2];
  const double a00 = K->fx * iz, a02 = -K->fx * xc[0] * iz * iz;
  const double a11 = K->fy * iz, a12 = -K->fy * xc[1] * iz * iz;
  /* d P / d(dw, dt) = [-[P]x, I] */
  const double M[3][6] = {{0, xr[2], -xr[1], 1, 0, 0}, {-xr[2], 0, xr[0], 0, 1, 0}, {xr[1], -xr[0], 0, 0, 0, 1}};
  double Mc[3][6];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 6; ++k) Mc[r][k] = Rc[3 * r] * M[0][k] + Rc[3 * r + 1] * M[1][k] + Rc[3 * r + 2] * M[2][k];
  double J[2][6];
  for (int k = 0; k < 6; ++k) {
    J[0][k] = a00 * Mc[0][k] + a02 * Mc[2][k];
    J[1][k] = a11 * Mc[1][k] + a12 * Mc[2][k];
  }
  for (int r = 0; r < 6; ++r) {
    g[r] += wgt * (J[0][r] * du + J[1][r] * dv);
    for (int k = 0; k < 6; ++k) H[6 * r + k] += wgt * (J[0][r] * J[0][k] + J[1][r] * J[1][k]);
  }
}

static int rig_chol6(const double Hin[36], const double b[6], double x[6]) {
  double L[36] = {0};
  for (int i = 0; i < 6; ++i) {
    for (int j = 0; j <= i; ++j) {
      double s = Hin[6 * i + j];
      for (int k = 0; k < j; ++k) s -= L[6 * i + k] * L[6 * j + k];
      if (i == j) {
        if (!(s > 0.0)) return 0;
        L[6 * i + i] = sqrt(s);
      } else {
        L[6 * i + j] = s / L[6 * j + j];
      }
    }
  }
  double y[6];
  for (int i = 0; i < 6; ++i) {
    double s = b[i];
    for (int k = 0; k < i; ++k) s -= L[6 * i + k] * y[k];
    y[i] = s / L[6 * i + i];
  }
  for (int i = 5; i >= 0; --i) {
    double s = y[i];
    for (int k = i + 1; k < 6; ++k) s -= L[6 * k + i] * x[k];
    x[i] = s / L[6 * i + i];
  }
  return 1;
}

static double rig_eval_truncated(const orc_pose *P, const orc_rig_corr *c, const orc_rig_camera *cams, double tau2,
                                 double H[36], double g[6], int64_t *count) {
  memset(H, 0, 36 * sizeof(double));
  memset(g, 0, 6 * sizeof(double));
  double cost = 0.0;
  int64_t cnt = 0;
  for (int64_t i = 0; i < c->n; ++i) {
    double xr[3], xc[3];
    rig_point(P, cams, c, i, xr, xc);
    const double w = rig_w(c, i);
    if (!(xc[2] > 0.0)) { cost += w * tau2; continue; }
    const orc_rig_camera *k = &cams[c->cam[i]];
    const double du = k->K.fx * xc[0] / xc[2] + k->K.cx - (double)c->u[i];
    const double dv = k->K.fy * xc[1] / xc[2] + k->K.cy - (double)c->v[i];
    const double r2 = du * du + dv * dv;
    if (r2 < tau2) {
      ++cnt;
      cost += w * r2;
      rig_accumulate(&k->K, k->R, xr, xc, du, dv, w, H, g);
    } else {
      cost += w * tau2;
    }
  }
  *count = cnt;
  return cost;
}

int orc_rig_lo(const orc_pose *start, const orc_rig_corr *c, const orc_rig_camera *cams, double tau, int32_t iters,
               orc_pose *out, double *cost, int64_t *count) {
  const double tau2 = tau * tau;
  double H[36], g[6];
  orc_pose cur = *start;
  int64_t cnt;
  double cur_cost = rig_eval_truncated(&cur, c, cams, tau2, H, g, &cnt);
  int accepted = 0;
  for (int it = 0; it < iters; ++it) {
    double rhs[6], d[6];
    for (int k = 0; k < 6; ++k) rhs[k] = -g[k];
    if (!rig_chol6(H, rhs, d)) break;
    if (orc_step_converged(d)) break;
    orc_pose cand;
    orc_pose_update(&cur, d, &cand);
    double H2[36], g2[6];
    int64_t cnt2;
    const double nc = rig_eval_truncated(&cand, c, cams, tau2, H2, g2, &cnt2);
    if (!(nc <= cur_cost)) break;
    cur = cand;
    cur_cost = nc;
    cnt = cnt2;
    memcpy(H, H2, sizeof(H));
    memcpy(g, g2, sizeof(g));
    ++accepted;
  }
  *out = cur;
  *cost = cur_cost;
  *count = cnt;
  return accepted;
}

static void rig_mask(const orc_pose *P, const orc_rig_corr *c, const orc_rig_camera *cams, double tau2, uint8_t *m) {
  for (int64_t i = 0; i < c->n; ++i) {
    double xr[3], xc[3];
    rig_point(P, cams, c, i, xr, xc);
    m[i] = 0;
    if (!(xc[2] > 0.0)) continue;
    const orc_camera *K = &cams[c->cam[i]].K;
    const double du = K->fx * xc[0] / xc[2] + K->cx - (double)c->u[i];
    const double dv = K->fy * xc[1] / xc[2] + K->cy - (double)c->v[i];
    if (du * du + dv * dv < tau2) m[i] = 1;
  }
}

static double rig_eval_cauchy(const orc_pose *P, const orc_rig_corr *c, const uint8_t *in_set,
                              const orc_rig_camera *cams, double tau2, double s2, double H[36], double g[6]) {
  memset(H, 0, 36 * sizeof(double));
  memset(g, 0, 6 * sizeof(double));
  double cost = 0.0;
  for (int64_t i = 0; i < c->n; ++i) {
    if (!in_set[i]) continue;
    double xr[3], xc[3];
    rig_point(P, cams, c, i, xr, xc);
    const double w = rig_w(c, i);
    if (!(xc[2] > 0.0)) { cost += w * s2 * log1p(tau2 / s2); continue; }
    const orc_rig_camera *k = &cams[c->cam[i]];
    const double du = k->K.fx * xc[0] / xc[2] + k->K.cx - (double)c->u[i];
    const double dv = k->K.fy * xc[1] / xc[2] + k->K.cy - (double)c->v[i];
    const double r2 = du * du + dv * dv;
    cost += w * s2 * log1p(r2 / s2);
    rig_accumulate(&k->K, k->R, xr, xc, du, dv, w / (1.0 + r2 / s2), H, g);
  }
  return cost;
}

int orc_rig_refine(const orc_pose *start, const orc_rig_corr *c, const orc_rig_camera *cams, double tau, double s,
                   int32_t iters, orc_pose *out, double *cost, int64_t *n_inl) {
  const double tau2 = tau * tau, s2 = s * s;
  double H[36], g[6];
  uint8_t *in_set = (uint8_t *)malloc(c->n > 0 ? (size_t)c->n : 1);
  rig_mask(start, c, cams, tau2, in_set);
  int64_t ni = 0;
  for (int64_t i = 0; i < c->n; ++i) ni += in_set[i];
  orc_pose cur = *start;
  double cur_cost = rig_eval_cauchy(&cur, c, in_set, cams, tau2, s2, H, g);
  int accepted = 0;
  for (int it = 0; it < iters; ++it) {
    double rhs[6], d[6];
    for (int k = 0; k < 6; ++k) rhs[k] = -g[k];
    if (!rig_chol6(H, rhs, d)) break;
    if (orc_step_converged(d)) break;
    orc_pose cand;
    orc_pose_update(&cur, d, &cand);
    double H2[36], g2[6];
    const double nc = rig_eval_cauchy(&cand, c, in_set, cams, tau2, s2, H2, g2);
    if (!(nc <= cur_cost)) break;
    cur = cand;
    cur_cost = nc;
    memcpy(H, H2, sizeof(H));
    memcpy(g, g2, sizeof(g));
    ++accepted;
  }
  free(in_set);
  *out = cur;
  *cost = cur_cost;
  *n_inl = ni;
  return accepted;
}

/* ------------------------------------------------------------------------- */
/* LO-RANSAC driver for a rig query.                                           */
/* ------------------------------------------------------------------------- */
typedef struct {
  orc_pose pose;
  int64_t h;
  int32_t j, count;
  double msac;
} rig_cand;

static int rig_cand_less(const rig_cand *a, const rig_cand *b) {
  if (a->msac != b->msac) return a->msac < b->msac;
  if (a->count != b->count) return a->count > b->count;
  if (a->h != b->h) return a->h < b->h;
  return a->j < b->j;
}

int orc_rig_lo_ransac(const orc_rig_corr *c, const orc_rig_camera *cams, int32_t n_cams, const orc_params *p,
                      orc_pose *pose, uint8_t *mask, orc_stats *st) {
  (void)n_cams;
  memset(st, 0, sizeof(*st));
  st->best_h = -1;
  st->best_j = -1;
  for (int k = 0; k < 9; ++k) pose->R[k] = (k % 4 == 0) ? 1.0 : 0.0;
  pose->t[0] = pose->t[1] = pose->t[2] = 0.0;
  if (mask) memset(mask, 0, (size_t)(c->n > 0 ? c->n : 0));
  const int64_t n = c->n;
  const double tau = p->threshold_px;

  /* scoring set: stride subsample, cameras carried along */
  int64_t m = n;
  if (p->max_score_points > 0 && n > p->max_score_points) m = p->max_score_points;
  float *S = (float *)malloc((size_t)(m > 0 ? m : 1) * 6 * sizeof(float));
  int32_t *Scam = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
  float *Su = S, *Sv = S + m, *SX = S + 2 * m, *SY = S + 3 * m, *SZ = S + 4 * m, *Sw = S + 5 * m;
  for (int64_t jx = 0; jx < m; ++jx) {
    const int64_t i = (m == n) ? jx : (int64_t)(((unsigned __int128)jx * (uint64_t)n) / (uint64_t)m);
    Su[jx] = c->u[i]; Sv[jx] = c->v[i]; SX[jx] = c->X[i]; SY[jx] = c->Y[i]; SZ[jx] = c->Z[i];
    Sw[jx] = c->w ? c->w[i] : 1.0f;
    Scam[jx] = c->cam[i];
  }
  const orc_rig_corr Sc = {Su, Sv, SX, SY, SZ, c->w ? Sw : NULL, Scam, m};

  int have_best = 0;
  double best_cost = INFINITY;
  int64_t best_count = 0;
  orc_pose best;
  const int64_t total = p->fixed_samples > 0 ? p->fixed_samples : p->max_iters;
  const int64_t batch = p->batch > 0 ? p->batch : 1024;
  int64_t drawn = 0;
  rig_cand *cands = (rig_cand *)malloc((size_t)(8 * batch) * sizeof(rig_cand));
  orc_pose *cp = (orc_pose *)malloc((size_t)(8 * batch) * sizeof(orc_pose));
  int32_t *cc = (int32_t *)malloc((size_t)(8 * batch) * sizeof(int32_t));
  double *cm = (double *)malloc((size_t)(8 * batch) * sizeof(double));
  while (m >= 3 && drawn < total) {
    const int64_t B = total - drawn < batch ? total - drawn : batch;
    int64_t nc = 0;
    for (int64_t h = drawn; h < drawn + B; ++h) {
      int32_t idx[3];
      const int ok = p->exhaustive ? orc_unrank_triple((uint64_t)h, m, idx)
                                   : orc_sample_triple(p->seed, p->query_id, (uint64_t)h, m, idx);
      if (!ok) continue;
      double o[9], f[9], Xw[9];
      for (int k = 0; k < 3; ++k) {
        const orc_rig_camera *rc = &cams[Scam[idx[k]]];
        const double d[3] = {((double)Su[idx[k]] - rc->K.cx) / rc->K.fx, ((double)Sv[idx[k]] - rc->K.cy) / rc->K.fy, 1.0};
        for (int a = 0; a < 3; ++a) {
          o[3 * k + a] = -(rc->R[a] * rc->t[0] + rc->R[3 + a] * rc->t[1] + rc->R[6 + a] * rc->t[2]);
          f[3 * k + a] = rc->R[a] * d[0] + rc->R[3 + a] * d[1] + rc->R[6 + a] * d[2];
        }
        Xw[3 * k] = SX[idx[k]]; Xw[3 * k + 1] = SY[idx[k]]; Xw[3 * k + 2] = SZ[idx[k]];
      }
      orc_pose sol[8];
      int32_t ill;
      const int ns = orc_gp3p(o, f, Xw, sol, NULL, &ill);
      for (int jj = 0; jj < ns; ++jj) {
        cands[nc].pose = sol[jj];
        cands[nc].h = h;
        cands[nc].j = jj;
        cp[nc] = sol[jj];
        ++nc;
      }
    }
    orc_rig_score(cp, nc, &Sc, cams, tau, cc, cm);
    for (int64_t k = 0; k < nc; ++k) { cands[k].count = cc[k]; cands[k].msac = cm[k]; }
    st->candidates += nc;
    st->residuals += nc * m;
    const double gate = best_cost;
    int32_t chosen[32];
    int nch = 0;
    const int kmax = p->lo_top_k < 1 ? 1 : (p->lo_top_k < 32 ? p->lo_top_k : 32);
    for (int sel = 0; sel < kmax; ++sel) {
      int64_t arg = -1;
      for (int64_t k = 0; k < nc; ++k) {
        if (!(cands[k].msac < gate)) continue;
        int taken = 0;
        for (int q = 0; q < nch; ++q) taken |= (chosen[q] == k);
        if (taken) continue;
        if (arg < 0 || rig_cand_less(&cands[k], &cands[arg])) arg = k;
      }
      if (arg < 0) break;
      chosen[nch++] = (int32_t)arg;
    }
    for (int q = 0; q < nch; ++q) {
      orc_pose lo_pose;
      double lo_cost;
      int64_t lo_count;
      orc_rig_lo(&cands[chosen[q]].pose, &Sc, cams, tau, p->lo_iters, &lo_pose, &lo_cost, &lo_count);
      st->lo_runs++;
      if (lo_cost < best_cost) {
        best_cost = lo_cost;
        best_count = lo_count;
        best = lo_pose;
        have_best = 1;
        st->best_h = cands[chosen[q]].h;
        st->best_j = cands[chosen[q]].j;
      }
    }
    drawn += B;
    st->batches++;
    if (p->fixed_samples <= 0) {
      const double eps = (double)best_count / (double)m;
      int64_t need = orc_required_samples(eps, p->confidence, p->max_iters);
      if (need < p->min_iters) need = p->min_iters;
      if (need > p->max_iters) need = p->max_iters;
      if (drawn >= need) break;
    }
  }
  st->samples = drawn;
  free(cands); free(cp); free(cc); free(cm);
  free(S); free(Scam);
  if (!have_best) { st->status = 1; return 1; }
  st->best_count = best_count;
  st->best_msac = best_cost;
  orc_pose fin;
  double fcost;
  int64_t ninl;
  orc_rig_refine(&best, c, cams, tau, p->cauchy_scale_px, p->final_iters, &fin, &fcost, &ninl);
  *pose = fin;
  st->final_cost = fcost;
  uint8_t *mk = mask ? mask : (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
  rig_mask(&fin, c, cams, tau * tau, mk);
  int64_t fc = 0;
  for (int64_t i = 0; i < n; ++i) fc += mk[i];
  st->full_count = fc;
  if (!mask) free(mk);
  st->status = 0;
  return 0;
}
