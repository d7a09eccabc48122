/*
 * imloc_oracle.c -- FP64 CPU oracle for the ImLoc pose-estimation hot path.
 *
 * TEST INFRASTRUCTURE ONLY (see imloc_oracle.h).  Plain loops, FP64, no
 * blocking or fusion beyond what each definition states.  The only parallelism
 * is an OpenMP loop over independent pose candidates in the scoring step, which
 * does not change any result.
 *
 * Readings taken where the paper (Sec. 3.3 "Pose Estimation" / "2D-3D
 * Lifting") is silent, in the order they are used below:
 *   - a RANSAC "iteration" is one minimal sample; each gives 0-4 candidates;
 *   - residuals are squared pixel distances through the query intrinsics; a
 *     point with camera depth <= 0 is an outlier; inlier iff r^2 < tau^2;
 *   - the score is MSAC: sum_i w_i min(r_i^2, tau^2), lower is better;
 *   - the local optimisation is Gauss-Newton on that truncated cost with the
 *     inlier set re-evaluated at every iterate, a left update on SO(3), and a
 *     step that raises the cost rejected (which ends the run);
 *   - the stopping rule is the standard RANSAC bound for minimal size 3;
 *   - the final Cauchy loss is rho(r^2) = s^2 ln(1 + r^2/s^2) over the inliers
 *     of the full set at the best pose, held fixed during the refinement;
 *   - depth is z-depth; poses are cam_from_world; the centre of pixel
 *     (row i, col j) is (j + 0.5, i + 0.5); bilinear taps sit at
 *     (db_u - 0.5, db_v - 0.5); a tap footprint leaving the image, or any used
 *     tap that is not finite and positive, makes the depth invalid.
 */
#include "imloc_oracle.h"

#include <float.h>
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as    */
/* easy as 1, 2, 3", SC 2011): ten rounds of two 64x64->128 multiplies, the   */
/* high halves xor-ed with the other words and the round key, key bumped by   */
/* the Weyl constants between rounds.                                          */
/* ------------------------------------------------------------------------- */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    unsigned __int128 p0 = (unsigned __int128)M0 * x0;
    unsigned __int128 p1 = (unsigned __int128)M1 * x2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t y0 = hi1 ^ x1 ^ k0;
    uint64_t y1 = lo1;
    uint64_t y2 = hi0 ^ x3 ^ k1;
    uint64_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += W0; k1 += W1;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Minimal sampling (Sec. 3.3: batches of minimal sets). */
int orc_sample_triple(uint64_t seed, uint64_t query_id, uint64_t h, int64_t n, int32_t idx[3]) {
  idx[0] = idx[1] = idx[2] = -1;
  if (n < 3) return 0;
  for (uint64_t attempt = 0; attempt < 16; ++attempt) {
    uint64_t ctr[4] = {h, query_id, attempt, 0};
    uint64_t key[2] = {seed, 0};
    uint64_t w[4];
    orc_philox4x64_10(ctr, key, w);
    int32_t a[3];
    for (int k = 0; k < 3; ++k)
      a[k] = (int32_t)(((unsigned __int128)w[k] * (uint64_t)n) >> 64);
    if (a[0] != a[1] && a[0] != a[2] && a[1] != a[2]) {
      idx[0] = a[0]; idx[1] = a[1]; idx[2] = a[2];
      return 1;
    }
  }
  return 0;
}

static uint64_t choose(uint64_t n, uint64_t k) {
  if (k > n) return 0;
  uint64_t r = 1;
  for (uint64_t i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

/* Combinatorial number system: h = C(k,3) + C(j,2) + C(i,1), i < j < k. */
int orc_unrank_triple(uint64_t h, int64_t n, int32_t idx[3]) {
  idx[0] = idx[1] = idx[2] = -1;
  if (n < 3 || h >= choose((uint64_t)n, 3)) return 0;
  uint64_t rem = h;
  int64_t k = 2;
  while (choose((uint64_t)(k + 1), 3) <= rem) ++k;
  rem -= choose((uint64_t)k, 3);
  int64_t j = 1;
  while (choose((uint64_t)(j + 1), 2) <= rem) ++j;
  rem -= choose((uint64_t)j, 2);
  idx[0] = (int32_t)rem; idx[1] = (int32_t)j; idx[2] = (int32_t)k;
  return 1;
}

/* ------------------------------------------------------------------------- */
/* Small linear algebra.                                                      */
/* ------------------------------------------------------------------------- */
static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void sub3(const double a[3], const double b[3], double o[3]) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static void cross3(const double a[3], const double b[3], double o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }

/* x_cam = R X + t */
static void transform(const orc_pose *P, const double X[3], double o[3]) {
  for (int r = 0; r < 3; ++r) o[r] = P->R[3 * r] * X[0] + P->R[3 * r + 1] * X[1] + P->R[3 * r + 2] * X[2] + P->t[r];
}

/* Rotation angle of M = Ra * Rb^T, radians: atan2 of sin (norm of the skew
 * part) and cos ((trace - 1) / 2), accurate also for tiny angles. */
static double rot_angle_between(const double Ra[9], const double Rb[9]) {
  double M[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += Ra[3 * r + k] * Rb[3 * c + k];
      M[3 * r + c] = s;
    }
  double sx = 0.5 * (M[7] - M[5]), sy = 0.5 * (M[2] - M[6]), sz = 0.5 * (M[3] - M[1]);
  double sn = sqrt(sx * sx + sy * sy + sz * sz), cs = 0.5 * (M[0] + M[4] + M[8] - 1.0);
  return atan2(sn, cs);
}

/* Rodrigues: Exp(w) = I + A [w]x + B [w]x^2, A = sin(th)/th, B = (1-cos(th))/th^2. */
static void so3_exp(const double w[3], double R[9]) {
  double th2 = dot3(w, w), th = sqrt(th2), A, B;
  if (th < 1e-4) {
    A = 1.0 - th2 / 6.0 + th2 * th2 / 120.0;
    B = 0.5 - th2 / 24.0 + th2 * th2 / 720.0;
  } else {
    A = sin(th) / th;
    B = (1.0 - cos(th)) / th2;
  }
  double K[9] = {0, -w[2], w[1], w[2], 0, -w[0], -w[1], w[0], 0};
  double K2[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int m = 0; m < 3; ++m) s += K[3 * r + m] * K[3 * m + c];
      K2[3 * r + c] = s;
    }
  for (int i = 0; i < 9; ++i) R[i] = A * K[i] + B * K2[i];
  R[0] += 1.0; R[4] += 1.0; R[8] += 1.0;
}

/* Left update: x' = Exp(dw) x + dt  =>  R' = Exp(dw) R, t' = Exp(dw) t + dt. */
static void pose_update(const orc_pose *P, const double d[6], orc_pose *o) {
  double E[9];
  so3_exp(d, E);
  orc_pose q;
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int m = 0; m < 3; ++m) s += E[3 * r + m] * P->R[3 * m + c];
      q.R[3 * r + c] = s;
    }
    q.t[r] = E[3 * r] * P->t[0] + E[3 * r + 1] * P->t[1] + E[3 * r + 2] * P->t[2] + d[3 + r];
  }
  *o = q;
}

/* Solve H x = b for symmetric positive definite 6x6 H by Cholesky.  0 if not PD. */
static int chol6_solve(const double Hin[36], const double b[6], double x[6]) {
  double L[36];
  memset(L, 0, sizeof(L));
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

/* ------------------------------------------------------------------------- */
/* Real roots of a polynomial of degree <= 4 (ascending coefficients): the   */
/* roots of the derivative split the line into monotone pieces, each piece   */
/* holds at most one root, found by bisection on a sign change.               */
/* ------------------------------------------------------------------------- */
static double poly_eval(const double *c, int d, double x) {
  double s = c[d];
  for (int k = d - 1; k >= 0; --k) s = s * x + c[k];
  return s;
}
static double poly_absscale(const double *c, int d, double x) {
  double s = 0.0, p = 1.0, ax = fabs(x);
  for (int k = 0; k <= d; ++k) { s += fabs(c[k]) * p; p *= ax; }
  return s;
}

static double bisect_root(const double *c, int d, double lo, double hi) {
  double flo = poly_eval(c, d, lo);
  for (int it = 0; it < 400; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    double fm = poly_eval(c, d, mid);
    if (fm == 0.0) return mid;
    if ((fm < 0.0) == (flo < 0.0)) { lo = mid; flo = fm; } else { hi = mid; }
  }
  return 0.5 * (lo + hi);
}

/* Returns the number of distinct real roots, ascending.  *near_double is set
 * when a critical value is within rel_tol of zero relative to the evaluation
 * scale, i.e. where a double root may appear or vanish under perturbation. */
static int real_roots(const double *cin, int d, double *roots, double rel_tol, int *near_double) {
  double c[5];
  double m = 0.0;
  for (int k = 0; k <= d; ++k) { c[k] = cin[k]; if (fabs(c[k]) > m) m = fabs(c[k]); }
  if (m == 0.0) return 0;
  while (d > 0 && fabs(c[d]) <= 1e-14 * m) --d;
  if (d == 0) return 0;
  if (d == 1) { roots[0] = -c[0] / c[1]; return 1; }
  double dc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = 1; k <= d; ++k) dc[k - 1] = k * c[k];
  double crit[4];
  int dummy = 0;
  int nc = real_roots(dc, d - 1, crit, rel_tol, &dummy);
  double bound = 0.0;
  for (int k = 0; k < d; ++k) { double r = fabs(c[k] / c[d]); if (r > bound) bound = r; }
  bound = 1.0 + bound;
  double pts[6];
  int np = 0;
  pts[np++] = -bound;
  for (int i = 0; i < nc; ++i) {
    if (crit[i] > -bound && crit[i] < bound) pts[np++] = crit[i];
    double fv = poly_eval(c, d, crit[i]);
    if (fabs(fv) <= rel_tol * poly_absscale(c, d, crit[i])) *near_double = 1;
  }
  pts[np++] = bound;
  int nr = 0;
  for (int i = 0; i + 1 < np; ++i) {
    double a = pts[i], b = pts[i + 1];
    double fa = poly_eval(c, d, a), fb = poly_eval(c, d, b);
    if (fa == 0.0) {
      if (nr == 0 || roots[nr - 1] != a) roots[nr++] = a;
      continue;
    }
    if (fb == 0.0) continue; /* recorded as the left end of the next piece */
    if ((fa < 0.0) != (fb < 0.0)) roots[nr++] = bisect_root(c, d, a, b);
  }
  return nr;
}

/* Polynomial product, ascending coefficients. */
static void poly_mul(const double *a, int da, const double *b, int db, double *o) {
  for (int k = 0; k <= da + db; ++k) o[k] = 0.0;
  for (int i = 0; i <= da; ++i)
    for (int j = 0; j <= db; ++j) o[i + j] += a[i] * b[j];
}

/* Rigid transform that maps the triangle P onto the congruent triangle Q,
 * built from orthonormal frames on each triangle: R Fp = Fq. */
static int frame_of(const double p1[3], const double p2[3], const double p3[3], double F[9]) {
  double e1[3], e3[3], e2[3], a[3];
  sub3(p2, p1, e1);
  double n1 = norm3(e1);
  if (!(n1 > 0.0)) return 0;
  for (int k = 0; k < 3; ++k) e1[k] /= n1;
  sub3(p3, p1, a);
  cross3(e1, a, e3);
  double n3 = norm3(e3);
  if (!(n3 > 1e-12 * norm3(a))) return 0;
  for (int k = 0; k < 3; ++k) e3[k] /= n3;
  cross3(e3, e1, e2);
  for (int r = 0; r < 3; ++r) { F[3 * r] = e1[r]; F[3 * r + 1] = e2[r]; F[3 * r + 2] = e3[r]; }
  return 1;
}

static int pose_from_triangles(const double P[3][3], const double Q[3][3], orc_pose *o) {
  double Fp[9], Fq[9];
  if (!frame_of(P[0], P[1], P[2], Fp) || !frame_of(Q[0], Q[1], Q[2], Fq)) return 0;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int m = 0; m < 3; ++m) s += Fq[3 * r + m] * Fp[3 * c + m];
      o->R[3 * r + c] = s;
    }
  for (int r = 0; r < 3; ++r)
    o->t[r] = Q[0][r] - (o->R[3 * r] * P[0][0] + o->R[3 * r + 1] * P[0][1] + o->R[3 * r + 2] * P[0][2]);
  return 1;
}

/* Newton polishing of the three distances on the law-of-cosines system
 *   s2^2 + s3^2 - 2 s2 s3 ca = a^2,  s1^2 + s3^2 - 2 s1 s3 cb = b^2,
 *   s1^2 + s2^2 - 2 s1 s2 cg = c^2;
 * a step is kept only while it lowers the residual norm. */
static void polish_depths(double s1, double s2, double s3, double a2, double b2, double c2, double ca,
                          double cb, double cg, double *o1, double *o2, double *o3) {
  double s[3] = {s1, s2, s3};
  for (int it = 0; it < 8; ++it) {
    double F[3] = {s[1] * s[1] + s[2] * s[2] - 2.0 * s[1] * s[2] * ca - a2,
                   s[0] * s[0] + s[2] * s[2] - 2.0 * s[0] * s[2] * cb - b2,
                   s[0] * s[0] + s[1] * s[1] - 2.0 * s[0] * s[1] * cg - c2};
    double J[3][3] = {{0.0, 2.0 * s[1] - 2.0 * s[2] * ca, 2.0 * s[2] - 2.0 * s[1] * ca},
                      {2.0 * s[0] - 2.0 * s[2] * cb, 0.0, 2.0 * s[2] - 2.0 * s[0] * cb},
                      {2.0 * s[0] - 2.0 * s[1] * cg, 2.0 * s[1] - 2.0 * s[0] * cg, 0.0}};
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                 J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (!(fabs(det) > 0.0)) break;
    double d[3];
    for (int c = 0; c < 3; ++c) {
      double M[3][3];
      memcpy(M, J, sizeof(M));
      for (int r = 0; r < 3; ++r) M[r][c] = F[r];
      d[c] = (M[0][0] * (M[1][1] * M[2][2] - M[1][2] * M[2][1]) - M[0][1] * (M[1][0] * M[2][2] - M[1][2] * M[2][0]) +
              M[0][2] * (M[1][0] * M[2][1] - M[1][1] * M[2][0])) / det;
    }
    double n[3] = {s[0] - d[0], s[1] - d[1], s[2] - d[2]};
    double Fn[3] = {n[1] * n[1] + n[2] * n[2] - 2.0 * n[1] * n[2] * ca - a2,
                    n[0] * n[0] + n[2] * n[2] - 2.0 * n[0] * n[2] * cb - b2,
                    n[0] * n[0] + n[1] * n[1] - 2.0 * n[0] * n[1] * cg - c2};
    if (!(Fn[0] * Fn[0] + Fn[1] * Fn[1] + Fn[2] * Fn[2] < F[0] * F[0] + F[1] * F[1] + F[2] * F[2])) break;
    s[0] = n[0]; s[1] = n[1]; s[2] = n[2];
  }
  *o1 = s[0]; *o2 = s[1]; *o3 = s[2];
}

/* ------------------------------------------------------------------------- */
/* P3P, Grunert's solution as set out in the Haralick et al. (1994) review.  */
/* Unknown distances s1, s2, s3 along unit bearings j1, j2, j3; with          */
/* a = |P2-P3|, b = |P1-P3|, c = |P1-P2| and the bearing angle cosines        */
/* ca = j2.j3, cb = j1.j3, cg = j1.j2 the law of cosines gives three          */
/* equations.  With s2 = u s1 and s3 = v s1, eliminating s1 leaves two conics */
/* in (u, v); one of them is linear in u once u^2 is replaced using the       */
/* other, and substituting that u back gives a quartic in v.                   */
/* ------------------------------------------------------------------------- */
int orc_p3p(const double uv[6], const double Xw[9], const orc_camera *K, orc_pose out[4], int32_t *ill) {
  *ill = 0;
  double j[3][3], P[3][3];
  for (int k = 0; k < 3; ++k) {
    double b[3] = {(uv[2 * k] - K->cx) / K->fx, (uv[2 * k + 1] - K->cy) / K->fy, 1.0};
    double nb = norm3(b);
    for (int r = 0; r < 3; ++r) { j[k][r] = b[r] / nb; P[k][r] = Xw[3 * k + r]; }
  }
  double d23[3], d13[3], d12[3], cr[3];
  sub3(P[1], P[2], d23); sub3(P[0], P[2], d13); sub3(P[0], P[1], d12);
  double a2 = dot3(d23, d23), b2 = dot3(d13, d13), c2 = dot3(d12, d12);
  cross3(d12, d13, cr);
  double scale = sqrt(a2 + b2 + c2);
  if (!(b2 > 0.0) || !(c2 > 0.0) || !(a2 > 0.0) || !(norm3(cr) > 1e-9 * scale * scale)) { *ill = 1; return 0; }
  double ca = dot3(j[1], j[2]), cb = dot3(j[0], j[2]), cg = dot3(j[0], j[1]);

  double q = (a2 - c2) / b2, r = c2 / b2;
  double N[3] = {q + 1.0, -2.0 * q * cb, q - 1.0};  /* numerator of u(v) */
  double D[2] = {2.0 * cg, -2.0 * ca};              /* denominator of u(v) */
  double L[3] = {1.0, -2.0 * cb, 1.0};              /* 1 + v^2 - 2 v cb */
  /* quartic: D^2 + N^2 - 2 cg N D - r L D^2 = 0 */
  double DD[3], NN[5], ND[4], LDD[5], Qp[5];
  poly_mul(D, 1, D, 1, DD);
  poly_mul(N, 2, N, 2, NN);
  poly_mul(N, 2, D, 1, ND);
  poly_mul(L, 2, DD, 2, LDD);
  for (int k = 0; k < 5; ++k) {
    Qp[k] = NN[k] - r * LDD[k];
    if (k < 3) Qp[k] += DD[k];
    if (k < 4) Qp[k] -= 2.0 * cg * ND[k];
  }
  double vr[4];
  int near_double = 0;
  int nv = real_roots(Qp, 4, vr, 1e-6, &near_double);
  if (near_double) *ill = 1;

  int ns = 0;
  for (int iv = 0; iv < nv; ++iv) {
    double v = vr[iv];
    double dv = poly_eval(D, 1, v);
    double slope_den = fabs(D[0]) + fabs(D[1] * v);
    if (fabs(dv) <= 1e-9 * slope_den) { *ill = 1; continue; }
    double u = poly_eval(N, 2, v) / dv;
    double Lv = poly_eval(L, 2, v);
    if (!(Lv > 0.0)) { *ill = 1; continue; }
    double s1 = sqrt(b2 / Lv), s2 = u * s1, s3 = v * s1;
    double smax = fmax(fabs(s1), fmax(fabs(s2), fabs(s3)));
    if (fabs(s2) <= 1e-9 * smax || fabs(s3) <= 1e-9 * smax) *ill = 1;
    if (!(s1 > 0.0 && s2 > 0.0 && s3 > 0.0)) continue;
    polish_depths(s1, s2, s3, a2, b2, c2, ca, cb, cg, &s1, &s2, &s3);
    /* slope of the quartic at the root, relative: a small value is a near-double root */
    double dq[4];
    for (int k = 1; k < 5; ++k) dq[k - 1] = k * Qp[k];
    if (fabs(poly_eval(dq, 3, v)) * (1.0 + fabs(v)) <= 1e-6 * poly_absscale(Qp, 4, v)) *ill = 1;
    double Qc[3][3];
    double s[3] = {s1, s2, s3};
    for (int k = 0; k < 3; ++k)
      for (int rr = 0; rr < 3; ++rr) Qc[k][rr] = s[k] * j[k][rr];
    orc_pose cand;
    if (!pose_from_triangles(P, Qc, &cand)) { *ill = 1; continue; }
    int dup = 0;
    for (int e = 0; e < ns; ++e) {
      double dt[3];
      sub3(cand.t, out[e].t, dt);
      if (rot_angle_between(cand.R, out[e].R) < 1e-9 && norm3(dt) < 1e-9 * fmax(1.0, norm3(out[e].t))) dup = 1;
    }
    if (dup) { *ill = 1; continue; }
    if (ns < 4) out[ns++] = cand;
  }
  /* canonical order: camera depth of point 0 ascending, then of point 1 */
  for (int a = 1; a < ns; ++a) {
    orc_pose key = out[a];
    double ka[3], kb[3];
    transform(&key, P[0], ka);
    transform(&key, P[1], kb);
    int b = a - 1;
    while (b >= 0) {
      double za[3], zb[3];
      transform(&out[b], P[0], za);
      transform(&out[b], P[1], zb);
      if (za[2] > ka[2] || (za[2] == ka[2] && zb[2] > kb[2])) { out[b + 1] = out[b]; --b; } else break;
    }
    out[b + 1] = key;
  }
  return ns;
}

/* ------------------------------------------------------------------------- */
/* Scoring (Sec. 3.3 "Pose Estimation"): MSAC sum of clipped squared pixel  */
/* errors, confidence-weighted, every hypothesis against every scored point. */
/* ------------------------------------------------------------------------- */
static double corr_w(const orc_corr *c, int64_t i) { return c->w ? (double)c->w[i] : 1.0; }

void orc_score(const orc_pose *poses, int64_t np, const orc_corr *c, const orc_camera *K,
               double tau, int32_t *count, double *msac) {
  const double tau2 = tau * tau;
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t p = 0; p < np; ++p) {
    int32_t cnt = 0;
    double sum = 0.0;
    for (int64_t i = 0; i < c->n; ++i) {
      double X[3] = {c->X[i], c->Y[i], c->Z[i]}, xc[3];
      transform(&poses[p], X, xc);
      double w = corr_w(c, i);
      if (!(xc[2] > 0.0)) { sum += w * tau2; continue; }
      double px = K->fx * xc[0] / xc[2] + K->cx, py = K->fy * xc[1] / xc[2] + K->cy;
      double du = px - (double)c->u[i], dv = py - (double)c->v[i];
      double r2 = du * du + dv * dv;
      if (r2 < tau2) { ++cnt; sum += w * r2; } else { sum += w * tau2; }
    }
    count[p] = cnt;
    msac[p] = sum;
  }
}

/* Ambiguity band of one residual (reading of the float32/float64 question of
 * the scoring step, Sec. 3.3): a bound on how far the pixel distance that a
 * float32 evaluation of the test acts on can sit from the exact one.  The
 * float32 evaluation it bounds: the rows p0 = P0/tau, p1 = P1/tau, p2 = P2 of
 * P = K [R | t] rounded to float32; a' = p0.X~, b' = p1.X~, w = p2.X~ by three
 * fused multiply-adds each (X~ = (X, Y, Z, 1) from the float32 inputs);
 * u' = u * fl(1/tau); du' = a' - u' w and dv' = b' - v' w by one fused
 * multiply-add each; e' = du'^2 + dv'^2 (a product and a fused multiply-add);
 * inlier iff e' < w |w|, i.e. iff rho' = sqrt(e' / (w |w|)) < 1.  With unit
 * roundoff u = 2^-24, g_k = k u / (1 - k u), A = sum_j |P0j X~j|,
 * B = sum_j |P1j X~j|, W = sum_j |P2j X~j|, the exact depth z = P2.X~ and the
 * exact distance r = tau rho (standard model of each rounding, no underflow):
 *   |da'| <= g4 A / tau, |db'| <= g4 B / tau, |dw| <= g4 W = k |z|
 *   |u' - u/tau| <= g3 |u| / tau                (1/tau, product, double)
 *   |du' - du| <= (1 + u) Pa / tau + u |du|, Pa = g4 A + g3 |u| (|z| + g4 W) + g4 |u| W
 * (likewise dv' with B, v, Pb).  The vector (du', dv') then moves
 * sqrt(du^2 + dv^2) by at most (1 + u) hypot(Pa, Pb) / tau + u rho |z|; 1/|w|
 * moves by at most k / (1 - k) relative; the roundings of e' and w |w| scale
 * rho' by a factor within 1.5 u' of 1 (u' = 1.001 u).  Collecting,
 *   |rho' tau - r| <= beta = (1.5 u' r + ((1 + u) hypot(Pa, Pb) / |z| + u r
 *                             + k r) / (1 - k)) / (1 - 1.5 u'),
 * taken at the residual's own r, so the float32 decision equals the exact one
 * whenever |r - tau| >= beta.  The sign of w is right when |z| > g4 W; a point
 * with |z| <= 8 u W is ambiguous (it may be either). */
static void residual_band(const double P[3][4], const orc_pose *pose, const orc_camera *K, const double Xt[4],
                          double u, double v, double tau, double band_abs, int32_t with_f32, double *r,
                          double *beta, int *behind) {
  const double uq = ldexp(1.0, -24), uq1 = 1.001 * uq;
  const double g3 = 3.0 * uq / (1.0 - 3.0 * uq), g4 = 4.0 * uq / (1.0 - 4.0 * uq);
  double xc[3];
  transform(pose, Xt, xc);
  double A = 0, B = 0, W = 0;
  for (int k = 0; k < 4; ++k) { A += fabs(P[0][k] * Xt[k]); B += fabs(P[1][k] * Xt[k]); W += fabs(P[2][k] * Xt[k]); }
  const double z = xc[2];
  const double wsign_err = with_f32 ? 8.0 * uq * W : 0.0;
  *r = NAN;
  *beta = INFINITY;
  if (!(z > wsign_err)) {
    /* behind the camera (1), or (float32) possibly on either side of its
     * plane (2); a NaN depth is behind */
    *behind = z > -wsign_err ? 2 : 1;
    return;
  }
  *behind = 0;
  const double px = K->fx * xc[0] / z + K->cx, py = K->fy * xc[1] / z + K->cy;
  const double d = sqrt((px - u) * (px - u) + (py - v) * (py - v));
  double b = band_abs;
  if (with_f32) {
    const double k = g4 * W / z;
    const double Pa = g4 * A + g3 * fabs(u) * (z + g4 * W) + g4 * fabs(u) * W;
    const double Pb = g4 * B + g3 * fabs(v) * (z + g4 * W) + g4 * fabs(v) * W;
    const double b32 = (1.5 * uq1 * d + ((1.0 + uq) * hypot(Pa, Pb) / z + uq * d + k * d) / (1.0 - k)) /
                       (1.0 - 1.5 * uq1);
    if (b32 > b) b = b32;
  }
  *r = d;
  *beta = b;
}

/* rows of K [R | t] */
static void proj_rows(const orc_pose *pose, const orc_camera *K, double P[3][4]) {
  const double *R = pose->R, *t = pose->t;
  for (int k = 0; k < 3; ++k) {
    P[0][k] = K->fx * R[k] + K->cx * R[6 + k];
    P[1][k] = K->fy * R[3 + k] + K->cy * R[6 + k];
    P[2][k] = R[6 + k];
  }
  P[0][3] = K->fx * t[0] + K->cx * t[2];
  P[1][3] = K->fy * t[1] + K->cy * t[2];
  P[2][3] = t[2];
}

void orc_residual_band(const orc_pose *pose, const orc_corr *c, const orc_camera *K, double tau, double band_abs,
                       int32_t with_f32, double *r, double *beta) {
  double P[3][4];
  proj_rows(pose, K, P);
  for (int64_t i = 0; i < c->n; ++i) {
    const double Xt[4] = {c->X[i], c->Y[i], c->Z[i], 1.0};
    int behind;
    residual_band(P, pose, K, Xt, c->u[i], c->v[i], tau, band_abs, with_f32, &r[i], &beta[i], &behind);
  }
}

void orc_score_band(const orc_pose *poses, int64_t np, const orc_corr *c, const orc_camera *K,
                    double tau, double band_abs, int32_t with_f32,
                    int32_t *count_lo, int32_t *count_hi, double *msac_err_bound) {
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t p = 0; p < np; ++p) {
    double P[3][4];
    proj_rows(&poses[p], K, P);
    int32_t lo = 0, hi = 0;
    double errb = 0.0;
    for (int64_t i = 0; i < c->n; ++i) {
      const double Xt[4] = {c->X[i], c->Y[i], c->Z[i], 1.0};
      const double w = corr_w(c, i);
      double r, beta;
      int behind;
      residual_band(P, &poses[p], K, Xt, c->u[i], c->v[i], tau, band_abs, with_f32, &r, &beta, &behind);
      if (behind) {
        if (behind == 2) { ++hi; errb += w * tau * tau; }
        continue;
      }
      if (r < tau - beta) ++lo;
      if (r < tau + beta) ++hi;
      if (r < tau + beta) errb += w * (2.0 * fmin(r + beta, tau + beta) * beta + beta * beta);
    }
    count_lo[p] = lo;
    count_hi[p] = hi;
    if (msac_err_bound) msac_err_bound[p] = errb;
  }
}

/* ------------------------------------------------------------------------- */
/* Normal equations of the reprojection error.  Residual r = pi(R X + t) - x, */
/* Jacobian w.r.t. (dw, dt) of the left update: d x_c = dw x x_c + dt.        */
/* ------------------------------------------------------------------------- */
static void accumulate_normal(const orc_camera *K, const double xc[3], double du, double dv, double wgt,
                              double H[36], double g[6]) {
  double x = xc[0], y = xc[1], z = xc[2], iz = 1.0 / z;
  /* d(pixel)/d(x_c) */
  double a00 = K->fx * iz, a02 = -K->fx * x * iz * iz;
  double a11 = K->fy * iz, a12 = -K->fy * y * iz * iz;
  /* d(x_c)/d(dw) = -[x_c]_x = [[0, z, -y], [-z, 0, x], [y, -x, 0]] ; d(x_c)/d(dt) = I */
  double M[3][6] = {{0, z, -y, 1, 0, 0}, {-z, 0, x, 0, 1, 0}, {y, -x, 0, 0, 0, 1}};
  double J[2][6];
  for (int k = 0; k < 6; ++k) {
    J[0][k] = a00 * M[0][k] + a02 * M[2][k];
    J[1][k] = a11 * M[1][k] + a12 * M[2][k];
  }
  for (int r = 0; r < 6; ++r) {
    g[r] += wgt * (J[0][r] * du + J[1][r] * dv);
    for (int c = 0; c < 6; ++c) H[6 * r + c] += wgt * (J[0][r] * J[0][c] + J[1][r] * J[1][c]);
  }
}

/* Truncated cost at a pose, and the normal equations over its inliers. */
static double eval_truncated(const orc_pose *P, const orc_corr *c, const orc_camera *K, double tau2,
                             double H[36], double g[6], int64_t *count) {
  memset(H, 0, 36 * sizeof(double));
  memset(g, 0, 6 * sizeof(double));
  double cost = 0.0;
  int64_t cnt = 0;
  for (int64_t i = 0; i < c->n; ++i) {
    double X[3] = {c->X[i], c->Y[i], c->Z[i]}, xc[3];
    transform(P, X, xc);
    double w = corr_w(c, i);
    if (!(xc[2] > 0.0)) { cost += w * tau2; continue; }
    double du = K->fx * xc[0] / xc[2] + K->cx - (double)c->u[i];
    double dv = K->fy * xc[1] / xc[2] + K->cy - (double)c->v[i];
    double r2 = du * du + dv * dv;
    if (r2 < tau2) {
      ++cnt;
      cost += w * r2;
      accumulate_normal(K, xc, du, dv, w, H, g);
    } else {
      cost += w * tau2;
    }
  }
  *count = cnt;
  return cost;
}

double orc_normal_equations(const orc_pose *P, const orc_corr *c, const orc_camera *K, double tau, double H[36],
                            double g[6], int64_t *count) {
  return eval_truncated(P, c, K, tau * tau, H, g, count);
}

void orc_pose_update(const orc_pose *P, const double d[6], orc_pose *o) { pose_update(P, d, o); }

/* Converged: a Gauss-Newton step (dw in rad, dt in scene units) shorter
 * than 1e-10 is not taken and ends the run (the refinement the paper follows
 * also stops on a short step). */
#define ORC_STEP_TOL2 1e-20
int orc_step_converged(const double d[6]) {
  double s = 0.0;
  for (int k = 0; k < 6; ++k) s += d[k] * d[k];
  return s < ORC_STEP_TOL2;
}

int orc_lo(const orc_pose *start, const orc_corr *c, const orc_camera *K, double tau, int32_t iters,
           orc_pose *out, double *cost, int64_t *count) {
  double tau2 = tau * tau, H[36], g[6];
  orc_pose cur = *start;
  int64_t cnt;
  double cur_cost = eval_truncated(&cur, c, K, tau2, H, g, &cnt);
  int accepted = 0;
  for (int it = 0; it < iters; ++it) {
    double rhs[6], d[6];
    for (int k = 0; k < 6; ++k) rhs[k] = -g[k];
    if (!chol6_solve(H, rhs, d)) break;
    if (orc_step_converged(d)) break;
    orc_pose cand;
    pose_update(&cur, d, &cand);
    double H2[36], g2[6];
    int64_t cnt2;
    double new_cost = eval_truncated(&cand, c, K, tau2, H2, g2, &cnt2);
    if (!(new_cost <= cur_cost)) break;
    cur = cand;
    cur_cost = new_cost;
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

/* Cauchy cost over the fixed set I, and its IRLS normal equations. */
static double eval_cauchy(const orc_pose *P, const orc_corr *c, const uint8_t *in_set, const orc_camera *K,
                          double tau2, double s2, double H[36], double g[6]) {
  memset(H, 0, 36 * sizeof(double));
  memset(g, 0, 6 * sizeof(double));
  double cost = 0.0;
  for (int64_t i = 0; i < c->n; ++i) {
    if (!in_set[i]) continue;
    double X[3] = {c->X[i], c->Y[i], c->Z[i]}, xc[3];
    transform(P, X, xc);
    double w = corr_w(c, i);
    if (!(xc[2] > 0.0)) { cost += w * s2 * log1p(tau2 / s2); continue; }
    double du = K->fx * xc[0] / xc[2] + K->cx - (double)c->u[i];
    double dv = K->fy * xc[1] / xc[2] + K->cy - (double)c->v[i];
    double r2 = du * du + dv * dv;
    cost += w * s2 * log1p(r2 / s2);
    accumulate_normal(K, xc, du, dv, w / (1.0 + r2 / s2), H, g);
  }
  return cost;
}

static void inlier_mask(const orc_pose *P, const orc_corr *c, const orc_camera *K, double tau2, uint8_t *m) {
  for (int64_t i = 0; i < c->n; ++i) {
    double X[3] = {c->X[i], c->Y[i], c->Z[i]}, xc[3];
    transform(P, X, xc);
    m[i] = 0;
    if (!(xc[2] > 0.0)) continue;
    double du = K->fx * xc[0] / xc[2] + K->cx - (double)c->u[i];
    double dv = K->fy * xc[1] / xc[2] + K->cy - (double)c->v[i];
    if (du * du + dv * dv < tau2) m[i] = 1;
  }
}

int orc_refine(const orc_pose *start, const orc_corr *c, const orc_camera *K, double tau, double s,
               int32_t iters, orc_pose *out, double *cost, int64_t *n_inl) {
  double tau2 = tau * tau, s2 = s * s, H[36], g[6];
  uint8_t *in_set = (uint8_t *)malloc(c->n > 0 ? (size_t)c->n : 1);
  inlier_mask(start, c, K, tau2, in_set);
  int64_t ni = 0;
  for (int64_t i = 0; i < c->n; ++i) ni += in_set[i];
  orc_pose cur = *start;
  double cur_cost = eval_cauchy(&cur, c, in_set, K, tau2, s2, H, g);
  int accepted = 0;
  for (int it = 0; it < iters; ++it) {
    double rhs[6], d[6];
    for (int k = 0; k < 6; ++k) rhs[k] = -g[k];
    if (!chol6_solve(H, rhs, d)) break;
    if (orc_step_converged(d)) break;
    orc_pose cand;
    pose_update(&cur, d, &cand);
    double H2[36], g2[6];
    double new_cost = eval_cauchy(&cand, c, in_set, K, tau2, s2, H2, g2);
    if (!(new_cost <= cur_cost)) break;
    cur = cand;
    cur_cost = new_cost;
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

/* Standard RANSAC bound: k = ceil(ln(1 - p) / ln(1 - eps^3)). */
int64_t orc_required_samples(double eps, double confidence, int64_t max_iters) {
  if (!(eps > 0.0)) return max_iters;
  if (eps >= 1.0) return 0;
  double denom = log1p(-eps * eps * eps);
  if (!(denom < 0.0)) return max_iters;
  double k = ceil(log(1.0 - confidence) / denom);
  if (!(k < (double)max_iters)) return max_iters;
  if (k < 0.0) return 0;
  return (int64_t)k;
}

/* ------------------------------------------------------------------------- */
/* LO-RANSAC driver.                                                          */
/* ------------------------------------------------------------------------- */
typedef struct {
  orc_pose pose;
  int64_t h;
  int32_t j;
  int32_t count;
  double msac;
} orc_cand;

static int cand_less(const orc_cand *a, const orc_cand *b) {
  if (a->msac != b->msac) return a->msac < b->msac;
  if (a->count != b->count) return a->count > b->count;
  if (a->h != b->h) return a->h < b->h;
  return a->j < b->j;
}

int orc_lo_ransac_pnp(const orc_corr *c, const orc_camera *K, const orc_params *p, orc_pose *pose,
                      uint8_t *mask, orc_stats *st) {
  memset(st, 0, sizeof(*st));
  st->best_h = -1;
  st->best_j = -1;
  for (int k = 0; k < 9; ++k) pose->R[k] = (k % 4 == 0) ? 1.0 : 0.0;
  pose->t[0] = pose->t[1] = pose->t[2] = 0.0;
  if (mask) memset(mask, 0, (size_t)(c->n > 0 ? c->n : 0));
  const int64_t n = c->n;
  const double tau = p->threshold_px, tau2 = tau * tau;

  /* scoring set S: stride subsample (Sec. 3.3 "uniform subsampling") */
  int64_t m = n;
  if (p->max_score_points > 0 && n > p->max_score_points) m = p->max_score_points;
  float *S = (float *)malloc((size_t)(m > 0 ? m : 1) * 6 * sizeof(float));
  float *Su = S, *Sv = S + m, *SX = S + 2 * m, *SY = S + 3 * m, *SZ = S + 4 * m, *Sw = S + 5 * m;
  for (int64_t jx = 0; jx < m; ++jx) {
    int64_t i = (m == n) ? jx : (int64_t)(((unsigned __int128)jx * (uint64_t)n) / (uint64_t)m);
    Su[jx] = c->u[i]; Sv[jx] = c->v[i]; SX[jx] = c->X[i]; SY[jx] = c->Y[i]; SZ[jx] = c->Z[i];
    Sw[jx] = c->w ? c->w[i] : 1.0f;
  }
  orc_corr Sc = {Su, Sv, SX, SY, SZ, c->w ? Sw : NULL, m};

  int have_best = 0;
  double best_cost = INFINITY;
  int64_t best_count = 0;
  orc_pose best;
  const int64_t total = p->fixed_samples > 0 ? p->fixed_samples : p->max_iters;
  const int64_t batch = p->batch > 0 ? p->batch : 1024;
  int64_t drawn = 0;
  orc_cand *cands = (orc_cand *)malloc((size_t)(4 * batch) * sizeof(orc_cand));
  orc_pose *cp = (orc_pose *)malloc((size_t)(4 * batch) * sizeof(orc_pose));
  int32_t *cc = (int32_t *)malloc((size_t)(4 * batch) * sizeof(int32_t));
  double *cm = (double *)malloc((size_t)(4 * batch) * sizeof(double));

  while (m >= 3 && drawn < total) {
    int64_t B = total - drawn < batch ? total - drawn : batch;
    int64_t nc = 0;
    for (int64_t h = drawn; h < drawn + B; ++h) {
      int32_t idx[3];
      int ok = p->exhaustive ? orc_unrank_triple((uint64_t)h, m, idx)
                             : orc_sample_triple(p->seed, p->query_id, (uint64_t)h, m, idx);
      if (!ok) continue;
      double uv[6], Xw[9];
      for (int k = 0; k < 3; ++k) {
        uv[2 * k] = Su[idx[k]]; uv[2 * k + 1] = Sv[idx[k]];
        Xw[3 * k] = SX[idx[k]]; Xw[3 * k + 1] = SY[idx[k]]; Xw[3 * k + 2] = SZ[idx[k]];
      }
      orc_pose sol[4];
      int32_t ill;
      int ns = orc_p3p(uv, Xw, K, sol, &ill);
      for (int jj = 0; jj < ns; ++jj) {
        cands[nc].pose = sol[jj];
        cands[nc].h = h;
        cands[nc].j = jj;
        cp[nc] = sol[jj];
        ++nc;
      }
    }
    orc_score(cp, nc, &Sc, K, tau, cc, cm);
    for (int64_t k = 0; k < nc; ++k) { cands[k].count = cc[k]; cands[k].msac = cm[k]; }
    st->candidates += nc;
    st->residuals += nc * m;

    /* top-k of the batch whose score beats the running best */
    const double gate = best_cost;
    int32_t chosen[32];
    int nch = 0;
    int kmax = p->lo_top_k < 1 ? 1 : (p->lo_top_k < 32 ? p->lo_top_k : 32);
    for (int sel = 0; sel < kmax; ++sel) {
      int64_t arg = -1;
      for (int64_t k = 0; k < nc; ++k) {
        if (!(cands[k].msac < gate)) continue;
        int taken = 0;
        for (int q = 0; q < nch; ++q) taken |= (chosen[q] == k);
        if (taken) continue;
        if (arg < 0 || cand_less(&cands[k], &cands[arg])) arg = k;
      }
      if (arg < 0) break;
      chosen[nch++] = (int32_t)arg;
    }
    for (int q = 0; q < nch; ++q) {
      orc_pose lo_pose;
      double lo_cost;
      int64_t lo_count;
      orc_lo(&cands[chosen[q]].pose, &Sc, K, tau, p->lo_iters, &lo_pose, &lo_cost, &lo_count);
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
      double eps = (double)best_count / (double)m;
      int64_t req = orc_required_samples(eps, p->confidence, p->max_iters);
      int64_t need = req > p->min_iters ? req : p->min_iters;
      if (need > p->max_iters) need = p->max_iters;
      if (drawn >= need) break;
    }
  }
  st->samples = drawn;
  free(cands); free(cp); free(cc); free(cm);
  free(S);
  if (!have_best) { st->status = 1; return 1; }
  st->best_count = best_count;
  st->best_msac = best_cost;

  /* final refinement on all inliers of the full set (Sec. 3.3) */
  orc_pose fin;
  double fcost;
  int64_t ninl;
  orc_refine(&best, c, K, tau, p->cauchy_scale_px, p->final_iters, &fin, &fcost, &ninl);
  *pose = fin;
  st->final_cost = fcost;
  uint8_t *mk = mask ? mask : (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
  inlier_mask(&fin, c, K, tau2, mk);
  int64_t fc = 0;
  for (int64_t i = 0; i < n; ++i) fc += mk[i];
  st->full_count = fc;
  if (!mask) free(mk);
  st->status = 0;
  return 0;
}

/* ------------------------------------------------------------------------- */
/* Lifting (Sec. 3.3 "Query Time Matching and 2D-3D Lifting").                */
/* ------------------------------------------------------------------------- */
static int depth_ok(float d) { return isfinite(d) && d > 0.0f; }

/* ------------------------------------------------------------------------- */
/* 8-bit log-depth codes (Sec. 3.3 "Data Compression", Sec. 4.3 "Depth       */
/* Quantization"): depth clipped to [0.25, 128] m and quantised uniformly in  */
/* log depth.  Reading: code 0 marks a pixel without depth; codes 1..255 are  */
/* the levels d(c) = 0.25 * (128 / 0.25)^((c - 1) / 254), endpoints included; */
/* encoding rounds log depth to the nearest level (halves away from zero).    */
/* ------------------------------------------------------------------------- */
#define ORC_LOG8_DMIN 0.25
#define ORC_LOG8_DMAX 128.0
#define ORC_LOG8_STEPS 254.0

double orc_log8_decode(uint8_t c) {
  if (c == 0) return 0.0;
  return ORC_LOG8_DMIN * pow(ORC_LOG8_DMAX / ORC_LOG8_DMIN, ((double)c - 1.0) / ORC_LOG8_STEPS);
}

uint8_t orc_log8_encode(float depth) {
  double d = depth;
  if (!(isfinite(d) && d > 0.0)) return 0;
  if (d < ORC_LOG8_DMIN) d = ORC_LOG8_DMIN;
  if (d > ORC_LOG8_DMAX) d = ORC_LOG8_DMAX;
  const double level = ORC_LOG8_STEPS * log(d / ORC_LOG8_DMIN) / log(ORC_LOG8_DMAX / ORC_LOG8_DMIN);
  return (uint8_t)(1 + (int)round(level));
}

void orc_log8_encode_array(const float *depth, int64_t n, uint8_t *codes) {
  for (int64_t i = 0; i < n; ++i) codes[i] = orc_log8_encode(depth[i]);
}

/* Depth texel idx of the float32 maps or the code maps (exactly one given);
 * returns 0 if the texel holds no valid depth. */
static int depth_tap(const float *depth, const uint8_t *codes, int64_t idx, double *d) {
  if (codes) {
    if (codes[idx] == 0) return 0;
    *d = orc_log8_decode(codes[idx]);
    return 1;
  }
  if (!depth_ok(depth[idx])) return 0;
  *d = depth[idx];
  return 1;
}

static int64_t lift_maps(const float *q_u, const float *q_v, const float *db_u, const float *db_v,
                         const float *conf, const int32_t *view, int64_t n_matches, int32_t subpixel,
                         const float *depth, const uint8_t *codes, int32_t n_views, int32_t H, int32_t W,
                         const orc_camera *cams, const orc_pose *poses, float min_conf, double *out_u,
                         double *out_v, double *out_X, double *out_Y, double *out_Z, double *out_w,
                         int64_t *out_src) {
  int64_t nout = 0;
  for (int64_t mi = 0; mi < n_matches; ++mi) {
    if (!(conf[mi] > min_conf)) continue;
    int32_t k = view[mi];
    if (k < 0 || k >= n_views) continue;
    double qu = q_u[mi], qv = q_v[mi], du = db_u[mi], dv = db_v[mi];
    if (!isfinite(qu) || !isfinite(qv) || !isfinite(du) || !isfinite(dv)) continue;
    const int64_t base = (int64_t)k * H * W;
    double d;
    if (subpixel) {
      double x = du - 0.5, y = dv - 0.5;
      double x0 = floor(x), y0 = floor(y);
      if (x0 < 0.0 || y0 < 0.0 || x0 + 1.0 > (double)(W - 1) || y0 + 1.0 > (double)(H - 1)) continue;
      int64_t c0 = (int64_t)x0, r0 = (int64_t)y0;
      double d00, d01, d10, d11;
      if (!depth_tap(depth, codes, base + r0 * W + c0, &d00) || !depth_tap(depth, codes, base + r0 * W + c0 + 1, &d01) ||
          !depth_tap(depth, codes, base + (r0 + 1) * W + c0, &d10) ||
          !depth_tap(depth, codes, base + (r0 + 1) * W + c0 + 1, &d11))
        continue;
      double ax = x - x0, ay = y - y0;
      d = (1.0 - ay) * ((1.0 - ax) * d00 + ax * d01) + ay * ((1.0 - ax) * d10 + ax * d11);
    } else {
      double cf = floor(du), rf = floor(dv);
      if (cf < 0.0 || rf < 0.0 || cf > (double)(W - 1) || rf > (double)(H - 1)) continue;
      if (!depth_tap(depth, codes, base + (int64_t)rf * W + (int64_t)cf, &d)) continue;
    }
    const orc_camera *Kc = &cams[k];
    const orc_pose *T = &poses[k];
    double xc[3] = {d * (du - Kc->cx) / Kc->fx, d * (dv - Kc->cy) / Kc->fy, d};
    double e[3] = {xc[0] - T->t[0], xc[1] - T->t[1], xc[2] - T->t[2]};
    /* X_w = R^T (x_c - t) */
    double Xw[3];
    for (int r = 0; r < 3; ++r) Xw[r] = T->R[r] * e[0] + T->R[3 + r] * e[1] + T->R[6 + r] * e[2];
    out_u[nout] = qu; out_v[nout] = qv;
    out_X[nout] = Xw[0]; out_Y[nout] = Xw[1]; out_Z[nout] = Xw[2];
    out_w[nout] = conf[mi];
    out_src[nout] = mi;
    ++nout;
  }
  return nout;
}

int64_t orc_lift(const float *q_u, const float *q_v, const float *db_u, const float *db_v, const float *conf,
                 const int32_t *view, int64_t n_matches, int32_t subpixel, const float *depth, int32_t n_views,
                 int32_t H, int32_t W, const orc_camera *cams, const orc_pose *poses, float min_conf,
                 double *out_u, double *out_v, double *out_X, double *out_Y, double *out_Z, double *out_w,
                 int64_t *out_src) {
  return lift_maps(q_u, q_v, db_u, db_v, conf, view, n_matches, subpixel, depth, NULL, n_views, H, W, cams, poses,
                   min_conf, out_u, out_v, out_X, out_Y, out_Z, out_w, out_src);
}

int64_t orc_lift_log8(const float *q_u, const float *q_v, const float *db_u, const float *db_v, const float *conf,
                      const int32_t *view, int64_t n_matches, int32_t subpixel, const uint8_t *codes,
                      int32_t n_views, int32_t H, int32_t W, const orc_camera *cams, const orc_pose *poses,
                      float min_conf, double *out_u, double *out_v, double *out_X, double *out_Y, double *out_Z,
                      double *out_w, int64_t *out_src) {
  return lift_maps(q_u, q_v, db_u, db_v, conf, view, n_matches, subpixel, NULL, codes, n_views, H, W, cams, poses,
                   min_conf, out_u, out_v, out_X, out_Y, out_Z, out_w, out_src);
}

void orc_set_threads(int32_t n) { omp_set_num_threads(n >= 1 ? n : 1); }

int32_t orc_max_threads(void) { return (int32_t)omp_get_max_threads(); }
