// gp3p_device.h -- generalised P3P in float64 for multi-camera rigs (ImLoc
// appendix "LaMAR Hololens Results": generalised absolute pose for rig
// queries).
//
// Three rays in the rig frame, origin o_i and unit direction f_i, must pass
// through three world points at depths l_i: the rig-frame points o_i + l_i f_i
// keep the world distances d_ij.  With x = l1 the (1,2) and (1,3) distances
// are monic quadratics in l2 and l3 whose coefficients are polynomials in x:
//   l2^2 + B12(x) l2 + C12(x) = 0,   l3^2 + B13(x) l3 + C13(x) = 0.
// Using them to remove l2^2 and l3^2 from the (2,3) distance leaves
//   b l2 l3 + P(x) l2 + R(x) l3 + Q(x) = 0,
// so l3 = -(P l2 + Q) / (b l2 + R).  Put into the (1,3) quadratic, that is a
// quadratic A2 l2^2 + A1 l2 + A0 = 0 (A_k of degree 2, 3, 4 in x), and its
// resultant with the (1,2) quadratic is a polynomial of degree 8 in x.  Its
// real roots on the interval of x where l2 and l3 are real are isolated by
// derivative splitting and refined by safeguarded Newton; l2 is the common
// root of the two quadratics, l3 follows; all three depths are Newton-polished
// on the three distance equations, and the pose aligns the rig-frame triangle
// with the world triangle.
//
// The pieces are written for eight cooperating lanes per sample: at each
// level of the derivative splitting the monotone pieces are independent, so
// lane j refines the root of piece j; the per-level bookkeeping (which roots
// count, where the next level's pieces start and end) is a short scan every
// lane repeats over the level's results.  Lane j then lifts root j to the
// three depths, and a second scan removes duplicates and orders the
// solutions.  Pieces with no root keep their slot and repeat the previous
// cut point, so the next level's extra pieces are empty: the sequence of
// non-empty pieces, and every value computed on them, is that of the plain
// one-lane recursion.
#pragma once

#include "imloc_device.h"

namespace imloc {

// polynomial helpers, coefficients in increasing degree
__host__ __device__ inline void pmul(const double* a, int da, const double* b, int db, double* o) {
  for (int k = 0; k <= da + db; ++k) o[k] = 0.0;
  for (int i = 0; i <= da; ++i)
    for (int j = 0; j <= db; ++j) o[i + j] = fma(a[i], b[j], o[i + j]);
}

__host__ __device__ inline double peval(const double* c, int d, double x) {
  double r = c[d];
  for (int k = d - 1; k >= 0; --k) r = fma(r, x, c[k]);
  return r;
}

// Coefficients (degree D - K) of the K-th derivative of the degree-D
// polynomial c: c[e + K] (e + K) (e + K - 1) ... (e + 1), one rounding per
// factor, largest factor first (the order of repeated differentiation).
template <int D, int K>
__host__ __device__ inline void deriv_coeffs(const double* c, double* o) {
#pragma unroll
  for (int e = 0; e <= D - K; ++e) {
    double v = c[e + K];
#pragma unroll
    for (int m = e + K; m > e; --m) v *= (double)m;
    o[e] = v;
  }
}

// Root of the degree-DEG polynomial p (derivative dp) on the piece [a, b]
// of one level of the derivative splitting: p is monotone there, so a sign
// change brackets exactly one root, found by Newton steps kept inside the
// shrinking bracket (else bisection) until a step is below kRootStep (s lies
// in [-1, 1]).  A Newton step that lands on a bracket end counts as kept, so
// a converged iteration stops at once; a Newton step rejected right after a
// step below kRootNoise means the iteration has reached the rounding noise of
// p near the root, and it stops there too (bisecting on would only shrink a
// bracket Newton approached from one side).  Returns 0 (no root), 1 (root)
// or 2 (p(a) == 0: the root is a, and counts only if the level's previous
// root differs from it).  A zero at b counts on the last piece of the level
// only.
constexpr double kRootStep = 1e-14;
constexpr double kRootNoise = 1e-9;

template <int DEG>
__host__ __device__ inline int piece_root(const double* p, const double* dp, double a, double b, bool last_piece,
                                          double& root) {
  if (!(b > a)) return 0;
  const double fa = peval(p, DEG, a);
  const double fb = peval(p, DEG, b);
  if (fa == 0.0) { root = a; return 2; }
  if (fb == 0.0) {
    root = b;
    return last_piece ? 1 : 0;
  }
  if ((fa < 0.0) == (fb < 0.0)) return 0;
  double x = 0.5 * (a + b), dx_old = b - a;
  for (int it = 0; it < 100; ++it) {
    const double fx = peval(p, DEG, x);
    if (fx == 0.0) break;
    if ((fx < 0.0) == (fa < 0.0)) a = x; else b = x;
    const double dfx = peval(dp, DEG - 1, x);
    double xn = x - fx / dfx;
    if (!(xn >= a && xn <= b) || !(fabs(xn - x) < 0.5 * dx_old)) {
      if (dx_old <= kRootNoise) break;
      xn = 0.5 * (a + b);
    }
    dx_old = fabs(xn - x);
    x = xn;
    if (dx_old <= kRootStep) break;
  }
  root = x;
  return 1;
}

// Bookkeeping of one level with N pieces, given every piece's result
// (kind[i], root[i]): the roots that count, in order, and the cut points of
// the next level, [-1, slot_0, ..., slot_{N-1}, 1], where slot_i is the last
// counted root of pieces 0..i (-1 if none).  Lane j receives its next piece
// [a, b] and whether its own root counts.
template <int N>
__host__ __device__ inline void level_scan(const int* kind, const double* root, int j, double& a, double& b,
                                           bool& counted) {
  double last = -1.0;
  bool have = false;
  a = -1.0;
  b = 1.0;
  counted = false;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int k = kind[i];
    const double r = root[i];
    const bool c = k == 1 || (k == 2 && (!have || last != r));
    if (c) { last = r; have = true; }
    if (i == j - 1) a = last;
    if (i == j) { b = last; counted = c; }
  }
}

struct GP3PIn {
  double o[3][3], f[3][3], d2[3];
};

__host__ __device__ inline void gp3p_res(const GP3PIn& g, const double l[3], double r[3]) {
  const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
  for (int e = 0; e < 3; ++e) {
    double v[3];
    for (int c = 0; c < 3; ++c) v[c] = g.o[pa[e]][c] + l[pa[e]] * g.f[pa[e]][c] - g.o[pb[e]][c] - l[pb[e]] * g.f[pb[e]][c];
    r[e] = dot3(v, v) - g.d2[e];
  }
}

__host__ __device__ inline void gp3p_polish(const GP3PIn& g, double l[3]) {
  const int pa[3] = {0, 0, 1}, pb[3] = {1, 2, 2};
  for (int it = 0; it < 8; ++it) {
    double r[3];
    gp3p_res(g, l, r);
    const double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double J[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int e = 0; e < 3; ++e) {
      double v[3];
      for (int c = 0; c < 3; ++c) v[c] = g.o[pa[e]][c] + l[pa[e]] * g.f[pa[e]][c] - g.o[pb[e]][c] - l[pb[e]] * g.f[pb[e]][c];
      J[3 * e + pa[e]] = 2.0 * dot3(v, g.f[pa[e]]);
      J[3 * e + pb[e]] = -2.0 * dot3(v, g.f[pb[e]]);
    }
    const double det = det3(J);
    if (!(fabs(det) > 0.0)) return;
    double A[9], n[3], r2[3];
    adj3(J, A);
    for (int k = 0; k < 3; ++k) n[k] = l[k] - (A[3 * k] * r[0] + A[3 * k + 1] * r[1] + A[3 * k + 2] * r[2]) / det;
    gp3p_res(g, n, r2);
    if (!(r2[0] * r2[0] + r2[1] * r2[1] + r2[2] * r2[2] < rr)) return;
    l[0] = n[0]; l[1] = n[1]; l[2] = n[2];
  }
}

// interval of x = l1 on which the (1,k) distance has a real l_k
__host__ __device__ inline bool gp3p_interval(const GP3PIn& g, int k, double& lo, double& hi) {
  double D[3];
  for (int c = 0; c < 3; ++c) D[c] = g.o[0][c] - g.o[k][c];
  const double ck = dot3(g.f[0], g.f[k]), ek = dot3(D, g.f[k]), g1 = dot3(D, g.f[0]);
  const double kk = dot3(D, D) - g.d2[k - 1];
  const double A = ck * ck - 1.0, B = 2.0 * (ck * ek - g1), C = ek * ek - kk;
  if (!(A < 0.0)) return false;
  const double dq = B * B - 4.0 * A * C;
  if (dq < 0.0) return false;
  const double r1 = (-B + sqrt(dq)) / (2.0 * A), r2 = (-B - sqrt(dq)) / (2.0 * A);
  lo = fmin(r1, r2);
  hi = fmax(r1, r2);
  return true;
}

// The degree-8 resultant of one sample and what lifting its roots to depths
// needs.  x = l1 = mid + half s maps the feasible interval onto s in [-1, 1];
// every polynomial is in s, coefficients in increasing degree.
struct GP3PPoly {
  double mid, half, bb, dsum;
  double B12[2], C12[3], B13[2], C13[3], P[2], R[2], Q[3];
  double A2[3], A1[4], A0[5];
  double oct[9];  // the resultant, divided by its largest coefficient magnitude
};

// Builds the resultant of one sample; returns its degree once negligible
// leading coefficients are dropped (0: no feasible interval or no roots).
__host__ __device__ inline int gp3p_poly(const GP3PIn& g, GP3PPoly& y) {
  double lo2, hi2, lo3, hi3;
  if (!gp3p_interval(g, 1, lo2, hi2) || !gp3p_interval(g, 2, lo3, hi3)) return 0;
  const double lo = fmax(0.0, fmax(lo2, lo3)), hi = fmin(hi2, hi3);
  if (!(hi > lo)) return 0;
  const double mid = 0.5 * (lo + hi), half = 0.5 * (hi - lo);
  y.mid = mid;
  y.half = half;
  double D12[3], D13[3], D23[3];
  for (int c = 0; c < 3; ++c) {
    D12[c] = g.o[0][c] - g.o[1][c];
    D13[c] = g.o[0][c] - g.o[2][c];
    D23[c] = g.o[1][c] - g.o[2][c];
  }
  const double c12 = dot3(g.f[0], g.f[1]), c13 = dot3(g.f[0], g.f[2]), c23 = dot3(g.f[1], g.f[2]);
  // polynomials in s, x = mid + half s
  const double xs[2] = {mid, half};
  double(&B12)[2] = y.B12;
  double(&C12)[3] = y.C12;
  double(&B13)[2] = y.B13;
  double(&C13)[3] = y.C13;
  {
    const double e2 = dot3(D12, g.f[1]), g1 = dot3(D12, g.f[0]), k12 = dot3(D12, D12) - g.d2[0];
    const double e3 = dot3(D13, g.f[2]), h1 = dot3(D13, g.f[0]), k13 = dot3(D13, D13) - g.d2[1];
    // B12 = -2 c12 x - 2 e2 ; C12 = x^2 + 2 g1 x + k12
    B12[0] = -2.0 * c12 * xs[0] - 2.0 * e2; B12[1] = -2.0 * c12 * xs[1];
    C12[0] = xs[0] * xs[0] + 2.0 * g1 * xs[0] + k12; C12[1] = 2.0 * xs[0] * xs[1] + 2.0 * g1 * xs[1];
    C12[2] = xs[1] * xs[1];
    B13[0] = -2.0 * c13 * xs[0] - 2.0 * e3; B13[1] = -2.0 * c13 * xs[1];
    C13[0] = xs[0] * xs[0] + 2.0 * h1 * xs[0] + k13; C13[1] = 2.0 * xs[0] * xs[1] + 2.0 * h1 * xs[1];
    C13[2] = xs[1] * xs[1];
  }
  const double bb = -2.0 * c23, c2 = 2.0 * dot3(D23, g.f[1]), c3 = -2.0 * dot3(D23, g.f[2]);
  const double c0 = dot3(D23, D23) - g.d2[2];
  y.bb = bb;
  y.dsum = g.d2[0] + g.d2[1] + g.d2[2];
  double(&P)[2] = y.P;
  double(&R)[2] = y.R;
  double(&Q)[3] = y.Q;
  P[0] = c2 - B12[0]; P[1] = -B12[1];
  R[0] = c3 - B13[0]; R[1] = -B13[1];
  Q[0] = c0 - C12[0] - C13[0]; Q[1] = -C12[1] - C13[1]; Q[2] = -C12[2] - C13[2];
  // A2 = P^2 - b B13 P + b^2 C13
  double(&A2)[3] = y.A2;
  double(&A1)[4] = y.A1;
  double(&A0)[5] = y.A0;
  double t1[5], t2[5];
  pmul(P, 1, P, 1, A2);
  pmul(B13, 1, P, 1, t1);
  for (int e = 0; e <= 2; ++e) A2[e] += -bb * t1[e] + bb * bb * C13[e];
  // A1 = 2 P Q - B13 (P R + b Q) + 2 b C13 R
  double PQ[4], PR[3], bQ[3], S1[3], T[4], CR[4];
  pmul(P, 1, Q, 2, PQ);
  pmul(P, 1, R, 1, PR);
  for (int e = 0; e <= 2; ++e) { bQ[e] = bb * Q[e]; S1[e] = PR[e] + bQ[e]; }
  pmul(B13, 1, S1, 2, T);
  pmul(C13, 2, R, 1, CR);
  for (int e = 0; e <= 3; ++e) A1[e] = 2.0 * PQ[e] - T[e] + 2.0 * bb * CR[e];
  // A0 = Q^2 - B13 Q R + C13 R^2
  double QQ[5], QR[4], RR[3];
  pmul(Q, 2, Q, 2, QQ);
  pmul(Q, 2, R, 1, QR);
  pmul(R, 1, R, 1, RR);
  pmul(B13, 1, QR, 3, t1);
  pmul(C13, 2, RR, 2, t2);
  for (int e = 0; e <= 4; ++e) A0[e] = QQ[e] - t1[e] + t2[e];
  // Res = (A2 C12 - A0)^2 - (A2 B12 - A1)(A1 C12 - A0 B12)
  double U[5], V[4], W[6], a2c12[5], a2b12[4], a1c12[6], a0b12[6];
  pmul(A2, 2, C12, 2, a2c12);
  for (int e = 0; e <= 4; ++e) U[e] = a2c12[e] - A0[e];
  pmul(A2, 2, B12, 1, a2b12);
  for (int e = 0; e <= 3; ++e) V[e] = a2b12[e] - A1[e];
  pmul(A1, 3, C12, 2, a1c12);
  pmul(A0, 4, B12, 1, a0b12);
  for (int e = 0; e <= 5; ++e) W[e] = a1c12[e] - a0b12[e];
  double UU[9], VW[9];
  double(&oct)[9] = y.oct;
  pmul(U, 4, U, 4, UU);
  pmul(V, 3, W, 5, VW);
  double scale = 0.0;
  for (int e = 0; e <= 8; ++e) { oct[e] = UU[e] - VW[e]; scale = fmax(scale, fabs(oct[e])); }
  if (!(scale > 0.0)) return 0;
  for (int e = 0; e <= 8; ++e) oct[e] /= scale;
  int d = 8;
  while (d > 0 && fabs(oct[d]) < 1e-14) --d;
  return d;
}

// Depths (l1, l2, l3) of the root s of the resultant: l2 is the common root
// of the two quadratics in l2, l3 follows from the bilinear relation; all
// three are Newton-polished.  False when the root gives no valid solution
// (a depth not positive, or a residual above 1e-6 of the squared sides).
__host__ __device__ inline bool gp3p_lift(const GP3PIn& g, const GP3PPoly& y, double s, double l[3]) {
  const double x = y.mid + y.half * s;
  const double b12 = peval(y.B12, 1, s), c12v = peval(y.C12, 2, s);
  const double a2 = peval(y.A2, 2, s), a1 = peval(y.A1, 3, s), a0 = peval(y.A0, 4, s);
  l[0] = x;
  l[1] = 0.0;
  l[2] = 0.0;
  const double den = a2 * b12 - a1;
  bool ok = false;
  if (fabs(den) > 1e-300) {
    l[1] = -(a2 * c12v - a0) / den;
    ok = true;
  }
  // otherwise the larger root of the (1,2) quadratic
  const double disc = b12 * b12 - 4.0 * c12v;
  if (!ok && disc >= 0.0) { l[1] = 0.5 * (-b12 + sqrt(disc)); ok = true; }
  if (!ok) return false;
  const double pv = peval(y.P, 1, s), qv = peval(y.Q, 2, s), rv = peval(y.R, 1, s);
  const double den3 = y.bb * l[1] + rv;
  if (fabs(den3) > 1e-300) {
    l[2] = -(pv * l[1] + qv) / den3;
  } else {
    const double b13 = peval(y.B13, 1, s), c13v = peval(y.C13, 2, s);
    const double d3 = b13 * b13 - 4.0 * c13v;
    if (d3 < 0.0) return false;
    l[2] = 0.5 * (-b13 + sqrt(d3));
  }
  if (!(l[0] > 0.0 && l[1] > 0.0 && l[2] > 0.0)) return false;
  gp3p_polish(g, l);
  if (!(l[0] > 0.0 && l[1] > 0.0 && l[2] > 0.0)) return false;
  double res[3];
  gp3p_res(g, l, res);
  return fabs(res[0]) + fabs(res[1]) + fabs(res[2]) < 1e-6 * y.dsum;
}

// Solutions of one sample from its lifted roots (ok[i], depths l0/l1/l2[i],
// i < N, in root order): a solution within 1e-9 (relative, summed over the
// depths) of an earlier kept one is a duplicate; the kept ones are ordered by
// l1, then l2, ties by root order.  Returns whether lane j's solution is kept
// and its rank among the kept ones.
template <int N>
__host__ __device__ inline bool gp3p_keep_rank(const int* ok, const double* l0, const double* l1, const double* l2,
                                               int j, int& rank) {
  bool keep[N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    bool k = ok[i] != 0;
    const double tol = 1e-9 * (l0[i] + l1[i] + l2[i]);
#pragma unroll
    for (int e = 0; e < i; ++e)
      if (keep[e] && fabs(l0[e] - l0[i]) + fabs(l1[e] - l1[i]) + fabs(l2[e] - l2[i]) <= tol) k = false;
    keep[i] = k;
  }
  bool mine = false;
  double m0 = 0.0, m1 = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i)
    if (i == j) { mine = keep[i]; m0 = l0[i]; m1 = l1[i]; }
  rank = 0;
#pragma unroll
  for (int e = 0; e < N; ++e) {
    const bool before = l0[e] < m0 || (l0[e] == m0 && (l1[e] < m1 || (l1[e] == m1 && e < j)));
    if (keep[e] && e != j && before) ++rank;
  }
  return mine;
}

// Pose with P_i = R X_i + t from the rig-frame triangle P and the world
// triangle X (frames of two edges and their cross product, two Newton-Schulz
// steps towards the nearest rotation).
__host__ __device__ inline bool gp3p_pose(const double P[3][3], const double X[3][3], Pose& out) {
  double a[3], b[3], c[3], A[3], B[3], C[3];
  for (int k = 0; k < 3; ++k) {
    a[k] = X[0][k] - X[1][k]; b[k] = X[0][k] - X[2][k];
    A[k] = P[0][k] - P[1][k]; B[k] = P[0][k] - P[2][k];
  }
  cross3(a, b, c);
  cross3(A, B, C);
  double Mx[9], My[9], adj[9];
  for (int r = 0; r < 3; ++r) {
    Mx[3 * r] = a[r]; Mx[3 * r + 1] = b[r]; Mx[3 * r + 2] = c[r];
    My[3 * r] = A[r]; My[3 * r + 1] = B[r]; My[3 * r + 2] = C[r];
  }
  const double det = det3(Mx);
  if (!(fabs(det) > 0.0)) return false;
  adj3(Mx, adj);
  double* R = out.R;
  for (int r = 0; r < 3; ++r)
    for (int cc = 0; cc < 3; ++cc)
      R[3 * r + cc] = (My[3 * r] * adj[cc] + My[3 * r + 1] * adj[3 + cc] + My[3 * r + 2] * adj[6 + cc]) / det;
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
    for (int e = 0; e < 9; ++e) R[e] = Rn[e];
  }
  for (int r = 0; r < 3; ++r) out.t[r] = P[0][r] - (R[3 * r] * X[0][0] + R[3 * r + 1] * X[0][1] + R[3 * r + 2] * X[0][2]);
  return true;
}

}  // namespace imloc
