// imloc_device.h -- device-side building blocks of the pose-estimation path
// (gfx950).  Included by the kernel translation units only.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace imloc {

constexpr int kWave = 64;

struct Cam { double fx, fy, cx, cy; };

// Pointers read from a device-side table carry no address space; viewing them
// as global lets the compiler emit global (not flat) loads.
template <class T>
__device__ inline const __attribute__((address_space(1))) T* gmem(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}
struct Pose { double R[9]; double t[3]; };

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC 2011): per round two 64x64->128 products;
// the high halves are xor-ed with the other two words and the round key; the
// key advances by the Weyl constants.
// ---------------------------------------------------------------------------
__device__ inline void philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3, uint64_t k0, uint64_t k1,
                                     uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += W0; k1 += W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// Minimal sample h: three distinct indices of [0, n) from the stream keyed by
// (seed, 0) at counter (h, query, attempt, 0); index = high word of word * n.
__device__ inline bool sample_triple(uint64_t seed, uint64_t query, uint64_t h, uint64_t n, int idx[3]) {
  if (n < 3) return false;
  for (uint64_t attempt = 0; attempt < 16; ++attempt) {
    uint64_t w[4];
    philox4x64_10(h, query, attempt, 0, seed, 0, w);
    const int a = (int)__umul64hi(w[0], n), b = (int)__umul64hi(w[1], n), c = (int)__umul64hi(w[2], n);
    if (a != b && a != c && b != c) {
      idx[0] = a; idx[1] = b; idx[2] = c;
      return true;
    }
  }
  return false;
}

__device__ inline uint64_t binom(uint64_t n, uint64_t k) {
  if (k > n) return 0;
  uint64_t r = 1;
  for (uint64_t i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

// h-th 3-combination of [0, n), colexicographic (combinatorial number system).
__device__ inline bool unrank_triple(uint64_t h, uint64_t n, int idx[3]) {
  if (n < 3 || h >= binom(n, 3)) return false;
  uint64_t k = 2;
  while (binom(k + 1, 3) <= h) ++k;
  h -= binom(k, 3);
  uint64_t j = 1;
  while (binom(j + 1, 2) <= h) ++j;
  h -= binom(j, 2);
  idx[0] = (int)h; idx[1] = (int)j; idx[2] = (int)k;
  return true;
}

// ---------------------------------------------------------------------------
// Small dense algebra (float64).
// ---------------------------------------------------------------------------
__host__ __device__ inline double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
__host__ __device__ inline void cross3(const double a[3], const double b[3], double o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
__host__ __device__ inline double det3(const double M[9]) {
  return M[0] * (M[4] * M[8] - M[5] * M[7]) - M[1] * (M[3] * M[8] - M[5] * M[6]) + M[2] * (M[3] * M[7] - M[4] * M[6]);
}
// adjugate (transpose of the cofactor matrix)
__host__ __device__ inline void adj3(const double M[9], double A[9]) {
  A[0] = M[4] * M[8] - M[5] * M[7];
  A[1] = M[2] * M[7] - M[1] * M[8];
  A[2] = M[1] * M[5] - M[2] * M[4];
  A[3] = M[5] * M[6] - M[3] * M[8];
  A[4] = M[0] * M[8] - M[2] * M[6];
  A[5] = M[2] * M[3] - M[0] * M[5];
  A[6] = M[3] * M[7] - M[4] * M[6];
  A[7] = M[1] * M[6] - M[0] * M[7];
  A[8] = M[0] * M[4] - M[1] * M[3];
}
__device__ inline double trace_prod(const double A[9], const double B[9]) {
  double s = 0.0;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) s += A[3 * r + c] * B[3 * c + r];
  return s;
}

// Exp on SO(3) (Rodrigues): A = sin(th) / th and B = (1 - cos(th)) / th^2;
// below th = 0.5 their Taylor series in th^2 to 9 terms (truncation below
// 1e-19), which a Gauss-Newton step almost always is.
__device__ inline void so3_exp(const double w[3], double E[9]) {
  const double th2 = dot3(w, w);
  double A, B;
  if (th2 < 0.25) {
    // 1/(2k+1)! and 1/(2k+2)!, k = 8 .. 0, in Horner order
    A = 1.0 / 355687428096000.0;
    A = fma(A, -th2, 1.0 / 1307674368000.0);
    A = fma(A, -th2, 1.0 / 6227020800.0);
    A = fma(A, -th2, 1.0 / 39916800.0);
    A = fma(A, -th2, 1.0 / 362880.0);
    A = fma(A, -th2, 1.0 / 5040.0);
    A = fma(A, -th2, 1.0 / 120.0);
    A = fma(A, -th2, 1.0 / 6.0);
    A = fma(A, -th2, 1.0);
    B = 1.0 / 6402373705728000.0;
    B = fma(B, -th2, 1.0 / 20922789888000.0);
    B = fma(B, -th2, 1.0 / 87178291200.0);
    B = fma(B, -th2, 1.0 / 479001600.0);
    B = fma(B, -th2, 1.0 / 3628800.0);
    B = fma(B, -th2, 1.0 / 40320.0);
    B = fma(B, -th2, 1.0 / 720.0);
    B = fma(B, -th2, 1.0 / 24.0);
    B = fma(B, -th2, 0.5);
  } else {
    const double th = sqrt(th2);
    double s, c;
    sincos(th, &s, &c);
    A = s / th;
    B = (1.0 - c) / th2;
  }
  const double x = w[0], y = w[1], z = w[2];
  // I + A [w]x + B [w]x^2, with [w]x^2 = w w^T - th2 I
  E[0] = 1.0 + B * (x * x - th2);
  E[1] = -A * z + B * x * y;
  E[2] = A * y + B * x * z;
  E[3] = A * z + B * x * y;
  E[4] = 1.0 + B * (y * y - th2);
  E[5] = -A * x + B * y * z;
  E[6] = -A * y + B * x * z;
  E[7] = A * x + B * y * z;
  E[8] = 1.0 + B * (z * z - th2);
}

// x' = Exp(dw) x + dt : R' = Exp(dw) R, t' = Exp(dw) t + dt.
__device__ inline void pose_left_update(const Pose& P, const double d[6], Pose& o) {
  double E[9];
  so3_exp(d, E);
  for (int r = 0; r < 3; ++r) {
    for (int c = 0; c < 3; ++c) o.R[3 * r + c] = E[3 * r] * P.R[c] + E[3 * r + 1] * P.R[3 + c] + E[3 * r + 2] * P.R[6 + c];
    o.t[r] = E[3 * r] * P.t[0] + E[3 * r + 1] * P.t[1] + E[3 * r + 2] * P.t[2] + d[3 + r];
  }
}

// Solve H x = b, H symmetric positive definite 6x6 given by its upper triangle
// packed row-wise (21 entries).  false if a pivot is not positive.
__device__ inline bool chol6_solve_packed(const double Hp[21], const double b[6], double x[6]) {
  double L[6][6];
  int k = 0;
  double H[6][6];
  for (int r = 0; r < 6; ++r)
    for (int c = r; c < 6; ++c) { H[r][c] = Hp[k]; H[c][r] = Hp[k]; ++k; }
  for (int i = 0; i < 6; ++i) {
    for (int j = 0; j <= i; ++j) {
      double s = H[i][j];
      for (int m = 0; m < j; ++m) s -= L[i][m] * L[j][m];
      if (i == j) {
        if (!(s > 0.0)) return false;
        L[i][i] = sqrt(s);
      } else {
        L[i][j] = s / L[j][j];
      }
    }
  }
  double y[6];
  for (int i = 0; i < 6; ++i) {
    double s = b[i];
    for (int m = 0; m < i; ++m) s -= L[i][m] * y[m];
    y[i] = s / L[i][i];
  }
  for (int i = 5; i >= 0; --i) {
    double s = y[i];
    for (int m = i + 1; m < 6; ++m) s -= L[m][i] * x[m];
    x[i] = s / L[i][i];
  }
  return true;
}

// ---------------------------------------------------------------------------
// P3P in float64, as an intersection of a pencil of conics.
//
// Unknowns: depths l = (l1, l2, l3) > 0 along unit bearings y_i.  With
// b_ij = -y_i.y_j and a_ij = |x_i - x_j|^2 each pair gives the quadric
// l^T M_ij l = a_ij (M_ij has ones on the (i,i), (j,j) diagonal entries and
// b_ij off the diagonal).  Eliminating the right-hand sides gives two
// homogeneous conics D1 = M12 - (a12/a23) M23 and D2 = M13 - (a13/a23) M23
// through all solutions.  A degenerate member D0 = D1 + g D2 of their pencil
// (det = 0, a cubic in g) is a pair of lines through the solutions; each line
// meets D1 or D2 in at most two points, scaled by l^T M23 l = a23.  The pose
// follows from the three camera-frame points l_i y_i.
// ---------------------------------------------------------------------------

// Real roots of c3 x^3 + c2 x^2 + c1 x + c0 on [lo, hi], ascending, each
// passed to emit(root).  The interval is split at the critical points, so
// the cubic is monotone on each of the (at most three) brackets; every
// bracket with a sign change is shrunk by 24 bisection steps and then
// polished by 4 Newton steps kept inside it.  The brackets are refined
// together, branch-free, as independent chains (a lone wave per SIMD is
// bound by instruction issue, so one shared loop beats three divergent ones).
__device__ inline double cubic_at(double c0, double c1, double c2, double c3, double x) {
  return ((c3 * x + c2) * x + c1) * x + c0;
}

template <class Emit>
__device__ inline void cubic_roots_in(double c0, double c1, double c2, double c3, double lo, double hi, Emit&& emit) {
  // critical points: 3 c3 x^2 + 2 c2 x + c1 = 0
  const double qa = 3.0 * c3, qb = 2.0 * c2, qc = c1;
  double x1 = 0.0, x2 = 0.0;
  bool u1 = false, u2 = false;
  const double scale = fabs(qa) + fabs(qb) + fabs(qc);
  if (fabs(qa) > 1e-300 + 1e-15 * scale) {
    const double disc = qb * qb - 4.0 * qa * qc;
    if (disc > 0.0) {
      const double q = -0.5 * (qb + copysign(sqrt(disc), qb));
      x1 = q / qa;
      x2 = (q != 0.0) ? qc / q : x1;
      if (x1 > x2) { const double tt = x1; x1 = x2; x2 = tt; }
      u1 = true;
      u2 = true;
    }
  } else if (fabs(qb) > 0.0) {
    x1 = -qc / qb;
    u1 = true;
  }
  u1 = u1 && x1 > lo && x1 < hi;
  u2 = u2 && x2 > lo && x2 < hi;
  // brackets [lo, m1], [m1, m2], [m2, hi] over the split points in range
  const double m1 = u1 ? x1 : (u2 ? x2 : hi);
  const double m2 = (u1 && u2) ? x2 : hi;
  const int nb = 1 + (int)u1 + (int)u2;
  double A[3] = {lo, m1, m2}, B[3] = {m1, m2, hi};
  bool run[3], neg[3], at_a[3], at_b[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    const double fa = cubic_at(c0, c1, c2, c3, A[t]), fb = cubic_at(c0, c1, c2, c3, B[t]);
    const bool live = t < nb;
    at_a[t] = live && fa == 0.0;
    at_b[t] = live && !at_a[t] && fb == 0.0 && t == nb - 1;
    run[t] = live && !at_a[t] && !at_b[t] && ((fa < 0.0) != (fb < 0.0));
    neg[t] = fa < 0.0;
  }
  if (run[0] || run[1] || run[2]) {
    for (int it = 0; it < 24; ++it) {
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const double m = 0.5 * (A[t] + B[t]);
        const bool left = (cubic_at(c0, c1, c2, c3, m) < 0.0) == neg[t];
        A[t] = left ? m : A[t];
        B[t] = left ? B[t] : m;
      }
    }
    double x[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) x[t] = 0.5 * (A[t] + B[t]);
    for (int it = 0; it < 4; ++it) {
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const double f = cubic_at(c0, c1, c2, c3, x[t]);
        const double df = (qa * x[t] + qb) * x[t] + qc;
        const double xn = df != 0.0 ? x[t] - f / df : x[t];
        x[t] = fmin(fmax(xn, A[t]), B[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) A[t] = x[t];
  }
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    if (at_a[t]) emit(t == 0 ? lo : (t == 1 ? m1 : m2));
    else if (run[t]) emit(A[t]);
    else if (at_b[t]) emit(hi);
  }
}

// Eigenvector of symmetric M for eigenvalue s: the longest cross product of
// two rows of (M - s I).
__device__ inline void sym_eigvec(const double M[9], double s, double v[3]) {
  double r0[3] = {M[0] - s, M[1], M[2]}, r1[3] = {M[3], M[4] - s, M[5]}, r2[3] = {M[6], M[7], M[8] - s};
  double a[3], b[3], c[3];
  cross3(r0, r1, a);
  cross3(r0, r2, b);
  cross3(r1, r2, c);
  const double na = dot3(a, a), nb = dot3(b, b), nc = dot3(c, c);
  const double* best = a;
  double nbest = na;
  if (nb > nbest) { best = b; nbest = nb; }
  if (nc > nbest) { best = c; nbest = nc; }
  const double inv = nbest > 0.0 ? 1.0 / sqrt(nbest) : 0.0;
  v[0] = best[0] * inv; v[1] = best[1] * inv; v[2] = best[2] * inv;
}

// Newton polishing of the depths on the three quadrics; a step is kept while
// it lowers the squared residual.
__device__ inline void polish_depths(double l[3], double a12, double a13, double a23, double b12, double b13,
                                     double b23) {
  for (int it = 0; it < 6; ++it) {
    const double F0 = l[0] * l[0] + l[1] * l[1] + 2.0 * b12 * l[0] * l[1] - a12;
    const double F1 = l[0] * l[0] + l[2] * l[2] + 2.0 * b13 * l[0] * l[2] - a13;
    const double F2 = l[1] * l[1] + l[2] * l[2] + 2.0 * b23 * l[1] * l[2] - a23;
    const double J[9] = {2.0 * (l[0] + b12 * l[1]), 2.0 * (l[1] + b12 * l[0]), 0.0,
                         2.0 * (l[0] + b13 * l[2]), 0.0, 2.0 * (l[2] + b13 * l[0]),
                         0.0, 2.0 * (l[1] + b23 * l[2]), 2.0 * (l[2] + b23 * l[1])};
    const double det = det3(J);
    if (!(fabs(det) > 0.0)) return;
    double A[9];
    adj3(J, A);
    const double F[3] = {F0, F1, F2};
    const double idet = 1.0 / det;
    double n[3];
    for (int r = 0; r < 3; ++r) n[r] = l[r] - (A[3 * r] * F[0] + A[3 * r + 1] * F[1] + A[3 * r + 2] * F[2]) * idet;
    const double G0 = n[0] * n[0] + n[1] * n[1] + 2.0 * b12 * n[0] * n[1] - a12;
    const double G1 = n[0] * n[0] + n[2] * n[2] + 2.0 * b13 * n[0] * n[2] - a13;
    const double G2 = n[1] * n[1] + n[2] * n[2] + 2.0 * b23 * n[1] * n[2] - a23;
    if (!(G0 * G0 + G1 * G1 + G2 * G2 < F0 * F0 + F1 * F1 + F2 * F2)) return;
    l[0] = n[0]; l[1] = n[1]; l[2] = n[2];
  }
}

// Shared part of one sample's P3P: squared sides, bearing cosines, the two
// conics and the coefficients of the cubic det(D1 + g D2).
struct P3PSetup {
  double a12, a13, a23, b12, b13, b23;
  double D1[9], D2[9];
  double c0, c1, c2, c3;
};

// y: unit bearings (row per point), x: world points.  False for a degenerate
// world triangle (no solution).
__device__ inline bool p3p_setup(const double y[3][3], const double x[3][3], P3PSetup& s) {
  double d12[3], d13[3], d23[3];
  for (int k = 0; k < 3; ++k) { d12[k] = x[0][k] - x[1][k]; d13[k] = x[0][k] - x[2][k]; d23[k] = x[1][k] - x[2][k]; }
  s.a12 = dot3(d12, d12);
  s.a13 = dot3(d13, d13);
  s.a23 = dot3(d23, d23);
  double crs[3];
  cross3(d12, d13, crs);
  if (!(s.a12 > 0.0 && s.a13 > 0.0 && s.a23 > 0.0)) return false;
  if (!(sqrt(dot3(crs, crs)) > 1e-9 * (s.a12 + s.a13 + s.a23))) return false;
  s.b12 = -dot3(y[0], y[1]);
  s.b13 = -dot3(y[0], y[2]);
  s.b23 = -dot3(y[1], y[2]);
  const double ia23 = 1.0 / s.a23;
  const double r12 = s.a12 * ia23, r13 = s.a13 * ia23;
  const double D1[9] = {1.0, s.b12, 0.0, s.b12, 1.0 - r12, -r12 * s.b23, 0.0, -r12 * s.b23, -r12};
  const double D2[9] = {1.0, 0.0, s.b13, 0.0, -r13, -r13 * s.b23, s.b13, -r13 * s.b23, 1.0 - r13};
  double A1[9], A2[9];
  adj3(D1, A1);
  adj3(D2, A2);
  s.c0 = det3(D1);
  s.c1 = trace_prod(A1, D2);
  s.c2 = trace_prod(D1, A2);
  s.c3 = det3(D2);
  for (int e = 0; e < 9; ++e) { s.D1[e] = D1[e]; s.D2[e] = D2[e]; }
  return true;
}

// Degenerate pencil member D1 + g D2 (from_f, g = root) or e D1 + D2 (e =
// root), scaled to unit largest entry, with its trace T and second invariant
// S.  Returns its quality -S / (T^2 - 2 S), or 0 if it has none.
__device__ inline double p3p_member(const P3PSetup& s, double root, bool from_f, double M[9], double& T, double& S) {
  double mx = 0.0;
  for (int e = 0; e < 9; ++e) {
    M[e] = from_f ? s.D1[e] + root * s.D2[e] : root * s.D1[e] + s.D2[e];
    mx = fmax(mx, fabs(M[e]));
  }
  if (!(mx > 0.0)) return 0.0;
  const double imx = 1.0 / mx;
  for (int e = 0; e < 9; ++e) M[e] *= imx;
  T = M[0] + M[4] + M[8];
  S = (M[0] * M[4] - M[1] * M[3]) + (M[0] * M[8] - M[2] * M[6]) + (M[4] * M[8] - M[5] * M[7]);
  const double den = T * T - 2.0 * S;
  if (!(den > 0.0)) return 0.0;
  const double q = -S / den;
  return q > 0.0 ? q : 0.0;
}

// One of the two searches for degenerate members: from_f, the roots g of
// det(D1 + g D2) on [-1, 1]; otherwise the roots e of det(e D1 + D2) with
// |e| < 1.  Returns the quality of the first member of best quality (0: none)
// and its root.
__device__ inline double p3p_best_member(const P3PSetup& s, bool from_f, double& best_root) {
  double best_q = 0.0;
  best_root = 0.0;
  const double k0 = from_f ? s.c0 : s.c3, k1 = from_f ? s.c1 : s.c2;
  const double k2 = from_f ? s.c2 : s.c1, k3 = from_f ? s.c3 : s.c0;
  cubic_roots_in(k0, k1, k2, k3, -1.0, 1.0, [&](double r) {
    if (!from_f && !(fabs(r) < 1.0)) return;
    double M[9], T = 0.0, S = 0.0;
    const double q = p3p_member(s, r, from_f, M, T, S);
    if (q > best_q) { best_q = q; best_root = r; }
  });
  return best_q;
}

// Slot t = 2 line + intersection of the degenerate member D0 (trace T, second
// invariant S; from_f says which conic to cut its lines with): the depths of
// the solution on that slot, Newton-polished; false if the slot has none
// (no intersection, a depth not positive, or a residual above 1e-6 of the
// squared sides).
__device__ inline bool p3p_slot(const P3PSetup& s, const double D0[9], double T, double S, bool from_f, int t,
                                double l[3]) {
  // conic restricted to the lines: the pencil member farthest from D0
  const double* Q = from_f ? s.D2 : s.D1;
  const double half = 0.5 * T, disc = sqrt(half * half - S);
  const double s1 = half + disc, s2 = half - disc;  // s1 > 0 > s2
  double e1[3], e2[3], e3[3];
  sym_eigvec(D0, s1, e1);
  sym_eigvec(D0, s2, e2);
  cross3(e1, e2, e3);
  const double w1 = sqrt(s1), w2 = sqrt(-s2);
  const double sgn = (t >> 1) == 0 ? -1.0 : 1.0;
  double nrm[3], m[3];
  for (int c = 0; c < 3; ++c) nrm[c] = w1 * e1[c] + sgn * w2 * e2[c];
  cross3(nrm, e3, m);
  const double mn = sqrt(dot3(m, m));
  if (!(mn > 0.0)) return false;
  const double imn = 1.0 / mn;
  for (int c = 0; c < 3; ++c) m[c] *= imn;
  double Qe[3], Qm[3];
  for (int r = 0; r < 3; ++r) {
    Qe[r] = Q[3 * r] * e3[0] + Q[3 * r + 1] * e3[1] + Q[3 * r + 2] * e3[2];
    Qm[r] = Q[3 * r] * m[0] + Q[3 * r + 1] * m[1] + Q[3 * r + 2] * m[2];
  }
  const double A = dot3(e3, Qe), B = dot3(e3, Qm), C = dot3(m, Qm);
  const double dq = B * B - A * C;
  if (dq < 0.0) return false;
  const double sq = sqrt(dq);
  const double root_sign = (t & 1) == 0 ? 1.0 : -1.0;  // intersection 0: -B + sq, 1: -B - sq
  double v[3];
  if (fabs(A) >= fabs(C) && A != 0.0) {
    const double ra = (-B + root_sign * sq) / A;  // alpha / beta
    for (int c = 0; c < 3; ++c) v[c] = ra * e3[c] + m[c];
  } else if (C != 0.0) {
    const double ra = (-B + root_sign * sq) / C;  // beta / alpha
    for (int c = 0; c < 3; ++c) v[c] = e3[c] + ra * m[c];
  } else {
    for (int c = 0; c < 3; ++c) v[c] = (t & 1) == 0 ? e3[c] : m[c];
  }
  const double s23 = v[1] * v[1] + v[2] * v[2] + 2.0 * s.b23 * v[1] * v[2];
  if (!(s23 > 0.0)) return false;
  const double sc = sqrt(s.a23 / s23) * ((v[0] + v[1] + v[2]) < 0.0 ? -1.0 : 1.0);
  l[0] = sc * v[0];
  l[1] = sc * v[1];
  l[2] = sc * v[2];
  if (!(l[0] > 0.0 && l[1] > 0.0 && l[2] > 0.0)) return false;
  polish_depths(l, s.a12, s.a13, s.a23, s.b12, s.b13, s.b23);
  if (!(l[0] > 0.0 && l[1] > 0.0 && l[2] > 0.0)) return false;
  const double F0 = l[0] * l[0] + l[1] * l[1] + 2.0 * s.b12 * l[0] * l[1] - s.a12;
  const double F1 = l[0] * l[0] + l[2] * l[2] + 2.0 * s.b13 * l[0] * l[2] - s.a13;
  const double F2 = l[1] * l[1] + l[2] * l[2] + 2.0 * s.b23 * l[1] * l[2] - s.a23;
  return fabs(F0) + fabs(F1) + fabs(F2) < 1e-6 * (s.a12 + s.a13 + s.a23);
}

// Solutions of one sample from its four slots (ok[t], depths l0/l1/l2[t],
// camera depths k0/k1[t] of points 0 and 1): a slot within 1e-9 (relative,
// summed over the depths) of an earlier kept slot is a duplicate; the kept
// ones are ordered by (k0, k1, slot).  Returns whether slot j is kept and its
// rank among the kept ones.
__device__ inline bool p3p_keep_rank(const int* ok, const double* l0, const double* l1, const double* l2,
                                     const double* k0, const double* k1, int j, int& rank) {
  bool keep[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    bool k = ok[t] != 0;
    const double tol = 1e-9 * (l0[t] + l1[t] + l2[t]);
#pragma unroll
    for (int e = 0; e < t; ++e)
      if (keep[e] && fabs(l0[e] - l0[t]) + fabs(l1[e] - l1[t]) + fabs(l2[e] - l2[t]) <= tol) k = false;
    keep[t] = k;
  }
  bool mine = false;
  double m0 = 0.0, m1 = 0.0;
#pragma unroll
  for (int t = 0; t < 4; ++t)
    if (t == j) { mine = keep[t]; m0 = k0[t]; m1 = k1[t]; }
  rank = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const bool before = k0[e] < m0 || (k0[e] == m0 && (k1[e] < m1 || (k1[e] == m1 && e < j)));
    if (keep[e] && e != j && before) ++rank;
  }
  return mine;
}

// Inverse of the world triangle frame X = [x1 - x2, x1 - x3, (x1 - x2) x
// (x1 - x3)] (columns), shared by all solutions of a sample.
__device__ inline void p3p_frame_inverse(const double x[3][3], double Xi[9]) {
  double d12[3], d13[3], crs[3];
  for (int k = 0; k < 3; ++k) { d12[k] = x[0][k] - x[1][k]; d13[k] = x[0][k] - x[2][k]; }
  cross3(d12, d13, crs);
  double X[9];
  for (int r = 0; r < 3; ++r) { X[3 * r] = d12[r]; X[3 * r + 1] = d13[r]; X[3 * r + 2] = crs[r]; }
  adj3(X, Xi);
  const double idet = 1.0 / det3(X);
  for (int e = 0; e < 9; ++e) Xi[e] *= idet;
}

// Pose of one P3P solution: R maps the world triangle frame onto the camera
// one (R = Y X^-1, then one Newton-Schulz step towards the nearest rotation),
// t = l1 y1 - R x1.  Xi from p3p_frame_inverse.
__device__ inline void p3p_pose(const double l[3], const double y[3][3], const double x[3][3], const double Xi[9],
                                Pose& P) {
  double z[3][3];
  for (int i = 0; i < 3; ++i)
    for (int c = 0; c < 3; ++c) z[i][c] = l[i] * y[i][c];
  double e12[3], e13[3], ec[3];
  for (int c = 0; c < 3; ++c) { e12[c] = z[0][c] - z[1][c]; e13[c] = z[0][c] - z[2][c]; }
  cross3(e12, e13, ec);
  double Y[9];
  for (int r = 0; r < 3; ++r) { Y[3 * r] = e12[r]; Y[3 * r + 1] = e13[r]; Y[3 * r + 2] = ec[r]; }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      P.R[3 * r + c] = Y[3 * r] * Xi[c] + Y[3 * r + 1] * Xi[3 + c] + Y[3 * r + 2] * Xi[6 + c];
  // R <- R (3 I - R^T R) / 2
  double RtR[9], Rn[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c)
      RtR[3 * r + c] = P.R[r] * P.R[c] + P.R[3 + r] * P.R[3 + c] + P.R[6 + r] * P.R[6 + c];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double s2 = 0.0;
      for (int m = 0; m < 3; ++m) s2 += P.R[3 * r + m] * ((m == c ? 3.0 : 0.0) - RtR[3 * m + c]);
      Rn[3 * r + c] = 0.5 * s2;
    }
  for (int e = 0; e < 9; ++e) P.R[e] = Rn[e];
  for (int r = 0; r < 3; ++r)
    P.t[r] = z[0][r] - (P.R[3 * r] * x[0][0] + P.R[3 * r + 1] * x[0][1] + P.R[3 * r + 2] * x[0][2]);
}

// 8-bit log-depth codes (ImLoc Sec. 3.3 "Data Compression"): depth clipped to
// [0.25, 128] m and quantised uniformly in log depth; code 0 = no depth,
// code c >= 1 = 0.25 * 512^((c - 1) / 254).
constexpr double kLog8DMin = 0.25;            // metres, level of code 1
constexpr double kLog8Log2Range = 9.0;        // log2(128 / 0.25)
constexpr double kLog8Steps = 254.0;          // levels 1..255

__device__ inline double log8_level(int c) {
  return c == 0 ? 0.0 : kLog8DMin * exp2(((double)(c - 1) * kLog8Log2Range) / kLog8Steps);
}

// nearest level in log depth (halves away from zero); 0 for depth not finite or <= 0
__device__ inline uint8_t log8_code(float f) {
  double d = f;
  if (!(d > 0.0 && d <= 3.4028234663852886e38)) return 0;
  d = fmin(fmax(d, kLog8DMin), kLog8DMin * 512.0);
  const double level = kLog8Steps * log2(d / kLog8DMin) / kLog8Log2Range;
  return (uint8_t)(1 + (int)round(level));
}

// Folded projection P = K [R | t] rows (a, b, w) = P [X, 1].
__device__ inline void projection_rows(const Pose& P, const Cam& K, double M[12]) {
  for (int c = 0; c < 3; ++c) {
    M[c] = K.fx * P.R[c] + K.cx * P.R[6 + c];
    M[4 + c] = K.fy * P.R[3 + c] + K.cy * P.R[6 + c];
    M[8 + c] = P.R[6 + c];
  }
  M[3] = K.fx * P.t[0] + K.cx * P.t[2];
  M[7] = K.fy * P.t[1] + K.cy * P.t[2];
  M[11] = P.t[2];
}

// ---------------------------------------------------------------------------
// Wave / block reductions.
// ---------------------------------------------------------------------------
__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}
__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}
__device__ inline long long wave_sum(long long v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

}  // namespace imloc
