/* Runs every entry point of the float64 oracle on small synthetic inputs, for
 * a build with AddressSanitizer and UndefinedBehaviorSanitizer (test
 * infrastructure: tests/test_sanitizers.py builds and runs it).  Exits 0 when
 * every call returns and the recovered poses are close to the truth. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "imloc_oracle.h"

static uint64_t g_state = 0x9E3779B97F4A7C15ull;
static double urand(void) { /* xorshift64*, uniform in [0, 1) */
  g_state ^= g_state >> 12; g_state ^= g_state << 25; g_state ^= g_state >> 27;
  return (double)((g_state * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}

static void rot_from_axis(double ax, double ay, double az, double ang, double R[9]) {
  const double n = sqrt(ax * ax + ay * ay + az * az);
  ax /= n; ay /= n; az /= n;
  const double c = cos(ang), s = sin(ang), C = 1 - c;
  R[0] = c + ax * ax * C;      R[1] = ax * ay * C - az * s; R[2] = ax * az * C + ay * s;
  R[3] = ay * ax * C + az * s; R[4] = c + ay * ay * C;      R[5] = ay * az * C - ax * s;
  R[6] = az * ax * C - ay * s; R[7] = az * ay * C + ax * s; R[8] = c + az * az * C;
}

/* n correspondences seen by pose (R, t) through K, a fraction `inl` exact */
static void make_query(int n, double inl, const orc_camera *K, const orc_pose *P, float *u, float *v, float *X,
                       float *Y, float *Z, float *w) {
  for (int i = 0; i < n; ++i) {
    const double px = urand() * 640, py = urand() * 480, z = 2 + 18 * urand();
    const double xc = (px - K->cx) / K->fx * z, yc = (py - K->cy) / K->fy * z;
    const double d[3] = {xc - P->t[0], yc - P->t[1], z - P->t[2]};
    double Xw[3];
    for (int r = 0; r < 3; ++r) Xw[r] = P->R[r] * d[0] + P->R[3 + r] * d[1] + P->R[6 + r] * d[2];
    const int good = urand() < inl;
    u[i] = (float)(good ? px : urand() * 640);
    v[i] = (float)(good ? py : urand() * 480);
    X[i] = (float)Xw[0]; Y[i] = (float)Xw[1]; Z[i] = (float)Xw[2];
    w[i] = (float)(0.1 + 0.9 * urand());
  }
}

static double rot_err(const orc_pose *a, const orc_pose *b) {
  double tr = 0;
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) tr += a->R[3 * r + c] * b->R[3 * r + c];
  double x = 0.5 * (tr - 1);
  return acos(x > 1 ? 1 : (x < -1 ? -1 : x));
}

int main(void) {
  int fails = 0;
  const orc_camera K = {500, 500, 320, 240};
  orc_pose P;
  rot_from_axis(0.3, -1, 0.2, 0.7, P.R);
  P.t[0] = 0.5; P.t[1] = -0.3; P.t[2] = 1.0;
  enum { N = 600 };
  float *u = malloc(N * 4), *v = malloc(N * 4), *X = malloc(N * 4), *Y = malloc(N * 4), *Z = malloc(N * 4),
        *w = malloc(N * 4);
  make_query(N, 0.5, &K, &P, u, v, X, Y, Z, w);
  const orc_corr c = {u, v, X, Y, Z, w, N};

  /* sampling, P3P, scoring, bands, local optimisation, refinement */
  int32_t idx[3];
  for (uint64_t h = 0; h < 50; ++h) orc_sample_triple(0, 3, h, N, idx);
  orc_unrank_triple(17, 12, idx);
  orc_pose cand[4];
  int32_t ill = 0;
  double uv[6], Xw[9];
  for (int k = 0; k < 3; ++k) { /* an exact triple from the inlier generator */
    float uu[1], vv[1], xx[1], yy[1], zz[1], ww[1];
    make_query(1, 1.0, &K, &P, uu, vv, xx, yy, zz, ww);
    uv[2 * k] = uu[0]; uv[2 * k + 1] = vv[0]; Xw[3 * k] = xx[0]; Xw[3 * k + 1] = yy[0]; Xw[3 * k + 2] = zz[0];
  }
  const int ns = orc_p3p(uv, Xw, &K, cand, &ill);
  if (ns < 1) { fprintf(stderr, "p3p found no solution\n"); ++fails; }
  int32_t cnt[4], lo[4], hi[4];
  double ms[4], eb[4], r[N], beta[N];
  orc_score(cand, ns > 0 ? ns : 1, &c, &K, 4.0, cnt, ms);
  orc_score_band(cand, ns > 0 ? ns : 1, &c, &K, 4.0, 1e-5, 1, lo, hi, eb);
  orc_residual_band(&P, &c, &K, 4.0, 1e-5, 1, r, beta);
  double H[36], g[6];
  int64_t count = 0;
  orc_normal_equations(&P, &c, &K, 4.0, H, g, &count);
  orc_pose out;
  double cost;
  orc_lo(&cand[0], &c, &K, 4.0, 10, &out, &cost, &count);
  orc_refine(&P, &c, &K, 4.0, 2.0, 10, &out, &cost, &count);
  orc_required_samples(0.3, 0.999, 100000);

  /* whole LO-RANSAC, fixed and adaptive, with a subsample */
  orc_params p;
  memset(&p, 0, sizeof(p));
  p.threshold_px = 4; p.fixed_samples = 256; p.batch = 128; p.lo_top_k = 3; p.lo_iters = 10;
  p.final_iters = 10; p.cauchy_scale_px = 2; p.confidence = 0.999; p.max_iters = 10000; p.min_iters = 128;
  uint8_t mask[N];
  orc_stats st;
  orc_pose best;
  orc_lo_ransac_pnp(&c, &K, &p, &best, mask, &st);
  if (rot_err(&best, &P) > 1e-3) { fprintf(stderr, "fixed-sample pose off\n"); ++fails; }
  p.fixed_samples = 0; p.max_score_points = 300;
  orc_lo_ransac_pnp(&c, &K, &p, &best, mask, &st);
  if (rot_err(&best, &P) > 1e-3) { fprintf(stderr, "adaptive pose off\n"); ++fails; }

  /* lifting through a fronto-parallel depth map, float32 and 8-bit codes */
  enum { VH = 12, VW = 16, NM = 40 };
  float depth[2 * VH * VW];
  uint8_t codes[2 * VH * VW];
  for (int i = 0; i < 2 * VH * VW; ++i) depth[i] = (i % 37 == 5) ? 0.0f : 3.0f;
  orc_log8_encode_array(depth, 2 * VH * VW, codes);
  for (int cc = 0; cc < 256; ++cc) (void)orc_log8_decode((uint8_t)cc);
  const orc_camera Kd[2] = {{20, 20, 8, 6}, {20, 20, 8, 6}};
  orc_pose Td[2];
  memcpy(&Td[0], &P, sizeof(P));
  memcpy(&Td[1], &P, sizeof(P));
  float qu[NM], qv[NM], du[NM], dv[NM], cf[NM];
  int32_t vw[NM];
  for (int i = 0; i < NM; ++i) {
    qu[i] = (float)(urand() * 640); qv[i] = (float)(urand() * 480);
    du[i] = (float)(urand() * VW * 1.1); dv[i] = (float)(urand() * VH * 1.1);
    cf[i] = (float)urand(); vw[i] = i % 3 - (i % 7 == 0);
  }
  double ou[NM], ov[NM], oX[NM], oY[NM], oZ[NM], ow[NM];
  int64_t src[NM];
  orc_lift(qu, qv, du, dv, cf, vw, NM, 1, depth, 2, VH, VW, Kd, Td, 0.05f, ou, ov, oX, oY, oZ, ow, src);
  orc_lift(qu, qv, du, dv, cf, vw, NM, 0, depth, 2, VH, VW, Kd, Td, 0.05f, ou, ov, oX, oY, oZ, ow, src);
  orc_lift_log8(qu, qv, du, dv, cf, vw, NM, 1, codes, 2, VH, VW, Kd, Td, 0.05f, ou, ov, oX, oY, oZ, ow, src);

  /* mapping depth on a tiny image with three views */
  enum { TH = 9, TW = 11, TV = 3 };
  float mu[TV * TH * TW], mv[TV * TH * TW], mc[TV * TH * TW];
  for (int i = 0; i < TV * TH * TW; ++i) {
    mu[i] = (float)(urand() * TW); mv[i] = (float)(urand() * TH); mc[i] = (float)urand();
  }
  mu[5] = NAN;
  orc_pose Tv[TV];
  orc_camera Kv[TV];
  for (int k = 0; k < TV; ++k) {
    rot_from_axis(0, 1, 0, 0.05 * (k + 1), Tv[k].R);
    Tv[k].t[0] = -0.3 * (k + 1); Tv[k].t[1] = 0; Tv[k].t[2] = 0;
    Kv[k] = (orc_camera){10, 10, 5.5, 4.5};
  }
  orc_pose T0;
  rot_from_axis(0, 0, 1, 0, T0.R);
  T0.t[0] = T0.t[1] = T0.t[2] = 0;
  const orc_tri_params tp = {0.05, 2.0, 2, 50};
  double tdepth[TH * TW], tcost[TH * TW], tcurv[TH * TW];
  int32_t tinl[TH * TW], tview[TH * TW];
  uint8_t tamb[TH * TW];
  orc_triangulate(TH, TW, &Kv[0], &T0, TV, Kv, Tv, mu, mv, mc, &tp, tdepth, tinl, tview, tamb, tcost, tcurv);

  /* a two-camera rig */
  orc_rig_camera rc[2];
  for (int k = 0; k < 2; ++k) {
    rc[k].K = K;
    rot_from_axis(0, 1, 0, k ? 0.4 : -0.4, rc[k].R);
    rc[k].t[0] = k ? 0.05 : -0.05; rc[k].t[1] = 0; rc[k].t[2] = 0;
  }
  int32_t cam[N];
  for (int i = 0; i < N; ++i) cam[i] = i < N / 2 ? 0 : 1;
  const orc_rig_corr rcc = {u, v, X, Y, Z, w, cam, N};
  orc_pose rposes[8];
  double depths[24];
  const double o[9] = {0, 0, 0, 0.1, 0, 0, 0, 0.1, 0}, f[9] = {0, 0, 1, 0.1, 0, 1, 0, 0.1, 1};
  orc_gp3p(o, f, Xw, rposes, depths, &ill);
  int32_t rcnt[1];
  double rms[1];
  orc_rig_score(&P, 1, &rcc, rc, 4.0, rcnt, rms);
  orc_rig_lo(&P, &rcc, rc, 4.0, 10, &out, &cost, &count);
  orc_rig_refine(&P, &rcc, rc, 4.0, 2.0, 10, &out, &cost, &count);
  p.fixed_samples = 128; p.max_score_points = 0;
  orc_rig_lo_ransac(&rcc, rc, 2, &p, &best, mask, &st);

  free(u); free(v); free(X); free(Y); free(Z); free(w);
  printf("oracle driver done: %d failure(s)\n", fails);
  return fails ? 1 : 0;
}
