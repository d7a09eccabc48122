/*
 * imloc_oracle.h -- FP64 CPU oracle for the ImLoc pose-estimation hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow, obviously-correct
 * definition that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no source with the GPU library and includes none of its headers.
 *
 * What it follows (ImLoc, Jiang et al., arXiv 2601.04185):
 *   - Sec. 3.3 "Query Time Matching and 2D-3D Lifting": give every
 *     query-to-database match a world point through the stored depth maps
 *     (bilinear at sub-pixel database coordinates, plain lookup otherwise),
 *     keep matches with valid depth and confidence above 0.05.
 *   - Sec. 3.3 "Pose Estimation": LO-RANSAC over P3P minimal sets; each
 *     hypothesis is scored by the MSAC sum of squared pixel errors clipped at
 *     the threshold, weighted by the matching confidences; a hypothesis that
 *     beats the running best is refined by Gauss-Newton on that clipped sum;
 *     sampling ends at a cap or once the standard RANSAC confidence bound is
 *     met; the best pose is then refined over every inlier with a Cauchy loss.
 *   - Sec. 1 cites the Haralick et al. (1994) review for PnP; the P3P here is
 *     Grunert's law-of-cosines elimination described in that review.
 * The paper prints no formulas; the readings taken where it is silent are the
 * ones listed with each function below.
 *
 * Everything is FP64.  Float32 inputs are promoted to double on entry.
 */
#ifndef IMLOC_ORACLE_H
#define IMLOC_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { double fx, fy, cx, cy; } orc_camera;      /* pinhole, no distortion */
typedef struct { double R[9]; double t[3]; } orc_pose;      /* cam_from_world, R row-major */

/* Correspondence set in structure-of-arrays form, float32 as the GPU sees it. */
typedef struct {
  const float *u, *v;          /* observed query pixel (continuous coords) */
  const float *X, *Y, *Z;      /* world point */
  const float *w;              /* confidence weight; NULL means all 1 */
  int64_t n;
} orc_corr;

typedef struct {
  double threshold_px;         /* tau: inlier iff squared error < tau^2 */
  int64_t fixed_samples;       /* > 0: draw exactly this many samples, no adaptive stop */
  int64_t batch;               /* samples per batch */
  int64_t min_iters, max_iters;
  double confidence;           /* stop when P(miss best) < 1 - confidence */
  int32_t lo_top_k;            /* candidates refined per batch (clamped to [1, 32]) */
  int32_t lo_iters;            /* Gauss-Newton iterations of the local optimisation */
  int64_t max_score_points;    /* 0: score all; else stride-subsample to this many */
  int32_t final_iters;         /* Cauchy IRLS iterations of the final refinement */
  double cauchy_scale_px;      /* s of the Cauchy loss */
  int32_t exhaustive;          /* 1: sample h is the h-th 3-combination (tiny n only) */
  uint64_t seed, query_id;
} orc_params;

typedef struct {
  int64_t samples, candidates, residuals;
  int64_t best_count;          /* inliers of the best model on the scoring set */
  int64_t full_count;          /* inliers on the full set at the final pose */
  int64_t batches;
  int32_t lo_runs, status;     /* status 0 = pose, 1 = no pose */
  double best_msac;            /* truncated cost of the best model on the scoring set */
  double final_cost;           /* Cauchy cost at the final pose */
  int64_t best_h; int32_t best_j;  /* sample / solution the best model grew from */
} orc_stats;

/* Philox4x64-10 block function (Salmon et al., SC'11). */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* Minimal sample h of a query: three distinct indices in [0, n).
 * Counter (h, query_id, attempt, 0), key (seed, 0); index k = floor(word_k * n / 2^64);
 * up to 16 attempts, else the sample is empty.  Returns 1 if valid. */
int orc_sample_triple(uint64_t seed, uint64_t query_id, uint64_t h, int64_t n, int32_t idx[3]);

/* h-th 3-combination of [0, n) in colexicographic order (exhaustive mode). */
int orc_unrank_triple(uint64_t h, int64_t n, int32_t idx[3]);

/* P3P (Grunert via Haralick et al. 1994).  Inputs: pixel coords uv[2*k+{0,1}],
 * world points Xw[3*k+{0,1,2}] for k = 0..2.  Writes up to 4 poses, ordered by
 * camera depth of point 0, then point 1.  *ill is set to 1 when a root is
 * near-double, a depth is near zero or the triple is near-degenerate, i.e.
 * where another correct formulation may return a different solution count. */
int orc_p3p(const double uv[6], const double Xw[9], const orc_camera *K,
            orc_pose out[4], int32_t *ill);

/* Truncated (MSAC) scoring of np poses against all points: count of inliers
 * (z > 0 and r^2 < tau^2) and sum_i w_i * min(r_i^2, tau^2), points behind the
 * camera contributing tau^2. */
void orc_score(const orc_pose *poses, int64_t np, const orc_corr *c,
               const orc_camera *K, double tau, int32_t *count, double *msac);

/* Same test with an ambiguity band per residual: count_lo counts residuals
 * inside tau - b_i, count_hi those inside tau + b_i, where
 * b_i = max(band_abs, f32_bound_i) and f32_bound_i (used when with_f32 != 0)
 * bounds the error of evaluating the residual in float32 from a float32-rounded
 * projection matrix (derivation at residual_band in imloc_oracle.c; a point
 * too close to the camera plane to sign its depth in float32 counts in
 * count_hi only). */
void orc_score_band(const orc_pose *poses, int64_t np, const orc_corr *c,
                    const orc_camera *K, double tau, double band_abs, int32_t with_f32,
                    int32_t *count_lo, int32_t *count_hi, double *msac_err_bound);

/* Per residual of one pose: the exact pixel distance r_i (NaN when the point is
 * behind the camera or, with with_f32, too close to its plane to sign the depth
 * in float32) and its band b_i as used by orc_score_band. */
void orc_residual_band(const orc_pose *pose, const orc_corr *c, const orc_camera *K, double tau, double band_abs,
                       int32_t with_f32, double *r, double *beta);

/* Truncated cost at a pose and the Gauss-Newton normal equations over its
 * inliers: H = sum_i w_i J_i^T J_i, g = sum_i w_i J_i^T r_i, with J_i the
 * Jacobian of the pixel residual w.r.t. the left update (dw, dt). */
double orc_normal_equations(const orc_pose *P, const orc_corr *c, const orc_camera *K, double tau, double H[36],
                            double g[6], int64_t *count);

/* Left update on SO(3) x R^3: R' = Exp(dw) R, t' = Exp(dw) t + dt. */
void orc_pose_update(const orc_pose *P, const double d[6], orc_pose *o);

/* 1 if the Gauss-Newton step d = (dw, dt) is shorter than 1e-10: such a
 * step is not taken and ends the run (local optimisation, refinement). */
int orc_step_converged(const double d[6]);

/* Local optimisation: Gauss-Newton on sum_i w_i min(r_i^2, tau^2) over the
 * given point set, inlier set re-evaluated at every iterate, left update on
 * SO(3), a step that raises the cost is rejected and ends the run, and so
 * does a step shorter than 1e-10 (Euclidean norm of (dw, dt)), not taken.
 * Returns the number of accepted steps; *cost / *count at the output pose. */
int orc_lo(const orc_pose *start, const orc_corr *c, const orc_camera *K, double tau,
           int32_t iters, orc_pose *out, double *cost, int64_t *count);

/* Final refinement: IRLS Gauss-Newton on sum_{i in I} w_i s^2 ln(1 + r_i^2/s^2)
 * over the fixed set I = inliers of the full set at the start pose (tau),
 * with the same two ends of a run as orc_lo.
 * Returns accepted steps; *cost at the output pose; *n_inl = |I|. */
int orc_refine(const orc_pose *start, const orc_corr *c, const orc_camera *K, double tau,
               double s, int32_t iters, orc_pose *out, double *cost, int64_t *n_inl);

/* Samples required by the stopping rule for inlier ratio eps, minimal size 3. */
int64_t orc_required_samples(double eps, double confidence, int64_t max_iters);

/* Whole LO-RANSAC PnP for one query.  mask (n bytes, may be NULL) receives the
 * inlier mask over all points at the final pose.  Returns status (0 pose, 1 none). */
int orc_lo_ransac_pnp(const orc_corr *c, const orc_camera *K, const orc_params *p,
                      orc_pose *pose, uint8_t *mask, orc_stats *stats);

/* Lifting: a world point for every image-to-image match.  Views: depth[k*H*W + row*W + col].
 * cams[k], poses[k] per view (cam_from_world).  subpixel != 0: bilinear depth at
 * (db_u - 0.5, db_v - 0.5); else lookup at (floor(db_v), floor(db_u)).
 * Keeps a match iff conf > min_conf (compared in float32), view in range and
 * depth valid.  Outputs in input order; returns the count. */
int64_t orc_lift(const float *q_u, const float *q_v, const float *db_u, const float *db_v,
                 const float *conf, const int32_t *view, int64_t n_matches, int32_t subpixel,
                 const float *depth, int32_t n_views, int32_t H, int32_t W,
                 const orc_camera *cams, const orc_pose *poses, float min_conf,
                 double *out_u, double *out_v, double *out_X, double *out_Y, double *out_Z,
                 double *out_w, int64_t *out_src);

/* 8-bit log-depth codes (Sec. 3.3 "Data Compression"; Sec. 4.3 "Depth
 * Quantization"): depth clipped to [0.25, 128] m, quantised uniformly in log
 * depth.  Code 0: no depth (not finite or <= 0); codes 1..255: levels
 * 0.25 * 512^((c - 1) / 254), the nearest level in log depth is chosen. */
double orc_log8_decode(uint8_t c);
uint8_t orc_log8_encode(float depth);
void orc_log8_encode_array(const float *depth, int64_t n, uint8_t *codes);

/* orc_lift on code maps codes[k*H*W + row*W + col]; a tap holding code 0 is
 * invalid, any other decodes to its level (float64) before interpolation. */
int64_t orc_lift_log8(const float *q_u, const float *q_v, const float *db_u, const float *db_v,
                      const float *conf, const int32_t *view, int64_t n_matches, int32_t subpixel,
                      const uint8_t *codes, int32_t n_views, int32_t H, int32_t W,
                      const orc_camera *cams, const orc_pose *poses, float min_conf,
                      double *out_u, double *out_v, double *out_X, double *out_Y, double *out_Z,
                      double *out_w, int64_t *out_src);

/* Depth of every pixel of a mapping image by 1-DoF triangulation of dense
 * matches (Sec. 3.3 "Depth Estimation by Dense Matching"; triangulate.c).
 * Matches mu, mv, conf: [V][H][W] float32, pixel (row i, col j) of the
 * mapping image matched to (mu, mv) of covisible view k.  Outputs [H][W]:
 * depth (z-depth, 0 = none), inliers of the winning hypothesis, the view
 * whose match gave it (-1 = none) and whether some angular test of the pixel
 * lay within 1e-9 rad of the threshold (then float rounding may decide). */
typedef struct {
  double min_conf;         /* a match is used iff conf >= min_conf (float32 comparison) */
  double angle_deg;        /* inlier iff angular error < angle_deg */
  int32_t min_inliers;     /* the depth is kept iff the inlier set has at least this many */
  int32_t max_refine_iters;
} orc_tri_params;

void orc_triangulate(int32_t H, int32_t W, const orc_camera *K0, const orc_pose *T0, int32_t V,
                     const orc_camera *Kv, const orc_pose *Tv, const float *mu, const float *mv,
                     const float *conf, const orc_tri_params *p, double *depth, int32_t *inliers,
                     int32_t *best_view, uint8_t *ambiguous, double *cost, double *curv);
/* (cost, curv: optional [H][W] outputs, the refinement cost at the kept depth
 * and its second derivative in l, 0 where no depth is kept) */
/* The pieces, for the tests: angle of depth l for one observation (C0 + l r0
 * seen from Ck along unit rk), the depth minimising it (0 if none), and the
 * refinement of l0 over n weighted observations. */
double orc_tri_angle(const double C0[3], const double r0[3], double l, const double Ck[3], const double rk[3]);
int orc_tri_hypothesis(const double C0[3], const double r0[3], const double Ck[3], const double rk[3], double *l);
double orc_tri_refine(const double C0[3], const double r0[3], double l0, int n, const double (*Ck)[3],
                      const double (*rk)[3], const double *w, int max_iters);

/* Multi-camera rig (generalised absolute pose; rig.c).  A rig camera has
 * intrinsics K and cam_from_rig (R, t); poses are rig_from_world; a world
 * point X seen by camera c projects through x_c = R_c (R X + t) + t_c. */
typedef struct {
  orc_camera K;
  double R[9], t[3];
} orc_rig_camera;

typedef struct {
  const float *u, *v, *X, *Y, *Z, *w;  /* as orc_corr (w may be NULL) */
  const int32_t *cam;                  /* camera of each correspondence */
  int64_t n;
} orc_rig_corr;

/* Generalised P3P: rays (origins o[3*i..], directions f[3*i..], rig frame)
 * through world points Xw.  Up to 8 rig poses, ordered by the depth along ray
 * 0, then ray 1; depths (3 per pose) if non-NULL.  *ill = 1 for near-double
 * roots or near-zero depths (another correct formulation may then differ). */
int orc_gp3p(const double o[9], const double f[9], const double Xw[9], orc_pose out[8], double depths[24],
             int32_t *ill);
void orc_rig_score(const orc_pose *poses, int64_t np, const orc_rig_corr *c, const orc_rig_camera *cams,
                   double tau, int32_t *count, double *msac);
int orc_rig_lo(const orc_pose *start, const orc_rig_corr *c, const orc_rig_camera *cams, double tau, int32_t iters,
               orc_pose *out, double *cost, int64_t *count);
int orc_rig_refine(const orc_pose *start, const orc_rig_corr *c, const orc_rig_camera *cams, double tau, double s,
                   int32_t iters, orc_pose *out, double *cost, int64_t *n_inl);
int orc_rig_lo_ransac(const orc_rig_corr *c, const orc_rig_camera *cams, int32_t n_cams, const orc_params *p,
                      orc_pose *pose, uint8_t *mask, orc_stats *st);

/* Host threads of the OpenMP loops (independent candidates only, so the
 * results do not depend on it): orc_set_threads(n) for n >= 1, and the
 * number the next parallel loop will use. */
void orc_set_threads(int32_t n);
int32_t orc_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
