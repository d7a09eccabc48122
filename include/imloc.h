/*
 * imloc.h -- C ABI of the MI355X pose-estimation library (libimloc.so).
 *
 * The library implements the query-time hot path of ImLoc (Jiang et al.,
 * arXiv 2601.04185, Sec. 3.3): dense query-to-database matches are lifted to
 * 2D-3D correspondences through the stored depth maps, intrinsics and poses
 * ("Query Time Matching and 2D-3D Lifting"), then the query pose is estimated
 * by LO-RANSAC over P3P minimal sets: MSAC scoring of clipped squared pixel
 * errors weighted by confidence, Gauss-Newton refinement of a hypothesis that
 * beats the running best, an adaptive stopping rule, and a last Cauchy-loss
 * refinement over every inlier ("Pose Estimation").  Every step runs in HIP kernels on the GPU.
 *
 * Conventions (the paper fixes none of them):
 *   - pinhole cameras without distortion; pixel (row i, col j) has its centre
 *     at (j + 0.5, i + 0.5);
 *   - poses are cam_from_world, x_cam = R X + t, R row-major;
 *   - depth maps store z-depth (distance along the optical axis).
 *
 * Memory: every array argument marked "device" is a caller-owned device
 * pointer on the context's device; "host" arguments are ordinary host
 * memory.  The library never frees or keeps a caller pointer beyond the call.
 * Scratch memory comes from a caller-provided workspace
 * (imloc_set_workspace); the library itself allocates no device memory after
 * imloc_create.  Host staging (pinned memory for query tables and results)
 * is allocated by imloc_create and imloc_set_staging only: a call that needs
 * more staging returns IMLOC_ENOMEM instead of growing it, and timing events
 * are created by imloc_set_timing, so the query calls allocate nothing.
 * Work is enqueued on the context's stream; calls that return host results
 * synchronise that stream before returning.
 *
 * Errors: functions return IMLOC_OK (0), IMLOC_NO_POSE (1, the call ran but
 * no pose candidate exists), or a negative code; imloc_last_error() gives a
 * message.  A context is used by one host thread at a time.
 */
#ifndef IMLOC_H
#define IMLOC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define IMLOC_OK 0
#define IMLOC_NO_POSE 1
#define IMLOC_PENDING 2     /* imloc_server_poll: the query has not finished yet */
#define IMLOC_EINVAL (-1)   /* bad argument (null pointer, size, threshold, intrinsics) */
#define IMLOC_ENOMEM (-2)   /* workspace or host staging too small: see imloc_workspace_bytes, imloc_staging_bytes */
#define IMLOC_EHIP (-3)     /* HIP runtime error */

#define IMLOC_FP32_SCORE 0  /* scoring in float32; P3P, local optimisation, refinement in float64 */
#define IMLOC_FP64_ALL 1    /* every step in float64 */

typedef struct imloc_ctx imloc_ctx;

typedef struct { double fx, fy, cx, cy; } imloc_camera;
typedef struct { double R[9]; double t[3]; } imloc_pose;   /* 12 doubles, R row-major */

/* 2D-3D correspondences, structure of arrays, float32, device pointers of
 * length n: observed query pixel (u, v), world point (X, Y, Z), weight w (the
 * matching confidence; NULL means every weight is 1). */
typedef struct {
  const float *u, *v, *X, *Y, *Z, *w;
} imloc_corr;

/* Output arrays of imloc_lift (device, capacity entries each; w and src may
 * be NULL if not wanted). */
typedef struct {
  float *u, *v, *X, *Y, *Z, *w;
  int32_t *src;    /* index of the match each correspondence came from */
} imloc_corr_out;

/* 2D-2D matches, device arrays of length n: query pixel, database pixel,
 * matching confidence, database view index. */
typedef struct {
  const float *q_u, *q_v, *db_u, *db_v, *conf;
  const int32_t *view;
} imloc_matches;

typedef struct {
  double threshold_px;       /* tau: a residual is an inlier iff r^2 < tau^2 (and depth > 0) */
  int64_t fixed_samples;     /* > 0: draw exactly this many minimal samples, no adaptive stop */
  int64_t batch;             /* samples per batch (the paper uses 1,000) */
  int64_t min_iters;         /* adaptive mode: never stop before this many samples */
  int64_t max_iters;         /* adaptive mode: cap (the paper: 100,000) */
  double confidence;         /* adaptive mode: stop when P(missing the best model) < 1 - confidence */
  int32_t lo_top_k;          /* candidates of a batch refined when they beat the running best (clamped to [1, 32]) */
  int32_t lo_iters;          /* Gauss-Newton iterations of the local optimisation, at most (a run also
                                ends at a cost-raising step or one shorter than 1e-10) */
  int64_t max_score_points;  /* 0: score every correspondence; else stride-subsample to this many */
  int32_t final_iters;       /* Cauchy refinement iterations, at most, with the same two ends (0: skip) */
  double cauchy_scale_px;    /* s of rho(r^2) = s^2 ln(1 + r^2 / s^2) */
  int32_t exhaustive;        /* 1: sample h is the h-th 3-combination instead of a Philox draw */
  int32_t precision;         /* IMLOC_FP32_SCORE or IMLOC_FP64_ALL */
  uint64_t seed, query_id;   /* Philox key word 0 and counter word 1 */
} imloc_ransac_params;

typedef struct {
  int64_t samples;           /* minimal samples drawn */
  int64_t candidates;        /* pose candidates scored (0-4 per sample) */
  int64_t residuals;         /* candidate x scored-point pairs evaluated */
  int64_t inlier_residuals;  /* of those, the ones inside the threshold */
  int64_t best_count;        /* inliers of the best model on the scoring set */
  int64_t full_count;        /* inliers of the final pose on the full set */
  int64_t batches;
  int32_t lo_runs;           /* local optimisations run */
  int32_t status;            /* IMLOC_OK or IMLOC_NO_POSE */
  double best_msac;          /* truncated cost of the best model on the scoring set */
  double final_cost;         /* Cauchy cost at the final pose */
  int64_t best_h;            /* sample the best model grew from */
  int32_t best_j;            /* its P3P solution index */
  int32_t score_launches;    /* scoring kernel launches (for per-launch timing) */
  /* device time in ms, if timing is on: sampling + P3P + the scoring work
   * list, the scoring kernel alone, selection, local optimisation with the
   * round's end, final refinement with the mask, and the whole call */
  float ms_sample, ms_score, ms_select, ms_lo, ms_refine, ms_total;
} imloc_stats;

/* Fill *p with the LO-RANSAC settings of Sec. 3.3 "Pose Estimation": batches
 * of 1,000 minimal sets, adaptive stop once the chance of having missed the
 * best model is below 1e-4 (at least one batch, at most 100,000 samples),
 * scoring on a uniform subsample of at most 10,000 points, local optimisation
 * (10 Gauss-Newton iterations) of a batch's best candidate when it beats the
 * running best, 10 Cauchy refinement iterations over the full set with
 * s = threshold_px / 2, float32 scoring, seed 0.  The paper states no pixel
 * threshold, so the caller gives it.  Host-only; touches no device.  Returns
 * IMLOC_EINVAL for a null p or a threshold that is not finite and > 0. */
int imloc_paper_params(double threshold_px, imloc_ransac_params *p);

/* ---- context ----------------------------------------------------------- */

/* Create a context on `device` that enqueues on `hip_stream` (a hipStream_t;
 * NULL = the null stream).  Returns IMLOC_OK or IMLOC_EHIP / IMLOC_EINVAL. */
int imloc_create(imloc_ctx **out, int device, void *hip_stream);
void imloc_destroy(imloc_ctx *ctx);
int imloc_set_stream(imloc_ctx *ctx, void *hip_stream);
const char *imloc_last_error(const imloc_ctx *ctx);

/* Hand the context a device scratch buffer of `bytes` bytes (caller-owned,
 * must stay valid while calls that use it are in flight). */
int imloc_set_workspace(imloc_ctx *ctx, void *device_ptr, size_t bytes);

/* Host staging.  imloc_create gives every context 1 MiB of pinned staging,
 * enough for a batch of about 1,400 queries; imloc_staging_bytes(nq, c) is
 * what a batch of nq queries with c rig cameras in total (0 without rigs)
 * needs (never less than the default), and imloc_set_staging replaces the
 * context's staging by `bytes` of pinned host memory (it waits for the
 * context's stream first and drops a captured graph that used the old
 * buffer; a server created on the context must not be stepping).
 * imloc_get_staging reports the current size.  A call whose tables do not
 * fit returns IMLOC_ENOMEM and names the size needed.  imloc_set_staging
 * returns IMLOC_EINVAL above 4 GiB and IMLOC_EHIP if the allocation fails. */
size_t imloc_staging_bytes(int32_t n_queries, int32_t n_rig_cameras);
int imloc_set_staging(imloc_ctx *ctx, size_t bytes);
size_t imloc_get_staging(const imloc_ctx *ctx);

/* Workspace bytes imloc_lo_ransac_pnp needs for up to n correspondences. */
size_t imloc_workspace_bytes(int64_t n, const imloc_ransac_params *p);

/* Workspace bytes imloc_lo_ransac_pnp_batch needs for nq queries of the given
 * sizes (host array) and parameters (host array of n_params = 1 or nq). */
size_t imloc_batch_workspace_bytes(int32_t nq, const int64_t *n, const imloc_ransac_params *p, int32_t n_params);

/* Workspace bytes of the stage entry points: imloc_score for n
 * correspondences and np poses, imloc_local_optimize for n correspondences
 * and np start poses, imloc_refine for n correspondences, imloc_sample_p3p
 * for count samples of n correspondences, imloc_lift and imloc_lift_log8 for n_matches matches over
 * n_views views. */
size_t imloc_score_workspace_bytes(int64_t n, int64_t np, int32_t precision);
size_t imloc_sample_workspace_bytes(int64_t n, int64_t count);
size_t imloc_lo_workspace_bytes(int64_t n, int32_t np);
size_t imloc_refine_workspace_bytes(int64_t n);
size_t imloc_lift_workspace_bytes(int64_t n_matches, int32_t n_views);

/* 1: record per-stage device time with HIP events into imloc_stats (the
 * first call with 1 creates the context's pool of 256 events; when a call
 * needs more spans than the pool holds, the stream is synchronised and the
 * pool reused, so timing perturbs long adaptive runs slightly). */
int imloc_set_timing(imloc_ctx *ctx, int enable);

/* 1: run batches with a fixed sample count as one captured hipGraph, replayed
 * while the batch shape (query count and sizes, parameters, workspace) stays
 * the same; 0 (default): enqueue every launch.  Results are identical.
 * imloc_graph_counters reports captures and replays so far. */
int imloc_set_graphs(imloc_ctx *ctx, int enable);
int imloc_graph_counters(const imloc_ctx *ctx, int64_t *captures, int64_t *launches);

/* Launch shape of the scoring kernel: candidates per work item (32, 64 or
 * 128, or 0, the default: picked per round, the largest tile that still
 * gives about four work items per compute unit) and workgroups (1 to 2^20;
 * each walks the round's work list with a grid stride; or 0, the default:
 * per round, about 1.5 per estimated work item, between 8 per compute unit
 * and 2^18).  Neither changes any result (per-candidate sums are
 * integer-accumulated), only the speed; the autotuner in the Python package
 * picks them by timing.  imloc_get_score_tuning reports 0 for a value picked
 * per round.  Returns IMLOC_EINVAL for other values. */
int imloc_set_score_tuning(imloc_ctx *ctx, int32_t candidates_per_item, int32_t workgroups);
int imloc_get_score_tuning(const imloc_ctx *ctx, int32_t *candidates_per_item, int32_t *workgroups);

/* Correspondence tile of the float32 scoring kernel: correspondences per work
 * item, 512, 1024, 2048 (default) or 4096.  A wave always scores a block of
 * 512 consecutive correspondences against a candidate, and the per-block
 * partial sums are added as integers, so the tile changes no result, only
 * the speed (longer items stage each candidate tile once for more
 * correspondences; shorter ones give more items to small rounds).  Float64
 * scoring keeps its own 512-correspondence items.  IMLOC_EINVAL for other
 * values. */
int imloc_set_score_points(imloc_ctx *ctx, int32_t points_per_item);
int imloc_get_score_points(const imloc_ctx *ctx, int32_t *points_per_item);

/* Launch form of the Gauss-Newton runs (local optimisation and final
 * refinement): 0 (default) picks by size, 1 = one launch per iteration in
 * which every workgroup of a problem re-reduces the previous partial sums,
 * 2 = an evaluation launch and a one-workgroup-per-problem decision launch
 * per iteration.  Every form sums the same 512-point chunk partials in the
 * same order, so results are identical; only the speed differs.  Returns
 * IMLOC_EINVAL for another value. */
int imloc_set_gn_mode(imloc_ctx *ctx, int32_t mode);

/* ---- the hot path -------------------------------------------------------- */

/* Give each query-to-database match a world point (Sec. 3.3 "Query Time Matching
 * and 2D-3D Lifting").  A match is kept iff conf > min_conf (float32
 * comparison; the paper uses 0.05), its view index is in [0, n_views), its
 * coordinates are finite, and its depth is valid: subpixel != 0 interpolates
 * bilinearly at (db_u - 0.5, db_v - 0.5) and needs all four taps inside the
 * image, finite and > 0; subpixel == 0 reads texel (floor(db_v), floor(db_u))
 * and needs it inside the image, finite and > 0.  The world point is
 * R_k^T (d K_k^-1 [db_u, db_v, 1]^T - t_k).  Kept matches are written in input
 * order (a stable compaction).
 *   m: device arrays of n_matches entries.  depth: device float32
 *   [n_views][H][W].  cams, poses: host arrays of n_views entries.
 *   out: device arrays of `capacity` entries.  n_out: device int32, receives
 *   the number kept (no host synchronisation).  Matches beyond `capacity`
 *   kept ones are dropped (n_out still counts them). */
int imloc_lift(imloc_ctx *ctx, const imloc_matches *m, int64_t n_matches, const float *depth, int32_t n_views,
               int32_t H, int32_t W, const imloc_camera *cams, const imloc_pose *poses, int32_t subpixel,
               float min_conf, const imloc_corr_out *out, int64_t capacity, int32_t *n_out);

/* 8-bit log-depth codes of stored depth maps (Sec. 3.3 "Data Compression":
 * depth clipped to [0.25, 128] m and quantised uniformly in log depth, 256
 * codes; Sec. 4.3 "Depth Quantization" bounds the relative error by 1.4 %).
 * Code 0 = no depth (depth not finite or <= 0); code c in 1..255 = the level
 * 0.25 * 512^((c - 1) / 254) m; a depth gets its nearest level in log depth
 * (halves away from zero), so the relative error is at most
 * exp(ln 512 / 508) - 1 = 1.24 %.
 *   depth: device float32 [count]; codes: device uint8 [count] (caller-owned).
 *   Asynchronous on the context's stream.  Returns IMLOC_EINVAL for a
 *   negative count or null arrays. */
int imloc_depth_encode_log8(imloc_ctx *ctx, const float *depth, int64_t count, uint8_t *codes);

/* imloc_lift on code maps: codes is device uint8 [n_views][H][W]; a tap with
 * code 0 is invalid, any other is decoded to its level (float64) before the
 * interpolation.  Every other argument, rule and the output are those of
 * imloc_lift; the maps take a quarter of the float32 maps' memory. */
int imloc_lift_log8(imloc_ctx *ctx, const imloc_matches *m, int64_t n_matches, const uint8_t *codes,
                    int32_t n_views, int32_t H, int32_t W, const imloc_camera *cams, const imloc_pose *poses,
                    int32_t subpixel, float min_conf, const imloc_corr_out *out, int64_t capacity, int32_t *n_out);

/* A camera of a multi-camera rig: intrinsics and the camera's pose in the
 * rig frame (cam_from_rig: x_cam = R x_rig + t). */
typedef struct {
  imloc_camera K;
  imloc_pose cam_from_rig;
} imloc_rig_camera;

/* LO-RANSAC for a multi-camera rig query: generalised absolute pose (the
 * appendix on LaMAR HoloLens rig queries, with the LO-RANSAC of Sec. 3.3
 * "Pose Estimation").  The unknown is rig_from_world (R, t); a world point X
 * seen by camera c projects through x_c = R_c (R X + t) + t_c and K_c.
 * Minimal samples are drawn as in imloc_lo_ransac_pnp; each yields up to 8
 * candidates from the generalised P3P (the distance equations of the three
 * rays of the sampled points in the rig frame, reduced to a degree-8
 * polynomial in the first depth); scoring, selection, local optimisation,
 * stopping and the final Cauchy refinement are those of imloc_lo_ransac_pnp
 * with every residual taken through its point's camera.
 *   pts: device arrays of n correspondences GROUPED BY CAMERA: camera c owns
 *   [cam_start[c], cam_start[c + 1]) (host array of n_cams + 1, from 0 to n).
 *   cams: host array of n_cams (1..8).  pose_out: rig_from_world.  mask,
 *   stats: as imloc_lo_ransac_pnp (mask in the caller's point order).
 *   Needs imloc_rig_workspace_bytes(n, n_cams, p) of workspace. */
size_t imloc_rig_workspace_bytes(int64_t n, int32_t n_cams, const imloc_ransac_params *p);
int imloc_rig_lo_ransac_pnp(imloc_ctx *ctx, const imloc_corr *pts, int64_t n, const imloc_rig_camera *cams,
                            int32_t n_cams, const int64_t *cam_start, const imloc_ransac_params *p,
                            imloc_pose *pose_out, uint8_t *mask, imloc_stats *stats);

/* Rig stages for the parity tests, as imloc_sample_p3p and imloc_score:
 * sampling + generalised P3P of `count` samples (up to 8 candidates each, in
 * order of the depth along the first ray, then the second), and scoring of np
 * rig poses.  Workspace: imloc_rig_stage_workspace_bytes(n, n_cams, count)
 * with count = samples or poses. */
size_t imloc_rig_stage_workspace_bytes(int64_t n, int32_t n_cams, int64_t count);
int imloc_rig_sample_gp3p(imloc_ctx *ctx, const imloc_corr *pts, int64_t n, const imloc_rig_camera *cams,
                          int32_t n_cams, const int64_t *cam_start, uint64_t seed, uint64_t query_id,
                          int32_t exhaustive, int64_t h0, int64_t count, double *poses, int64_t *h_out,
                          int32_t *j_out, int32_t *n_cand, int32_t *triples);
int imloc_rig_score(imloc_ctx *ctx, const imloc_corr *pts, int64_t n, const imloc_rig_camera *cams, int32_t n_cams,
                    const int64_t *cam_start, const double *poses, int64_t np, double tau, int32_t precision,
                    int32_t *count, double *msac);

/* Dense matches of a mapping image against n_views covisible views, device
 * arrays [n_views][H][W]: pixel (row, col) of the mapping image matched to
 * (u, v) of view k with confidence conf. */
typedef struct {
  const float *u, *v, *conf;
} imloc_dense_matches;

typedef struct {
  double min_conf;           /* a match is used iff conf >= min_conf (float32 comparison; the paper: 0.05) */
  double angle_deg;          /* a match is an inlier of a depth iff its angular error < angle_deg (2) */
  int32_t min_inliers;       /* the depth is kept iff the winning inlier set has >= min_inliers (4: "more than 3") */
  int32_t max_refine_iters;  /* Newton steps of the refinement, at most (50) */
} imloc_triangulation_params;

/* Mapping-time depth of every pixel by 1-DoF triangulation of dense matches
 * (Sec. 3.3 "Depth Estimation by Dense Matching").  With known poses the
 * pixel's point is X(l) = C0 + l R0^T K0^-1 [col + 0.5, row + 0.5, 1]^T (l =
 * z-depth); a match in view k is the unit ray r_k from its centre C_k, and the
 * angular error of depth l for it is the angle between X(l) - C_k and r_k.
 * Each used match gives one hypothesis, the depth minimising its own angular
 * error (when that minimum lies at a finite l > 0); the hypothesis with the
 * most matches within angle_deg wins (ties: lowest view); its depth is refined
 * by minimising the confidence-weighted sum of squared angular errors over
 * its inliers (a fixed set; Newton's method to a step below 1e-12 l) and kept
 * iff it has at least min_inliers inliers, else the depth is 0.
 *   K_map, T_map: the mapping camera (host); K_views, T_views: host arrays of
 *   n_views (1..32) entries, cam_from_world.  m: device arrays.  Outputs
 *   (device [H][W], each may be NULL): depth (float32 z-depth in metres, 0 =
 *   none), inliers (int32, the winning set's size), codes (uint8 8-bit
 *   log-depth codes of depth, as imloc_depth_encode_log8).  Asynchronous on
 *   the context's stream; needs imloc_triangulate_workspace_bytes(H, W,
 *   n_views) of workspace (16 B per pixel: the queue of pixels to refine).  IMLOC_EINVAL for n_views outside 1..32, H or W < 1, null
 *   inputs or bad intrinsics. */
size_t imloc_triangulate_workspace_bytes(int32_t H, int32_t W, int32_t n_views);
int imloc_triangulate_depth(imloc_ctx *ctx, int32_t H, int32_t W, const imloc_camera *K_map,
                            const imloc_pose *T_map, int32_t n_views, const imloc_camera *K_views,
                            const imloc_pose *T_views, const imloc_dense_matches *m,
                            const imloc_triangulation_params *p, float *depth, int32_t *inliers, uint8_t *codes);

/* LO-RANSAC PnP for one query (Sec. 3.3 "Pose Estimation").  Minimal sample
 * h draws three distinct indices of the scoring set from Philox4x64-10 with
 * key (seed, 0) and counter (h, query_id, attempt, 0), index = floor(word *
 * size / 2^64), redrawn while not distinct (at most 16 attempts).  P3P gives
 * up to four candidates per sample; each is scored against every scored
 * correspondence by sum_i w_i min(r_i^2, tau^2) (points behind the camera
 * count tau^2).  Per batch the lo_top_k lowest-scoring candidates that beat
 * the running best are refined by at most lo_iters Gauss-Newton iterations
 * on that truncated cost (a step that raises the cost, or is shorter than
 * 1e-10 in (rad, scene units), is not taken and ends the run), and the
 * lowest refined cost becomes the best model.  The
 * adaptive rule stops once samples >= min(max_iters, max(min_iters,
 * ceil(ln(1 - confidence) / ln(1 - eps^3)))), eps = best inlier ratio.  The
 * best pose is then refined by at most final_iters Cauchy IRLS iterations
 * (the same two ends) over the inliers of the full set.
 *   pts: device arrays of n entries.  pose_out, stats: host (stats may be
 *   NULL).  inlier_mask: device uint8 [n] (may be NULL): 1 where the point
 *   is an inlier of the final pose.  Returns IMLOC_OK, IMLOC_NO_POSE (n < 3 or
 *   no candidate; pose = identity, mask = 0) or an error. */
int imloc_lo_ransac_pnp(imloc_ctx *ctx, const imloc_corr *pts, int64_t n, const imloc_camera *K_query,
                        const imloc_ransac_params *p, imloc_pose *pose_out, uint8_t *inlier_mask,
                        imloc_stats *stats);

/* imloc_lo_ransac_pnp for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, rules and results, but the device scratch is a fixed
 * array of imloc_noalloc_max_bytes() bytes (32 MiB) inside the library,
 * which every GPU the library runs on holds until the process ends, and the
 * call never captures a graph.  It allocates nothing: no device or host
 * memory, no events, no streams (the context's pinned staging from
 * imloc_create serves the tables).  A query whose scratch would exceed the
 * array returns IMLOC_ENOMEM (imloc_workspace_bytes(n, p) is the size it
 * needs; a 50,000-point query with 10,000 samples per batch needs about
 * 8 MB).  Every call on one GPU shares that GPU's array and leaves its
 * contents behind, so calls that overlap on one GPU (two host threads, or
 * two contexts on different streams) race: serialise them. */
int imloc_lo_ransac_pnp_noalloc(imloc_ctx *ctx, const imloc_corr *pts, int64_t n, const imloc_camera *K_query,
                                const imloc_ransac_params *p, imloc_pose *pose_out, uint8_t *inlier_mask,
                                imloc_stats *stats);
size_t imloc_noalloc_max_bytes(void);

/* The same for nq independent queries in one batched pipeline: the samples,
 * P3P solves, scoring, selection and local optimisation of all queries run in
 * shared launches.  Each query's result equals what imloc_lo_ransac_pnp gives
 * for it alone (same Philox counters, same reduction order).
 *   pts, n, K, params: host arrays of nq entries (params may have 1 entry,
 *   shared).  poses, stats, status: host arrays of nq entries (stats may be
 *   NULL).  masks: host array of nq device pointers (array or entries may be
 *   NULL). */
int imloc_lo_ransac_pnp_batch(imloc_ctx *ctx, const imloc_corr *pts, const int64_t *n, const imloc_camera *K,
                              int32_t nq, const imloc_ransac_params *params, int32_t n_params, imloc_pose *poses,
                              uint8_t *const *masks, imloc_stats *stats, int32_t *status);

/* ---- stages of the path, for inspection and parity checks ---------------- */

/* Draw samples [h0, h0 + count) and solve P3P on each (float64).  Writes the
 * candidates, compacted in an unspecified order: poses (device double
 * [4*count][12]), sample index h_out (device int64 [4*count]), solution index
 * j_out (device int32 [4*count], rank in the canonical order: camera depth of
 * the first sample point ascending, then of the second), n_cand (device
 * int32, the count).  triples (device int32 [count][3], may be NULL) receives
 * each sample's indices, -1 for an empty sample. */
int imloc_sample_p3p(imloc_ctx *ctx, const imloc_corr *pts, int64_t n, const imloc_camera *K, uint64_t seed,
                     uint64_t query_id, int32_t exhaustive, int64_t h0, int64_t count, double *poses,
                     int64_t *h_out, int32_t *j_out, int32_t *n_cand, int32_t *triples);

/* Score np poses (device double [np][12]) against n correspondences: inlier
 * count (device int32 [np]) and truncated cost (device double [np]).
 * precision as in imloc_ransac_params. */
int imloc_score(imloc_ctx *ctx, const imloc_corr *pts, int64_t n, const imloc_camera *K, const double *poses,
                int64_t np, double threshold_px, int32_t precision, int32_t *count, double *msac);

/* The loop's choice of local-optimisation starts (Sec. 3.3 "Pose
 * Estimation": hypotheses that beat the best so far are refined): score np
 * poses (device double [np][12]) as imloc_score does, then take the k (1..32)
 * with the smallest truncated cost below gate (+inf: every pose), ordered by
 * that cost, then the larger inlier count, then the smaller pose index.  sel
 * (device int32 [k]) receives their pose indices in that order, n_sel
 * (device int32) how many there are (fewer than k when fewer poses pass the
 * gate).  Workspace as imloc_score.  IMLOC_EINVAL for k outside [1, 32] or a
 * NaN gate.  Returns once the results are written. */
int imloc_select_top_k(imloc_ctx *ctx, const imloc_corr *pts, int64_t n, const imloc_camera *K, const double *poses,
                       int64_t np, double threshold_px, int32_t precision, int32_t k, double gate, int32_t *sel,
                       int32_t *n_sel);

/* Local optimisation of np start poses (device double [np][12]) on n
 * correspondences: at most iters Gauss-Newton steps each, a run ending at a
 * step that raises the truncated cost or is shorter than 1e-10; out_poses
 * (device double [np][12]), cost (device double [np]), count (device int64
 * [np]). */
int imloc_local_optimize(imloc_ctx *ctx, const imloc_corr *pts, int64_t n, const imloc_camera *K,
                         const double *start, int32_t np, double threshold_px, int32_t iters, double *out_poses,
                         double *cost, int64_t *count);

/* Final Cauchy refinement of one start pose (device double [12]) over the
 * inliers of the n correspondences at that pose, at most iters IRLS steps (a
 * step that raises the cost or is shorter than 1e-10 ends the run); out_pose
 * (device double [12]), cost (device double), mask (device uint8 [n], may be
 * NULL) at the refined pose. */
int imloc_refine(imloc_ctx *ctx, const imloc_corr *pts, int64_t n, const imloc_camera *K, const double *start,
                 double threshold_px, double cauchy_scale_px, int32_t iters, double *out_pose, double *cost,
                 uint8_t *mask);

/* ---- serving: continuous batching ---------------------------------------- */

/* A server keeps up to max_slots queries resident on the device.  Queries are
 * admitted first come first served when a slot is free and their buffers fit
 * the two pools: 4 * batch candidate slots from the candidate pool, and n
 * bytes (plus 24 bytes per point of a subsampled scoring set) from the byte
 * pool.  Every step runs one round (one batch of minimal samples, scoring,
 * selection, local optimisation, stopping rule) for every resident query at
 * once; queries whose stopping rule fires get their final refinement and mask
 * in the same step and leave.  A query's result is the one
 * imloc_lo_ransac_pnp gives for it alone. */
typedef struct imloc_server imloc_server;

typedef struct {
  int32_t max_slots;        /* resident queries at most (<= 4096) */
  int32_t max_top_k;        /* largest lo_top_k accepted (<= 32) */
  int64_t max_n;            /* largest query accepted (correspondences) */
  int64_t candidate_pool;   /* candidate slots shared by the resident queries */
  int64_t byte_pool;        /* bytes shared by the resident queries: a query of n
                             * correspondences takes 1,024 ceil(n / 512) bytes
                             * plus a 256-byte-aligned count table for its
                             * refinement's in-set, and 24 m more for a
                             * gathered scoring subset of m points */
} imloc_server_config;

/* Workspace bytes a server needs; the server uses the context's workspace
 * (imloc_set_workspace) from creation until it is destroyed, and the context
 * serves no other call meanwhile. */
size_t imloc_server_workspace_bytes(const imloc_server_config *cfg);
int imloc_server_create(imloc_ctx *ctx, const imloc_server_config *cfg, imloc_server **out);
void imloc_server_destroy(imloc_server *srv);

/* Queue a query (arguments as for imloc_lo_ransac_pnp; the arrays must stay
 * valid until the query has finished).  *ticket identifies it. */
int imloc_server_submit(imloc_server *srv, const imloc_corr *pts, int64_t n, const imloc_camera *K,
                        const imloc_ransac_params *p, uint8_t *inlier_mask, int64_t *ticket);

/* One step: admit what fits, enqueue one round for every resident query (the
 * queries whose stopping rule fires get their final refinement and mask in
 * that round), then read back the round enqueued by the previous step, if it
 * is still in flight, and retire its finished queries.  While queries wait
 * in the queue the new round is left in flight, to be read back by the next
 * step (a two-deep pipeline: the host's admission and bookkeeping overlap the
 * device's rounds, and a query finished in it is reported one step later);
 * otherwise the step reads the new round back before it returns.  Keep
 * stepping until every ticket is done; a step with nothing resident and
 * nothing in flight does nothing.  done_tickets (host, capacity entries, may
 * be NULL) receives the tickets finished in this step; *n_done their number,
 * *n_resident the queries holding a slot, *n_queued those waiting.  The
 * server's context needs imloc_staging_bytes(2 * max_slots + 2, 0) of
 * staging (two halves); IMLOC_ENOMEM otherwise. */
int imloc_server_step(imloc_server *srv, int64_t *done_tickets, int32_t capacity, int32_t *n_done,
                      int32_t *n_resident, int32_t *n_queued);

/* Result of a finished query (once per ticket): IMLOC_OK or IMLOC_NO_POSE with
 * pose and stats (host) filled, or IMLOC_PENDING. */
int imloc_server_poll(imloc_server *srv, int64_t ticket, imloc_pose *pose, imloc_stats *stats);

/* Pool occupancy: candidate slots and bytes held by resident queries. */
int imloc_server_usage(const imloc_server *srv, int64_t *candidate_slots_used, int64_t *bytes_used);

#ifdef __cplusplus
}
#endif
#endif
