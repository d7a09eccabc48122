// imloc_kernels.h -- device data structures and host-side launchers of the
// HIP kernels (internal to libimloc.so; the public interface is
// include/imloc.h).
//
// Every kernel of the LO-RANSAC path works on a batch of queries described by
// a device-resident table of QueryDesc; a single query is a batch of one, so
// a query's arithmetic is the same alone and in a mix.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace imloc {

// Float32 structure-of-arrays correspondences on the device (w may be null).
struct CorrF32 {
  const float *u, *v, *X, *Y, *Z, *w;
};

struct CamH { double fx, fy, cx, cy; };

constexpr int kMaxTopK = 32;       // local optimisations per query and batch, at most
constexpr int kMaxCams = 8;        // cameras of a rig query, at most
constexpr int kScorePPL32 = 8;     // correspondences per lane, float32 scoring (fixes the summation order)
constexpr int kScoreWaveBlock = 64 * kScorePPL32;  // a wave's 512 consecutive correspondences, float32 scoring
constexpr int kScoreMaxPoints = 4096;  // the largest float32 work item (correspondences)
constexpr int kScoreMaxBlocks = 1 << 18;  // the largest grid picked per round (workgroups)
constexpr int kScorePPL64 = 2;     // correspondences per lane, float64 scoring
constexpr double kGainScale = 4294967296.0;  // fixed-point scale of the accumulated truncated-cost gain

// Per-query running state of one LO-RANSAC, resident on the device.
struct BestState {
  double pose[12];
  double cost;               // truncated cost of the best model (+inf if none)
  int64_t count;             // its inliers on the scoring set
  int64_t h;                 // sample it grew from
  int32_t j;                 // P3P solution index
  int32_t have;              // a best model exists
  int64_t lo_runs;
  int64_t candidates;        // candidates scored so far
  int64_t inlier_residuals;  // inside-threshold residuals seen by scoring
  double weight_sum;         // sum of weights over the scoring set
  double final_cost;
  int64_t full_count;
  int64_t drawn;             // samples drawn so far
  int64_t batches;
  int32_t active;            // still sampling
  int32_t finished;          // 0 sampling, 1 sampling ended (final refinement pending), 2 retired
};

// Device descriptor of one query of a batch.
struct QueryDesc {
  CorrF32 full;          // all correspondences
  CorrF32 S;             // scoring set (the full set, or its stride subsample)
  int64_t n, m;          // sizes of the two
  double fx, fy, cx, cy;
  double tau;            // inlier threshold (px)
  double cauchy_s;       // scale of the final Cauchy loss
  double confidence;
  uint64_t seed, qid;
  int64_t total;         // sample budget: fixed count, or the adaptive cap
  int64_t batch;         // samples per round
  int64_t min_iters;
  int32_t fixed;         // 1: exactly `total` samples
  int32_t exhaustive;
  int32_t precision;     // 0: float32 scoring, 1: float64 scoring
  int32_t k;             // local optimisations per round
  int32_t lo_iters, final_iters;
  int64_t cand_off;      // first candidate slot of this query
  int64_t cap;           // candidate slots (4 per sample of a round)
  int64_t in_set_off;    // offset of this query's bytes in the in-set array
  int64_t B;             // samples of the current round (0: inactive)
  uint8_t* mask;         // inlier mask output (device) or null
  int32_t fresh;         // 1: admitted with this table upload (initialise, gather its subset)
  int32_t ncam;          // 0: one camera (fx, fy, cx, cy; poses cam_from_world); 1..kMaxCams: a rig
  const double* rig;     // rig cameras (device) [ncam][16]: fx, fy, cx, cy, cam_from_rig R (9), t (3)
  int64_t proj_off;      // first float of this query's projection rows: 16 per camera per candidate slot
  int64_t segS[kMaxCams + 1];  // rig: camera c owns scoring-set points [segS[c], segS[c + 1])
  int64_t segF[kMaxCams + 1];  // rig: camera c owns full-set points [segF[c], segF[c + 1])
};

// Camera of point i of a rig query (segments seg[0..ncam]); 0 for one camera.
__host__ __device__ inline int cam_of(const int64_t* seg, int ncam, int64_t i) {
  int c = 0;
  while (c + 1 < ncam && i >= seg[c + 1]) ++c;
  return c;
}

// Rows per candidate slot: one set of 16 floats per camera.
__host__ __device__ inline int rows_per_slot(const QueryDesc& d) { return d.ncam > 0 ? d.ncam : 1; }

// Candidate arrays of all queries of a batch (device), indexed by slot.
struct CandBuf {
  double* pose;      // [slots][12]
  float* proj;       // per query from proj_off: [slots][cameras][16] float32 rows of K [R | t] (rig: of
                     // K_c [R_c R | R_c t + t_c]), rows a and b divided by tau (12 used)
  int64_t* h;        // [slots] sample index
  int32_t* j;        // [slots] solution index
  uint32_t* cnt;     // [slots] inlier count (accumulated by scoring)
  uint64_t* gain;    // [slots] sum of w (1 - r^2 / tau^2) over inliers, fixed point 2^-32 (accumulated)
  int32_t* n;        // [queries] candidates of the current round
  int32_t* sel_done; // [queries] selection workgroups finished (zeroed by the work-list kernel)
};

// --- lift ------------------------------------------------------------------
struct LiftArgs {
  const float *q_u, *q_v, *db_u, *db_v, *conf;
  const int32_t* view;
  int64_t n;
  const float* depth;     // float32 maps, or
  const uint8_t* codes;   // 8-bit log-depth code maps (exactly one is set)
  int32_t n_views, H, W;
  const double* cams;   // device [n_views][4]
  const double* poses;  // device [n_views][12]
  int32_t subpixel;
  float min_conf;
  float *out_u, *out_v, *out_X, *out_Y, *out_Z, *out_w;
  int32_t* out_src;
  int64_t capacity;
  int32_t* n_out;
  int32_t* block_counts;  // scratch [blocks]
};
int lift_blocks(int64_t n);
hipError_t launch_lift(const LiftArgs& a, hipStream_t s);
// 8-bit log-depth codes of n float32 depths (depth and codes 16- and 4-byte aligned)
hipError_t launch_log8_encode(const float* depth, int64_t n, uint8_t* codes, hipStream_t s);

// --- mapping-time depth by 1-DoF triangulation ------------------------------
// a pixel whose depth is refined: its winning hypothesis and inlier set
struct TriTask {
  double l;
  int32_t p;
  uint32_t set;
};
struct TriArgs {
  int32_t H, W, V;               // mapping image size, covisible views (<= 32)
  const double* views;           // device [V + 1][16]: fx, fy, cx, cy, R^T (9), C0 - Ck (3); entry 0 = mapping camera
  const float *mu, *mv, *conf;   // device [V][H][W]
  float min_conf;
  double cos2_thr;               // cos^2 of the angular threshold
  int32_t min_inliers, max_iters;
  float* depth;                  // device [H][W] or null
  int32_t* inliers;              // device [H][W] or null
  uint8_t* codes;                // device [H][W] 8-bit log-depth codes, or null
  int32_t* n_tasks;              // device scratch: length of the refinement queue
  TriTask* tasks;                // device scratch [H * W]: the pixels to refine
};
hipError_t launch_triangulate(const TriArgs& a, hipStream_t s);

// --- small utilities ---------------------------------------------------------
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t s);
hipError_t launch_gather_subset(const CorrF32& c, int64_t n, int64_t m, float* dst /*[6][m]*/, hipStream_t s);
// stride subsets of every query whose scoring set is not its full set (the
// table says from where to where); max_m bounds the subset sizes
hipError_t launch_gather_subsets(const QueryDesc* qd, int nq, int64_t max_m, hipStream_t s);

// --- round bookkeeping ---------------------------------------------------------
// init: state and the weight sum of the scoring set of every fresh query.
// begin: also set up the first round (every query of the table is fresh)
hipError_t launch_init_queries(QueryDesc* qd, BestState* st, int32_t* n_cand, int nq, bool begin, hipStream_t s);
// finished queries (final refinement and mask done) leave the round loop
hipError_t launch_retire(BestState* st, int nq, hipStream_t s);
// begin: samples of this round per query, zero candidate counts.
hipError_t launch_begin_round(QueryDesc* qd, const BestState* st, CandBuf cb, int nq, hipStream_t s);
// end: take the round's local optimisations into the running best, advance
// the sample count, apply the stopping rule, and (begin_next) set up the next
// round; *active_count receives the number of queries that keep sampling.
hipError_t launch_round_end(QueryDesc* qd, CandBuf cb, const int32_t* sel, const int32_t* n_sel,
                            const double* lo_pose, const double* lo_cost, const int64_t* lo_count, int nq, int kmax,
                            BestState* st, int32_t* active_count, bool begin_next, hipStream_t s);

// --- sampling + P3P ----------------------------------------------------------
// Samples [drawn, drawn + B) of every query; max_b bounds B.
hipError_t launch_sample_p3p(const QueryDesc* qd, const BestState* st, CandBuf cb, int nq, int64_t max_b,
                             int32_t* triples, hipStream_t s);
// Rig queries of the batch (the one-camera ones are skipped): generalised P3P,
// up to 8 candidates per sample.
hipError_t launch_sample_gp3p(const QueryDesc* qd, const BestState* st, CandBuf cb, int nq, int64_t max_b,
                              int32_t* triples, hipStream_t s);
// Candidates from given float64 poses (query 0): projection rows, zeroed accumulators.
hipError_t launch_set_candidates(const QueryDesc* qd, const double* poses, int64_t np, CandBuf cb, hipStream_t s);

// --- scoring -----------------------------------------------------------------
struct ScoreTune {
  int ct;       // candidates per work item (32, 64 or 128)
  int blocks;   // workgroups of the launch (each strides over the work list)
  int pts;      // correspondences per float32 work item (512, 1024, 2048 or 4096)
};
hipError_t launch_worklist(const QueryDesc* qd, CandBuf cb, int nq, ScoreTune tune, int64_t* item_off,
                           hipStream_t s);
hipError_t launch_score(const QueryDesc* qd, CandBuf cb, BestState* st, int nq, const int64_t* item_off,
                        ScoreTune tune, int precision, hipStream_t s);
// truncated cost of the candidates of query 0: count and msac outputs
hipError_t launch_candidate_costs(const QueryDesc* qd, const BestState* st, CandBuf cb, int64_t np, int32_t* count,
                                  double* msac, hipStream_t s);

// --- selection / local optimisation / refinement ------------------------------
// scratch: select_scratch_bytes(nq); max_cap bounds the queries' candidate slots
size_t select_scratch_bytes(int nq);
hipError_t launch_select(const QueryDesc* qd, const BestState* st, CandBuf cb, int nq, int kmax, int64_t max_cap,
                         void* scratch, int32_t* sel, int32_t* n_sel, hipStream_t s);

// Gauss-Newton problems.  LO: problem p = q * kmax + slot starts from the
// candidate sel[q * kMaxTopK + slot] (or from start_direct[p] when given, all
// on query 0) and runs on the scoring set of its query.  Refine: problem q
// starts from the best pose of query q (or start_direct[q]) and runs on its
// full set, if the query has just finished sampling.
int gn_chunks(int64_t n);
// bytes of the final refinement's compacted in-set of a query of n points
int64_t gn_inset_bytes(int64_t n);
size_t gn_scratch_bytes(int nprob, int chunks_max);
// any_rig: some problem belongs to a rig query (selects the kernel variant
// that takes residuals through rig cameras).  gn_mode: 0 = pick the launch
// form by size, 1 = fused (one launch per iteration), 2 = split (evaluation
// and decision launches); every form gives identical results.
hipError_t launch_lo(const QueryDesc* qd, CandBuf cb, const int32_t* sel, const int32_t* n_sel,
                     const double* start_direct, int nprob, int kmax, int chunks_max, int iters_max, void* scratch,
                     double* out_pose, double* out_cost, int64_t* out_count, bool any_rig, bool any_weighted,
                     int gn_mode, hipStream_t s);
hipError_t launch_refine(const QueryDesc* qd, BestState* st, const double* start_direct, int nq, int chunks_max,
                         int iters_max, uint8_t* in_set, void* scratch, double* out_pose, double* out_cost,
                         bool any_rig, int gn_mode, bool fuse_mask, bool* mask_done, hipStream_t s);
// mask and inlier count of the final pose of every query that just finished
// (all != 0: of every query, each with a pose)
hipError_t launch_mask(const QueryDesc* qd, BestState* st, const double* fin_pose, int nq, int64_t max_n, int all,
                       hipStream_t s);

}  // namespace imloc
