// imloc_kernels.h -- host-side launchers of the HIP kernels (internal to
// libimloc.so; the public interface is include/imloc.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace imloc {

// Float32 structure-of-arrays correspondences on the device (w may be null).
struct CorrF32 {
  const float *u, *v, *X, *Y, *Z, *w;
};

struct CamH { double fx, fy, cx, cy; };

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
};

// Candidate arrays of one batch (device).
struct CandBuf {
  double* pose;     // [cap][12]
  float* proj;      // [cap][16] float32 rows of K [R | t], rows a and b divided by tau (12 used)
  int64_t* h;       // [cap]
  int32_t* j;       // [cap]
  int32_t* n;       // device count
  int32_t* count;   // [cap] inliers after reduction
  double* msac;     // [cap]
  int64_t cap;
};

// --- lift ------------------------------------------------------------------
struct LiftArgs {
  const float *q_u, *q_v, *db_u, *db_v, *conf;
  const int32_t* view;
  int64_t n;
  const float* depth;
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

// --- sampling + P3P ----------------------------------------------------------
hipError_t launch_sample_p3p(const CorrF32& c, int64_t m, CamH K, uint64_t seed, uint64_t query, int exhaustive,
                             int64_t h0, int64_t count, double tau, const CandBuf& cb, int32_t* triples,
                             hipStream_t s);
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t s);

// Float32 projection rows (rows a, b divided by tau) from float64 poses.
hipError_t launch_make_proj(const double* poses, int64_t np, CamH K, double tau, float* proj, hipStream_t s);

// --- scoring -----------------------------------------------------------------
struct ScorePlan {
  int ppl;        // points per lane
  int ct;         // candidates per tile
  int chunks;     // point chunks (blocks along x)
  int tiles;      // candidate tiles (blocks along y)
  int64_t cap;    // candidate capacity (row stride of the partial arrays)
};
ScorePlan plan_score(int64_t m, int64_t cand_cap, int precision);
size_t score_partial_bytes(const ScorePlan& p);
hipError_t launch_score(const CorrF32& c, int64_t m, CamH K, double tau, int precision, const ScorePlan& plan,
                        const CandBuf& cb, uint32_t* part_cnt, float* part_gain, double* part_gain64,
                        hipStream_t s);
// sums the partials of each candidate in chunk order; msac = tau^2 (C - sum gain)
hipError_t launch_reduce_scores(const ScorePlan& plan, const CandBuf& cb, double tau, const uint32_t* part_cnt,
                                const float* part_gain, const double* part_gain64, int precision, BestState* st,
                                hipStream_t s);
hipError_t launch_weight_sum(const CorrF32& c, int64_t m, BestState* st, hipStream_t s);
hipError_t launch_gather_subset(const CorrF32& c, int64_t n, int64_t m, float* dst /*[6][m]*/, hipStream_t s);

// --- selection / local optimisation / refinement ------------------------------
hipError_t launch_select(const CandBuf& cb, int32_t k, const BestState* st, int32_t* sel, int32_t* n_sel,
                         hipStream_t s);
hipError_t launch_lo(const CorrF32& c, int64_t m, CamH K, double tau, int32_t iters, const double* cand_pose,
                     const int32_t* sel, const int32_t* n_sel, int32_t k, double* out_pose, double* out_cost,
                     int64_t* out_count, hipStream_t s);
hipError_t launch_update_best(const CandBuf& cb, const int32_t* sel, const int32_t* n_sel, const double* lo_pose,
                              const double* lo_cost, const int64_t* lo_count, BestState* st, hipStream_t s);
hipError_t launch_refine(const CorrF32& c, int64_t n, CamH K, double tau, double scale, int32_t iters,
                         const double* start, uint8_t* in_set, double* out_pose, double* out_cost, hipStream_t s);
hipError_t launch_mask(const CorrF32& c, int64_t n, CamH K, double tau, const double* pose, uint8_t* mask,
                       int64_t* count, hipStream_t s);
hipError_t launch_init_state(BestState* st, hipStream_t s);

}  // namespace imloc
