// runtime.cpp -- the C ABI of libimloc.so (include/imloc.h): context,
// workspace carving, argument checks and the orchestration of the kernels of
// the pose-estimation path (ImLoc Sec. 3.3).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "imloc.h"
#include "imloc_kernels.h"

using namespace imloc;

struct imloc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool timing = false;
  std::string err;
  void* pinned = nullptr;  // host staging for small device->host reads
  size_t pinned_bytes = 0;
  std::vector<hipEvent_t> events;
  size_t next_event = 0;
};

namespace {

constexpr int kMaxTopK = 32;

int set_err(imloc_ctx* c, int code, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return code;
}

#define HIP_TRY(ctx, expr)                                                                     \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) return set_err(ctx, IMLOC_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// Bump allocator over the caller's workspace.
struct Arena {
  char* base;
  size_t size;
  size_t off = 0;
  bool ok = true;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(base ? base + off : nullptr);
    off += count * sizeof(T);
    if (off > size) ok = false;
    return p;
  }
};

bool cam_ok(const imloc_camera* K) {
  return K && std::isfinite(K->fx) && std::isfinite(K->fy) && std::isfinite(K->cx) && std::isfinite(K->cy) &&
         K->fx > 0.0 && K->fy > 0.0;
}

bool corr_ok(const imloc_corr* p) { return p && p->u && p->v && p->X && p->Y && p->Z; }

CorrF32 to_corr(const imloc_corr* p) { return CorrF32{p->u, p->v, p->X, p->Y, p->Z, p->w}; }
CamH to_cam(const imloc_camera* K) { return CamH{K->fx, K->fy, K->cx, K->cy}; }

// Sizes derived from the parameters of one query.
struct QueryShape {
  int64_t n, m;        // correspondences, scoring-set size
  bool subset;
  int64_t total;       // samples to draw at most
  int64_t batch;       // samples per batch
  int64_t cap;         // candidate capacity per batch
  int32_t k;           // top-k refined per batch
  ScorePlan plan;
};

QueryShape shape_of(int64_t n, const imloc_ransac_params* p) {
  QueryShape s;
  s.n = n;
  s.subset = p->max_score_points > 0 && n > p->max_score_points;
  s.m = s.subset ? p->max_score_points : n;
  s.total = p->fixed_samples > 0 ? p->fixed_samples : p->max_iters;
  s.batch = p->batch > 0 ? p->batch : 1024;
  if (s.batch > s.total) s.batch = s.total;
  if (s.batch < 1) s.batch = 1;
  s.cap = 4 * s.batch;
  s.k = p->lo_top_k < 1 ? 1 : (p->lo_top_k > kMaxTopK ? kMaxTopK : p->lo_top_k);
  s.plan = plan_score(s.m, s.cap, p->precision);
  return s;
}

// Device buffers of one single-query run, carved from the workspace.
struct QueryBufs {
  float* subset;
  BestState* st;
  CandBuf cb;
  uint32_t* part_cnt;
  double* part_gain;
  int32_t* sel;
  int32_t* n_sel;
  double* lo_pose;
  double* lo_cost;
  int64_t* lo_count;
  double* fin_pose;
  double* fin_cost;
  uint8_t* in_set;
};

QueryBufs carve(Arena& a, const QueryShape& s) {
  QueryBufs b;
  b.subset = s.subset ? a.take<float>(6 * (size_t)s.m) : nullptr;
  b.st = a.take<BestState>(1);
  b.cb.cap = s.cap;
  b.cb.pose = a.take<double>(12 * (size_t)s.cap);
  b.cb.proj = a.take<float>(16 * (size_t)s.cap);
  b.cb.h = a.take<int64_t>((size_t)s.cap);
  b.cb.j = a.take<int32_t>((size_t)s.cap);
  b.cb.n = a.take<int32_t>(1);
  b.cb.count = a.take<int32_t>((size_t)s.cap);
  b.cb.msac = a.take<double>((size_t)s.cap);
  b.part_cnt = a.take<uint32_t>((size_t)s.plan.chunks * (size_t)s.cap);
  b.part_gain = a.take<double>((size_t)s.plan.chunks * (size_t)s.cap);
  b.sel = a.take<int32_t>(kMaxTopK);
  b.n_sel = a.take<int32_t>(1);
  b.lo_pose = a.take<double>(12 * kMaxTopK);
  b.lo_cost = a.take<double>(kMaxTopK);
  b.lo_count = a.take<int64_t>(kMaxTopK);
  b.fin_pose = a.take<double>(12);
  b.fin_cost = a.take<double>(1);
  b.in_set = a.take<uint8_t>((size_t)(s.n > 0 ? s.n : 1));
  return b;
}

int check_params(imloc_ctx* ctx, const imloc_ransac_params* p) {
  if (!p) return set_err(ctx, IMLOC_EINVAL, "params is null");
  if (!(p->threshold_px > 0.0) || !std::isfinite(p->threshold_px))
    return set_err(ctx, IMLOC_EINVAL, "threshold_px must be finite and > 0");
  if (p->fixed_samples <= 0 && (p->max_iters <= 0 || !(p->confidence > 0.0 && p->confidence < 1.0)))
    return set_err(ctx, IMLOC_EINVAL, "adaptive mode needs max_iters > 0 and 0 < confidence < 1");
  if (p->precision != IMLOC_FP32_SCORE && p->precision != IMLOC_FP64_ALL)
    return set_err(ctx, IMLOC_EINVAL, "unknown precision %d", p->precision);
  if (p->final_iters > 0 && !(p->cauchy_scale_px > 0.0)) return set_err(ctx, IMLOC_EINVAL, "cauchy_scale_px must be > 0");
  if (p->lo_iters < 0 || p->final_iters < 0) return set_err(ctx, IMLOC_EINVAL, "negative iteration count");
  if (p->max_score_points < 0) return set_err(ctx, IMLOC_EINVAL, "max_score_points < 0");
  if (p->max_score_points > 0 && p->max_score_points < 3) return set_err(ctx, IMLOC_EINVAL, "max_score_points < 3");
  return IMLOC_OK;
}

// Stopping rule: samples needed for inlier ratio eps (minimal size 3).
int64_t required_samples(double eps, double conf, int64_t max_iters) {
  if (!(eps > 0.0)) return max_iters;
  if (eps >= 1.0) return 0;
  const double denom = std::log1p(-eps * eps * eps);
  if (!(denom < 0.0)) return max_iters;
  const double k = std::ceil(std::log(1.0 - conf) / denom);
  if (!(k < (double)max_iters)) return max_iters;
  if (k < 0.0) return 0;
  return (int64_t)k;
}

hipEvent_t take_event(imloc_ctx* c) {
  if (c->next_event == c->events.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->events.push_back(e);
  }
  return c->events[c->next_event++];
}

// Per-stage timing with HIP events on the context stream.
struct Timer {
  imloc_ctx* c;
  struct Span { int stage; hipEvent_t a, b; };
  std::vector<Span> spans;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  explicit Timer(imloc_ctx* cc) : c(cc) { c->next_event = 0; }
  hipEvent_t begin() {
    if (!c->timing) return nullptr;
    hipEvent_t e = take_event(c);
    if (e) hipEventRecord(e, c->stream);
    return e;
  }
  void end(int stage, hipEvent_t a) {
    if (!c->timing || !a) return;
    hipEvent_t e = take_event(c);
    if (!e) return;
    hipEventRecord(e, c->stream);
    spans.push_back({stage, a, e});
  }
  void fill(imloc_stats* st) {
    if (!c->timing || !st) return;
    float acc[6] = {0, 0, 0, 0, 0, 0};
    for (auto& s : spans) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, s.a, s.b) == hipSuccess) acc[s.stage] += ms;
    }
    st->ms_sample = acc[0]; st->ms_score = acc[1]; st->ms_select = acc[2];
    st->ms_lo = acc[3]; st->ms_refine = acc[4]; st->ms_total = acc[5];
  }
};
enum { kStSample = 0, kStScore = 1, kStSelect = 2, kStLO = 3, kStRefine = 4, kStTotal = 5 };

void identity_pose(imloc_pose* p) {
  for (int e = 0; e < 9; ++e) p->R[e] = (e % 4 == 0) ? 1.0 : 0.0;
  p->t[0] = p->t[1] = p->t[2] = 0.0;
}

}  // namespace

extern "C" {

int imloc_create(imloc_ctx** out, int device, void* hip_stream) {
  if (!out) return IMLOC_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return IMLOC_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return IMLOC_EHIP;
  imloc_ctx* c = new imloc_ctx();
  c->device = device;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  c->pinned_bytes = 4096;
  if (hipHostMalloc(&c->pinned, c->pinned_bytes, hipHostMallocDefault) != hipSuccess) {
    delete c;
    return IMLOC_EHIP;
  }
  *out = c;
  return IMLOC_OK;
}

void imloc_destroy(imloc_ctx* c) {
  if (!c) return;
  hipSetDevice(c->device);
  hipStreamSynchronize(c->stream);
  for (auto e : c->events) hipEventDestroy(e);
  if (c->pinned) hipHostFree(c->pinned);
  delete c;
}

int imloc_set_stream(imloc_ctx* c, void* s) {
  if (!c) return IMLOC_EINVAL;
  c->stream = reinterpret_cast<hipStream_t>(s);
  return IMLOC_OK;
}

const char* imloc_last_error(const imloc_ctx* c) { return c ? c->err.c_str() : "null context"; }

int imloc_set_workspace(imloc_ctx* c, void* p, size_t bytes) {
  if (!c) return IMLOC_EINVAL;
  if (!p && bytes) return set_err(c, IMLOC_EINVAL, "workspace pointer is null");
  c->ws = reinterpret_cast<char*>(p);
  c->ws_bytes = bytes;
  return IMLOC_OK;
}

int imloc_set_timing(imloc_ctx* c, int enable) {
  if (!c) return IMLOC_EINVAL;
  c->timing = enable != 0;
  return IMLOC_OK;
}

size_t imloc_workspace_bytes(int64_t n, const imloc_ransac_params* p) {
  if (!p || n < 0) return 0;
  QueryShape s = shape_of(n, p);
  Arena a{nullptr, (size_t)-1};
  carve(a, s);
  return a.off + 256;
}

size_t imloc_score_workspace_bytes(int64_t n, int64_t np, int32_t precision) {
  if (n < 0 || np < 0) return 0;
  Arena a{nullptr, (size_t)-1};
  ScorePlan pl = plan_score(n, np > 0 ? np : 1, precision);
  a.take<BestState>(1);
  a.take<float>(16 * (size_t)(np > 0 ? np : 1));
  a.take<int32_t>(1);
  a.take<uint32_t>((size_t)pl.chunks * (size_t)pl.cap);
  a.take<double>((size_t)pl.chunks * (size_t)pl.cap);
  return a.off + 256;
}

size_t imloc_lift_workspace_bytes(int64_t n_matches, int32_t n_views) {
  if (n_matches < 0 || n_views < 0) return 0;
  Arena a{nullptr, (size_t)-1};
  const int nb = lift_blocks(n_matches);
  a.take<double>(4 * (size_t)(n_views > 0 ? n_views : 1));
  a.take<double>(12 * (size_t)(n_views > 0 ? n_views : 1));
  a.take<int32_t>((size_t)(nb > 0 ? nb : 1));
  return a.off + 256;
}

int imloc_lift(imloc_ctx* ctx, const imloc_matches* m, int64_t n_matches, const float* depth, int32_t n_views,
               int32_t H, int32_t W, const imloc_camera* cams, const imloc_pose* poses, int32_t subpixel,
               float min_conf, const imloc_corr_out* out, int64_t capacity, int32_t* n_out) {
  if (!ctx) return IMLOC_EINVAL;
  if (n_matches < 0 || n_matches > INT32_MAX) return set_err(ctx, IMLOC_EINVAL, "n_matches out of range");
  if (!n_out || !out) return set_err(ctx, IMLOC_EINVAL, "null output");
  if (n_matches > 0) {
    if (!m || !m->q_u || !m->q_v || !m->db_u || !m->db_v || !m->conf || !m->view)
      return set_err(ctx, IMLOC_EINVAL, "null match array");
    if (!depth || n_views <= 0 || H < 2 || W < 2 || !cams || !poses)
      return set_err(ctx, IMLOC_EINVAL, "bad depth maps / views");
    if (capacity < 0 || (capacity > 0 && (!out->u || !out->v || !out->X || !out->Y || !out->Z)))
      return set_err(ctx, IMLOC_EINVAL, "bad output arrays");
    for (int k = 0; k < n_views; ++k)
      if (!cam_ok(&cams[k])) return set_err(ctx, IMLOC_EINVAL, "view %d: bad intrinsics", k);
  }
  hipSetDevice(ctx->device);
  Arena a{ctx->ws, ctx->ws_bytes};
  const int nb = lift_blocks(n_matches);
  double* dcams = a.take<double>(4 * (size_t)(n_views > 0 ? n_views : 1));
  double* dposes = a.take<double>(12 * (size_t)(n_views > 0 ? n_views : 1));
  int32_t* blk = a.take<int32_t>((size_t)(nb > 0 ? nb : 1));
  if (!a.ok) return set_err(ctx, IMLOC_ENOMEM, "workspace too small for lift: need %zu bytes", a.off);
  if (n_matches > 0) {
    std::vector<double> hc(4 * (size_t)n_views), hp(12 * (size_t)n_views);
    for (int k = 0; k < n_views; ++k) {
      hc[4 * k] = cams[k].fx; hc[4 * k + 1] = cams[k].fy; hc[4 * k + 2] = cams[k].cx; hc[4 * k + 3] = cams[k].cy;
      for (int e = 0; e < 9; ++e) hp[12 * k + e] = poses[k].R[e];
      for (int e = 0; e < 3; ++e) hp[12 * k + 9 + e] = poses[k].t[e];
    }
    // synchronous copies: the host vectors die at return
    HIP_TRY(ctx, hipMemcpyAsync(dcams, hc.data(), hc.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(dposes, hp.data(), hp.size() * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  }
  LiftArgs la;
  la.q_u = m ? m->q_u : nullptr; la.q_v = m ? m->q_v : nullptr; la.db_u = m ? m->db_u : nullptr;
  la.db_v = m ? m->db_v : nullptr; la.conf = m ? m->conf : nullptr; la.view = m ? m->view : nullptr;
  la.n = n_matches; la.depth = depth; la.n_views = n_views; la.H = H; la.W = W;
  la.cams = dcams; la.poses = dposes; la.subpixel = subpixel; la.min_conf = min_conf;
  la.out_u = out->u; la.out_v = out->v; la.out_X = out->X; la.out_Y = out->Y; la.out_Z = out->Z;
  la.out_w = out->w; la.out_src = out->src; la.capacity = capacity; la.n_out = n_out; la.block_counts = blk;
  HIP_TRY(ctx, launch_lift(la, ctx->stream));
  return IMLOC_OK;
}

int imloc_lo_ransac_pnp(imloc_ctx* ctx, const imloc_corr* pts, int64_t n, const imloc_camera* K,
                        const imloc_ransac_params* p, imloc_pose* pose_out, uint8_t* mask, imloc_stats* stats) {
  if (!ctx) return IMLOC_EINVAL;
  int rc = check_params(ctx, p);
  if (rc) return rc;
  if (!pose_out) return set_err(ctx, IMLOC_EINVAL, "pose_out is null");
  if (n < 0 || n > INT32_MAX) return set_err(ctx, IMLOC_EINVAL, "n out of range");
  if (n > 0 && !corr_ok(pts)) return set_err(ctx, IMLOC_EINVAL, "null correspondence array");
  if (!cam_ok(K)) return set_err(ctx, IMLOC_EINVAL, "bad query intrinsics");
  hipSetDevice(ctx->device);
  hipStream_t s = ctx->stream;
  const QueryShape sh = shape_of(n, p);
  Arena a{ctx->ws, ctx->ws_bytes};
  QueryBufs b = carve(a, sh);
  if (!a.ok) return set_err(ctx, IMLOC_ENOMEM, "workspace too small: need %zu bytes, have %zu", a.off, ctx->ws_bytes);
  if (stats) std::memset(stats, 0, sizeof(*stats));
  identity_pose(pose_out);

  Timer tm(ctx);
  hipEvent_t ev_total = tm.begin();
  const CamH cam = to_cam(K);
  const CorrF32 full = n > 0 ? to_corr(pts) : CorrF32{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  CorrF32 S = full;
  if (sh.subset) {
    HIP_TRY(ctx, launch_gather_subset(full, n, sh.m, b.subset, s));
    const int64_t m = sh.m;
    S = CorrF32{b.subset, b.subset + m, b.subset + 2 * m, b.subset + 3 * m, b.subset + 4 * m, b.subset + 5 * m};
  }
  HIP_TRY(ctx, launch_init_state(b.st, s));
  HIP_TRY(ctx, launch_weight_sum(S, sh.m, b.st, s));

  BestState* hst = reinterpret_cast<BestState*>(ctx->pinned);
  int64_t drawn = 0, batches = 0;
  int32_t score_launches = 0;
  while (sh.m >= 3 && drawn < sh.total) {
    const int64_t B = std::min(sh.batch, sh.total - drawn);
    hipEvent_t e0 = tm.begin();
    HIP_TRY(ctx, launch_fill_i32(b.cb.n, 1, 0, s));
    HIP_TRY(ctx, launch_sample_p3p(S, sh.m, cam, p->seed, p->query_id, p->exhaustive, drawn, B, p->threshold_px,
                                   b.cb, nullptr, s));
    tm.end(kStSample, e0);
    hipEvent_t e1 = tm.begin();
    HIP_TRY(ctx, launch_score(S, sh.m, cam, p->threshold_px, p->precision, sh.plan, b.cb, b.part_cnt,
                              reinterpret_cast<float*>(b.part_gain), b.part_gain, s));
    ++score_launches;
    tm.end(kStScore, e1);
    hipEvent_t e2 = tm.begin();
    HIP_TRY(ctx, launch_reduce_scores(sh.plan, b.cb, p->threshold_px, b.part_cnt, reinterpret_cast<float*>(b.part_gain),
                                      b.part_gain, p->precision, b.st, s));
    HIP_TRY(ctx, launch_select(b.cb, sh.k, b.st, b.sel, b.n_sel, s));
    tm.end(kStSelect, e2);
    hipEvent_t e3 = tm.begin();
    if (sh.k > 0) {
      HIP_TRY(ctx, launch_lo(S, sh.m, cam, p->threshold_px, p->lo_iters, b.cb.pose, b.sel, b.n_sel, sh.k, b.lo_pose,
                             b.lo_cost, b.lo_count, s));
      HIP_TRY(ctx, launch_update_best(b.cb, b.sel, b.n_sel, b.lo_pose, b.lo_cost, b.lo_count, b.st, s));
    }
    tm.end(kStLO, e3);
    drawn += B;
    ++batches;
    if (p->fixed_samples <= 0) {
      HIP_TRY(ctx, hipMemcpyAsync(hst, b.st, sizeof(BestState), hipMemcpyDeviceToHost, s));
      HIP_TRY(ctx, hipStreamSynchronize(s));
      const double eps = (double)hst->count / (double)sh.m;
      int64_t need = required_samples(eps, p->confidence, p->max_iters);
      if (need < p->min_iters) need = p->min_iters;
      if (need > p->max_iters) need = p->max_iters;
      if (drawn >= need) break;
    }
  }
  HIP_TRY(ctx, hipMemcpyAsync(hst, b.st, sizeof(BestState), hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  const bool have = hst->have != 0;
  int status = have ? IMLOC_OK : IMLOC_NO_POSE;
  if (have) {
    hipEvent_t e4 = tm.begin();
    HIP_TRY(ctx, launch_refine(full, n, cam, p->threshold_px, p->cauchy_scale_px > 0 ? p->cauchy_scale_px : 1.0,
                               p->final_iters, b.st->pose, b.in_set, b.fin_pose, b.fin_cost, s));
    HIP_TRY(ctx, launch_mask(full, n, cam, p->threshold_px, b.fin_pose, mask, &b.st->full_count, s));
    tm.end(kStRefine, e4);
  } else if (mask && n > 0) {
    HIP_TRY(ctx, launch_fill_u8(mask, n, 0, s));
  }
  tm.end(kStTotal, ev_total);
  double* hpose = reinterpret_cast<double*>(reinterpret_cast<char*>(ctx->pinned) + 1024);
  HIP_TRY(ctx, hipMemcpyAsync(hst, b.st, sizeof(BestState), hipMemcpyDeviceToHost, s));
  if (have) {
    HIP_TRY(ctx, hipMemcpyAsync(hpose, b.fin_pose, 12 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipMemcpyAsync(hpose + 12, b.fin_cost, sizeof(double), hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(ctx, hipStreamSynchronize(s));
  if (have) {
    for (int e = 0; e < 9; ++e) pose_out->R[e] = hpose[e];
    for (int e = 0; e < 3; ++e) pose_out->t[e] = hpose[9 + e];
  }
  if (stats) {
    stats->samples = drawn;
    stats->candidates = hst->candidates;
    stats->residuals = hst->candidates * sh.m;
    stats->inlier_residuals = hst->inlier_residuals;
    stats->best_count = have ? hst->count : 0;
    stats->full_count = have ? hst->full_count : 0;
    stats->batches = batches;
    stats->lo_runs = (int32_t)hst->lo_runs;
    stats->status = status;
    stats->best_msac = have ? hst->cost : 0.0;
    stats->final_cost = have ? hpose[12] : 0.0;
    stats->best_h = have ? hst->h : -1;
    stats->best_j = have ? hst->j : -1;
    stats->score_launches = score_launches;
    tm.fill(stats);
  }
  return status;
}

int imloc_sample_p3p(imloc_ctx* ctx, const imloc_corr* pts, int64_t n, const imloc_camera* K, uint64_t seed,
                     uint64_t query_id, int32_t exhaustive, int64_t h0, int64_t count, double* poses, int64_t* h_out,
                     int32_t* j_out, int32_t* n_cand, int32_t* triples) {
  if (!ctx) return IMLOC_EINVAL;
  if (n < 0 || n > INT32_MAX || count < 0 || h0 < 0) return set_err(ctx, IMLOC_EINVAL, "bad sizes");
  if (n > 0 && !corr_ok(pts)) return set_err(ctx, IMLOC_EINVAL, "null correspondence array");
  if (!cam_ok(K)) return set_err(ctx, IMLOC_EINVAL, "bad intrinsics");
  if (!poses || !h_out || !j_out || !n_cand) return set_err(ctx, IMLOC_EINVAL, "null output");
  hipSetDevice(ctx->device);
  Arena a{ctx->ws, ctx->ws_bytes};
  float* proj = a.take<float>(16 * (size_t)(4 * count > 0 ? 4 * count : 1));
  if (!a.ok) return set_err(ctx, IMLOC_ENOMEM, "workspace too small: need %zu bytes", a.off);
  CandBuf cb;
  cb.pose = poses; cb.proj = proj; cb.h = h_out; cb.j = j_out; cb.n = n_cand; cb.count = nullptr; cb.msac = nullptr;
  cb.cap = 4 * count;
  HIP_TRY(ctx, launch_fill_i32(n_cand, 1, 0, ctx->stream));
  const CorrF32 c = n > 0 ? to_corr(pts) : CorrF32{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  HIP_TRY(ctx, launch_sample_p3p(c, n, to_cam(K), seed, query_id, exhaustive, h0, count, 1.0, cb, triples, ctx->stream));
  return IMLOC_OK;
}

int imloc_score(imloc_ctx* ctx, const imloc_corr* pts, int64_t n, const imloc_camera* K, const double* poses,
                int64_t np, double tau, int32_t precision, int32_t* count, double* msac) {
  if (!ctx) return IMLOC_EINVAL;
  if (n < 0 || n > INT32_MAX || np < 0 || np > INT32_MAX) return set_err(ctx, IMLOC_EINVAL, "bad sizes");
  if (n > 0 && !corr_ok(pts)) return set_err(ctx, IMLOC_EINVAL, "null correspondence array");
  if (!cam_ok(K)) return set_err(ctx, IMLOC_EINVAL, "bad intrinsics");
  if (!(tau > 0.0)) return set_err(ctx, IMLOC_EINVAL, "threshold must be > 0");
  if (precision != IMLOC_FP32_SCORE && precision != IMLOC_FP64_ALL) return set_err(ctx, IMLOC_EINVAL, "bad precision");
  if (np == 0) return IMLOC_OK;
  if (!poses || !count || !msac) return set_err(ctx, IMLOC_EINVAL, "null pose / output array");
  hipSetDevice(ctx->device);
  hipStream_t s = ctx->stream;
  Arena a{ctx->ws, ctx->ws_bytes};
  ScorePlan pl = plan_score(n, np, precision);
  BestState* st = a.take<BestState>(1);
  float* proj = a.take<float>(16 * (size_t)np);
  int32_t* ncand = a.take<int32_t>(1);
  uint32_t* pc = a.take<uint32_t>((size_t)pl.chunks * (size_t)pl.cap);
  double* pg = a.take<double>((size_t)pl.chunks * (size_t)pl.cap);
  if (!a.ok) return set_err(ctx, IMLOC_ENOMEM, "workspace too small: need %zu bytes", a.off);
  const CorrF32 c = n > 0 ? to_corr(pts) : CorrF32{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  CandBuf cb;
  cb.pose = const_cast<double*>(poses); cb.proj = proj; cb.h = nullptr; cb.j = nullptr; cb.n = ncand;
  cb.count = count; cb.msac = msac; cb.cap = np;
  HIP_TRY(ctx, launch_init_state(st, s));
  HIP_TRY(ctx, launch_weight_sum(c, n, st, s));
  HIP_TRY(ctx, launch_fill_i32(ncand, 1, (int32_t)np, s));
  HIP_TRY(ctx, launch_make_proj(poses, np, to_cam(K), tau, proj, s));
  HIP_TRY(ctx, launch_score(c, n, to_cam(K), tau, precision, pl, cb, pc, reinterpret_cast<float*>(pg), pg, s));
  HIP_TRY(ctx, launch_reduce_scores(pl, cb, tau, pc, reinterpret_cast<float*>(pg), pg, precision, st, s));
  return IMLOC_OK;
}

int imloc_local_optimize(imloc_ctx* ctx, const imloc_corr* pts, int64_t n, const imloc_camera* K, const double* start,
                         int32_t np, double tau, int32_t iters, double* out_poses, double* cost, int64_t* count) {
  if (!ctx) return IMLOC_EINVAL;
  if (n < 0 || n > INT32_MAX || np < 0 || iters < 0) return set_err(ctx, IMLOC_EINVAL, "bad sizes");
  if (n > 0 && !corr_ok(pts)) return set_err(ctx, IMLOC_EINVAL, "null correspondence array");
  if (!cam_ok(K)) return set_err(ctx, IMLOC_EINVAL, "bad intrinsics");
  if (!(tau > 0.0)) return set_err(ctx, IMLOC_EINVAL, "threshold must be > 0");
  if (np == 0) return IMLOC_OK;
  if (!start || !out_poses || !cost) return set_err(ctx, IMLOC_EINVAL, "null pose / output array");
  hipSetDevice(ctx->device);
  const CorrF32 c = n > 0 ? to_corr(pts) : CorrF32{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  HIP_TRY(ctx, launch_lo(c, n, to_cam(K), tau, iters, start, nullptr, nullptr, np, out_poses, cost, count, ctx->stream));
  return IMLOC_OK;
}

int imloc_refine(imloc_ctx* ctx, const imloc_corr* pts, int64_t n, const imloc_camera* K, const double* start,
                 double tau, double scale, int32_t iters, double* out_pose, double* cost, uint8_t* mask) {
  if (!ctx) return IMLOC_EINVAL;
  if (n < 0 || n > INT32_MAX || iters < 0) return set_err(ctx, IMLOC_EINVAL, "bad sizes");
  if (n > 0 && !corr_ok(pts)) return set_err(ctx, IMLOC_EINVAL, "null correspondence array");
  if (!cam_ok(K)) return set_err(ctx, IMLOC_EINVAL, "bad intrinsics");
  if (!(tau > 0.0) || !(scale > 0.0)) return set_err(ctx, IMLOC_EINVAL, "threshold and scale must be > 0");
  if (!start || !out_pose || !cost) return set_err(ctx, IMLOC_EINVAL, "null pose / output array");
  hipSetDevice(ctx->device);
  Arena a{ctx->ws, ctx->ws_bytes};
  uint8_t* in_set = a.take<uint8_t>((size_t)(n > 0 ? n : 1));
  if (!a.ok) return set_err(ctx, IMLOC_ENOMEM, "workspace too small: need %zu bytes", a.off);
  const CorrF32 c = n > 0 ? to_corr(pts) : CorrF32{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  HIP_TRY(ctx, launch_refine(c, n, to_cam(K), tau, scale, iters, start, in_set, out_pose, cost, ctx->stream));
  if (mask) HIP_TRY(ctx, launch_mask(c, n, to_cam(K), tau, out_pose, mask, nullptr, ctx->stream));
  return IMLOC_OK;
}

size_t imloc_batch_workspace_bytes(int32_t nq, const int64_t* n, const imloc_ransac_params* p) {
  if (nq <= 0 || !n || !p) return 0;
  size_t mx = 0;
  for (int32_t q = 0; q < nq; ++q) mx = std::max(mx, imloc_workspace_bytes(n[q], p));
  return mx;
}

int imloc_lo_ransac_pnp_batch(imloc_ctx* ctx, const imloc_corr* pts, const int64_t* n, const imloc_camera* K,
                              int32_t nq, const imloc_ransac_params* params, int32_t n_params, imloc_pose* poses,
                              uint8_t* const* masks, imloc_stats* stats, int32_t* status) {
  if (!ctx) return IMLOC_EINVAL;
  if (nq < 0 || (nq > 0 && (!pts || !n || !K || !params || !poses || !status)))
    return set_err(ctx, IMLOC_EINVAL, "bad batch arguments");
  if (n_params != 1 && n_params != nq) return set_err(ctx, IMLOC_EINVAL, "n_params must be 1 or nq");
  for (int32_t q = 0; q < nq; ++q) {
    const imloc_ransac_params* p = &params[n_params == 1 ? 0 : q];
    int rc = imloc_lo_ransac_pnp(ctx, &pts[q], n[q], &K[q], p, &poses[q], masks ? masks[q] : nullptr,
                                 stats ? &stats[q] : nullptr);
    if (rc < 0) return rc;
    status[q] = rc;
  }
  return IMLOC_OK;
}

}  // extern "C"
