// runtime.cpp -- the C ABI of libimloc.so (include/imloc.h): context,
// workspace carving, argument checks and the orchestration of the kernels of
// the pose-estimation path (ImLoc Sec. 3.3).
//
// Queries run as batches: a device table of QueryDesc drives every kernel,
// and a single query is a batch of one.  A round draws one batch of minimal
// samples for every query still sampling, solves P3P, scores, selects, runs
// the local optimisations and applies the stopping rule; after the last round
// the final refinement and the inlier mask run for every query.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "imloc.h"
#include "imloc_kernels.h"

using namespace imloc;

// Device scratch of the allocation-free entry point
// (imloc_lo_ransac_pnp_noalloc): a fixed array that every GPU the library
// runs on holds until the process ends.  Host code never passes `scratch`
// itself to a kernel (on the host it is only a stand-in symbol): its device
// address is looked up once per device, with that device current, and kept.
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Called by imloc_create with `device` current.
hipError_t noalloc_setup(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  if (g_scratch_ptr[device]) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = p;
  return hipSuccess;
}

void* noalloc_scratch(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return device >= 0 && device < kMaxDevices ? g_scratch_ptr[device] : nullptr;
}
}  // namespace

// Vector with room for N elements inside the object: a call on up to N
// queries builds its host-side plan without touching the heap (the
// allocation-free entry point relies on this for its one query).
template <class T, int N>
class SmallVec {
 public:
  SmallVec() = default;
  explicit SmallVec(size_t n) { resize(n); }
  SmallVec(const SmallVec&) = delete;
  SmallVec& operator=(const SmallVec&) = delete;
  void resize(size_t n) {
    if (p_ == inl_ && n <= (size_t)N) {
      for (size_t i = n_; i < n; ++i) inl_[i] = T();
      n_ = n;
      return;
    }
    if (p_ == inl_) heap_.assign(inl_, inl_ + n_);
    heap_.resize(n);
    p_ = heap_.data();
    n_ = n;
  }
  void assign(size_t n, const T& v) {
    resize(n);
    for (size_t i = 0; i < n; ++i) p_[i] = v;
  }
  void push_back(const T& v) {
    resize(n_ + 1);
    p_[n_ - 1] = v;
  }
  T& operator[](size_t i) { return p_[i]; }
  const T& operator[](size_t i) const { return p_[i]; }
  T& back() { return p_[n_ - 1]; }
  const T& back() const { return p_[n_ - 1]; }
  const T* data() const { return p_; }
  size_t size() const { return n_; }

 private:
  T inl_[N] = {};
  std::vector<T> heap_;
  T* p_ = inl_;
  size_t n_ = 0;
};

struct imloc_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool timing = false;
  char err[512] = "";
  // Host staging (pinned): query tables and view tables in, states and poses
  // out.  Allocated by imloc_create / imloc_set_staging only; a call that
  // needs more returns IMLOC_ENOMEM.  `staging_ev` is recorded after the last
  // asynchronous copy that uses it, so the host waits for that copy (and only
  // that) before writing the buffer again.
  char* pinned = nullptr;
  size_t pinned_bytes = 0;
  hipEvent_t staging_ev = nullptr;
  bool staging_pending = false;
  // recorded behind a synchronous call's work and polled (wait_stream)
  hipEvent_t done_ev = nullptr;
  // timing events, created when timing is switched on (imloc_set_timing)
  std::vector<hipEvent_t> events;
  size_t next_event = 0;
  ScoreTune tune{0, 0, 2048};  // ct == 0, blocks == 0: the tile and the grid are picked per round (round_tune)
  int cus = 256;
  int gn_mode = 0;  // Gauss-Newton launch form: 0 by size, 1 fused, 2 split
  // hipGraph replay of the fixed-sample pipeline
  bool graphs = false;
  hipStream_t gstream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::string gkey;
  int64_t graph_launches = 0, graph_captures = 0;
};

namespace {

int set_err(imloc_ctx* c, int code, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    snprintf(c->err, sizeof(c->err), "%s", buf);
  }
  return code;
}

#define HIP_TRY(ctx, expr)                                                                          \
  do {                                                                                              \
    hipError_t e_ = (expr);                                                                         \
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
const CorrF32 kNoCorr{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};

int check_params(imloc_ctx* ctx, const imloc_ransac_params* p) {
  if (!p) return set_err(ctx, IMLOC_EINVAL, "params is null");
  if (!(p->threshold_px > 0.0) || !std::isfinite(p->threshold_px))
    return set_err(ctx, IMLOC_EINVAL, "threshold_px must be finite and > 0");
  if (p->fixed_samples <= 0 && (p->max_iters <= 0 || !(p->confidence > 0.0 && p->confidence < 1.0)))
    return set_err(ctx, IMLOC_EINVAL, "adaptive mode needs max_iters > 0 and 0 < confidence < 1");
  if (p->precision != IMLOC_FP32_SCORE && p->precision != IMLOC_FP64_ALL)
    return set_err(ctx, IMLOC_EINVAL, "unknown precision %d", p->precision);
  if (p->final_iters > 0 && !(p->cauchy_scale_px > 0.0))
    return set_err(ctx, IMLOC_EINVAL, "cauchy_scale_px must be > 0");
  if (p->lo_iters < 0 || p->final_iters < 0) return set_err(ctx, IMLOC_EINVAL, "negative iteration count");
  if (p->lo_iters > 1000 || p->final_iters > 1000) return set_err(ctx, IMLOC_EINVAL, "iteration count above 1000");
  if (p->max_score_points < 0) return set_err(ctx, IMLOC_EINVAL, "max_score_points < 0");
  if (p->max_score_points > 0 && p->max_score_points < 3) return set_err(ctx, IMLOC_EINVAL, "max_score_points < 3");
  return IMLOC_OK;
}

// Host-side plan of one query.
struct QPlan {
  int64_t n, m;
  bool subset;
  int64_t total, batch, cap;
  int k;
  int ncam = 0;  // 0: one camera; else the cameras of a rig
};

// Scoring launch shape: the context's fixed one, or (ct == 0) the largest
// candidate tile of 128, 64 and 32 that still gives about four work items per
// CU, so that small rounds keep every CU busy; est holds per query the
// expected candidates (one per sample) and scoring points.  Neither the tile
// nor the correspondences per item change a result (per-candidate sums are
// integer-accumulated over fixed wave blocks).
using EstList = SmallVec<std::pair<int64_t, int64_t>, 4>;
ScoreTune round_tune(const imloc_ctx* c, const std::pair<int64_t, int64_t>* est, size_t n_est) {
  ScoreTune t = c->tune;
  if (t.ct > 0 && t.blocks > 0) return t;
  const int64_t pts = t.pts;
  auto items_for = [&](int ct) {
    int64_t items = 0;
    for (size_t q = 0; q < n_est; ++q) items += (est[q].first + ct - 1) / ct * ((est[q].second + pts - 1) / pts);
    return items;
  };
  if (t.ct == 0) {
    t.ct = 32;
    for (int ct : {128, 64})
      if (items_for(ct) >= 4 * (int64_t)c->cus) {
        t.ct = ct;
        break;
      }
  }
  if (t.blocks == 0) {
    // About one work item per workgroup: the hardware dispatcher then hands
    // the next item to whichever workgroup slot frees first, so ragged items
    // (a query's last tile and chunk) leave a tail of about one item, where a
    // grid of a few resident workgroups striding over many items each leaves
    // a tail of a whole workgroup's share (3.7 % of the 256-query batch's
    // scoring).  A P3P sample gives 1.4 candidates on average, up to 4.
    const int64_t items = items_for(t.ct);
    t.blocks = (int)std::min<int64_t>(kScoreMaxBlocks, std::max<int64_t>(8 * (int64_t)c->cus, items + items / 2));
  }
  return t;
}

// Scoring points of a query for the estimate above (a rig cuts its segments
// apart: about one more partial item per further camera).
int64_t est_points(const QPlan& pl) { return pl.m + (pl.ncam > 1 ? (int64_t)(pl.ncam - 1) * 2048 : 0); }

// Host view of a rig query (ncam == 0: a one-camera query).
struct RigHost {
  int32_t ncam;
  const imloc_rig_camera* cams;  // [ncam]
  const int64_t* cam_start;      // [ncam + 1], correspondences grouped by camera
};

int rig_check(imloc_ctx* ctx, const RigHost& r, int64_t n) {
  if (r.ncam < 1 || r.ncam > kMaxCams) return set_err(ctx, IMLOC_EINVAL, "n_cams must be in 1..%d", kMaxCams);
  if (!r.cams || !r.cam_start) return set_err(ctx, IMLOC_EINVAL, "null rig arrays");
  if (r.cam_start[0] != 0 || r.cam_start[r.ncam] != n)
    return set_err(ctx, IMLOC_EINVAL, "cam_start must run from 0 to n");
  for (int c = 0; c < r.ncam; ++c) {
    if (r.cam_start[c + 1] < r.cam_start[c]) return set_err(ctx, IMLOC_EINVAL, "cam_start must not decrease");
    const imloc_rig_camera& k = r.cams[c];
    if (!(k.K.fx > 0.0 && k.K.fy > 0.0 && std::isfinite(k.K.cx) && std::isfinite(k.K.cy)))
      return set_err(ctx, IMLOC_EINVAL, "rig camera %d: bad intrinsics", c);
    for (int e = 0; e < 9; ++e)
      if (!std::isfinite(k.cam_from_rig.R[e])) return set_err(ctx, IMLOC_EINVAL, "rig camera %d: bad pose", c);
    for (int e = 0; e < 3; ++e)
      if (!std::isfinite(k.cam_from_rig.t[e])) return set_err(ctx, IMLOC_EINVAL, "rig camera %d: bad pose", c);
  }
  return IMLOC_OK;
}

QPlan plan_query(int64_t n, const imloc_ransac_params* p, int ncam = 0) {
  QPlan s;
  s.ncam = ncam;
  s.n = n;
  s.subset = p->max_score_points > 0 && n > p->max_score_points;
  s.m = s.subset ? p->max_score_points : n;
  s.total = p->fixed_samples > 0 ? p->fixed_samples : p->max_iters;
  s.batch = p->batch > 0 ? p->batch : 1024;
  if (s.batch > s.total) s.batch = s.total;
  if (s.batch < 1) s.batch = 1;
  s.cap = (ncam > 0 ? 8 : 4) * s.batch;  // P3P gives at most 4 candidates, generalised P3P 8
  s.k = p->lo_top_k < 1 ? 1 : (p->lo_top_k > kMaxTopK ? kMaxTopK : p->lo_top_k);
  return s;
}

// Device buffers of one batch, carved from the workspace.
struct Engine {
  int nq = 0, kmax = 1, chunks_lo = 1, chunks_fin = 1, lo_iters = 0, fin_iters = 0;
  int64_t max_batch = 1, max_n = 0, slots = 0, max_rounds = 0;
  bool all_fixed = true;
  bool any_rig = false;
  bool any_single = false;  // some query has one camera (the P3P sampler has work)
  int64_t max_cap = 4, proj_floats = 16, rig_doubles = 0;
  QueryDesc* qd;
  double* rig;
  BestState* st;
  CandBuf cb;
  int64_t* item_off;
  int32_t* active_count;
  int32_t* sel;
  int32_t* n_sel;
  void* sel_part;
  double* lo_pose;
  double* lo_cost;
  int64_t* lo_count;
  double* fin_pose;
  double* fin_cost;
  uint8_t* in_set;
  void* gn_lo;
  void* gn_fin;
  float* subset;
  SmallVec<int64_t, 4> cand_off, in_set_off, subset_off, proj_off, rig_off;
};

void plan_engine(Engine& e, int nq, const QPlan* pl, const imloc_ransac_params* const* pp) {
  e.nq = nq;
  e.cand_off.resize(nq);
  e.in_set_off.resize(nq);
  e.subset_off.resize(nq);
  e.proj_off.resize(nq);
  e.rig_off.resize(nq);
  int64_t slots = 0, in_bytes = 0, sub = 0, proj = 0, rigd = 0;
  for (int q = 0; q < nq; ++q) {
    e.cand_off[q] = slots;
    slots += pl[q].cap;
    e.proj_off[q] = proj;
    proj += 16 * pl[q].cap * std::max(1, pl[q].ncam);
    e.rig_off[q] = rigd;
    rigd += 16 * pl[q].ncam;
    e.max_cap = std::max(e.max_cap, pl[q].cap);
    if (pl[q].ncam > 0) e.any_rig = true;
    else e.any_single = true;
    e.in_set_off[q] = in_bytes;
    in_bytes += (gn_inset_bytes(pl[q].n) + 255) & ~int64_t(255);
    e.subset_off[q] = sub;
    if (pl[q].subset) sub += 6 * pl[q].m;
    e.kmax = std::max(e.kmax, pl[q].k);
    e.chunks_lo = std::max(e.chunks_lo, gn_chunks(pl[q].m));
    e.chunks_fin = std::max(e.chunks_fin, gn_chunks(pl[q].n));
    e.lo_iters = std::max(e.lo_iters, (int)pp[q]->lo_iters);
    e.fin_iters = std::max(e.fin_iters, (int)pp[q]->final_iters);
    e.max_batch = std::max(e.max_batch, pl[q].batch);
    e.max_n = std::max(e.max_n, pl[q].n);
    e.max_rounds = std::max(e.max_rounds, (pl[q].total + pl[q].batch - 1) / pl[q].batch);
    if (pp[q]->fixed_samples <= 0) e.all_fixed = false;
  }
  e.slots = std::max<int64_t>(slots, 1);
  e.proj_floats = std::max<int64_t>(proj, 16);
  e.rig_doubles = rigd;
  e.in_set_off.push_back(in_bytes);
  e.subset_off.push_back(sub);
}

size_t result_bytes(int nq) { return (size_t)nq * (sizeof(BestState) + 13 * sizeof(double)); }

void carve_engine(Arena& a, Engine& e) {
  const int nq = e.nq;
  const size_t S = (size_t)e.slots;
  e.qd = a.take<QueryDesc>(nq);
  // states, final poses and final costs back to back, in the order of the host
  // staging buffer, so that one copy returns all results
  char* res = a.take<char>(result_bytes(nq));
  e.st = reinterpret_cast<BestState*>(res);
  // (sizing passes carve from a null base: no pointer arithmetic on it)
  e.fin_pose = res ? reinterpret_cast<double*>(res + (size_t)nq * sizeof(BestState)) : nullptr;
  e.fin_cost = res ? e.fin_pose + (size_t)nq * 12 : nullptr;
  e.cb.pose = a.take<double>(12 * S);
  e.cb.proj = a.take<float>((size_t)e.proj_floats);
  e.rig = a.take<double>((size_t)std::max<int64_t>(e.rig_doubles, 16));
  e.cb.h = a.take<int64_t>(S);
  e.cb.j = a.take<int32_t>(S);
  e.cb.cnt = a.take<uint32_t>(S);
  e.cb.gain = a.take<uint64_t>(S);
  e.cb.n = a.take<int32_t>(nq);
  e.cb.sel_done = a.take<int32_t>(nq);
  e.item_off = a.take<int64_t>(nq + 1);
  e.active_count = a.take<int32_t>(1);
  e.sel = a.take<int32_t>((size_t)nq * kMaxTopK);
  e.n_sel = a.take<int32_t>(nq);
  e.sel_part = a.take<char>(select_scratch_bytes(nq));
  e.lo_pose = a.take<double>((size_t)nq * e.kmax * 12);
  e.lo_cost = a.take<double>((size_t)nq * e.kmax);
  e.lo_count = a.take<int64_t>((size_t)nq * e.kmax);
  e.in_set = a.take<uint8_t>((size_t)std::max<int64_t>(e.in_set_off.back(), 1));
  e.gn_lo = a.take<char>(gn_scratch_bytes(nq * e.kmax, e.chunks_lo));
  e.gn_fin = a.take<char>(gn_scratch_bytes(nq, e.chunks_fin));
  e.subset = a.take<float>((size_t)std::max<int64_t>(e.subset_off.back(), 1));
}

// Host staging of the context: at least `bytes` of it, else an error naming
// the size to pass to imloc_set_staging.  Nothing is allocated here.
int staging_check(imloc_ctx* c, size_t bytes) {
  if (bytes <= c->pinned_bytes) return IMLOC_OK;
  return set_err(c, IMLOC_ENOMEM, "host staging too small: need %zu bytes, have %zu (imloc_set_staging)", bytes,
                 c->pinned_bytes);
}

// Wait until no queued copy reads or writes the staging buffer.
int staging_wait(imloc_ctx* c) {
  if (!c->staging_pending) return IMLOC_OK;
  HIP_TRY(c, hipEventSynchronize(c->staging_ev));
  c->staging_pending = false;
  return IMLOC_OK;
}

// Wait for the work enqueued on s so far: an event recorded behind it is
// polled for up to kSpinWait (a blocking wait wakes about 13 us after the
// work ends on this system, a sizeable part of a single query's latency),
// then waited on.
constexpr auto kSpinWait = std::chrono::microseconds(2000);
int wait_event(imloc_ctx* c, hipEvent_t ev) {
  const auto t0 = std::chrono::steady_clock::now();
  for (;;) {
    const hipError_t q = hipEventQuery(ev);
    if (q == hipSuccess) return IMLOC_OK;
    if (q != hipErrorNotReady) HIP_TRY(c, q);
    if (std::chrono::steady_clock::now() - t0 > kSpinWait) break;
  }
  HIP_TRY(c, hipEventSynchronize(ev));
  return IMLOC_OK;
}
int wait_stream(imloc_ctx* c, hipStream_t s) {
  HIP_TRY(c, hipEventRecord(c->done_ev, s));
  return wait_event(c, c->done_ev);
}

// After enqueueing copies that use the staging buffer on the context stream.
int staging_mark(imloc_ctx* c) {
  HIP_TRY(c, hipEventRecord(c->staging_ev, c->stream));
  c->staging_pending = true;
  return IMLOC_OK;
}

// Replace the staging buffer (setup calls only): waits for the stream, drops
// a captured graph that copies from or to the old buffer.
int staging_alloc(imloc_ctx* c, size_t bytes) {
  bytes = std::max<size_t>(bytes, 4096);
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  if (c->gexec) {
    if (c->gstream) hipStreamSynchronize(c->gstream);
    hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
    if (c->graph) hipGraphDestroy(c->graph);
    c->graph = nullptr;
    c->gkey.clear();
  }
  if (c->pinned) hipHostFree(c->pinned);
  c->pinned = nullptr;
  c->pinned_bytes = 0;
  c->staging_pending = false;
  HIP_TRY(c, hipHostMalloc(reinterpret_cast<void**>(&c->pinned), bytes, hipHostMallocDefault));
  c->pinned_bytes = bytes;
  return IMLOC_OK;
}

constexpr size_t kDefaultStaging = size_t(1) << 20;
constexpr size_t kTimingEvents = 256;  // events of the timing pool (reused within a call)

// Per-stage timing with HIP events on the context stream.  The events come
// from the pool created by imloc_set_timing; event 0 opens the whole call,
// the stage spans use the rest, and when the pool runs out the stream is
// synchronised, the closed spans are added up and the pool is reused.
struct Timer {
  imloc_ctx* c;
  struct Span { int stage; hipEvent_t a, b; };
  Span spans[kTimingEvents];  // closed spans not yet added up (fewer than events in the pool)
  size_t n_spans = 0;
  float acc[6] = {0, 0, 0, 0, 0, 0};
  bool on;
  explicit Timer(imloc_ctx* cc) : c(cc), on(cc->timing && cc->events.size() == kTimingEvents) {
    c->next_event = 1;
  }
  void add_up() {
    for (size_t k = 0; k < n_spans; ++k) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, spans[k].a, spans[k].b) == hipSuccess) acc[spans[k].stage] += ms;
    }
    n_spans = 0;
  }
  void fold() {
    (void)hipStreamSynchronize(c->stream);
    add_up();
    c->next_event = 1;
  }
  hipEvent_t total_begin() {
    if (!on) return nullptr;
    (void)hipEventRecord(c->events[0], c->stream);
    return c->events[0];
  }
  void total_end(hipEvent_t a) {  // the last event of the pool closes the whole call
    if (!on || !a) return;
    hipEvent_t e = c->events[kTimingEvents - 1];
    (void)hipEventRecord(e, c->stream);
    spans[n_spans++] = Span{5, a, e};
  }
  hipEvent_t begin() {
    if (!on) return nullptr;
    if (c->next_event + 2 > kTimingEvents - 1) fold();
    hipEvent_t e = c->events[c->next_event++];
    (void)hipEventRecord(e, c->stream);
    return e;
  }
  void end(int stage, hipEvent_t a) {
    if (!on || !a) return;
    hipEvent_t e = c->events[c->next_event++];
    (void)hipEventRecord(e, c->stream);
    spans[n_spans++] = Span{stage, a, e};
  }
  void fill(imloc_stats* st) {
    if (!on || !st) return;
    add_up();
    st->ms_sample = acc[0]; st->ms_score = acc[1]; st->ms_select = acc[2];
    st->ms_lo = acc[3]; st->ms_refine = acc[4]; st->ms_total = acc[5];
  }
};
enum { kStSample = 0, kStScore = 1, kStSelect = 2, kStLO = 3, kStRefine = 4, kStTotal = 5 };

void identity_pose(imloc_pose* p) {
  for (int e = 0; e < 9; ++e) p->R[e] = (e % 4 == 0) ? 1.0 : 0.0;
  p->t[0] = p->t[1] = p->t[2] = 0.0;
}

QueryDesc make_desc(const imloc_corr* pts, int64_t n, const imloc_camera* K, const imloc_ransac_params* p,
                    const QPlan& pl, const Engine& e, int q, uint8_t* mask, const RigHost* rig = nullptr) {
  QueryDesc d;
  std::memset(&d, 0, sizeof(d));
  d.full = n > 0 ? to_corr(pts) : kNoCorr;
  if (pl.subset) {
    const float* b = e.subset + e.subset_off[q];
    const int64_t m = pl.m;
    d.S = CorrF32{b, b + m, b + 2 * m, b + 3 * m, b + 4 * m, b + 5 * m};
  } else {
    d.S = d.full;
  }
  d.n = n;
  d.m = pl.m;
  if (K) { d.fx = K->fx; d.fy = K->fy; d.cx = K->cx; d.cy = K->cy; }
  d.tau = p->threshold_px;
  d.cauchy_s = p->cauchy_scale_px > 0.0 ? p->cauchy_scale_px : 1.0;
  d.confidence = p->confidence;
  d.seed = p->seed;
  d.qid = p->query_id;
  d.total = pl.total;
  d.batch = pl.batch;
  d.min_iters = p->min_iters;
  d.fixed = p->fixed_samples > 0 ? 1 : 0;
  d.exhaustive = p->exhaustive ? 1 : 0;
  d.precision = p->precision;
  d.k = pl.k;
  d.lo_iters = p->lo_iters;
  d.final_iters = p->final_iters;
  d.cand_off = e.cand_off[q];
  d.cap = pl.cap;
  d.in_set_off = e.in_set_off[q];
  d.B = 0;
  d.mask = mask;
  d.fresh = 1;
  d.proj_off = e.proj_off[q];
  d.ncam = 0;
  if (rig && rig->ncam > 0) {
    d.ncam = rig->ncam;
    d.rig = e.rig + e.rig_off[q];
    for (int c = 0; c <= rig->ncam; ++c) {
      d.segF[c] = rig->cam_start[c];
      // stride subset j -> point floor(j n / m): camera c starts at j = ceil(start_c m / n)
      d.segS[c] = pl.subset ? (int64_t)(((unsigned __int128)rig->cam_start[c] * (uint64_t)pl.m + (uint64_t)n - 1) /
                                        (uint64_t)n)
                            : rig->cam_start[c];
    }
  }
  return d;
}

// Rig tables of a batch in host staging: per camera fx, fy, cx, cy, R (9), t (3).
void fill_rig_tables(double* h, int nq, const RigHost* rigs, const Engine& e) {
  if (!rigs) return;
  for (int q = 0; q < nq; ++q) {
    for (int c = 0; c < rigs[q].ncam; ++c) {
      double* o = h + e.rig_off[q] + 16 * c;
      const imloc_rig_camera& k = rigs[q].cams[c];
      o[0] = k.K.fx; o[1] = k.K.fy; o[2] = k.K.cx; o[3] = k.K.cy;
      for (int x = 0; x < 9; ++x) o[4 + x] = k.cam_from_rig.R[x];
      for (int x = 0; x < 3; ++x) o[13 + x] = k.cam_from_rig.t[x];
    }
  }
}

// Device scratch of a call: the context's workspace, or the library's
// fixed array for the allocation-free entry point.
struct Scratch {
  char* base;
  size_t bytes;
};

// Validate, plan, carve and run a batch.  Outputs are host arrays of nq.
// `ws` is the device scratch; `may_capture` allows the captured-graph form.
int run_batch(imloc_ctx* ctx, int nq, const imloc_corr* pts, const int64_t* n, const imloc_camera* K,
              const imloc_ransac_params* params, int n_params, imloc_pose* poses, uint8_t* const* masks,
              imloc_stats* stats, int32_t* status, const RigHost* rigs, Scratch ws, bool may_capture) {
  SmallVec<const imloc_ransac_params*, 4> pp(nq);
  SmallVec<QPlan, 4> pl(nq);
  for (int q = 0; q < nq; ++q) {
    pp[q] = &params[n_params == 1 ? 0 : q];
    int rc = check_params(ctx, pp[q]);
    if (rc) return rc;
    if (n[q] < 0 || n[q] > INT32_MAX) return set_err(ctx, IMLOC_EINVAL, "query %d: n out of range", q);
    if (n[q] > 0 && !corr_ok(&pts[q])) return set_err(ctx, IMLOC_EINVAL, "query %d: null correspondence array", q);
    const int ncam = rigs ? rigs[q].ncam : 0;
    if (ncam > 0) {
      rc = rig_check(ctx, rigs[q], n[q]);
      if (rc) return rc;
    } else if (!cam_ok(&K[q])) {
      return set_err(ctx, IMLOC_EINVAL, "query %d: bad intrinsics", q);
    }
    pl[q] = plan_query(n[q], pp[q], ncam);
  }
  hipSetDevice(ctx->device);
  hipStream_t s = ctx->stream;
  Engine e;
  plan_engine(e, nq, pl.data(), pp.data());
  Arena a{ws.base, ws.bytes};
  carve_engine(a, e);
  if (!a.ok) return set_err(ctx, IMLOC_ENOMEM, "workspace too small: need %zu bytes, have %zu", a.off, ws.bytes);
  const size_t tab = (size_t)nq * sizeof(QueryDesc);
  const size_t outb = (size_t)nq * sizeof(BestState) + (size_t)nq * 13 * sizeof(double) + 64;
  const size_t rigb = (size_t)e.rig_doubles * sizeof(double);
  int rc0 = staging_check(ctx, tab + outb + 512 + rigb);
  if (rc0) return rc0;
  rc0 = staging_wait(ctx);  // an earlier asynchronous call may still copy from the staging buffer
  if (rc0) return rc0;
  QueryDesc* htab = reinterpret_cast<QueryDesc*>(ctx->pinned);
  for (int q = 0; q < nq; ++q)
    htab[q] = make_desc(&pts[q], n[q], rigs && rigs[q].ncam > 0 ? nullptr : &K[q], pp[q], pl[q], e, q,
                        masks ? masks[q] : nullptr, rigs ? &rigs[q] : nullptr);
  double* hrig = reinterpret_cast<double*>(ctx->pinned + tab + outb + 512);
  fill_rig_tables(hrig, nq, rigs, e);

  BestState* hst = reinterpret_cast<BestState*>(ctx->pinned + tab);
  double* hfin = reinterpret_cast<double*>(ctx->pinned + tab + (size_t)nq * sizeof(BestState));
  int32_t* hact = reinterpret_cast<int32_t*>(ctx->pinned + tab + outb);
  int64_t max_m_sub = 0;
  for (int q = 0; q < nq; ++q)
    if (pl[q].subset) max_m_sub = std::max(max_m_sub, pl[q].m);

  // a query with confidences needs the weighted local optimisation (the
  // unweighted one gives the same bits when every weight is 1)
  bool any_w = false;
  for (int q = 0; q < nq; ++q) any_w = any_w || (n[q] > 0 && pts[q].w != nullptr);
  Timer tm(ctx);
  int rounds = 0;
  EstList est(nq);
  for (int q = 0; q < nq; ++q) est[q] = {std::min(pl[q].batch, pl[q].total), est_points(pl[q])};
  const ScoreTune tune = round_tune(ctx, est.data(), est.size());
  // The whole pipeline of a batch, enqueued on stream `st_`: table upload,
  // rounds, final refinement, mask, readback into pinned memory.  `sync`
  // lets adaptive batches read the active count after every round.
  auto enqueue = [&](hipStream_t st_, bool sync) -> int {
    hipEvent_t ev_total = tm.total_begin();
    HIP_TRY(ctx, hipMemcpyAsync(e.qd, htab, tab, hipMemcpyHostToDevice, st_));
    if (rigb) HIP_TRY(ctx, hipMemcpyAsync(e.rig, hrig, rigb, hipMemcpyHostToDevice, st_));
    HIP_TRY(ctx, launch_gather_subsets(e.qd, nq, max_m_sub, st_));
    HIP_TRY(ctx, launch_init_queries(e.qd, e.st, e.cb.n, nq, true, st_));  // and the first round's setup
    rounds = 0;
    for (int64_t r = 0; r < e.max_rounds; ++r) {
      hipEvent_t e0 = tm.begin();
      if (e.any_single) HIP_TRY(ctx, launch_sample_p3p(e.qd, e.st, e.cb, nq, e.max_batch, nullptr, st_));
      if (e.any_rig) HIP_TRY(ctx, launch_sample_gp3p(e.qd, e.st, e.cb, nq, e.max_batch, nullptr, st_));
      HIP_TRY(ctx, launch_worklist(e.qd, e.cb, nq, tune, e.item_off, st_));
      tm.end(kStSample, e0);
      hipEvent_t e1 = tm.begin();  // the scoring span holds the scoring kernel alone
      HIP_TRY(ctx, launch_score(e.qd, e.cb, e.st, nq, e.item_off, tune, 0, st_));
      tm.end(kStScore, e1);
      hipEvent_t e2 = tm.begin();
      HIP_TRY(ctx, launch_select(e.qd, e.st, e.cb, nq, e.kmax, e.max_cap, e.sel_part, e.sel, e.n_sel, st_));
      tm.end(kStSelect, e2);
      hipEvent_t e3 = tm.begin();
      HIP_TRY(ctx, launch_lo(e.qd, e.cb, e.sel, e.n_sel, nullptr, nq * e.kmax, e.kmax, e.chunks_lo, e.lo_iters,
                             e.gn_lo, e.lo_pose, e.lo_cost, e.lo_count, e.any_rig, any_w, ctx->gn_mode, st_));
      HIP_TRY(ctx, launch_round_end(e.qd, e.cb, e.sel, e.n_sel, e.lo_pose, e.lo_cost, e.lo_count, nq, e.kmax, e.st,
                                    e.active_count, true, st_));
      tm.end(kStLO, e3);
      ++rounds;
      if (sync) {
        HIP_TRY(ctx, hipMemcpyAsync(hact, e.active_count, sizeof(int32_t), hipMemcpyDeviceToHost, st_));
        int rcw = wait_stream(ctx, st_);
        if (rcw) return rcw;
        if (*hact == 0) break;
      }
    }
    hipEvent_t e4 = tm.begin();
    bool mask_done = false;  // the fused final refinement writes the masks itself
    HIP_TRY(ctx, launch_refine(e.qd, e.st, nullptr, nq, e.chunks_fin, e.fin_iters, e.in_set, e.gn_fin, e.fin_pose,
                               e.fin_cost, e.any_rig, ctx->gn_mode, true, &mask_done, st_));
    if (!mask_done) HIP_TRY(ctx, launch_mask(e.qd, e.st, e.fin_pose, nq, e.max_n, 0, st_));
    tm.end(kStRefine, e4);
    tm.total_end(ev_total);
    HIP_TRY(ctx, hipMemcpyAsync(hst, e.st, result_bytes(nq), hipMemcpyDeviceToHost, st_));
    return IMLOC_OK;
  };

  if (may_capture && ctx->graphs && ctx->gstream && e.all_fixed && !ctx->timing) {
    // key of everything a captured graph bakes in: shapes, workspace, staging
    std::string key;
    char buf[160];
    snprintf(buf, sizeof(buf), "%d|%p|%p|%d|%d|%d|%d|%d|%d|", nq, (void*)ws.base, (void*)ctx->pinned, tune.ct,
             tune.blocks, tune.pts, e.lo_iters, e.fin_iters, ctx->gn_mode);
    key += buf;
    for (int q = 0; q < nq; ++q) {
      snprintf(buf, sizeof(buf), "%lld,%lld,%d,%lld,%lld,%d,%d;", (long long)pl[q].n, (long long)pl[q].m,
               (int)pl[q].subset, (long long)pl[q].total, (long long)pl[q].batch, pl[q].k, pl[q].ncam);
      key += buf;
    }
    if (key != ctx->gkey || !ctx->gexec) {
      if (ctx->gexec) hipGraphExecDestroy(ctx->gexec);
      if (ctx->graph) hipGraphDestroy(ctx->graph);
      ctx->gexec = nullptr;
      ctx->graph = nullptr;
      ctx->gkey.clear();
      HIP_TRY(ctx, hipStreamBeginCapture(ctx->gstream, hipStreamCaptureModeRelaxed));
      int rc = enqueue(ctx->gstream, false);
      hipGraph_t g = nullptr;
      hipError_t ce = hipStreamEndCapture(ctx->gstream, &g);
      if (rc) return rc;
      if (ce != hipSuccess) return set_err(ctx, IMLOC_EHIP, "graph capture failed: %s", hipGetErrorString(ce));
      ctx->graph = g;
      HIP_TRY(ctx, hipGraphInstantiate(&ctx->gexec, ctx->graph, nullptr, nullptr, 0));
      ctx->gkey = key;
      ctx->graph_captures++;
    }
    // captured on the internal stream, replayed on the caller's stream
    HIP_TRY(ctx, hipGraphLaunch(ctx->gexec, s));
    int rcw = wait_stream(ctx, s);
    if (rcw) return rcw;
    ctx->graph_launches++;
    rounds = (int)e.max_rounds;
  } else {
    int rc = enqueue(s, !e.all_fixed);
    if (rc) return rc;
    rc = wait_stream(ctx, s);
    if (rc) return rc;
  }

  imloc_stats shared_t;
  std::memset(&shared_t, 0, sizeof(shared_t));
  tm.fill(&shared_t);
  for (int q = 0; q < nq; ++q) {
    const BestState& b = hst[q];
    const bool have = b.have != 0;
    status[q] = have ? IMLOC_OK : IMLOC_NO_POSE;
    identity_pose(&poses[q]);
    if (have) {
      for (int x = 0; x < 9; ++x) poses[q].R[x] = hfin[12 * q + x];
      for (int x = 0; x < 3; ++x) poses[q].t[x] = hfin[12 * q + 9 + x];
    }
    if (stats) {
      imloc_stats& o = stats[q];
      o = shared_t;
      o.samples = b.drawn;
      o.candidates = b.candidates;
      o.residuals = b.candidates * pl[q].m;
      o.inlier_residuals = b.inlier_residuals;
      o.best_count = have ? b.count : 0;
      o.full_count = have ? b.full_count : 0;
      o.batches = b.batches;
      o.lo_runs = (int32_t)b.lo_runs;
      o.status = status[q];
      o.best_msac = have ? b.cost : 0.0;
      o.final_cost = have ? hfin[12 * nq + q] : 0.0;
      o.best_h = have ? b.h : -1;
      o.best_j = have ? b.j : -1;
      o.score_launches = rounds;
    }
  }
  return IMLOC_OK;
}

size_t batch_bytes(int nq, const int64_t* n, const imloc_ransac_params* params, int n_params,
                   const int32_t* ncam = nullptr) {
  std::vector<const imloc_ransac_params*> pp(nq);
  std::vector<QPlan> pl(nq);
  for (int q = 0; q < nq; ++q) {
    pp[q] = &params[n_params == 1 ? 0 : q];
    pl[q] = plan_query(n[q] < 0 ? 0 : n[q], pp[q], ncam ? ncam[q] : 0);
  }
  Engine e;
  plan_engine(e, nq, pl.data(), pp.data());
  Arena a{nullptr, (size_t)-1};
  carve_engine(a, e);
  return a.off + 256;
}

// A one-query engine for the stage entry points: the query's full set is its
// scoring set, `cap` candidate slots.
struct StageQuery {
  Engine e;
  QPlan pl;
  imloc_ransac_params p;
};

void stage_setup(StageQuery& sq, int64_t n, int64_t cap, double tau, int precision, int lo_iters, int final_iters,
                 double cauchy_s, int nprob_lo, int ncam = 0) {
  std::memset(&sq.p, 0, sizeof(sq.p));
  sq.p.threshold_px = tau;
  sq.p.fixed_samples = 1;
  sq.p.batch = 1;
  sq.p.lo_top_k = 1;
  sq.p.lo_iters = lo_iters;
  sq.p.final_iters = final_iters;
  sq.p.cauchy_scale_px = cauchy_s;
  sq.p.precision = precision;
  sq.pl = plan_query(n, &sq.p, ncam);
  sq.pl.cap = std::max<int64_t>(cap, 1);
  const imloc_ransac_params* pp = &sq.p;
  plan_engine(sq.e, 1, &sq.pl, &pp);
  sq.e.kmax = 1;
  sq.e.chunks_lo = gn_chunks(n);
  (void)nprob_lo;
}

size_t stage_bytes(StageQuery& sq, int nprob_lo) {
  Arena a{nullptr, (size_t)-1};
  carve_engine(a, sq.e);
  a.take<char>(gn_scratch_bytes(nprob_lo, sq.e.chunks_lo));
  return a.off + 256;
}

// Upload the one-query table (and optionally an initial state) and return the
// device pointers.
int stage_upload(imloc_ctx* ctx, StageQuery& sq, const imloc_corr* pts, int64_t n, const imloc_camera* K,
                 int64_t B, int64_t drawn, uint8_t* mask, const RigHost* rig = nullptr) {
  const size_t rig_at = 256 * ((sizeof(QueryDesc) + sizeof(BestState) + 512 + 255) / 256);
  int rc = staging_check(ctx, rig_at + (size_t)sq.e.rig_doubles * sizeof(double));
  if (rc) return rc;
  rc = staging_wait(ctx);  // the staging buffer may still feed an earlier copy
  if (rc) return rc;
  QueryDesc* htab = reinterpret_cast<QueryDesc*>(ctx->pinned);
  htab[0] = make_desc(pts, n, K, &sq.p, sq.pl, sq.e, 0, mask, rig);
  htab[0].B = B;
  HIP_TRY(ctx, hipMemcpyAsync(sq.e.qd, htab, sizeof(QueryDesc), hipMemcpyHostToDevice, ctx->stream));
  if (rig && sq.e.rig_doubles) {
    double* hrig = reinterpret_cast<double*>(ctx->pinned + rig_at);
    fill_rig_tables(hrig, 1, rig, sq.e);
    HIP_TRY(ctx, hipMemcpyAsync(sq.e.rig, hrig, (size_t)sq.e.rig_doubles * sizeof(double), hipMemcpyHostToDevice,
                                ctx->stream));
  }
  HIP_TRY(ctx, launch_init_queries(sq.e.qd, sq.e.st, sq.e.cb.n, 1, false, ctx->stream));
  if (drawn) {
    BestState* hb = reinterpret_cast<BestState*>(ctx->pinned + 256 * ((sizeof(QueryDesc) + 255) / 256));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(hb, sq.e.st, sizeof(BestState), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    hb->drawn = drawn;
    HIP_TRY(ctx, hipMemcpyAsync(sq.e.st, hb, sizeof(BestState), hipMemcpyHostToDevice, ctx->stream));
  }
  return staging_mark(ctx);
}

}  // namespace

extern "C" {

int imloc_create(imloc_ctx** out, int device, void* hip_stream) {
  if (!out) return IMLOC_EINVAL;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return IMLOC_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return IMLOC_EHIP;
  if (noalloc_setup(device) != hipSuccess) return IMLOC_EHIP;
  imloc_ctx* c = new imloc_ctx();
  c->device = device;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  if (hipEventCreateWithFlags(&c->staging_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->done_ev, hipEventDisableTiming) != hipSuccess ||
      staging_alloc(c, kDefaultStaging) != IMLOC_OK) {
    imloc_destroy(c);
    return IMLOC_EHIP;
  }
  int cus = 256;
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  c->cus = cus > 0 ? cus : 256;
  c->tune.ct = 0;      // the candidate tile and
  c->tune.blocks = 0;  // the grid of the scoring launch: picked per round
  *out = c;
  return IMLOC_OK;
}

void imloc_destroy(imloc_ctx* c) {
  if (!c) return;
  hipSetDevice(c->device);
  hipStreamSynchronize(c->stream);
  for (auto e : c->events) hipEventDestroy(e);
  if (c->gexec) hipGraphExecDestroy(c->gexec);
  if (c->graph) hipGraphDestroy(c->graph);
  if (c->staging_ev) hipEventDestroy(c->staging_ev);
  if (c->done_ev) hipEventDestroy(c->done_ev);
  if (c->gstream) {
    hipStreamSynchronize(c->gstream);
    hipStreamDestroy(c->gstream);
  }
  if (c->pinned) hipHostFree(c->pinned);
  delete c;
}

int imloc_set_stream(imloc_ctx* c, void* s) {
  if (!c) return IMLOC_EINVAL;
  c->stream = reinterpret_cast<hipStream_t>(s);
  return IMLOC_OK;
}

const char* imloc_last_error(const imloc_ctx* c) { return c ? c->err : "null context"; }

int imloc_set_workspace(imloc_ctx* c, void* p, size_t bytes) {
  if (!c) return IMLOC_EINVAL;
  if (!p && bytes) return set_err(c, IMLOC_EINVAL, "workspace pointer is null");
  c->ws = reinterpret_cast<char*>(p);
  c->ws_bytes = bytes;
  return IMLOC_OK;
}

int imloc_set_timing(imloc_ctx* c, int enable) {
  if (!c) return IMLOC_EINVAL;
  if (enable && c->events.size() < kTimingEvents) {
    hipSetDevice(c->device);
    while (c->events.size() < kTimingEvents) {
      hipEvent_t e;
      HIP_TRY(c, hipEventCreate(&e));
      c->events.push_back(e);
    }
  }
  c->timing = enable != 0;
  return IMLOC_OK;
}

int imloc_set_graphs(imloc_ctx* c, int enable) {
  if (!c) return IMLOC_EINVAL;
  if (enable && !c->gstream) {  // the capture stream
    hipSetDevice(c->device);
    HIP_TRY(c, hipStreamCreateWithFlags(&c->gstream, hipStreamNonBlocking));
  }
  c->graphs = enable != 0;
  return IMLOC_OK;
}

size_t imloc_staging_bytes(int32_t n_queries, int32_t n_rig_cameras) {
  const size_t nq = n_queries > 0 ? (size_t)n_queries : 0;
  const size_t nc = n_rig_cameras > 0 ? (size_t)n_rig_cameras : 0;
  const size_t batch = nq * (sizeof(QueryDesc) + sizeof(BestState) + 13 * sizeof(double)) + 64 + 512 +
                       nc * 16 * sizeof(double);
  return std::max(batch, kDefaultStaging);
}

int imloc_set_staging(imloc_ctx* c, size_t bytes) {
  if (!c) return IMLOC_EINVAL;
  if (bytes > (size_t(1) << 32)) return set_err(c, IMLOC_EINVAL, "staging above 4 GiB");
  hipSetDevice(c->device);
  return staging_alloc(c, bytes);
}

size_t imloc_get_staging(const imloc_ctx* c) { return c ? c->pinned_bytes : 0; }

int imloc_graph_counters(const imloc_ctx* c, int64_t* captures, int64_t* launches) {
  if (!c || !captures || !launches) return IMLOC_EINVAL;
  *captures = c->graph_captures;
  *launches = c->graph_launches;
  return IMLOC_OK;
}

int imloc_set_score_tuning(imloc_ctx* c, int32_t candidates_per_item, int32_t workgroups) {
  if (!c) return IMLOC_EINVAL;
  if (candidates_per_item != 0 && candidates_per_item != 32 && candidates_per_item != 64 && candidates_per_item != 128)
    return set_err(c, IMLOC_EINVAL, "candidates_per_item must be 0 (per round), 32, 64 or 128");
  if (workgroups < 0 || workgroups > (1 << 20)) return set_err(c, IMLOC_EINVAL, "workgroups out of range");
  c->tune.ct = candidates_per_item;
  c->tune.blocks = workgroups;
  return IMLOC_OK;
}

int imloc_set_gn_mode(imloc_ctx* c, int32_t mode) {
  if (!c) return IMLOC_EINVAL;
  if (mode < 0 || mode > 2) return set_err(c, IMLOC_EINVAL, "Gauss-Newton launch form must be 0, 1 or 2");
  c->gn_mode = mode;
  return IMLOC_OK;
}

int imloc_get_score_tuning(const imloc_ctx* c, int32_t* candidates_per_item, int32_t* workgroups) {
  if (!c || !candidates_per_item || !workgroups) return IMLOC_EINVAL;
  *candidates_per_item = c->tune.ct;
  *workgroups = c->tune.blocks;
  return IMLOC_OK;
}

int imloc_set_score_points(imloc_ctx* c, int32_t points_per_item) {
  if (!c) return IMLOC_EINVAL;
  if (points_per_item != 512 && points_per_item != 1024 && points_per_item != 2048 && points_per_item != kScoreMaxPoints)
    return set_err(c, IMLOC_EINVAL, "points_per_item must be 512, 1024, 2048 or 4096");
  c->tune.pts = points_per_item;
  return IMLOC_OK;
}

int imloc_get_score_points(const imloc_ctx* c, int32_t* points_per_item) {
  if (!c || !points_per_item) return IMLOC_EINVAL;
  *points_per_item = c->tune.pts;
  return IMLOC_OK;
}

int imloc_paper_params(double threshold_px, imloc_ransac_params* p) {
  if (!p || !(threshold_px > 0.0) || !std::isfinite(threshold_px)) return IMLOC_EINVAL;
  *p = imloc_ransac_params{};
  p->threshold_px = threshold_px;
  p->fixed_samples = 0;
  p->batch = 1000;
  p->min_iters = 1000;
  p->max_iters = 100000;
  p->confidence = 1.0 - 1e-4;
  p->lo_top_k = 1;
  p->lo_iters = 10;
  p->max_score_points = 10000;
  p->final_iters = 10;
  p->cauchy_scale_px = 0.5 * threshold_px;
  p->exhaustive = 0;
  p->precision = IMLOC_FP32_SCORE;
  p->seed = 0;
  p->query_id = 0;
  return IMLOC_OK;
}

size_t imloc_workspace_bytes(int64_t n, const imloc_ransac_params* p) {
  if (!p || n < 0) return 0;
  return batch_bytes(1, &n, p, 1);
}

size_t imloc_batch_workspace_bytes(int32_t nq, const int64_t* n, const imloc_ransac_params* p, int32_t n_params) {
  if (nq <= 0 || !n || !p || (n_params != 1 && n_params != nq)) return 0;
  return batch_bytes(nq, n, p, n_params);
}

size_t imloc_rig_workspace_bytes(int64_t n, int32_t n_cams, const imloc_ransac_params* p) {
  if (!p || n < 0 || n_cams < 1 || n_cams > kMaxCams) return 0;
  return batch_bytes(1, &n, p, 1, &n_cams);
}

size_t imloc_rig_stage_workspace_bytes(int64_t n, int32_t n_cams, int64_t count) {
  if (n < 0 || count < 0 || n_cams < 1 || n_cams > kMaxCams) return 0;
  StageQuery sq;
  stage_setup(sq, n, 8 * std::max<int64_t>(count, 1), 1.0, 1, 0, 0, 1.0, 1, n_cams);
  return stage_bytes(sq, 1);
}

size_t imloc_score_workspace_bytes(int64_t n, int64_t np, int32_t precision) {
  if (n < 0 || np < 0) return 0;
  StageQuery sq;
  stage_setup(sq, n, np, 1.0, precision, 0, 0, 1.0, 1);
  return stage_bytes(sq, 1);
}

size_t imloc_lo_workspace_bytes(int64_t n, int32_t np) {
  if (n < 0 || np < 0) return 0;
  StageQuery sq;
  stage_setup(sq, n, 1, 1.0, 0, 0, 0, 1.0, np);
  return stage_bytes(sq, std::max(np, 1));
}

size_t imloc_refine_workspace_bytes(int64_t n) {
  if (n < 0) return 0;
  StageQuery sq;
  stage_setup(sq, n, 1, 1.0, 0, 0, 0, 1.0, 1);
  return stage_bytes(sq, 1);
}

size_t imloc_sample_workspace_bytes(int64_t n, int64_t count) {
  if (n < 0 || count < 0) return 0;
  StageQuery sq;
  stage_setup(sq, n, 4 * std::max<int64_t>(count, 1), 1.0, 0, 0, 0, 1.0, 1);
  return stage_bytes(sq, 1);
}

size_t imloc_lift_workspace_bytes(int64_t n_matches, int32_t n_views) {
  if (n_matches < 0 || n_views < 0) return 0;
  Arena a{nullptr, (size_t)-1};
  const int nb = lift_blocks(n_matches);
  a.take<double>(16 * (size_t)(n_views > 0 ? n_views : 1));
  a.take<int32_t>((size_t)(nb > 0 ? nb : 1));
  return a.off + 256;
}

static int lift_impl(imloc_ctx* ctx, const imloc_matches* m, int64_t n_matches, const float* depth,
                     const uint8_t* codes, int32_t n_views, int32_t H, int32_t W, const imloc_camera* cams,
                     const imloc_pose* poses, int32_t subpixel, float min_conf, const imloc_corr_out* out,
                     int64_t capacity, int32_t* n_out) {
  if (!ctx) return IMLOC_EINVAL;
  if (n_matches < 0 || n_matches > INT32_MAX) return set_err(ctx, IMLOC_EINVAL, "n_matches out of range");
  if (!n_out || !out) return set_err(ctx, IMLOC_EINVAL, "null output");
  if (n_matches > 0) {
    if (!m || !m->q_u || !m->q_v || !m->db_u || !m->db_v || !m->conf || !m->view)
      return set_err(ctx, IMLOC_EINVAL, "null match array");
    if ((!depth && !codes) || n_views <= 0 || H < 2 || W < 2 || !cams || !poses)
      return set_err(ctx, IMLOC_EINVAL, "bad depth maps / views");
    if ((int64_t)n_views * H * W > ((int64_t)1 << 40)) return set_err(ctx, IMLOC_EINVAL, "depth maps too large");
    if (capacity < 0 || (capacity > 0 && (!out->u || !out->v || !out->X || !out->Y || !out->Z)))
      return set_err(ctx, IMLOC_EINVAL, "bad output arrays");
    for (int k = 0; k < n_views; ++k)
      if (!cam_ok(&cams[k])) return set_err(ctx, IMLOC_EINVAL, "view %d: bad intrinsics", k);
  }
  hipSetDevice(ctx->device);
  Arena a{ctx->ws, ctx->ws_bytes};
  const int nb = lift_blocks(n_matches);
  // the view table: intrinsics of every view, then the poses (one upload)
  double* dcams = a.take<double>(16 * (size_t)(n_views > 0 ? n_views : 1));
  double* dposes = dcams + 4 * (size_t)(n_views > 0 ? n_views : 1);
  int32_t* blk = a.take<int32_t>((size_t)(nb > 0 ? nb : 1));
  if (!a.ok) return set_err(ctx, IMLOC_ENOMEM, "workspace too small for lift: need %zu bytes", a.off);
  if (n_matches > 0) {
    const size_t hb = (size_t)n_views * 16 * sizeof(double);
    int rc = staging_check(ctx, hb + 512);
    if (rc) return rc;
    rc = staging_wait(ctx);  // the staging buffer may still feed an earlier copy
    if (rc) return rc;
    double* hc = reinterpret_cast<double*>(ctx->pinned);
    double* hp = hc + 4 * (size_t)n_views;
    for (int k = 0; k < n_views; ++k) {
      hc[4 * k] = cams[k].fx; hc[4 * k + 1] = cams[k].fy; hc[4 * k + 2] = cams[k].cx; hc[4 * k + 3] = cams[k].cy;
      for (int e = 0; e < 9; ++e) hp[12 * k + e] = poses[k].R[e];
      for (int e = 0; e < 3; ++e) hp[12 * k + 9 + e] = poses[k].t[e];
    }
    HIP_TRY(ctx, hipMemcpyAsync(dcams, hc, 16 * (size_t)n_views * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    rc = staging_mark(ctx);
    if (rc) return rc;
  }
  LiftArgs la;
  la.q_u = m ? m->q_u : nullptr; la.q_v = m ? m->q_v : nullptr; la.db_u = m ? m->db_u : nullptr;
  la.db_v = m ? m->db_v : nullptr; la.conf = m ? m->conf : nullptr; la.view = m ? m->view : nullptr;
  la.n = n_matches; la.depth = depth; la.codes = codes; la.n_views = n_views; la.H = H; la.W = W;
  la.cams = dcams; la.poses = dposes; la.subpixel = subpixel; la.min_conf = min_conf;
  la.out_u = out->u; la.out_v = out->v; la.out_X = out->X; la.out_Y = out->Y; la.out_Z = out->Z;
  la.out_w = out->w; la.out_src = out->src; la.capacity = capacity; la.n_out = n_out; la.block_counts = blk;
  HIP_TRY(ctx, launch_lift(la, ctx->stream));
  return IMLOC_OK;
}

int imloc_lift(imloc_ctx* ctx, const imloc_matches* m, int64_t n_matches, const float* depth, int32_t n_views,
               int32_t H, int32_t W, const imloc_camera* cams, const imloc_pose* poses, int32_t subpixel,
               float min_conf, const imloc_corr_out* out, int64_t capacity, int32_t* n_out) {
  return lift_impl(ctx, m, n_matches, depth, nullptr, n_views, H, W, cams, poses, subpixel, min_conf, out, capacity,
                   n_out);
}

int imloc_lift_log8(imloc_ctx* ctx, const imloc_matches* m, int64_t n_matches, const uint8_t* codes,
                    int32_t n_views, int32_t H, int32_t W, const imloc_camera* cams, const imloc_pose* poses,
                    int32_t subpixel, float min_conf, const imloc_corr_out* out, int64_t capacity, int32_t* n_out) {
  return lift_impl(ctx, m, n_matches, nullptr, codes, n_views, H, W, cams, poses, subpixel, min_conf, out, capacity,
                   n_out);
}

int imloc_depth_encode_log8(imloc_ctx* ctx, const float* depth, int64_t count, uint8_t* codes) {
  if (!ctx) return IMLOC_EINVAL;
  if (count < 0 || count > ((int64_t)1 << 40)) return set_err(ctx, IMLOC_EINVAL, "count out of range");
  if (count > 0 && (!depth || !codes)) return set_err(ctx, IMLOC_EINVAL, "null depth or code array");
  hipSetDevice(ctx->device);
  HIP_TRY(ctx, launch_log8_encode(depth, count, codes, ctx->stream));
  return IMLOC_OK;
}

size_t imloc_triangulate_workspace_bytes(int32_t H, int32_t W, int32_t n_views) {
  const int v = n_views < 0 ? 0 : n_views;
  const size_t hw = H > 0 && W > 0 ? (size_t)H * W : 0;
  auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
  return up((size_t)(v + 1) * 16 * sizeof(double)) + up(sizeof(int32_t)) + up(hw * sizeof(TriTask));
}

int imloc_triangulate_depth(imloc_ctx* ctx, int32_t H, int32_t W, const imloc_camera* K_map, const imloc_pose* T_map,
                            int32_t n_views, const imloc_camera* K_views, const imloc_pose* T_views,
                            const imloc_dense_matches* m, const imloc_triangulation_params* p, float* depth,
                            int32_t* inliers, uint8_t* codes) {
  if (!ctx) return IMLOC_EINVAL;
  if (H < 1 || W < 1 || (int64_t)H * W > INT32_MAX) return set_err(ctx, IMLOC_EINVAL, "bad image size");
  if (n_views < 1 || n_views > 32) return set_err(ctx, IMLOC_EINVAL, "n_views must be in 1..32");
  if (!K_map || !T_map || !K_views || !T_views || !m || !p) return set_err(ctx, IMLOC_EINVAL, "null argument");
  if (!m->u || !m->v || !m->conf) return set_err(ctx, IMLOC_EINVAL, "null match array");
  if (!cam_ok(K_map)) return set_err(ctx, IMLOC_EINVAL, "bad intrinsics of the mapping camera");
  for (int k = 0; k < n_views; ++k)
    if (!cam_ok(&K_views[k])) return set_err(ctx, IMLOC_EINVAL, "view %d: bad intrinsics", k);
  if (!(p->angle_deg > 0.0 && p->angle_deg < 90.0)) return set_err(ctx, IMLOC_EINVAL, "angle_deg must be in (0, 90)");
  if (p->max_refine_iters < 0) return set_err(ctx, IMLOC_EINVAL, "max_refine_iters < 0");
  hipSetDevice(ctx->device);
  Arena a{ctx->ws, ctx->ws_bytes};
  double* dviews = a.take<double>((size_t)(n_views + 1) * 16);
  int32_t* n_tasks = a.take<int32_t>(1);
  TriTask* tasks = a.take<TriTask>((size_t)H * W);
  if (!a.ok) return set_err(ctx, IMLOC_ENOMEM, "workspace too small for triangulation: need %zu bytes", a.off);
  const size_t hb = (size_t)(n_views + 1) * 16 * sizeof(double);
  int rc = staging_check(ctx, hb + 512);
  if (rc) return rc;
  rc = staging_wait(ctx);  // the staging buffer may still feed an earlier copy
  if (rc) return rc;
  double* h = reinterpret_cast<double*>(ctx->pinned);
  auto centre = [](const imloc_pose& T, double C[3]) {
    for (int r = 0; r < 3; ++r) C[r] = -(T.R[r] * T.t[0] + T.R[3 + r] * T.t[1] + T.R[6 + r] * T.t[2]);
  };
  double C0[3];
  centre(*T_map, C0);
  for (int e = 0; e <= n_views; ++e) {
    const imloc_camera& K = e == 0 ? *K_map : K_views[e - 1];
    const imloc_pose& T = e == 0 ? *T_map : T_views[e - 1];
    double* o = h + 16 * e;
    o[0] = K.fx; o[1] = K.fy; o[2] = K.cx; o[3] = K.cy;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) o[4 + 3 * r + c] = T.R[3 * c + r];  // R^T
    double C[3];
    centre(T, C);
    for (int c = 0; c < 3; ++c) o[13 + c] = e == 0 ? 0.0 : C0[c] - C[c];
  }
  HIP_TRY(ctx, hipMemcpyAsync(dviews, h, hb, hipMemcpyHostToDevice, ctx->stream));
  rc = staging_mark(ctx);
  if (rc) return rc;
  TriArgs ta;
  ta.H = H; ta.W = W; ta.V = n_views; ta.views = dviews;
  ta.mu = m->u; ta.mv = m->v; ta.conf = m->conf;
  ta.min_conf = (float)p->min_conf;
  const double th = p->angle_deg * (3.14159265358979323846 / 180.0);
  ta.cos2_thr = cos(th) * cos(th);
  ta.min_inliers = p->min_inliers;
  ta.max_iters = p->max_refine_iters;
  ta.depth = depth; ta.inliers = inliers; ta.codes = codes;
  ta.n_tasks = n_tasks; ta.tasks = tasks;
  HIP_TRY(ctx, launch_triangulate(ta, ctx->stream));
  return IMLOC_OK;
}

int imloc_lo_ransac_pnp(imloc_ctx* ctx, const imloc_corr* pts, int64_t n, const imloc_camera* K,
                        const imloc_ransac_params* p, imloc_pose* pose_out, uint8_t* mask, imloc_stats* stats) {
  if (!ctx) return IMLOC_EINVAL;
  if (!pose_out) return set_err(ctx, IMLOC_EINVAL, "pose_out is null");
  if (!p) return set_err(ctx, IMLOC_EINVAL, "params is null");
  imloc_corr none{};
  int32_t status = 0;
  uint8_t* masks[1] = {mask};
  int rc = run_batch(ctx, 1, pts ? pts : &none, &n, K, p, 1, pose_out, masks, stats, &status, nullptr,
                     Scratch{ctx->ws, ctx->ws_bytes}, true);
  return rc < 0 ? rc : status;
}

size_t imloc_noalloc_max_bytes(void) { return kNoAllocScratchBytes; }

int imloc_lo_ransac_pnp_noalloc(imloc_ctx* ctx, const imloc_corr* pts, int64_t n, const imloc_camera* K,
                                const imloc_ransac_params* p, imloc_pose* pose_out, uint8_t* mask,
                                imloc_stats* stats) {
  if (!ctx) return IMLOC_EINVAL;
  if (!pose_out) return set_err(ctx, IMLOC_EINVAL, "pose_out is null");
  if (!p) return set_err(ctx, IMLOC_EINVAL, "params is null");
  void* base = noalloc_scratch(ctx->device);
  if (!base) return set_err(ctx, IMLOC_EHIP, "device %d has no fixed scratch address", ctx->device);
  imloc_corr none{};
  int32_t status = 0;
  uint8_t* masks[1] = {mask};
  // the size check of run_batch (workspace too small -> IMLOC_ENOMEM) bounds the call by the array's size
  int rc = run_batch(ctx, 1, pts ? pts : &none, &n, K, p, 1, pose_out, masks, stats, &status, nullptr,
                     Scratch{reinterpret_cast<char*>(base), kNoAllocScratchBytes}, false);
  return rc < 0 ? rc : status;
}

int imloc_lo_ransac_pnp_batch(imloc_ctx* ctx, const imloc_corr* pts, const int64_t* n, const imloc_camera* K,
                              int32_t nq, const imloc_ransac_params* params, int32_t n_params, imloc_pose* poses,
                              uint8_t* const* masks, imloc_stats* stats, int32_t* status) {
  if (!ctx) return IMLOC_EINVAL;
  if (nq < 0 || (nq > 0 && (!pts || !n || !K || !params || !poses || !status)))
    return set_err(ctx, IMLOC_EINVAL, "bad batch arguments");
  if (nq > 65535) return set_err(ctx, IMLOC_EINVAL, "at most 65535 queries per batch");
  if (n_params != 1 && n_params != nq) return set_err(ctx, IMLOC_EINVAL, "n_params must be 1 or nq");
  if (nq == 0) return IMLOC_OK;
  return run_batch(ctx, nq, pts, n, K, params, n_params, poses, masks, stats, status, nullptr,
                   Scratch{ctx->ws, ctx->ws_bytes}, true);
}

int imloc_sample_p3p(imloc_ctx* ctx, const imloc_corr* pts, int64_t n, const imloc_camera* K, uint64_t seed,
                     uint64_t query_id, int32_t exhaustive, int64_t h0, int64_t count, double* poses, int64_t* h_out,
                     int32_t* j_out, int32_t* n_cand, int32_t* triples) {
  if (!ctx) return IMLOC_EINVAL;
  if (n < 0 || n > INT32_MAX || count < 0 || count > INT32_MAX || h0 < 0)
    return set_err(ctx, IMLOC_EINVAL, "bad sizes");
  if (n > 0 && !corr_ok(pts)) return set_err(ctx, IMLOC_EINVAL, "null correspondence array");
  if (!cam_ok(K)) return set_err(ctx, IMLOC_EINVAL, "bad intrinsics");
  if (!poses || !h_out || !j_out || !n_cand) return set_err(ctx, IMLOC_EINVAL, "null output");
  hipSetDevice(ctx->device);
  StageQuery sq;
  stage_setup(sq, n, 4 * std::max<int64_t>(count, 1), 1.0, 0, 0, 0, 1.0, 1);
  sq.p.seed = seed;
  sq.p.query_id = query_id;
  sq.p.exhaustive = exhaustive;
  Arena a{ctx->ws, ctx->ws_bytes};
  carve_engine(a, sq.e);
  if (!a.ok) return set_err(ctx, IMLOC_ENOMEM, "workspace too small: need %zu bytes", a.off);
  // the candidates go straight to the caller's arrays
  sq.e.cb.pose = poses;
  sq.e.cb.h = h_out;
  sq.e.cb.j = j_out;
  sq.e.cb.n = n_cand;
  int rc = stage_upload(ctx, sq, pts, n, K, count, h0, nullptr);
  if (rc) return rc;
  HIP_TRY(ctx, launch_fill_i32(n_cand, 1, 0, ctx->stream));
  HIP_TRY(ctx, launch_sample_p3p(sq.e.qd, sq.e.st, sq.e.cb, 1, count, triples, ctx->stream));
  return IMLOC_OK;
}

int imloc_rig_sample_gp3p(imloc_ctx* ctx, const imloc_corr* pts, int64_t n, const imloc_rig_camera* cams,
                          int32_t n_cams, const int64_t* cam_start, uint64_t seed, uint64_t query_id, int32_t exhaustive,
                          int64_t h0, int64_t count, double* poses, int64_t* h_out, int32_t* j_out, int32_t* n_cand,
                          int32_t* triples) {
  if (!ctx) return IMLOC_EINVAL;
  if (n < 0 || n > INT32_MAX || count < 0 || count > INT32_MAX || h0 < 0)
    return set_err(ctx, IMLOC_EINVAL, "bad sizes");
  if (n > 0 && !corr_ok(pts)) return set_err(ctx, IMLOC_EINVAL, "null correspondence array");
  const RigHost rig{n_cams, cams, cam_start};
  int rc = rig_check(ctx, rig, n);
  if (rc) return rc;
  if (!poses || !h_out || !j_out || !n_cand) return set_err(ctx, IMLOC_EINVAL, "null output");
  hipSetDevice(ctx->device);
  StageQuery sq;
  stage_setup(sq, n, 8 * std::max<int64_t>(count, 1), 1.0, 0, 0, 0, 1.0, 1, n_cams);
  sq.p.seed = seed;
  sq.p.query_id = query_id;
  sq.p.exhaustive = exhaustive;
  Arena a{ctx->ws, ctx->ws_bytes};
  carve_engine(a, sq.e);
  if (!a.ok) return set_err(ctx, IMLOC_ENOMEM, "workspace too small: need %zu bytes", a.off);
  sq.e.cb.pose = poses;
  sq.e.cb.h = h_out;
  sq.e.cb.j = j_out;
  sq.e.cb.n = n_cand;
  rc = stage_upload(ctx, sq, pts, n, nullptr, count, h0, nullptr, &rig);
  if (rc) return rc;
  HIP_TRY(ctx, launch_fill_i32(n_cand, 1, 0, ctx->stream));
  HIP_TRY(ctx, launch_sample_gp3p(sq.e.qd, sq.e.st, sq.e.cb, 1, count, triples, ctx->stream));
  return IMLOC_OK;
}

int imloc_rig_score(imloc_ctx* ctx, const imloc_corr* pts, int64_t n, const imloc_rig_camera* cams, int32_t n_cams,
                    const int64_t* cam_start, const double* poses, int64_t np, double tau, int32_t precision,
                    int32_t* count, double* msac) {
  if (!ctx) return IMLOC_EINVAL;
  if (n < 0 || n > INT32_MAX || np < 0 || np > INT32_MAX) return set_err(ctx, IMLOC_EINVAL, "bad sizes");
  if (n > 0 && !corr_ok(pts)) return set_err(ctx, IMLOC_EINVAL, "null correspondence array");
  const RigHost rig{n_cams, cams, cam_start};
  int rc = rig_check(ctx, rig, n);
  if (rc) return rc;
  if (!(tau > 0.0)) return set_err(ctx, IMLOC_EINVAL, "threshold must be > 0");
  if (precision != IMLOC_FP32_SCORE && precision != IMLOC_FP64_ALL) return set_err(ctx, IMLOC_EINVAL, "bad precision");
  if (np == 0) return IMLOC_OK;
  if (!poses || !count || !msac) return set_err(ctx, IMLOC_EINVAL, "null pose / output array");
  hipSetDevice(ctx->device);
  StageQuery sq;
  stage_setup(sq, n, np, tau, precision, 0, 0, 1.0, 1, n_cams);
  Arena a{ctx->ws, ctx->ws_bytes};
  carve_engine(a, sq.e);
  if (!a.ok) return set_err(ctx, IMLOC_ENOMEM, "workspace too small: need %zu bytes", a.off);
  rc = stage_upload(ctx, sq, pts, n, nullptr, 1, 0, nullptr, &rig);
  if (rc) return rc;
  hipStream_t s = ctx->stream;
  HIP_TRY(ctx, launch_set_candidates(sq.e.qd, poses, np, sq.e.cb, s));
  const std::pair<int64_t, int64_t> est1{np, est_points(sq.pl)};
  const ScoreTune tune = round_tune(ctx, &est1, 1);
  HIP_TRY(ctx, launch_worklist(sq.e.qd, sq.e.cb, 1, tune, sq.e.item_off, s));
  HIP_TRY(ctx, launch_score(sq.e.qd, sq.e.cb, sq.e.st, 1, sq.e.item_off, tune, precision, s));
  HIP_TRY(ctx, launch_candidate_costs(sq.e.qd, sq.e.st, sq.e.cb, np, count, msac, s));
  return IMLOC_OK;
}

int imloc_rig_lo_ransac_pnp(imloc_ctx* ctx, const imloc_corr* pts, int64_t n, const imloc_rig_camera* cams,
                            int32_t n_cams, const int64_t* cam_start, const imloc_ransac_params* p,
                            imloc_pose* pose_out, uint8_t* mask, imloc_stats* stats) {
  if (!ctx) return IMLOC_EINVAL;
  if (!pose_out) return set_err(ctx, IMLOC_EINVAL, "pose_out is null");
  if (!p) return set_err(ctx, IMLOC_EINVAL, "params is null");
  imloc_corr none{};
  int32_t status = 0;
  uint8_t* masks[1] = {mask};
  const RigHost rig{n_cams, cams, cam_start};
  imloc_camera unused{1.0, 1.0, 0.0, 0.0};
  int rc = run_batch(ctx, 1, pts ? pts : &none, &n, &unused, p, 1, pose_out, masks, stats, &status, &rig,
                     Scratch{ctx->ws, ctx->ws_bytes}, true);
  return rc < 0 ? rc : status;
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
  StageQuery sq;
  stage_setup(sq, n, np, tau, precision, 0, 0, 1.0, 1);
  Arena a{ctx->ws, ctx->ws_bytes};
  carve_engine(a, sq.e);
  if (!a.ok) return set_err(ctx, IMLOC_ENOMEM, "workspace too small: need %zu bytes", a.off);
  int rc = stage_upload(ctx, sq, pts, n, K, 1, 0, nullptr);
  if (rc) return rc;
  hipStream_t s = ctx->stream;
  HIP_TRY(ctx, launch_set_candidates(sq.e.qd, poses, np, sq.e.cb, s));
  const std::pair<int64_t, int64_t> est1{np, est_points(sq.pl)};
  const ScoreTune tune = round_tune(ctx, &est1, 1);
  HIP_TRY(ctx, launch_worklist(sq.e.qd, sq.e.cb, 1, tune, sq.e.item_off, s));
  HIP_TRY(ctx, launch_score(sq.e.qd, sq.e.cb, sq.e.st, 1, sq.e.item_off, tune, precision, s));
  HIP_TRY(ctx, launch_candidate_costs(sq.e.qd, sq.e.st, sq.e.cb, np, count, msac, s));
  return IMLOC_OK;
}

int imloc_select_top_k(imloc_ctx* ctx, const imloc_corr* pts, int64_t n, const imloc_camera* K, const double* poses,
                       int64_t np, double tau, int32_t precision, int32_t k, double gate, int32_t* sel,
                       int32_t* n_sel) {
  if (!ctx) return IMLOC_EINVAL;
  if (n < 0 || n > INT32_MAX || np < 0 || np > INT32_MAX) return set_err(ctx, IMLOC_EINVAL, "bad sizes");
  if (k < 1 || k > kMaxTopK) return set_err(ctx, IMLOC_EINVAL, "k must be in [1, %d]", kMaxTopK);
  if (std::isnan(gate)) return set_err(ctx, IMLOC_EINVAL, "gate is NaN");
  if (n > 0 && !corr_ok(pts)) return set_err(ctx, IMLOC_EINVAL, "null correspondence array");
  if (!cam_ok(K)) return set_err(ctx, IMLOC_EINVAL, "bad intrinsics");
  if (!(tau > 0.0)) return set_err(ctx, IMLOC_EINVAL, "threshold must be > 0");
  if (precision != IMLOC_FP32_SCORE && precision != IMLOC_FP64_ALL) return set_err(ctx, IMLOC_EINVAL, "bad precision");
  if (!sel || !n_sel || (np > 0 && !poses)) return set_err(ctx, IMLOC_EINVAL, "null pose / output array");
  hipSetDevice(ctx->device);
  StageQuery sq;
  stage_setup(sq, n, np, tau, precision, 0, 0, 1.0, 1);
  sq.pl.k = k;  // the query's k; the engine keeps one local optimisation slot (none runs here)
  Arena a{ctx->ws, ctx->ws_bytes};
  carve_engine(a, sq.e);
  if (!a.ok) return set_err(ctx, IMLOC_ENOMEM, "workspace too small: need %zu bytes", a.off);
  int rc = stage_upload(ctx, sq, pts, n, K, 1, 0, nullptr);
  if (rc) return rc;
  hipStream_t s = ctx->stream;
  if (!std::isinf(gate) || gate < 0.0) {  // the running best's cost (+inf after initialisation)
    double* hg = reinterpret_cast<double*>(ctx->pinned + 256 * ((sizeof(QueryDesc) + 255) / 256) + sizeof(BestState));
    *hg = gate;
    HIP_TRY(ctx, hipMemcpyAsync(&sq.e.st[0].cost, hg, sizeof(double), hipMemcpyHostToDevice, s));
  }
  HIP_TRY(ctx, launch_set_candidates(sq.e.qd, poses, np, sq.e.cb, s));
  const std::pair<int64_t, int64_t> est1{np, est_points(sq.pl)};
  const ScoreTune tune = round_tune(ctx, &est1, 1);
  HIP_TRY(ctx, launch_worklist(sq.e.qd, sq.e.cb, 1, tune, sq.e.item_off, s));
  HIP_TRY(ctx, launch_score(sq.e.qd, sq.e.cb, sq.e.st, 1, sq.e.item_off, tune, precision, s));
  HIP_TRY(ctx, launch_select(sq.e.qd, sq.e.st, sq.e.cb, 1, k, std::max<int64_t>(np, 1), sq.e.sel_part, sel, n_sel, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));  // the staging buffer held the gate
  return IMLOC_OK;
}

int imloc_local_optimize(imloc_ctx* ctx, const imloc_corr* pts, int64_t n, const imloc_camera* K, const double* start,
                         int32_t np, double tau, int32_t iters, double* out_poses, double* cost, int64_t* count) {
  if (!ctx) return IMLOC_EINVAL;
  if (n < 0 || n > INT32_MAX || np < 0 || np > 65535 || iters < 0 || iters > 1000)
    return set_err(ctx, IMLOC_EINVAL, "bad sizes");
  if (n > 0 && !corr_ok(pts)) return set_err(ctx, IMLOC_EINVAL, "null correspondence array");
  if (!cam_ok(K)) return set_err(ctx, IMLOC_EINVAL, "bad intrinsics");
  if (!(tau > 0.0)) return set_err(ctx, IMLOC_EINVAL, "threshold must be > 0");
  if (np == 0) return IMLOC_OK;
  if (!start || !out_poses || !cost) return set_err(ctx, IMLOC_EINVAL, "null pose / output array");
  hipSetDevice(ctx->device);
  StageQuery sq;
  stage_setup(sq, n, 1, tau, 0, iters, 0, 1.0, np);
  Arena a{ctx->ws, ctx->ws_bytes};
  carve_engine(a, sq.e);
  void* scratch = a.take<char>(gn_scratch_bytes(np, sq.e.chunks_lo));
  if (!a.ok) return set_err(ctx, IMLOC_ENOMEM, "workspace too small: need %zu bytes", a.off);
  int rc = stage_upload(ctx, sq, pts, n, K, 0, 0, nullptr);
  if (rc) return rc;
  HIP_TRY(ctx, launch_lo(sq.e.qd, sq.e.cb, nullptr, nullptr, start, np, 1, sq.e.chunks_lo, iters, scratch, out_poses,
                         cost, count, false, n > 0 && pts->w != nullptr, ctx->gn_mode, ctx->stream));
  return IMLOC_OK;
}

int imloc_refine(imloc_ctx* ctx, const imloc_corr* pts, int64_t n, const imloc_camera* K, const double* start,
                 double tau, double scale, int32_t iters, double* out_pose, double* cost, uint8_t* mask) {
  if (!ctx) return IMLOC_EINVAL;
  if (n < 0 || n > INT32_MAX || iters < 0 || iters > 1000) return set_err(ctx, IMLOC_EINVAL, "bad sizes");
  if (n > 0 && !corr_ok(pts)) return set_err(ctx, IMLOC_EINVAL, "null correspondence array");
  if (!cam_ok(K)) return set_err(ctx, IMLOC_EINVAL, "bad intrinsics");
  if (!(tau > 0.0) || !(scale > 0.0)) return set_err(ctx, IMLOC_EINVAL, "threshold and scale must be > 0");
  if (!start || !out_pose || !cost) return set_err(ctx, IMLOC_EINVAL, "null pose / output array");
  hipSetDevice(ctx->device);
  StageQuery sq;
  stage_setup(sq, n, 1, tau, 0, 0, iters, scale, 1);
  Arena a{ctx->ws, ctx->ws_bytes};
  carve_engine(a, sq.e);
  if (!a.ok) return set_err(ctx, IMLOC_ENOMEM, "workspace too small: need %zu bytes", a.off);
  int rc = stage_upload(ctx, sq, pts, n, K, 0, 0, mask);
  if (rc) return rc;
  HIP_TRY(ctx, launch_refine(sq.e.qd, sq.e.st, start, 1, sq.e.chunks_fin, iters, sq.e.in_set, sq.e.gn_fin, out_pose,
                             cost, false, ctx->gn_mode, false, nullptr, ctx->stream));
  if (mask) HIP_TRY(ctx, launch_mask(sq.e.qd, sq.e.st, out_pose, 1, n, 1, ctx->stream));
  return IMLOC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Serving: continuous batching over a resident slot table.
// ---------------------------------------------------------------------------
namespace {

// First-fit allocator over [0, cap) with coalescing of freed ranges.
struct RangePool {
  std::map<int64_t, int64_t> free_;  // offset -> length
  int64_t cap = 0, used = 0;
  void reset(int64_t c) {
    free_.clear();
    cap = c;
    used = 0;
    if (c > 0) free_[0] = c;
  }
  int64_t alloc(int64_t len) {
    if (len <= 0) return 0;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < len) continue;
      const int64_t off = it->first, rest = it->second - len;
      free_.erase(it);
      if (rest > 0) free_[off + len] = rest;
      used += len;
      return off;
    }
    return -1;
  }
  void release(int64_t off, int64_t len) {
    if (len <= 0) return;
    used -= len;
    auto it = free_.emplace(off, len).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

struct ServerQuery {
  int64_t ticket;
  imloc_corr pts;
  int64_t n;
  imloc_camera K;
  imloc_ransac_params p;
  uint8_t* mask;
};

struct ServerSlot {
  bool used = false;
  bool fresh = false;
  int64_t first_round = 0;  // the first round the query is part of
  ServerQuery q;
  QPlan pl;
  int64_t cand_off = 0, cand_len = 0, byte_off = 0, byte_len = 0;
};

struct Finished {
  int32_t status;
  imloc_pose pose;
  imloc_stats stats;
};

int64_t align256(int64_t x) { return (x + 255) & ~int64_t(255); }
// a query's share of a server's byte pool: its compacted in-set, then its
// gathered scoring subset
int64_t query_bytes(const QPlan& pl) {
  return align256(gn_inset_bytes(pl.n)) + (pl.subset ? align256(24 * pl.m) : 0);
}

}  // namespace

struct imloc_server {
  imloc_ctx* ctx;
  imloc_server_config cfg;
  Engine e;
  char* byte_pool;
  std::vector<ServerSlot> slots;
  std::deque<ServerQuery> queue;
  std::unordered_map<int64_t, Finished> done;
  RangePool cand_pool, bytes_pool;
  int64_t next_ticket = 0;
  int64_t rounds = 0;      // rounds enqueued so far
  // The round enqueued by the last step, still to be read back: its staging
  // half is (round & 1), its completion event ev[round & 1].
  bool inflight = false;
  int64_t inflight_round = 0;
  int inflight_nq = 0;
  hipEvent_t ev[2] = {nullptr, nullptr};
};

namespace {
// One half of a server's double-buffered staging: the slot table of a round,
// then the states, final poses and costs of every slot.
size_t server_half_bytes(int S) {
  return ((size_t)S * (sizeof(QueryDesc) + sizeof(BestState) + 13 * sizeof(double)) + 512 + 255) & ~size_t(255);
}
}  // namespace

namespace {

bool config_ok(const imloc_server_config* c) {
  return c && c->max_slots >= 1 && c->max_slots <= 4096 && c->max_top_k >= 1 && c->max_top_k <= kMaxTopK &&
         c->max_n >= 0 && c->max_n <= INT32_MAX && c->candidate_pool >= 4 && c->byte_pool >= 256;
}

// Slot-indexed engine of a server: candidate arrays sized by the candidate
// pool, in-set and subset bytes in one byte pool.
void server_engine(Engine& e, const imloc_server_config* c) {
  e.nq = c->max_slots;
  e.kmax = c->max_top_k;
  e.chunks_lo = gn_chunks(c->max_n);
  e.chunks_fin = gn_chunks(c->max_n);
  e.slots = c->candidate_pool;
  e.proj_floats = 16 * std::max<int64_t>(c->candidate_pool, 1);
  e.rig_doubles = 0;
  e.in_set_off.assign(1, 0);
  e.subset_off.assign(1, 0);
  e.proj_off.assign(1, 0);
  e.rig_off.assign(1, 0);
}

size_t server_carve(Arena& a, Engine& e, const imloc_server_config* c, char** byte_pool) {
  carve_engine(a, e);
  *byte_pool = a.take<char>((size_t)c->byte_pool);
  return a.off + 256;
}

}  // namespace

extern "C" {

size_t imloc_server_workspace_bytes(const imloc_server_config* cfg) {
  if (!config_ok(cfg)) return 0;
  Engine e;
  server_engine(e, cfg);
  Arena a{nullptr, (size_t)-1};
  char* bp;
  return server_carve(a, e, cfg, &bp);
}

int imloc_server_create(imloc_ctx* ctx, const imloc_server_config* cfg, imloc_server** out) {
  if (!ctx || !out) return IMLOC_EINVAL;
  *out = nullptr;
  if (!config_ok(cfg)) return set_err(ctx, IMLOC_EINVAL, "bad server configuration");
  imloc_server* srv = new imloc_server();
  srv->ctx = ctx;
  srv->cfg = *cfg;
  server_engine(srv->e, cfg);
  Arena a{ctx->ws, ctx->ws_bytes};
  server_carve(a, srv->e, cfg, &srv->byte_pool);
  if (!a.ok) {
    delete srv;
    return set_err(ctx, IMLOC_ENOMEM, "workspace too small for the server: need %zu bytes", a.off);
  }
  srv->slots.resize(cfg->max_slots);
  srv->cand_pool.reset(cfg->candidate_pool);
  srv->bytes_pool.reset(cfg->byte_pool);
  // every slot starts retired
  const size_t tab = (size_t)cfg->max_slots * sizeof(QueryDesc);
  int rc = staging_check(ctx, 2 * server_half_bytes(cfg->max_slots));
  if (!rc) rc = staging_wait(ctx);
  if (rc) {
    delete srv;
    return rc;
  }
  hipSetDevice(ctx->device);
  if (hipEventCreateWithFlags(&srv->ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&srv->ev[1], hipEventDisableTiming) != hipSuccess) {
    imloc_server_destroy(srv);
    return set_err(ctx, IMLOC_EHIP, "server event creation failed");
  }
  QueryDesc* htab = reinterpret_cast<QueryDesc*>(ctx->pinned);
  std::memset(htab, 0, tab);
  for (int q = 0; q < cfg->max_slots; ++q) htab[q].fresh = 1;
  hipStream_t s = ctx->stream;
  if (hipMemcpyAsync(srv->e.qd, htab, tab, hipMemcpyHostToDevice, s) != hipSuccess ||
      launch_init_queries(srv->e.qd, srv->e.st, srv->e.cb.n, cfg->max_slots, false, s) != hipSuccess ||
      launch_retire(srv->e.st, cfg->max_slots, s) != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
    imloc_server_destroy(srv);
    return set_err(ctx, IMLOC_EHIP, "server initialisation failed");
  }
  *out = srv;
  return IMLOC_OK;
}

void imloc_server_destroy(imloc_server* srv) {
  if (!srv) return;
  (void)hipStreamSynchronize(srv->ctx->stream);
  for (hipEvent_t e : srv->ev)
    if (e) (void)hipEventDestroy(e);
  delete srv;
}

int imloc_server_submit(imloc_server* srv, const imloc_corr* pts, int64_t n, const imloc_camera* K,
                        const imloc_ransac_params* p, uint8_t* mask, int64_t* ticket) {
  if (!srv || !ticket) return IMLOC_EINVAL;
  imloc_ctx* ctx = srv->ctx;
  int rc = check_params(ctx, p);
  if (rc) return rc;
  if (n < 0 || n > srv->cfg.max_n) return set_err(ctx, IMLOC_EINVAL, "n out of range for this server");
  if (n > 0 && !corr_ok(pts)) return set_err(ctx, IMLOC_EINVAL, "null correspondence array");
  if (!cam_ok(K)) return set_err(ctx, IMLOC_EINVAL, "bad intrinsics");
  if (p->lo_top_k > srv->cfg.max_top_k) return set_err(ctx, IMLOC_EINVAL, "lo_top_k above the server's maximum");
  const QPlan pl = plan_query(n, p);
  if (pl.cap > srv->cfg.candidate_pool || query_bytes(pl) > srv->cfg.byte_pool)
    return set_err(ctx, IMLOC_ENOMEM, "query larger than the server's pools");
  ServerQuery q;
  q.ticket = srv->next_ticket++;
  q.pts = n > 0 ? *pts : imloc_corr{};
  q.n = n;
  q.K = *K;
  q.p = *p;
  q.mask = mask;
  srv->queue.push_back(q);
  *ticket = q.ticket;
  return IMLOC_OK;
}

// Read back round r of a server (its staging half and event) and retire the
// queries that finished in it: slots admitted for a later round are left
// alone (their state in this read-back is the previous occupant's).
static int server_collect(imloc_server* srv, int64_t r, int nq, int64_t* done_tickets, int32_t capacity,
                          int32_t* ndone) {
  imloc_ctx* ctx = srv->ctx;
  const Engine& e = srv->e;
  const int S = srv->cfg.max_slots;
  int rcw = wait_event(ctx, srv->ev[r & 1]);
  if (rcw) return rcw;
  char* half = ctx->pinned + (size_t)(r & 1) * server_half_bytes(S);
  const size_t tab = (size_t)S * sizeof(QueryDesc);
  const BestState* hst = reinterpret_cast<const BestState*>(half + tab);
  const double* hfin = reinterpret_cast<const double*>(half + tab + (size_t)e.nq * sizeof(BestState));
  for (int i = 0; i < nq; ++i) {
    ServerSlot& sl = srv->slots[i];
    if (!sl.used || sl.first_round > r) continue;
    const BestState& b = hst[i];
    if (b.finished != 2) continue;
    Finished f;
    const bool have = b.have != 0;
    f.status = have ? IMLOC_OK : IMLOC_NO_POSE;
    identity_pose(&f.pose);
    if (have) {
      for (int x = 0; x < 9; ++x) f.pose.R[x] = hfin[12 * i + x];
      for (int x = 0; x < 3; ++x) f.pose.t[x] = hfin[12 * i + 9 + x];
    }
    std::memset(&f.stats, 0, sizeof(f.stats));
    f.stats.samples = b.drawn;
    f.stats.candidates = b.candidates;
    f.stats.residuals = b.candidates * sl.pl.m;
    f.stats.inlier_residuals = b.inlier_residuals;
    f.stats.best_count = have ? b.count : 0;
    f.stats.full_count = have ? b.full_count : 0;
    f.stats.batches = b.batches;
    f.stats.lo_runs = (int32_t)b.lo_runs;
    f.stats.status = f.status;
    f.stats.best_msac = have ? b.cost : 0.0;
    f.stats.final_cost = have ? hfin[12 * e.nq + i] : 0.0;
    f.stats.best_h = have ? b.h : -1;
    f.stats.best_j = have ? b.j : -1;
    f.stats.score_launches = (int32_t)b.batches;
    srv->done[sl.q.ticket] = f;
    if (done_tickets && *ndone < capacity) done_tickets[*ndone] = sl.q.ticket;
    ++*ndone;
    srv->cand_pool.release(sl.cand_off, sl.cand_len);
    srv->bytes_pool.release(sl.byte_off, sl.byte_len);
    sl.used = false;
  }
  return IMLOC_OK;
}

// One step: admit, enqueue round r for every resident query, then read back
// round r - 1 (enqueued by the previous step) while round r runs, so the
// host's work overlaps the device's.  A query that finished in round r - 1 is
// still in round r's table (retired on the device, so every kernel skips it)
// and its slot and pool ranges are freed here, for the next step's
// admission.  Round r stays in flight only while queries wait in the queue
// (then the next step's admission overlaps it); otherwise it is read back
// before the step returns.
int imloc_server_step(imloc_server* srv, int64_t* done_tickets, int32_t capacity, int32_t* n_done,
                      int32_t* n_resident, int32_t* n_queued) {
  if (!srv) return IMLOC_EINVAL;
  imloc_ctx* ctx = srv->ctx;
  Engine& e = srv->e;
  const int S = srv->cfg.max_slots;
  const int64_t r = srv->rounds;  // the round this step enqueues
  int32_t ndone = 0;
  // a previous round that has already completed is read back first, so that
  // its finished queries free their slots for this step's admission
  if (srv->inflight && hipEventQuery(srv->ev[srv->inflight_round & 1]) == hipSuccess) {
    const int rc = server_collect(srv, srv->inflight_round, srv->inflight_nq, done_tickets, capacity, &ndone);
    if (rc) return rc;
    srv->inflight = false;
  }
  // admission, first come first served: a slot and room in both pools
  while (!srv->queue.empty()) {
    const ServerQuery& q = srv->queue.front();
    int slot = -1;
    for (int i = 0; i < S; ++i)
      if (!srv->slots[i].used) { slot = i; break; }
    if (slot < 0) break;
    const QPlan pl = plan_query(q.n, &q.p);
    const int64_t co = srv->cand_pool.alloc(pl.cap);
    if (co < 0) break;
    const int64_t bl = query_bytes(pl);
    const int64_t bo = srv->bytes_pool.alloc(bl);
    if (bo < 0) {
      srv->cand_pool.release(co, pl.cap);
      break;
    }
    ServerSlot& sl = srv->slots[slot];
    sl.used = true;
    sl.fresh = true;
    sl.first_round = r;
    sl.q = q;
    sl.pl = pl;
    sl.cand_off = co;
    sl.cand_len = pl.cap;
    sl.byte_off = bo;
    sl.byte_len = bl;
    srv->queue.pop_front();
  }
  int nq = 0, kmax = 1, chunks_lo = 1, chunks_fin = 1, lo_iters = 0, fin_iters = 0;
  int64_t max_batch = 1, max_n = 0, max_m_sub = 0;
  bool any_w = false;  // a resident query with confidences: the weighted local optimisation
  EstList est;
  for (int i = 0; i < S; ++i) {
    const ServerSlot& sl = srv->slots[i];
    if (!sl.used) continue;
    any_w = any_w || (sl.q.n > 0 && sl.q.pts.w != nullptr);
    est.push_back({std::min(sl.pl.batch, sl.pl.total), est_points(sl.pl)});
    nq = i + 1;
    kmax = std::max(kmax, sl.pl.k);
    chunks_lo = std::max(chunks_lo, gn_chunks(sl.pl.m));
    chunks_fin = std::max(chunks_fin, gn_chunks(sl.pl.n));
    lo_iters = std::max(lo_iters, (int)sl.q.p.lo_iters);
    fin_iters = std::max(fin_iters, (int)sl.q.p.final_iters);
    max_batch = std::max(max_batch, sl.pl.batch);
    max_n = std::max(max_n, sl.pl.n);
    if (sl.pl.subset && sl.fresh) max_m_sub = std::max(max_m_sub, sl.pl.m);
  }
  if (nq > 0) {
    kmax = srv->cfg.max_top_k;  // problem index layout of the LO buffers
    const size_t tab = (size_t)nq * sizeof(QueryDesc);
    int rc = staging_check(ctx, 2 * server_half_bytes(S));
    if (rc) return rc;
    // the half of round r was last used by round r - 2, read back by the previous step
    char* half = ctx->pinned + (size_t)(r & 1) * server_half_bytes(S);
    QueryDesc* htab = reinterpret_cast<QueryDesc*>(half);
    for (int i = 0; i < nq; ++i) {
      ServerSlot& sl = srv->slots[i];
      if (!sl.used) {
        std::memset(&htab[i], 0, sizeof(QueryDesc));
        continue;
      }
      // per-slot view of the pools
      e.cand_off.assign(1, sl.cand_off);
      e.proj_off.assign(1, 16 * sl.cand_off);
      e.rig_off.assign(1, 0);
      e.in_set_off.assign(1, 0);
      e.subset_off.assign(1, 0);
      QueryDesc d = make_desc(&sl.q.pts, sl.q.n, &sl.q.K, &sl.q.p, sl.pl, e, 0, sl.q.mask);
      // the in-set bytes live in the byte pool, addressed relative to the in-set base
      d.in_set_off = (int64_t)((srv->byte_pool + sl.byte_off) - reinterpret_cast<char*>(e.in_set));
      if (sl.pl.subset) {
        const float* b = reinterpret_cast<const float*>(srv->byte_pool + sl.byte_off + align256(gn_inset_bytes(sl.pl.n)));
        const int64_t m = sl.pl.m;
        d.S = CorrF32{b, b + m, b + 2 * m, b + 3 * m, b + 4 * m, b + 5 * m};
      }
      d.fresh = sl.fresh ? 1 : 0;
      htab[i] = d;
      sl.fresh = false;
    }
    hipSetDevice(ctx->device);
    hipStream_t s = ctx->stream;
    HIP_TRY(ctx, hipMemcpyAsync(e.qd, htab, tab, hipMemcpyHostToDevice, s));
    HIP_TRY(ctx, launch_gather_subsets(e.qd, nq, max_m_sub, s));
    HIP_TRY(ctx, launch_init_queries(e.qd, e.st, e.cb.n, nq, false, s));
    HIP_TRY(ctx, launch_begin_round(e.qd, e.st, e.cb, nq, s));
    HIP_TRY(ctx, launch_sample_p3p(e.qd, e.st, e.cb, nq, max_batch, nullptr, s));
    const ScoreTune tune = round_tune(ctx, est.data(), est.size());
    HIP_TRY(ctx, launch_worklist(e.qd, e.cb, nq, tune, e.item_off, s));
    HIP_TRY(ctx, launch_score(e.qd, e.cb, e.st, nq, e.item_off, tune, 0, s));
    HIP_TRY(ctx, launch_select(e.qd, e.st, e.cb, nq, kmax, 4 * max_batch, e.sel_part, e.sel, e.n_sel, s));
    HIP_TRY(ctx, launch_lo(e.qd, e.cb, e.sel, e.n_sel, nullptr, nq * kmax, kmax, chunks_lo, lo_iters, e.gn_lo,
                           e.lo_pose, e.lo_cost, e.lo_count, false, any_w, ctx->gn_mode, s));
    HIP_TRY(ctx, launch_round_end(e.qd, e.cb, e.sel, e.n_sel, e.lo_pose, e.lo_cost, e.lo_count, nq, kmax, e.st,
                                  e.active_count, false, s));
    bool mask_done = false;  // the fused final refinement writes the masks itself
    HIP_TRY(ctx, launch_refine(e.qd, e.st, nullptr, nq, chunks_fin, fin_iters, e.in_set, e.gn_fin, e.fin_pose,
                               e.fin_cost, false, ctx->gn_mode, true, &mask_done, s));
    if (!mask_done) HIP_TRY(ctx, launch_mask(e.qd, e.st, e.fin_pose, nq, max_n, 0, s));
    HIP_TRY(ctx, launch_retire(e.st, nq, s));
    // the results block is laid out for all e.nq slots (the table may be shorter)
    HIP_TRY(ctx, hipMemcpyAsync(half + (size_t)S * sizeof(QueryDesc), e.st, result_bytes(e.nq),
                                hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipEventRecord(srv->ev[r & 1], s));
  }
  if (srv->inflight) {  // round r - 1 runs (or ran) ahead of round r: read it back now
    const int rc = server_collect(srv, srv->inflight_round, srv->inflight_nq, done_tickets, capacity, &ndone);
    if (rc) return rc;
    srv->inflight = false;
  }
  if (nq > 0) {
    srv->rounds = r + 1;
    if (srv->queue.empty()) {
      // nothing waits for admission, so there is no host work to overlap:
      // read round r back now (a query that finishes is reported at once
      // and no round is spent on it after it finished)
      const int rc = server_collect(srv, r, nq, done_tickets, capacity, &ndone);
      if (rc) return rc;
    } else {
      srv->inflight = true;
      srv->inflight_round = r;
      srv->inflight_nq = nq;
    }
  }
  int32_t resident = 0;
  for (int i = 0; i < S; ++i) resident += srv->slots[i].used ? 1 : 0;
  if (n_done) *n_done = ndone;
  if (n_resident) *n_resident = resident;
  if (n_queued) *n_queued = (int32_t)srv->queue.size();
  return IMLOC_OK;
}

int imloc_server_poll(imloc_server* srv, int64_t ticket, imloc_pose* pose, imloc_stats* stats) {
  if (!srv || !pose) return IMLOC_EINVAL;
  auto it = srv->done.find(ticket);
  if (it == srv->done.end()) {
    if (ticket < 0 || ticket >= srv->next_ticket) return set_err(srv->ctx, IMLOC_EINVAL, "unknown ticket");
    return IMLOC_PENDING;
  }
  *pose = it->second.pose;
  if (stats) *stats = it->second.stats;
  const int st = it->second.status;
  srv->done.erase(it);
  return st;
}

int imloc_server_usage(const imloc_server* srv, int64_t* candidate_slots_used, int64_t* bytes_used) {
  if (!srv || !candidate_slots_used || !bytes_used) return IMLOC_EINVAL;
  *candidate_slots_used = srv->cand_pool.used;
  *bytes_used = srv->bytes_pool.used;
  return IMLOC_OK;
}

}  // extern "C"
