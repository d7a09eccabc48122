"""MI355X pose-estimation hot path of ImLoc (arXiv 2601.04185, Sec. 3.3).

Thin ctypes binding of ``libimloc.so`` (C ABI in ``include/imloc.h``).  The
functions below carry the C names and only marshal arguments: every step of
lifting and LO-RANSAC PnP runs in the library's HIP kernels.  PyTorch supplies
device memory (tensors on ``cuda``) and the stream.

The library must be built first (``python -m paper_2601_04185_amd.build`` or
``__graft_entry__.build()``); importing the binding without it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libimloc.so")

IMLOC_OK = 0
IMLOC_NO_POSE = 1
IMLOC_PENDING = 2
IMLOC_EINVAL = -1
IMLOC_ENOMEM = -2
IMLOC_EHIP = -3
IMLOC_FP32_SCORE = 0
IMLOC_FP64_ALL = 1

EXPORTED = ["imloc_create", "imloc_destroy", "imloc_set_stream", "imloc_last_error", "imloc_set_workspace",
            "imloc_workspace_bytes", "imloc_batch_workspace_bytes", "imloc_score_workspace_bytes",
            "imloc_lift_workspace_bytes", "imloc_lo_workspace_bytes", "imloc_refine_workspace_bytes",
            "imloc_sample_workspace_bytes", "imloc_set_timing", "imloc_set_score_tuning", "imloc_get_score_tuning",
            "imloc_set_score_points", "imloc_get_score_points",
            "imloc_set_graphs", "imloc_graph_counters", "imloc_server_workspace_bytes", "imloc_server_create",
            "imloc_server_destroy", "imloc_server_submit", "imloc_server_step", "imloc_server_poll",
            "imloc_server_usage",
            "imloc_lift", "imloc_lift_log8", "imloc_depth_encode_log8", "imloc_triangulate_workspace_bytes",
            "imloc_triangulate_depth", "imloc_rig_workspace_bytes", "imloc_rig_lo_ransac_pnp",
            "imloc_rig_stage_workspace_bytes", "imloc_rig_sample_gp3p", "imloc_rig_score",
            "imloc_lo_ransac_pnp", "imloc_lo_ransac_pnp_batch", "imloc_sample_p3p", "imloc_score", "imloc_select_top_k",
            "imloc_local_optimize", "imloc_refine", "imloc_paper_params",
            "imloc_set_gn_mode", "imloc_staging_bytes", "imloc_set_staging", "imloc_get_staging",
            "imloc_lo_ransac_pnp_noalloc", "imloc_noalloc_max_bytes"]


class ImlocError(RuntimeError):
    pass


class Camera(C.Structure):
    _fields_ = [("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double)]


class Pose(C.Structure):
    _fields_ = [("R", C.c_double * 9), ("t", C.c_double * 3)]


class Corr(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("u", "v", "X", "Y", "Z", "w")]


class CorrOut(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("u", "v", "X", "Y", "Z", "w", "src")]


class Matches(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("q_u", "q_v", "db_u", "db_v", "conf", "view")]


class RansacParams(C.Structure):
    _fields_ = [("threshold_px", C.c_double), ("fixed_samples", C.c_int64), ("batch", C.c_int64),
                ("min_iters", C.c_int64), ("max_iters", C.c_int64), ("confidence", C.c_double),
                ("lo_top_k", C.c_int32), ("lo_iters", C.c_int32), ("max_score_points", C.c_int64),
                ("final_iters", C.c_int32), ("cauchy_scale_px", C.c_double), ("exhaustive", C.c_int32),
                ("precision", C.c_int32), ("seed", C.c_uint64), ("query_id", C.c_uint64)]


class Stats(C.Structure):
    _fields_ = [("samples", C.c_int64), ("candidates", C.c_int64), ("residuals", C.c_int64),
                ("inlier_residuals", C.c_int64), ("best_count", C.c_int64), ("full_count", C.c_int64),
                ("batches", C.c_int64), ("lo_runs", C.c_int32), ("status", C.c_int32), ("best_msac", C.c_double),
                ("final_cost", C.c_double), ("best_h", C.c_int64), ("best_j", C.c_int32),
                ("score_launches", C.c_int32), ("ms_sample", C.c_float), ("ms_score", C.c_float),
                ("ms_select", C.c_float), ("ms_lo", C.c_float), ("ms_refine", C.c_float), ("ms_total", C.c_float)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class ServerConfig(C.Structure):
    _fields_ = [("max_slots", C.c_int32), ("max_top_k", C.c_int32), ("max_n", C.c_int64),
                ("candidate_pool", C.c_int64), ("byte_pool", C.c_int64)]


_lib = None


def lib():
    """Load libimloc.so (fails loudly when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2601_04185_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dbl, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_uint64
        sig = {
            "imloc_create": ([C.POINTER(vp), C.c_int, vp], C.c_int),
            "imloc_destroy": ([vp], None),
            "imloc_set_stream": ([vp, vp], C.c_int),
            "imloc_last_error": ([vp], C.c_char_p),
            "imloc_set_workspace": ([vp, vp, C.c_size_t], C.c_int),
            "imloc_workspace_bytes": ([i64, vp], C.c_size_t),
            "imloc_batch_workspace_bytes": ([i32, vp, vp, i32], C.c_size_t),
            "imloc_sample_workspace_bytes": ([i64, i64], C.c_size_t),
            "imloc_set_score_tuning": ([vp, i32, i32], C.c_int),
            "imloc_set_graphs": ([vp, C.c_int], C.c_int),
            "imloc_graph_counters": ([vp, vp, vp], C.c_int),
            "imloc_server_workspace_bytes": ([vp], C.c_size_t),
            "imloc_server_create": ([vp, vp, C.POINTER(vp)], C.c_int),
            "imloc_server_destroy": ([vp], None),
            "imloc_server_submit": ([vp, vp, i64, vp, vp, vp, vp], C.c_int),
            "imloc_server_step": ([vp, vp, i32, vp, vp, vp], C.c_int),
            "imloc_server_poll": ([vp, i64, vp, vp], C.c_int),
            "imloc_server_usage": ([vp, vp, vp], C.c_int),
            "imloc_get_score_tuning": ([vp, vp, vp], C.c_int),
            "imloc_set_score_points": ([vp, i32], C.c_int),
            "imloc_get_score_points": ([vp, vp], C.c_int),
            "imloc_score_workspace_bytes": ([i64, i64, i32], C.c_size_t),
            "imloc_lift_workspace_bytes": ([i64, i32], C.c_size_t),
            "imloc_lo_workspace_bytes": ([i64, i32], C.c_size_t),
            "imloc_refine_workspace_bytes": ([i64], C.c_size_t),
            "imloc_set_timing": ([vp, C.c_int], C.c_int),
            "imloc_paper_params": ([dbl, vp], C.c_int),
            "imloc_set_gn_mode": ([vp, i32], C.c_int),
            "imloc_staging_bytes": ([i32, i32], C.c_size_t),
            "imloc_set_staging": ([vp, C.c_size_t], C.c_int),
            "imloc_get_staging": ([vp], C.c_size_t),
            "imloc_lo_ransac_pnp_noalloc": ([vp, vp, i64, vp, vp, vp, vp, vp], C.c_int),
            "imloc_noalloc_max_bytes": ([], C.c_size_t),
            "imloc_lift": ([vp, vp, i64, vp, i32, i32, i32, vp, vp, i32, C.c_float, vp, i64, vp], C.c_int),
            "imloc_lift_log8": ([vp, vp, i64, vp, i32, i32, i32, vp, vp, i32, C.c_float, vp, i64, vp], C.c_int),
            "imloc_depth_encode_log8": ([vp, vp, i64, vp], C.c_int),
            "imloc_triangulate_workspace_bytes": ([i32, i32, i32], C.c_size_t),
            "imloc_rig_workspace_bytes": ([i64, i32, vp], C.c_size_t),
            "imloc_rig_lo_ransac_pnp": ([vp, vp, i64, vp, i32, vp, vp, vp, vp, vp], C.c_int),
            "imloc_rig_stage_workspace_bytes": ([i64, i32, i64], C.c_size_t),
            "imloc_rig_sample_gp3p": ([vp, vp, i64, vp, i32, vp, u64, u64, i32, i64, i64, vp, vp, vp, vp, vp], C.c_int),
            "imloc_rig_score": ([vp, vp, i64, vp, i32, vp, vp, i64, C.c_double, i32, vp, vp], C.c_int),
            "imloc_triangulate_depth": ([vp, i32, i32, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp], C.c_int),
            "imloc_lo_ransac_pnp": ([vp, vp, i64, vp, vp, vp, vp, vp], C.c_int),
            "imloc_lo_ransac_pnp_batch": ([vp, vp, vp, vp, i32, vp, i32, vp, vp, vp, vp], C.c_int),
            "imloc_sample_p3p": ([vp, vp, i64, vp, u64, u64, i32, i64, i64, vp, vp, vp, vp, vp], C.c_int),
            "imloc_score": ([vp, vp, i64, vp, vp, i64, dbl, i32, vp, vp], C.c_int),
            "imloc_select_top_k": ([vp, vp, i64, vp, vp, i64, dbl, i32, i32, dbl, vp, vp], C.c_int),
            "imloc_local_optimize": ([vp, vp, i64, vp, vp, i32, dbl, i32, vp, vp, vp], C.c_int),
            "imloc_refine": ([vp, vp, i64, vp, vp, dbl, dbl, i32, vp, vp, vp], C.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _cam(K) -> Camera:
    return Camera(*[float(x) for x in K])


def make_params(threshold_px=4.0, fixed_samples=0, batch=1024, min_iters=1024, max_iters=100000, confidence=0.9999,
                lo_top_k=8, lo_iters=10, max_score_points=0, final_iters=10, cauchy_scale_px=None, exhaustive=0,
                precision=IMLOC_FP32_SCORE, seed=0, query_id=0) -> RansacParams:
    if cauchy_scale_px is None:
        cauchy_scale_px = 0.5 * threshold_px
    return RansacParams(float(threshold_px), int(fixed_samples), int(batch), int(min_iters), int(max_iters),
                        float(confidence), int(lo_top_k), int(lo_iters), int(max_score_points), int(final_iters),
                        float(cauchy_scale_px), int(exhaustive), int(precision), int(seed), int(query_id))


def paper_params(threshold_px=6.0, **overrides) -> RansacParams:
    """The LO-RANSAC settings of Sec. 3.3 "Pose Estimation" as filled in by
    imloc_paper_params (batches of 1,000, subsample 10,000, confidence
    1 - 1e-4, cap 100,000, top-1 local optimisation); keyword arguments
    override single fields afterwards."""
    p = RansacParams()
    rc = lib().imloc_paper_params(float(threshold_px), C.byref(p))
    if rc != IMLOC_OK:
        raise ImlocError(f"imloc_paper_params failed ({rc})")
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


class Context:
    """An imloc_ctx bound to a device and a torch stream, with a workspace
    tensor that grows on demand."""

    def __init__(self, device: int = 0, stream=None, timing: bool = False, graphs: bool = False):
        import torch
        self.torch = torch
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = C.c_void_p()
        rc = lib().imloc_create(C.byref(h), device, C.c_void_p(self.stream.cuda_stream))
        if rc != IMLOC_OK:
            raise ImlocError(f"imloc_create failed ({rc})")
        self.h = h
        self.ws = None
        lib().imloc_set_timing(self.h, 1 if timing else 0)
        lib().imloc_set_graphs(self.h, 1 if graphs else 0)

    def graph_counters(self):
        a, b = C.c_int64(), C.c_int64()
        self.check(lib().imloc_graph_counters(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def close(self):
        if getattr(self, "h", None):
            lib().imloc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def error(self) -> str:
        return lib().imloc_last_error(self.h).decode()

    def check(self, rc: int) -> int:
        if rc < 0:
            raise ImlocError(f"imloc error {rc}: {self.error()}")
        return rc

    def set_score_tuning(self, candidates_per_item: int, workgroups: int):
        self.check(lib().imloc_set_score_tuning(self.h, int(candidates_per_item), int(workgroups)))

    def set_gn_mode(self, mode: int):
        """Gauss-Newton launch form: 0 by size, 1 fused, 2 split (identical results)."""
        self.check(lib().imloc_set_gn_mode(self.h, int(mode)))

    def score_tuning(self):
        a, b = C.c_int32(), C.c_int32()
        self.check(lib().imloc_get_score_tuning(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def set_score_points(self, points_per_item: int):
        """Correspondences per float32 scoring work item (512, 1024, 2048, 4096; no result changes)."""
        self.check(lib().imloc_set_score_points(self.h, int(points_per_item)))

    def score_points(self) -> int:
        a = C.c_int32()
        self.check(lib().imloc_get_score_points(self.h, C.byref(a)))
        return a.value

    def ensure_staging(self, n_queries: int, n_rig_cameras: int = 0):
        """Grow the context's pinned host staging (a setup call, outside the
        query calls) so that a batch of n_queries fits."""
        need = lib().imloc_staging_bytes(int(n_queries), int(n_rig_cameras))
        if lib().imloc_get_staging(self.h) < need:
            self.check(lib().imloc_set_staging(self.h, need))

    def ensure_workspace(self, nbytes: int):
        if self.ws is None or self.ws.numel() < nbytes:
            self.ws = self.torch.empty(int(nbytes), dtype=self.torch.uint8, device=f"cuda:{self.device}")
            self.check(lib().imloc_set_workspace(self.h, C.c_void_p(self.ws.data_ptr()), self.ws.numel()))


def corr_struct(u, v, X, Y, Z, w=None) -> Corr:
    for t in (u, v, X, Y, Z) + ((w,) if w is not None else ()):
        assert t.is_cuda and t.dtype.is_floating_point and t.element_size() == 4 and t.is_contiguous()
    return Corr(*[t.data_ptr() for t in (u, v, X, Y, Z)], None if w is None else w.data_ptr())


def imloc_lo_ransac_pnp(ctx: Context, corr: dict, K, params: RansacParams, mask=None):
    """corr: dict of float32 cuda tensors u, v, X, Y, Z (and optional w).
    Returns (status, R (3x3), t (3,), stats dict)."""
    n = int(corr["u"].numel())
    cs = corr_struct(corr["u"], corr["v"], corr["X"], corr["Y"], corr["Z"], corr.get("w"))
    ctx.ensure_workspace(lib().imloc_workspace_bytes(n, C.byref(params)))
    pose = Pose()
    st = Stats()
    cam = _cam(K)
    rc = ctx.check(lib().imloc_lo_ransac_pnp(ctx.h, C.byref(cs), n, C.byref(cam), C.byref(params), C.byref(pose),
                                             _ptr(mask), C.byref(st)))
    R = np.array(pose.R[:], dtype=np.float64).reshape(3, 3)
    t = np.array(pose.t[:], dtype=np.float64)
    return rc, R, t, st.as_dict()


def imloc_lo_ransac_pnp_noalloc(ctx: Context, corr: dict, K, params: RansacParams, mask=None):
    """imloc_lo_ransac_pnp on the library's fixed device scratch (no workspace
    is set up: the call allocates nothing).  Same arguments and results."""
    n = int(corr["u"].numel())
    cs = corr_struct(corr["u"], corr["v"], corr["X"], corr["Y"], corr["Z"], corr.get("w"))
    pose = Pose()
    st = Stats()
    cam = _cam(K)
    rc = ctx.check(lib().imloc_lo_ransac_pnp_noalloc(ctx.h, C.byref(cs), n, C.byref(cam), C.byref(params),
                                                     C.byref(pose), _ptr(mask), C.byref(st)))
    R = np.array(pose.R[:], dtype=np.float64).reshape(3, 3)
    t = np.array(pose.t[:], dtype=np.float64)
    return rc, R, t, st.as_dict()


class BatchQueries:
    """The host-side descriptors of a batch of queries -- device pointers of
    every query's arrays, sizes, intrinsics and parameters -- validated and
    packed once, for callers that run the same device buffers repeatedly
    (their contents may change between calls).  imloc_lo_ransac_pnp_batch
    accepts it in place of the three lists; the library still builds, uploads
    and runs everything per call."""

    def __init__(self, corrs: list, Ks: list, params):
        self.nq = nq = len(corrs)
        self.corrs = corrs  # keeps the tensors alive
        self.ns = (C.c_int64 * nq)(*[int(c["u"].numel()) for c in corrs])
        self.cs = (Corr * nq)(*[corr_struct(c["u"], c["v"], c["X"], c["Y"], c["Z"], c.get("w")) for c in corrs])
        self.cams = (Camera * nq)(*[_cam(K) for K in Ks])
        plist = params if isinstance(params, (list, tuple)) else [params]
        self.np = len(plist)
        self.pa = (RansacParams * self.np)(*plist)
        self.ws_bytes = lib().imloc_batch_workspace_bytes(nq, self.ns, self.pa, self.np)


_STATS_DTYPE = None


def imloc_lo_ransac_pnp_batch(ctx: Context, corrs, Ks: list = None, params=None, masks=None, arrays=False):
    """corrs: list of dicts of float32 cuda tensors (with Ks and params: one
    RansacParams or a list), or a BatchQueries.  Returns (status list, list
    of (R, t), list of stats dicts); with arrays=True, (status (nq,) int32,
    poses (nq, 12) float64 -- R row-major, then t --, stats as a structured
    array with the fields of the stats dicts)."""
    global _STATS_DTYPE
    b = corrs if isinstance(corrs, BatchQueries) else BatchQueries(corrs, Ks, params)
    nq = b.nq
    ctx.ensure_workspace(b.ws_bytes)
    ctx.ensure_staging(nq)
    poses = (Pose * nq)()
    stats = (Stats * nq)()
    status = (C.c_int32 * nq)()
    mk = None
    if masks is not None:
        mk = (C.c_void_p * nq)(*[None if m is None else m.data_ptr() for m in masks])
    ctx.check(lib().imloc_lo_ransac_pnp_batch(ctx.h, b.cs, b.ns, b.cams, nq, b.pa, b.np, poses, mk, stats, status))
    if arrays:
        if _STATS_DTYPE is None:
            _STATS_DTYPE = np.ctypeslib.as_array((Stats * 1)()).dtype
        return (np.frombuffer(status, dtype=np.int32).copy(),
                np.frombuffer(poses, dtype=np.float64).reshape(nq, 12).copy(),
                np.frombuffer(stats, dtype=_STATS_DTYPE).copy())
    out = [(np.array(p.R[:]).reshape(3, 3), np.array(p.t[:])) for p in poses]
    return list(status), out, [s.as_dict() for s in stats]


class RigCamera(C.Structure):
    _fields_ = [("K", Camera), ("cam_from_rig", Pose)]


def rig_struct(rig):
    """rig: list of (K (fx, fy, cx, cy), cam_from_rig as 12 numbers R row-major, t)."""
    out = (RigCamera * len(rig))()
    for k, (K, T) in enumerate(rig):
        T = np.asarray(T, np.float64).reshape(12)
        out[k] = RigCamera(_cam(K), Pose((C.c_double * 9)(*T[:9]), (C.c_double * 3)(*T[9:])))
    return out


def _cam_start(cam_start):
    a = np.ascontiguousarray(np.asarray(cam_start, np.int64))
    return (C.c_int64 * len(a))(*a.tolist())


def imloc_rig_lo_ransac_pnp(ctx: Context, corr: dict, rig, cam_start, params: RansacParams, mask=None):
    """LO-RANSAC for a multi-camera rig query.  corr: dict of float32 cuda
    tensors grouped by camera (camera c owns [cam_start[c], cam_start[c+1])).
    Returns (status, R, t (rig_from_world), stats dict)."""
    n = int(corr["u"].numel())
    cs = corr_struct(corr["u"], corr["v"], corr["X"], corr["Y"], corr["Z"], corr.get("w"))
    cams = rig_struct(rig)
    starts = _cam_start(cam_start)
    ctx.ensure_workspace(lib().imloc_rig_workspace_bytes(n, len(rig), C.byref(params)))
    pose = Pose()
    st = Stats()
    rc = ctx.check(lib().imloc_rig_lo_ransac_pnp(ctx.h, C.byref(cs), n, cams, len(rig), starts, C.byref(params),
                                                 C.byref(pose), _ptr(mask), C.byref(st)))
    return rc, np.array(pose.R[:]).reshape(3, 3), np.array(pose.t[:]), st.as_dict()


def imloc_rig_sample_gp3p(ctx: Context, corr: dict, rig, cam_start, seed: int, query_id: int, h0: int, count: int,
                          exhaustive=0, want_triples=False):
    """-> dict of cuda tensors poses (nc, 12) float64 (rig_from_world), h (nc,), j (nc,) and triples."""
    torch = ctx.torch
    dev = corr["u"].device
    n = int(corr["u"].numel())
    cs = corr_struct(corr["u"], corr["v"], corr["X"], corr["Y"], corr["Z"], corr.get("w"))
    cap = 8 * max(count, 1)
    poses = torch.empty((cap, 12), dtype=torch.float64, device=dev)
    h = torch.empty(cap, dtype=torch.int64, device=dev)
    j = torch.empty(cap, dtype=torch.int32, device=dev)
    nc = torch.zeros(1, dtype=torch.int32, device=dev)
    tri = torch.empty((max(count, 1), 3), dtype=torch.int32, device=dev) if want_triples else None
    ctx.ensure_workspace(lib().imloc_rig_stage_workspace_bytes(n, len(rig), count))
    ctx.check(lib().imloc_rig_sample_gp3p(ctx.h, C.byref(cs), n, rig_struct(rig), len(rig), _cam_start(cam_start),
                                          seed, query_id, exhaustive, h0, count, _ptr(poses), _ptr(h), _ptr(j),
                                          _ptr(nc), _ptr(tri)))
    k = int(nc.item())
    out = dict(poses=poses[:k], h=h[:k], j=j[:k])
    if want_triples:
        out["triples"] = tri[:count]
    return out


def imloc_rig_score(ctx: Context, corr: dict, rig, cam_start, poses, threshold_px: float, precision=IMLOC_FP32_SCORE):
    """poses: cuda float64 (np, 12) rig_from_world -> (count int32, msac float64) cuda tensors."""
    torch = ctx.torch
    n = int(corr["u"].numel())
    npz = int(poses.shape[0])
    cs = corr_struct(corr["u"], corr["v"], corr["X"], corr["Y"], corr["Z"], corr.get("w"))
    cnt = torch.empty(max(npz, 1), dtype=torch.int32, device=poses.device)
    ms = torch.empty(max(npz, 1), dtype=torch.float64, device=poses.device)
    ctx.ensure_workspace(lib().imloc_rig_stage_workspace_bytes(n, len(rig), npz))
    ctx.check(lib().imloc_rig_score(ctx.h, C.byref(cs), n, rig_struct(rig), len(rig), _cam_start(cam_start),
                                    _ptr(poses.contiguous()), npz, float(threshold_px), int(precision), _ptr(cnt),
                                    _ptr(ms)))
    return cnt[:npz], ms[:npz]


def imloc_lift(ctx: Context, matches: dict, depth, cams, poses, subpixel=True, min_conf=0.05, capacity=None):
    """matches: dict of cuda tensors q_u, q_v, db_u, db_v, conf (float32), view (int32).
    depth: cuda float32 (K, H, W) depth maps, or cuda uint8 (K, H, W) 8-bit
    log-depth codes (imloc_lift_log8).  cams: (K, 4) host; poses: (K, 12) host.
    Returns dict of cuda tensors u, v, X, Y, Z, w (float32), src (int32) and n (int)."""
    torch = ctx.torch
    n = int(matches["q_u"].numel())
    cap = n if capacity is None else int(capacity)
    nv, H, W = depth.shape
    dev = depth.device
    if depth.dtype not in (torch.uint8, torch.float32) or not depth.is_contiguous():
        raise ValueError("depth must be contiguous float32 maps or uint8 code maps")
    # one allocation for the seven output arrays and the count (the library
    # always writes the count)
    c1 = (max(cap, 1) + 63) // 64 * 64  # each array 256-byte aligned
    buf = torch.empty(7 * c1 + 1, dtype=torch.float32, device=dev)
    out = {k: buf[i * c1:(i + 1) * c1] for i, k in enumerate(("u", "v", "X", "Y", "Z", "w"))}
    out["src"] = buf[6 * c1:7 * c1].view(torch.int32)
    n_out = buf[7 * c1:].view(torch.int32)
    m = Matches(*[matches[k].data_ptr() for k in ("q_u", "q_v", "db_u", "db_v", "conf", "view")])
    co = CorrOut(*[out[k].data_ptr() for k in ("u", "v", "X", "Y", "Z", "w", "src")])
    # Camera and Pose are rows of 4 and 12 doubles
    cams_a = np.ascontiguousarray(np.asarray(cams, np.float64).reshape(nv, 4))
    poses_a = np.ascontiguousarray(np.asarray(poses, np.float64).reshape(nv, 12))
    ctx.ensure_workspace(lib().imloc_lift_workspace_bytes(n, nv))
    fn = lib().imloc_lift_log8 if depth.dtype == torch.uint8 else lib().imloc_lift
    ctx.check(fn(ctx.h, C.byref(m), n, C.c_void_p(depth.data_ptr()), nv, H, W, cams_a.ctypes.data_as(C.c_void_p),
                 poses_a.ctypes.data_as(C.c_void_p), 1 if subpixel else 0, C.c_float(min_conf), C.byref(co), cap,
                 C.c_void_p(n_out.data_ptr())))
    k = int(n_out.item())
    res = {key: v[:min(k, cap)] for key, v in out.items()}
    res["n"] = k
    return res


def imloc_depth_encode_log8(ctx: Context, depth):
    """8-bit log-depth codes (cuda uint8, same shape) of cuda float32 depths."""
    torch = ctx.torch
    d = depth.contiguous()
    if d.dtype != torch.float32:
        raise ValueError("depth must be float32")
    codes = torch.empty(d.shape, dtype=torch.uint8, device=d.device)
    ctx.check(lib().imloc_depth_encode_log8(ctx.h, _ptr(d), d.numel(), _ptr(codes)))
    return codes


class DenseMatches(C.Structure):
    _fields_ = [("u", C.c_void_p), ("v", C.c_void_p), ("conf", C.c_void_p)]


class TriangulationParams(C.Structure):
    _fields_ = [("min_conf", C.c_double), ("angle_deg", C.c_double), ("min_inliers", C.c_int32),
                ("max_refine_iters", C.c_int32)]


def _pose12(T) -> Pose:
    T = np.asarray(T, np.float64).reshape(12)
    return Pose((C.c_double * 9)(*T[:9]), (C.c_double * 3)(*T[9:]))


def imloc_triangulate_depth(ctx: Context, K_map, T_map, K_views, T_views, mu, mv, conf, min_conf=0.05,
                            angle_deg=2.0, min_inliers=4, max_refine_iters=50, want_codes=False):
    """mu, mv, conf: cuda float32 (V, H, W) dense matches of the mapping image
    in its V covisible views.  K_*: (fx, fy, cx, cy); T_*: 12 numbers
    cam_from_world.  Returns dict of cuda tensors depth (H, W) float32,
    inliers (H, W) int32 and, if asked, codes (H, W) uint8."""
    torch = ctx.torch
    V, H, W = (int(x) for x in mu.shape)
    dev = mu.device
    depth = torch.empty((H, W), dtype=torch.float32, device=dev)
    inl = torch.empty((H, W), dtype=torch.int32, device=dev)
    codes = torch.empty((H, W), dtype=torch.uint8, device=dev) if want_codes else None
    Kv = np.asarray(K_views, np.float64).reshape(V, 4)
    Tv = np.asarray(T_views, np.float64).reshape(V, 12)
    cams = (Camera * V)(*[_cam(k) for k in Kv])
    poses = (Pose * V)(*[_pose12(t) for t in Tv])
    m = DenseMatches(mu.contiguous().data_ptr(), mv.contiguous().data_ptr(), conf.contiguous().data_ptr())
    prm = TriangulationParams(float(min_conf), float(angle_deg), int(min_inliers), int(max_refine_iters))
    ctx.ensure_workspace(lib().imloc_triangulate_workspace_bytes(H, W, V))
    k0 = _cam(K_map)
    t0 = _pose12(T_map)
    ctx.check(lib().imloc_triangulate_depth(ctx.h, H, W, C.byref(k0), C.byref(t0), V, cams, poses, C.byref(m),
                                            C.byref(prm), _ptr(depth), _ptr(inl), _ptr(codes)))
    out = dict(depth=depth, inliers=inl)
    if want_codes:
        out["codes"] = codes
    return out


def imloc_sample_p3p(ctx: Context, corr: dict, K, seed: int, query_id: int, h0: int, count: int, exhaustive=0,
                     want_triples=False):
    """-> dict of cuda tensors poses (nc, 12) float64, h (nc,), j (nc,), and triples (count, 3)."""
    torch = ctx.torch
    dev = corr["u"].device
    n = int(corr["u"].numel())
    cs = corr_struct(corr["u"], corr["v"], corr["X"], corr["Y"], corr["Z"], corr.get("w"))
    cap = 4 * max(count, 1)
    poses = torch.empty((cap, 12), dtype=torch.float64, device=dev)
    h = torch.empty(cap, dtype=torch.int64, device=dev)
    j = torch.empty(cap, dtype=torch.int32, device=dev)
    nc = torch.zeros(1, dtype=torch.int32, device=dev)
    tri = torch.empty((max(count, 1), 3), dtype=torch.int32, device=dev) if want_triples else None
    ctx.ensure_workspace(lib().imloc_sample_workspace_bytes(n, count))
    cam = _cam(K)
    ctx.check(lib().imloc_sample_p3p(ctx.h, C.byref(cs), n, C.byref(cam), seed, query_id, exhaustive, h0, count,
                                     _ptr(poses), _ptr(h), _ptr(j), _ptr(nc), _ptr(tri)))
    k = int(nc.item())
    out = dict(poses=poses[:k], h=h[:k], j=j[:k])
    if want_triples:
        out["triples"] = tri[:count]
    return out


def imloc_score(ctx: Context, corr: dict, K, poses, threshold_px: float, precision=IMLOC_FP32_SCORE):
    """poses: cuda float64 (np, 12).  -> (count int32 (np,), msac float64 (np,)) cuda tensors."""
    torch = ctx.torch
    n = int(corr["u"].numel())
    npz = int(poses.shape[0])
    cs = corr_struct(corr["u"], corr["v"], corr["X"], corr["Y"], corr["Z"], corr.get("w"))
    cnt = torch.empty(max(npz, 1), dtype=torch.int32, device=poses.device)
    ms = torch.empty(max(npz, 1), dtype=torch.float64, device=poses.device)
    ctx.ensure_workspace(lib().imloc_score_workspace_bytes(n, npz, int(precision)))
    cam = _cam(K)
    ctx.check(lib().imloc_score(ctx.h, C.byref(cs), n, C.byref(cam), _ptr(poses.contiguous()), npz, float(threshold_px),
                                int(precision), _ptr(cnt), _ptr(ms)))
    return cnt[:npz], ms[:npz]


def imloc_select_top_k(ctx: Context, corr: dict, K, poses, threshold_px: float, k: int, gate: float = float("inf"),
                       precision=IMLOC_FP32_SCORE):
    """poses: cuda float64 (np, 12).  Scores them as imloc_score does and
    returns the indices (cuda int32) of the k with the smallest truncated
    cost below gate, in order (ties: larger inlier count, then smaller index)."""
    torch = ctx.torch
    n = int(corr["u"].numel())
    npz = int(poses.shape[0])
    cs = corr_struct(corr["u"], corr["v"], corr["X"], corr["Y"], corr["Z"], corr.get("w"))
    sel = torch.full((max(int(k), 1),), -1, dtype=torch.int32, device=poses.device)
    nsel = torch.zeros(1, dtype=torch.int32, device=poses.device)
    ctx.ensure_workspace(lib().imloc_score_workspace_bytes(n, npz, int(precision)))
    cam = _cam(K)
    ctx.check(lib().imloc_select_top_k(ctx.h, C.byref(cs), n, C.byref(cam), _ptr(poses.contiguous()), npz,
                                       float(threshold_px), int(precision), int(k), float(gate), _ptr(sel), _ptr(nsel)))
    return sel[:int(nsel.item())]


def imloc_local_optimize(ctx: Context, corr: dict, K, start, threshold_px: float, iters: int = 10):
    """start: cuda float64 (np, 12) -> (poses (np, 12), cost (np,), count (np,))."""
    torch = ctx.torch
    n = int(corr["u"].numel())
    npz = int(start.shape[0])
    cs = corr_struct(corr["u"], corr["v"], corr["X"], corr["Y"], corr["Z"], corr.get("w"))
    out = torch.empty((max(npz, 1), 12), dtype=torch.float64, device=start.device)
    cost = torch.empty(max(npz, 1), dtype=torch.float64, device=start.device)
    cnt = torch.empty(max(npz, 1), dtype=torch.int64, device=start.device)
    ctx.ensure_workspace(lib().imloc_lo_workspace_bytes(n, npz))
    cam = _cam(K)
    ctx.check(lib().imloc_local_optimize(ctx.h, C.byref(cs), n, C.byref(cam), _ptr(start.contiguous()), npz,
                                         float(threshold_px), int(iters), _ptr(out), _ptr(cost), _ptr(cnt)))
    return out[:npz], cost[:npz], cnt[:npz]


def imloc_refine(ctx: Context, corr: dict, K, start, threshold_px: float, scale_px: float, iters: int = 10,
                 mask=None):
    """start: cuda float64 (12,) -> (pose (12,), cost (1,))."""
    torch = ctx.torch
    n = int(corr["u"].numel())
    cs = corr_struct(corr["u"], corr["v"], corr["X"], corr["Y"], corr["Z"], corr.get("w"))
    out = torch.empty(12, dtype=torch.float64, device=start.device)
    cost = torch.empty(1, dtype=torch.float64, device=start.device)
    ctx.ensure_workspace(lib().imloc_refine_workspace_bytes(n))
    cam = _cam(K)
    ctx.check(lib().imloc_refine(ctx.h, C.byref(cs), n, C.byref(cam), _ptr(start.contiguous()), float(threshold_px),
                                 float(scale_px), int(iters), _ptr(out), _ptr(cost), _ptr(mask)))
    return out, cost


def to_device(query_or_corr, device="cuda:0") -> dict:
    """Synthetic numpy correspondences (a synth.Query or dict) -> dict of cuda tensors."""
    import torch
    d = query_or_corr.corr() if hasattr(query_or_corr, "corr") else query_or_corr
    out = {}
    for k in ("u", "v", "X", "Y", "Z", "w"):
        a = d.get(k)
        out[k] = None if a is None else torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
    return out


class Server:
    """Continuous-batching front end of imloc_server_* on a context of its own.

    submit() queues a query (its tensors are kept alive until it finishes),
    step() admits what fits and runs one round for every resident query,
    poll() returns a finished query's result once."""

    def __init__(self, device: int = 0, max_slots: int = 64, max_top_k: int = 8, max_n: int = 200000,
                 candidate_pool: int | None = None, byte_pool: int | None = None, stream=None):
        self.ctx = Context(device, stream=stream)
        if candidate_pool is None:
            candidate_pool = max_slots * 4 * 1024
        if byte_pool is None:  # each query's refinement in-set: 1 KiB per 512 points and its count table
            byte_pool = max_slots * (1024 * ((max_n + 511) // 512) + 2 * ((max_n + 511) // 512) + 512)
        self.cfg = ServerConfig(int(max_slots), int(max_top_k), int(max_n), int(candidate_pool), int(byte_pool))
        nbytes = lib().imloc_server_workspace_bytes(C.byref(self.cfg))
        if nbytes == 0:
            raise ImlocError("bad server configuration")
        self.ctx.ensure_workspace(nbytes)
        self.ctx.ensure_staging(2 * max_slots + 2)  # two halves: one round in flight, one being built
        h = C.c_void_p()
        self.ctx.check(lib().imloc_server_create(self.ctx.h, C.byref(self.cfg), C.byref(h)))
        self.h = h
        self._keep = {}
        self._buf = (C.c_int64 * 4096)()

    def close(self):
        if getattr(self, "h", None):
            lib().imloc_server_destroy(self.h)
            self.h = None
        self.ctx.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, corr: dict, K, params: RansacParams, mask=None) -> int:
        n = int(corr["u"].numel())
        cs = corr_struct(corr["u"], corr["v"], corr["X"], corr["Y"], corr["Z"], corr.get("w"))
        cam = _cam(K)
        t = C.c_int64()
        self.ctx.check(lib().imloc_server_submit(self.h, C.byref(cs), n, C.byref(cam), C.byref(params), _ptr(mask),
                                                 C.byref(t)))
        self._keep[t.value] = (corr, mask)
        return t.value

    def step(self):
        """-> (finished tickets, resident, queued)."""
        nd, nr, nqd = C.c_int32(), C.c_int32(), C.c_int32()
        self.ctx.check(lib().imloc_server_step(self.h, self._buf, len(self._buf), C.byref(nd), C.byref(nr),
                                               C.byref(nqd)))
        done = [self._buf[i] for i in range(min(nd.value, len(self._buf)))]
        return done, nr.value, nqd.value

    def poll(self, ticket: int):
        """-> None while pending, else (status, R, t, stats)."""
        pose = Pose()
        st = Stats()
        rc = self.ctx.check(lib().imloc_server_poll(self.h, int(ticket), C.byref(pose), C.byref(st)))
        if rc == IMLOC_PENDING:
            return None
        self._keep.pop(ticket, None)
        return rc, np.array(pose.R[:]).reshape(3, 3), np.array(pose.t[:]), st.as_dict()

    def usage(self):
        a, b = C.c_int64(), C.c_int64()
        self.ctx.check(lib().imloc_server_usage(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value
