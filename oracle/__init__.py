"""FP64 CPU oracle of the ImLoc pose-estimation hot path (ctypes binding).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library (``paper_2601_04185_amd``) and never imports it.

The C source (``imloc_oracle.c``) holds the definitions; this module only
marshals numpy arrays.  Which passage of the paper each function follows is
stated in ``imloc_oracle.h``:
  lift              -- Sec. 3.3 "Query Time Matching and 2D-3D Lifting"
  sample / p3p      -- Sec. 3.3 "Pose Estimation" (minimal sets, P3P solver)
  score             -- Sec. 3.3 (truncated, confidence-weighted reprojection error)
  lo                -- Sec. 3.3 (Gauss-Newton on the truncated cost)
  required_samples  -- Sec. 3.3 (stop when P(missing the best model) is small)
  refine            -- Sec. 3.3 (final robust Cauchy refinement on all inliers)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (plain C11 + OpenMP)."""
    if force or not os.path.exists(_SO):
        srcs = [os.path.join(_HERE, f) for f in ("imloc_oracle.c", "triangulate.c", "rig.c")]
        tmp = _SO + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-std=gnu11", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
               "-Wno-unused-parameter", *srcs, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _SO)
    return _SO


class Camera(C.Structure):
    _fields_ = [("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double)]


class Corr(C.Structure):
    _fields_ = [("u", C.c_void_p), ("v", C.c_void_p), ("X", C.c_void_p), ("Y", C.c_void_p),
                ("Z", C.c_void_p), ("w", C.c_void_p), ("n", C.c_int64)]


class Params(C.Structure):
    _fields_ = [("threshold_px", C.c_double), ("fixed_samples", C.c_int64), ("batch", C.c_int64),
                ("min_iters", C.c_int64), ("max_iters", C.c_int64), ("confidence", C.c_double),
                ("lo_top_k", C.c_int32), ("lo_iters", C.c_int32), ("max_score_points", C.c_int64),
                ("final_iters", C.c_int32), ("cauchy_scale_px", C.c_double), ("exhaustive", C.c_int32),
                ("seed", C.c_uint64), ("query_id", C.c_uint64)]


class Stats(C.Structure):
    _fields_ = [("samples", C.c_int64), ("candidates", C.c_int64), ("residuals", C.c_int64),
                ("best_count", C.c_int64), ("full_count", C.c_int64), ("batches", C.c_int64),
                ("lo_runs", C.c_int32), ("status", C.c_int32), ("best_msac", C.c_double),
                ("final_cost", C.c_double), ("best_h", C.c_int64), ("best_j", C.c_int32)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        L = C.CDLL(_SO)
        vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
        L.orc_philox4x64_10.argtypes = [vp, vp, vp]
        L.orc_sample_triple.argtypes = [C.c_uint64, C.c_uint64, C.c_uint64, i64, vp]
        L.orc_sample_triple.restype = C.c_int
        L.orc_unrank_triple.argtypes = [C.c_uint64, i64, vp]
        L.orc_unrank_triple.restype = C.c_int
        L.orc_p3p.argtypes = [vp, vp, vp, vp, vp]
        L.orc_p3p.restype = C.c_int
        L.orc_score.argtypes = [vp, i64, vp, vp, dbl, vp, vp]
        L.orc_score_band.argtypes = [vp, i64, vp, vp, dbl, dbl, i32, vp, vp, vp]
        L.orc_residual_band.argtypes = [vp, vp, vp, dbl, dbl, i32, vp, vp]
        L.orc_lo.argtypes = [vp, vp, vp, dbl, i32, vp, vp, vp]
        L.orc_lo.restype = C.c_int
        L.orc_refine.argtypes = [vp, vp, vp, dbl, dbl, i32, vp, vp, vp]
        L.orc_refine.restype = C.c_int
        L.orc_required_samples.argtypes = [dbl, dbl, i64]
        L.orc_required_samples.restype = i64
        L.orc_lo_ransac_pnp.argtypes = [vp, vp, vp, vp, vp, vp]
        L.orc_lo_ransac_pnp.restype = C.c_int
        L.orc_lift.argtypes = [vp, vp, vp, vp, vp, vp, i64, i32, vp, i32, i32, i32, vp, vp, C.c_float,
                               vp, vp, vp, vp, vp, vp, vp]
        L.orc_lift.restype = i64
        L.orc_lift_log8.argtypes = L.orc_lift.argtypes
        L.orc_lift_log8.restype = i64
        L.orc_log8_decode.argtypes = [C.c_uint8]
        L.orc_log8_decode.restype = dbl
        L.orc_log8_encode.argtypes = [C.c_float]
        L.orc_log8_encode.restype = C.c_uint8
        L.orc_log8_encode_array.argtypes = [vp, i64, vp]
        L.orc_gp3p.argtypes = [vp, vp, vp, vp, vp, vp]
        L.orc_gp3p.restype = C.c_int
        L.orc_rig_score.argtypes = [vp, i64, vp, vp, dbl, vp, vp]
        L.orc_rig_lo.argtypes = [vp, vp, vp, dbl, i32, vp, vp, vp]
        L.orc_rig_lo.restype = C.c_int
        L.orc_rig_refine.argtypes = [vp, vp, vp, dbl, dbl, i32, vp, vp, vp]
        L.orc_rig_refine.restype = C.c_int
        L.orc_rig_lo_ransac.argtypes = [vp, vp, i32, vp, vp, vp, vp]
        L.orc_rig_lo_ransac.restype = C.c_int
        L.orc_triangulate.argtypes = [i32, i32, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.orc_tri_angle.argtypes = [vp, vp, dbl, vp, vp]
        L.orc_tri_angle.restype = dbl
        L.orc_tri_hypothesis.argtypes = [vp, vp, vp, vp, vp]
        L.orc_tri_hypothesis.restype = C.c_int
        L.orc_tri_refine.argtypes = [vp, vp, dbl, C.c_int, vp, vp, vp, C.c_int]
        L.orc_tri_refine.restype = dbl
        L.orc_normal_equations.argtypes = [vp, vp, vp, dbl, vp, vp, vp]
        L.orc_normal_equations.restype = dbl
        L.orc_pose_update.argtypes = [vp, vp, vp]
        L.orc_set_threads.argtypes = [i32]
        L.orc_max_threads.restype = i32
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _cam(K) -> Camera:
    fx, fy, cx, cy = [float(x) for x in K]
    return Camera(fx, fy, cx, cy)


def pose_array(R, t) -> np.ndarray:
    """(R, t) -> the 12-double layout of orc_pose (R row-major, then t)."""
    return np.concatenate([np.asarray(R, np.float64).reshape(9), np.asarray(t, np.float64).reshape(3)])


def split_pose(a):
    a = np.asarray(a, np.float64)
    return a[:9].reshape(3, 3).copy(), a[9:12].copy()


class _CorrHold:
    """Keeps float32 SoA copies alive while the C side reads them."""

    def __init__(self, corr):
        self.arrs = {}
        for k in ("u", "v", "X", "Y", "Z"):
            self.arrs[k] = np.ascontiguousarray(corr[k], dtype=np.float32)
        w = corr.get("w")
        self.arrs["w"] = None if w is None else np.ascontiguousarray(w, dtype=np.float32)
        n = self.arrs["u"].shape[0]
        self.c = Corr(*[self.arrs[k].ctypes.data for k in ("u", "v", "X", "Y", "Z")],
                      None if self.arrs["w"] is None else self.arrs["w"].ctypes.data, n)


def philox(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, np.uint64)
    k = np.asarray(key, np.uint64)
    o = np.zeros(4, np.uint64)
    lib().orc_philox4x64_10(_p(c), _p(k), _p(o))
    return o


def sample_triple(seed: int, query_id: int, h: int, n: int):
    idx = np.zeros(3, np.int32)
    ok = lib().orc_sample_triple(seed, query_id, h, n, _p(idx))
    return bool(ok), idx


def unrank_triple(h: int, n: int):
    idx = np.zeros(3, np.int32)
    ok = lib().orc_unrank_triple(h, n, _p(idx))
    return bool(ok), idx


def p3p(uv, Xw, K):
    """uv: (3,2) pixels, Xw: (3,3) world points -> (list of (R, t), ill flag)."""
    uv = np.ascontiguousarray(uv, np.float64).reshape(6)
    Xw = np.ascontiguousarray(Xw, np.float64).reshape(9)
    out = np.zeros((4, 12), np.float64)
    ill = np.zeros(1, np.int32)
    cam = _cam(K)
    ns = lib().orc_p3p(_p(uv), _p(Xw), C.byref(cam), _p(out), _p(ill))
    return [split_pose(out[k]) for k in range(ns)], bool(ill[0])


def _poses(poses) -> np.ndarray:
    if isinstance(poses, np.ndarray) and poses.ndim == 2 and poses.shape[1] == 12:
        return np.ascontiguousarray(poses, np.float64)
    return np.ascontiguousarray(np.stack([pose_array(R, t) for R, t in poses]), np.float64)


def score(poses, corr, K, tau):
    P = _poses(poses)
    h = _CorrHold(corr)
    cnt = np.zeros(P.shape[0], np.int32)
    ms = np.zeros(P.shape[0], np.float64)
    cam = _cam(K)
    lib().orc_score(_p(P), P.shape[0], C.byref(h.c), C.byref(cam), float(tau), _p(cnt), _p(ms))
    return cnt, ms


def score_band(poses, corr, K, tau, band_abs=1e-5, with_f32=True):
    P = _poses(poses)
    h = _CorrHold(corr)
    lo = np.zeros(P.shape[0], np.int32)
    hi = np.zeros(P.shape[0], np.int32)
    eb = np.zeros(P.shape[0], np.float64)
    cam = _cam(K)
    lib().orc_score_band(_p(P), P.shape[0], C.byref(h.c), C.byref(cam), float(tau), float(band_abs),
                         1 if with_f32 else 0, _p(lo), _p(hi), _p(eb))
    return lo, hi, eb


def residual_band(pose, corr, K, tau, band_abs=1e-5, with_f32=True):
    """-> (r, beta) per residual at one pose: exact pixel distance (NaN behind
    the camera or on its plane within float32 resolution) and the ambiguity
    band that score_band applies (inf where unbounded)."""
    P = _poses([pose])
    h = _CorrHold(corr)
    n = h.c.n
    r = np.zeros(max(n, 1), np.float64)
    beta = np.zeros(max(n, 1), np.float64)
    cam = _cam(K)
    lib().orc_residual_band(_p(P), C.byref(h.c), C.byref(cam), float(tau), float(band_abs), 1 if with_f32 else 0,
                            _p(r), _p(beta))
    return r[:n], beta[:n]


def lo(start, corr, K, tau, iters=10):
    s = pose_array(*start) if isinstance(start, tuple) else np.asarray(start, np.float64)
    out = np.zeros(12, np.float64)
    cost = np.zeros(1, np.float64)
    cnt = np.zeros(1, np.int64)
    h = _CorrHold(corr)
    cam = _cam(K)
    acc = lib().orc_lo(_p(s), C.byref(h.c), C.byref(cam), float(tau), int(iters), _p(out), _p(cost), _p(cnt))
    R, t = split_pose(out)
    return R, t, float(cost[0]), int(cnt[0]), int(acc)


def normal_equations(pose, corr, K, tau):
    """-> (cost, H (6,6), g (6,), inlier count) at the pose."""
    s = pose_array(*pose) if isinstance(pose, tuple) else np.asarray(pose, np.float64)
    H = np.zeros(36, np.float64)
    g = np.zeros(6, np.float64)
    cnt = np.zeros(1, np.int64)
    h = _CorrHold(corr)
    cam = _cam(K)
    cost = lib().orc_normal_equations(_p(s), C.byref(h.c), C.byref(cam), float(tau), _p(H), _p(g), _p(cnt))
    return float(cost), H.reshape(6, 6), g, int(cnt[0])


def pose_update(pose, d):
    s = pose_array(*pose) if isinstance(pose, tuple) else np.asarray(pose, np.float64)
    dd = np.ascontiguousarray(d, np.float64)
    out = np.zeros(12, np.float64)
    lib().orc_pose_update(_p(s), _p(dd), _p(out))
    return split_pose(out)


def refine(start, corr, K, tau, s, iters=10):
    st = pose_array(*start) if isinstance(start, tuple) else np.asarray(start, np.float64)
    out = np.zeros(12, np.float64)
    cost = np.zeros(1, np.float64)
    ninl = np.zeros(1, np.int64)
    h = _CorrHold(corr)
    cam = _cam(K)
    acc = lib().orc_refine(_p(st), C.byref(h.c), C.byref(cam), float(tau), float(s), int(iters), _p(out),
                           _p(cost), _p(ninl))
    R, t = split_pose(out)
    return R, t, float(cost[0]), int(ninl[0]), int(acc)


def required_samples(eps: float, confidence: float, max_iters: int = 100000) -> int:
    return int(lib().orc_required_samples(float(eps), float(confidence), int(max_iters)))


DEFAULT_PARAMS = dict(threshold_px=4.0, fixed_samples=0, batch=1024, min_iters=1024, max_iters=100000,
                      confidence=0.9999, lo_top_k=8, lo_iters=10, max_score_points=0, final_iters=10,
                      cauchy_scale_px=None, exhaustive=0, seed=0, query_id=0)


def make_params(**kw) -> Params:
    d = dict(DEFAULT_PARAMS)
    d.update(kw)
    if d["cauchy_scale_px"] is None:
        d["cauchy_scale_px"] = 0.5 * d["threshold_px"]
    return Params(float(d["threshold_px"]), int(d["fixed_samples"]), int(d["batch"]), int(d["min_iters"]),
                  int(d["max_iters"]), float(d["confidence"]), int(d["lo_top_k"]), int(d["lo_iters"]),
                  int(d["max_score_points"]), int(d["final_iters"]), float(d["cauchy_scale_px"]),
                  int(d["exhaustive"]), int(d["seed"]), int(d["query_id"]))


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops (results do not depend on it)."""
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def lo_ransac_pnp(corr, K, **params):
    """Whole LO-RANSAC PnP for one query -> dict(R, t, mask, stats...)."""
    h = _CorrHold(corr)
    n = h.c.n
    cam = _cam(K)
    prm = make_params(**params)
    pose = np.zeros(12, np.float64)
    mask = np.zeros(max(n, 1), np.uint8)
    st = Stats()
    status = lib().orc_lo_ransac_pnp(C.byref(h.c), C.byref(cam), C.byref(prm), _p(pose), _p(mask), C.byref(st))
    R, t = split_pose(pose)
    out = dict(R=R, t=t, mask=mask[:n].copy(), status=int(status))
    for f, _ in Stats._fields_:
        out[f] = getattr(st, f)
    return out


def lift(matches, depth, cams, poses, min_conf=0.05, subpixel=True):
    """matches: dict q_u, q_v, db_u, db_v, conf (float32), view (int32).
    depth: (K, H, W) float32 depth maps, or uint8 8-bit log-depth codes.
    cams: (K, 4).  poses: (K, 12) cam_from_world."""
    f32 = lambda a: np.ascontiguousarray(a, np.float32)
    qu, qv, du, dv, cf = (f32(matches[k]) for k in ("q_u", "q_v", "db_u", "db_v", "conf"))
    vw = np.ascontiguousarray(matches["view"], np.int32)
    codes = np.asarray(depth).dtype == np.uint8
    D = np.ascontiguousarray(depth, np.uint8) if codes else f32(depth)
    nv, H, W = D.shape
    cams_a = np.ascontiguousarray(np.asarray(cams, np.float64).reshape(nv, 4))
    poses_a = np.ascontiguousarray(np.asarray(poses, np.float64).reshape(nv, 12))
    n = qu.shape[0]
    outs = [np.zeros(max(n, 1), np.float64) for _ in range(6)]
    src = np.zeros(max(n, 1), np.int64)
    fn = lib().orc_lift_log8 if codes else lib().orc_lift
    cnt = fn(_p(qu), _p(qv), _p(du), _p(dv), _p(cf), _p(vw), n, 1 if subpixel else 0, _p(D), nv, H, W,
             _p(cams_a), _p(poses_a), C.c_float(np.float32(min_conf)), *[_p(o) for o in outs], _p(src))
    names = ("u", "v", "X", "Y", "Z", "w")
    res = {k: o[:cnt].copy() for k, o in zip(names, outs)}
    res["src"] = src[:cnt].copy()
    return res


def log8_decode(code: int) -> float:
    """Depth level of an 8-bit log-depth code (0: no depth)."""
    return float(lib().orc_log8_decode(int(code)))


def log8_encode(depth) -> np.ndarray:
    """8-bit log-depth codes of float32 depths (any shape)."""
    d = np.ascontiguousarray(depth, np.float32)
    out = np.zeros(d.shape, np.uint8)
    lib().orc_log8_encode_array(_p(d), d.size, _p(out))
    return out


class TriParams(C.Structure):
    _fields_ = [("min_conf", C.c_double), ("angle_deg", C.c_double), ("min_inliers", C.c_int32),
                ("max_refine_iters", C.c_int32)]


def _tri_cams(Ks):
    Ks = np.asarray(Ks, np.float64).reshape(-1, 4)
    return (Camera * len(Ks))(*[Camera(*map(float, k)) for k in Ks])


def _tri_poses(Ts):
    Ts = np.ascontiguousarray(np.asarray(Ts, np.float64).reshape(-1, 12))
    return Ts


def triangulate(K0, T0, Ks, Ts, mu, mv, conf, min_conf=0.05, angle_deg=2.0, min_inliers=4, max_refine_iters=50):
    """Depth of every pixel of a mapping image (H x W) from dense matches
    mu, mv, conf of shape (V, H, W).  T0, Ts: cam_from_world as 12 numbers
    (R row-major, t).  Returns dict depth (H, W) float64, inliers, best_view,
    ambiguous."""
    mu = np.ascontiguousarray(mu, np.float32)
    mv = np.ascontiguousarray(mv, np.float32)
    cf = np.ascontiguousarray(conf, np.float32)
    V, H, W = mu.shape
    depth = np.zeros((H, W), np.float64)
    inl = np.zeros((H, W), np.int32)
    bv = np.zeros((H, W), np.int32)
    amb = np.zeros((H, W), np.uint8)
    cost = np.zeros((H, W), np.float64)
    curv = np.zeros((H, W), np.float64)
    T0a = _tri_poses(T0)
    Tsa = _tri_poses(Ts)
    prm = TriParams(float(min_conf), float(angle_deg), int(min_inliers), int(max_refine_iters))
    lib().orc_triangulate(H, W, _tri_cams([K0]), _p(T0a), V, _tri_cams(Ks), _p(Tsa), _p(mu), _p(mv), _p(cf),
                          C.byref(prm), _p(depth), _p(inl), _p(bv), _p(amb), _p(cost), _p(curv))
    return dict(depth=depth, inliers=inl, best_view=bv, ambiguous=amb.astype(bool), cost=cost, curv=curv)


def tri_angle(C0, r0, l, Ck, rk) -> float:
    a = [np.ascontiguousarray(x, np.float64) for x in (C0, r0, Ck, rk)]
    return float(lib().orc_tri_angle(_p(a[0]), _p(a[1]), float(l), _p(a[2]), _p(a[3])))


def tri_hypothesis(C0, r0, Ck, rk):
    a = [np.ascontiguousarray(x, np.float64) for x in (C0, r0, Ck, rk)]
    out = np.zeros(1)
    ok = lib().orc_tri_hypothesis(_p(a[0]), _p(a[1]), _p(a[2]), _p(a[3]), _p(out))
    return float(out[0]) if ok else None


def tri_refine(C0, r0, l0, Ck, rk, w, max_iters=50) -> float:
    Ck = np.ascontiguousarray(Ck, np.float64).reshape(-1, 3)
    rk = np.ascontiguousarray(rk, np.float64).reshape(-1, 3)
    w = np.ascontiguousarray(w, np.float64)
    C0 = np.ascontiguousarray(C0, np.float64)
    r0 = np.ascontiguousarray(r0, np.float64)
    return float(lib().orc_tri_refine(_p(C0), _p(r0), float(l0), len(w), _p(Ck), _p(rk), _p(w), int(max_iters)))


class RigCamera(C.Structure):
    _fields_ = [("K", Camera), ("R", C.c_double * 9), ("t", C.c_double * 3)]


class RigCorr(C.Structure):
    _fields_ = [("u", C.c_void_p), ("v", C.c_void_p), ("X", C.c_void_p), ("Y", C.c_void_p), ("Z", C.c_void_p),
                ("w", C.c_void_p), ("cam", C.c_void_p), ("n", C.c_int64)]


def _rig_cams(rig):
    """rig: sequence of (K (4,), cam_from_rig (12,))."""
    out = (RigCamera * len(rig))()
    for k, (K, T) in enumerate(rig):
        T = np.asarray(T, np.float64).reshape(12)
        out[k] = RigCamera(Camera(*map(float, K)), (C.c_double * 9)(*T[:9]), (C.c_double * 3)(*T[9:]))
    return out


class _RigCorrHold(_CorrHold):
    def __init__(self, corr):
        super().__init__(corr)
        self.cam = np.ascontiguousarray(corr["cam"], np.int32)
        a = self.arrs
        self.rc = RigCorr(*[a[k].ctypes.data for k in ("u", "v", "X", "Y", "Z")],
                          None if a["w"] is None else a["w"].ctypes.data, self.cam.ctypes.data, self.c.n)


def gp3p(o, f, Xw):
    """Generalised P3P: rays (origins o (3, 3), directions f (3, 3)) in the rig
    frame through world points Xw (3, 3).  -> (list of (R, t) rig_from_world,
    depths (k, 3), ill)."""
    o = np.ascontiguousarray(o, np.float64).reshape(9)
    f = np.ascontiguousarray(f, np.float64).reshape(9)
    X = np.ascontiguousarray(Xw, np.float64).reshape(9)
    out = np.zeros((8, 12))
    dep = np.zeros((8, 3))
    ill = np.zeros(1, np.int32)
    n = lib().orc_gp3p(_p(o), _p(f), _p(X), _p(out), _p(dep), _p(ill))
    return [split_pose(out[k]) for k in range(n)], dep[:n].copy(), bool(ill[0])


def rig_score(poses, corr, rig, tau):
    P = _poses(poses)
    h = _RigCorrHold(corr)
    cams = _rig_cams(rig)
    cnt = np.zeros(max(len(P), 1), np.int32)
    ms = np.zeros(max(len(P), 1), np.float64)
    lib().orc_rig_score(_p(P), len(P), C.byref(h.rc), cams, float(tau), _p(cnt), _p(ms))
    return cnt[:len(P)], ms[:len(P)]


def rig_lo(start, corr, rig, tau, iters=10):
    s = np.ascontiguousarray(start, np.float64).reshape(12)
    h = _RigCorrHold(corr)
    out = np.zeros(12)
    cost = np.zeros(1)
    cnt = np.zeros(1, np.int64)
    acc = lib().orc_rig_lo(_p(s), C.byref(h.rc), _rig_cams(rig), float(tau), int(iters), _p(out), _p(cost), _p(cnt))
    return dict(pose=out, cost=float(cost[0]), count=int(cnt[0]), accepted=int(acc))


def rig_refine(start, corr, rig, tau, s=None, iters=10):
    st = np.ascontiguousarray(start, np.float64).reshape(12)
    h = _RigCorrHold(corr)
    out = np.zeros(12)
    cost = np.zeros(1)
    ni = np.zeros(1, np.int64)
    s = 0.5 * tau if s is None else s
    acc = lib().orc_rig_refine(_p(st), C.byref(h.rc), _rig_cams(rig), float(tau), float(s), int(iters), _p(out),
                               _p(cost), _p(ni))
    return dict(pose=out, cost=float(cost[0]), n_inliers=int(ni[0]), accepted=int(acc))


def rig_lo_ransac(corr, rig, **params):
    """LO-RANSAC for a multi-camera rig query: corr has u, v, X, Y, Z, (w) and
    cam (int32 camera index); rig: list of (K, cam_from_rig).  -> dict(R, t
    (rig_from_world), mask, status, stats...)."""
    h = _RigCorrHold(corr)
    n = h.c.n
    prm = make_params(**params)
    pose = np.zeros(12, np.float64)
    mask = np.zeros(max(n, 1), np.uint8)
    st = Stats()
    status = lib().orc_rig_lo_ransac(C.byref(h.rc), _rig_cams(rig), len(rig), C.byref(prm), _p(pose), _p(mask),
                                     C.byref(st))
    R, t = split_pose(pose)
    out = dict(R=R, t=t, mask=mask[:n].copy(), status=int(status))
    for f_, _ in Stats._fields_:
        out[f_] = getattr(st, f_)
    return out
