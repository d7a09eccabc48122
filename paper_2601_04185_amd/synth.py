"""Seeded synthetic workloads shaped like the paper's localization queries.

This module only draws inputs with a known ground truth.  It holds none of the
pose-estimation arithmetic (no lifting, no P3P, no scoring, no refinement): it
is shared by the GPU-path tests, the oracle tests and the benchmark so that both
sides see the same float32 arrays.

The paper evaluates on Oxford Day & Night, LaMAR, Cambridge Landmarks and
Aachen, matching each query densely (RoMa) against its K best database views
(K = 10 or 50 at 560 x 560, Sec. 3.3 / Sec. 4).  Those datasets and the matcher
weights are not available, so every generator below stands in for them with
the same shapes: thousands of dense matches per retrieved view, inlier ratios
from a few percent to a majority, pixel noise of about one pixel.

Conventions: pinhole camera (fx, fy, cx, cy), poses are cam_from_world
(x_cam = R X + t), camera frame x right / y down / z forward, pixel (row i,
col j) has its centre at (j + 0.5, i + 0.5), depth is z-depth.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

DEFAULT_K = (500.0, 500.0, 320.0, 240.0)
DEFAULT_W, DEFAULT_H = 640, 480


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform on SO(3): normalised 4-D Gaussian quaternion."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def random_translation(rng: np.random.Generator, tmax: float) -> np.ndarray:
    """Uniform in the ball of radius tmax."""
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    return d * tmax * rng.random() ** (1.0 / 3.0)


def _frustum_points(rng, n, K, width, height, zmin, zmax):
    """Camera-frame points uniform in volume inside the viewing frustum:
    pixel uniform over the image, depth with density proportional to z^2."""
    fx, fy, cx, cy = K
    px = rng.random(n) * width
    py = rng.random(n) * height
    z = (zmin ** 3 + rng.random(n) * (zmax ** 3 - zmin ** 3)) ** (1.0 / 3.0)
    Xc = np.stack([(px - cx) / fx * z, (py - cy) / fy * z, z], axis=1)
    return px, py, Xc


@dataclass
class Query:
    """One query's 2D-3D correspondences (float32 SoA) plus its ground truth."""
    u: np.ndarray
    v: np.ndarray
    X: np.ndarray
    Y: np.ndarray
    Z: np.ndarray
    w: np.ndarray | None
    K: tuple
    R: np.ndarray
    t: np.ndarray
    is_inlier: np.ndarray
    view: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.u.shape[0])

    def corr(self) -> dict:
        return dict(u=self.u, v=self.v, X=self.X, Y=self.Y, Z=self.Z, w=self.w)


def make_query(seed: int, n: int, inlier_ratio: float, sigma_px: float, K=DEFAULT_K,
               width: int = DEFAULT_W, height: int = DEFAULT_H, zmin: float = 2.0, zmax: float = 20.0,
               tmax: float = 5.0, weights: str = "ones", n_views: int = 0) -> Query:
    """A single query: random pose (R uniform on SO(3), |t| <= tmax), inliers seen
    through the true pose with Gaussian pixel noise, outliers with a pixel uniform
    in the image and an independent 3-D point from the same frustum, shuffled."""
    rng = rng_for(seed)
    R = random_rotation(rng)
    t = random_translation(rng, tmax)
    n_in = int(round(n * inlier_ratio))
    n_out = n - n_in
    px, py, Xc = _frustum_points(rng, n_in, K, width, height, zmin, zmax)
    Xw_in = (Xc - t) @ R  # R^T (x_c - t), row-wise
    obs_u = px + rng.standard_normal(n_in) * sigma_px
    obs_v = py + rng.standard_normal(n_in) * sigma_px
    ou = rng.random(n_out) * width
    ov = rng.random(n_out) * height
    _, _, Xc_o = _frustum_points(rng, n_out, K, width, height, zmin, zmax)
    Xw_out = (Xc_o - t) @ R
    u = np.concatenate([obs_u, ou])
    v = np.concatenate([obs_v, ov])
    Xw = np.concatenate([Xw_in, Xw_out])
    inl = np.concatenate([np.ones(n_in, bool), np.zeros(n_out, bool)])
    perm = rng.permutation(n)
    u, v, Xw, inl = u[perm], v[perm], Xw[perm], inl[perm]
    if weights == "ones":
        w = None
    else:
        w = (0.05 + 0.95 * rng.random(n)).astype(np.float32)
        w = np.maximum(w, np.float32(0.0500001))
    view = (np.arange(n) * max(n_views, 1) // max(n, 1)).astype(np.int32)[perm] if n_views else None
    f = lambda a: np.ascontiguousarray(a, np.float32)
    return Query(f(u), f(v), f(Xw[:, 0]), f(Xw[:, 1]), f(Xw[:, 2]), w, tuple(K), R, t, inl, view,
                 dict(seed=seed, inlier_ratio=inlier_ratio, sigma_px=sigma_px))


# ---------------------------------------------------------------------------
# The benchmark workloads (seeds are 1000 + config index).
# ---------------------------------------------------------------------------

def config1_single_small() -> Query:
    """2,000 correspondences, 40 % inliers, sigma 1 px (1,024 samples, tau 4 px)."""
    return make_query(1001, 2000, 0.40, 1.0)


def config2_single_large(n_views: int = 10, per_view: int = 5000) -> Query:
    """K = 10 views x 5,000 = 50,000 correspondences, 25 % inliers, sigma 1.5 px
    (10,000 samples, tau 6 px, LO on the top-8)."""
    return make_query(1002, n_views * per_view, 0.25, 1.5, n_views=n_views)


def config3_batch(n_queries: int = 256, n_lo: int = 5000, n_hi: int = 80000, seed: int = 1003):
    """256 queries, correspondence counts uniform in [5,000, 80,000], inlier
    ratios uniform in [10 %, 60 %], sigma 1 px (4,096 samples each)."""
    rng = rng_for(seed)
    ns = rng.integers(n_lo, n_hi + 1, size=n_queries)
    eps = rng.uniform(0.10, 0.60, size=n_queries)
    return [make_query(seed * 1000 + q, int(ns[q]), float(eps[q]), 1.0) for q in range(n_queries)]


def serving_arrivals(n_queries: int, rate_qps: float, seed: int = 1005, n_min: int = 2000,
                     n_max: int = 200000, mu: float = math.log(20000.0), sigma_ln: float = 0.77):
    """Poisson arrival times and per-query sizes of the serving workload:
    correspondence counts log-normal clamped to [2,000, 200,000], inlier
    ratios uniform in [5 %, 60 %]."""
    rng = rng_for(seed)
    gaps = rng.exponential(1.0 / rate_qps, size=n_queries)
    arrivals = np.cumsum(gaps) - gaps[0]
    ns = np.clip(np.exp(rng.normal(mu, sigma_ln, size=n_queries)), n_min, n_max).astype(np.int64)
    eps = rng.uniform(0.05, 0.60, size=n_queries)
    return arrivals, ns, eps


# ---------------------------------------------------------------------------
# Box-and-plane scene with rendered depth maps (end-to-end lifting workload).
# ---------------------------------------------------------------------------

def look_at(center: np.ndarray, target: np.ndarray, up=(0.0, 0.0, 1.0)):
    z = target - center
    z = z / np.linalg.norm(z)
    x = np.cross(z, np.asarray(up, float))
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z])
    return R, -R @ center


@dataclass
class Scene:
    boxes: np.ndarray  # (B, 2, 3) min / max corners


def make_scene(rng: np.random.Generator, n_boxes: int | None = None, half: float = 20.0) -> Scene:
    if n_boxes is None:
        n_boxes = int(rng.integers(5, 16))
    lo = np.zeros((n_boxes, 3))
    size = rng.uniform(1.0, 5.0, size=(n_boxes, 3))
    lo[:, :2] = rng.uniform(-half * 0.6, half * 0.6 - size[:, :2])
    lo[:, 2] = 0.0
    return Scene(np.stack([lo, lo + size], axis=1))


def ray_cast(scene: Scene, origin: np.ndarray, dirs: np.ndarray, half: float = 20.0) -> np.ndarray:
    """Distance along each (unnormalised) direction to the first surface of the
    ground plane z = 0 (inside the square) or of any box; inf when nothing is hit."""
    tbest = np.full(dirs.shape[0], np.inf)
    with np.errstate(divide="ignore", invalid="ignore"):
        tg = -origin[2] / dirs[:, 2]
        hit = (tg > 1e-9) & np.isfinite(tg)
        p = origin[None, :] + tg[:, None] * dirs
        hit &= (np.abs(p[:, 0]) <= half) & (np.abs(p[:, 1]) <= half)
        tbest = np.where(hit, tg, tbest)
        for b in scene.boxes:
            t0 = (b[0][None, :] - origin[None, :]) / dirs
            t1 = (b[1][None, :] - origin[None, :]) / dirs
            tmin = np.nanmax(np.minimum(t0, t1), axis=1)
            tmax = np.nanmin(np.maximum(t0, t1), axis=1)
            ok = (tmax >= tmin) & (tmin > 1e-9)
            tbest = np.where(ok & (tmin < tbest), tmin, tbest)
    return tbest


def render_depth(scene: Scene, R: np.ndarray, t: np.ndarray, K, width: int, height: int):
    """z-depth per pixel centre by ray casting in float64."""
    fx, fy, cx, cy = K
    jj, ii = np.meshgrid(np.arange(width) + 0.5, np.arange(height) + 0.5)
    dc = np.stack([(jj - cx) / fx, (ii - cy) / fy, np.ones_like(jj)], axis=-1).reshape(-1, 3)
    C0 = -R.T @ t
    dw = dc @ R  # R^T d per row
    s = ray_cast(scene, C0, dw)
    return s.reshape(height, width)  # z-depth because d_c has unit z


def _blob_mask(rng, height, width, frac):
    m = np.zeros((height, width), bool)
    jj, ii = np.meshgrid(np.arange(width), np.arange(height))
    while m.mean() < frac:
        r = rng.uniform(3, 20)
        c = rng.uniform(0, width), rng.uniform(0, height)
        m |= (jj - c[0]) ** 2 + (ii - c[1]) ** 2 < r * r
    return m


@dataclass
class LiftWorkload:
    depth: np.ndarray      # (K, H, W) float32
    cams: np.ndarray       # (K, 4) float64
    poses: np.ndarray      # (K, 12) float64 cam_from_world
    matches: dict          # q_u, q_v, db_u, db_v, conf float32, view int32
    K_query: tuple
    R: np.ndarray
    t: np.ndarray
    correct: np.ndarray    # per match: generated as a correct match


def config4_lift_scene(n_views: int = 20, per_view: int = 8000, correct_frac: float = 0.30,
                       width: int = DEFAULT_W, height: int = DEFAULT_H, seed: int = 1004,
                       zclip=(0.5, 30.0), invalid_frac: float = 0.05) -> LiftWorkload:
    """Box-and-plane world, n_views database RGB-D views near one query at about
    1.5 m height looking inward; depth clipped to [0.5, 30] m (0 beyond), about
    5 % invalid zeros in blobs; per view, per_view query->database matches, a
    fraction correct to within 1 px (a uniform disk offset), the rest random;
    confidence uniform in (0.05, 1]."""
    rng = rng_for(seed)
    K = DEFAULT_K
    scene = make_scene(rng)
    ang0 = rng.uniform(0, 2 * np.pi)

    def cam_at(angle, radius, height_m, jitter):
        c = np.array([radius * np.cos(angle), radius * np.sin(angle), height_m])
        target = np.array([0.0, 0.0, 1.0]) + rng.normal(0, jitter, 3)
        return look_at(c, target)

    Rq, tq = cam_at(ang0, 16.0, 1.5, 1.0)
    depth = np.zeros((n_views, height, width), np.float32)
    cams = np.tile(np.array(K, np.float64), (n_views, 1))
    poses = np.zeros((n_views, 12))
    Rs, ts = [], []
    for k in range(n_views):
        ang = ang0 + rng.uniform(-0.5, 0.5)
        Rk, tk = cam_at(ang, rng.uniform(12.0, 19.0), rng.uniform(1.2, 1.8), 2.0)
        Rs.append(Rk)
        ts.append(tk)
        poses[k, :9] = Rk.reshape(9)
        poses[k, 9:] = tk
        d = render_depth(scene, Rk, tk, K, width, height)
        d = np.where((d >= zclip[0]) & (d <= zclip[1]), d, 0.0)
        d[_blob_mask(rng, height, width, invalid_frac)] = 0.0
        depth[k] = d.astype(np.float32)

    fx, fy, cx, cy = K
    Cq = -Rq.T @ tq
    q_u, q_v, db_u, db_v, view, corr = [], [], [], [], [], []
    for k in range(n_views):
        Rk, tk = Rs[k], ts[k]
        n_cor = int(round(per_view * correct_frac))
        got_u, got_v, got_du, got_dv = [], [], [], []
        tries = 0
        while sum(len(a) for a in got_u) < n_cor and tries < 50:
            tries += 1
            m = 4 * n_cor
            pu = rng.random(m) * width
            pv = rng.random(m) * height
            dcam = np.stack([(pu - cx) / fx, (pv - cy) / fy, np.ones(m)], 1)
            s = ray_cast(scene, Cq, dcam @ Rq)
            ok = np.isfinite(s)
            s = np.where(ok, s, 1.0)
            Xw = Cq[None, :] + s[:, None] * (dcam @ Rq)
            xk = Xw @ Rk.T + tk
            zk = xk[:, 2]
            ok &= zk > zclip[0]
            with np.errstate(divide="ignore", invalid="ignore"):
                du = fx * xk[:, 0] / zk + cx
                dv = fy * xk[:, 1] / zk + cy
            ok &= (du >= 1.0) & (du <= width - 1.0) & (dv >= 1.0) & (dv <= height - 1.0)
            # visibility in view k: the rendered depth at that pixel agrees with zk
            ci = np.clip(np.floor(np.nan_to_num(du)).astype(int), 0, width - 1)
            ri = np.clip(np.floor(np.nan_to_num(dv)).astype(int), 0, height - 1)
            dk = depth[k][ri, ci]
            ok &= (dk > 0) & (np.abs(dk - zk) < 0.02 * zk)
            rad = np.sqrt(rng.random(m))
            phi = rng.random(m) * 2 * np.pi
            got_u.append(pu[ok]); got_v.append(pv[ok])
            got_du.append((du + rad * np.cos(phi))[ok]); got_dv.append((dv + rad * np.sin(phi))[ok])
        cu = np.concatenate(got_u)[:n_cor]
        cv_ = np.concatenate(got_v)[:n_cor]
        cdu = np.concatenate(got_du)[:n_cor]
        cdv = np.concatenate(got_dv)[:n_cor]
        nr = per_view - cu.shape[0]
        ru, rv = rng.random(nr) * width, rng.random(nr) * height
        rdu, rdv = rng.random(nr) * width, rng.random(nr) * height
        q_u += [cu, ru]; q_v += [cv_, rv]; db_u += [cdu, rdu]; db_v += [cdv, rdv]
        view += [np.full(per_view, k, np.int32)]
        corr += [np.ones(cu.shape[0], bool), np.zeros(nr, bool)]
    n = n_views * per_view
    perm = rng.permutation(n)
    cat = lambda L: np.concatenate(L)[perm]
    conf = (1.0 - rng.random(n) * 0.95).astype(np.float32)  # (0.05, 1]
    f = lambda a: np.ascontiguousarray(a, np.float32)
    matches = dict(q_u=f(cat(q_u)), q_v=f(cat(q_v)), db_u=f(cat(db_u)), db_v=f(cat(db_v)), conf=conf,
                   view=np.ascontiguousarray(cat(view), np.int32))
    return LiftWorkload(depth, cams, poses, matches, K, Rq, tq, cat(corr))


# ---------------------------------------------------------------------------
# Dense matches of a mapping image against its covisible views (mapping-time
# depth estimation workload).
# ---------------------------------------------------------------------------

@dataclass
class DenseMatchWorkload:
    K0: tuple
    T0: np.ndarray        # (12,) cam_from_world of the mapping image
    Ks: np.ndarray        # (V, 4)
    Ts: np.ndarray        # (V, 12)
    mu: np.ndarray        # (V, H, W) float32 matched column coordinate in view k
    mv: np.ndarray        # (V, H, W) float32
    conf: np.ndarray      # (V, H, W) float32
    depth_true: np.ndarray  # (H, W) float64 z-depth of the mapping image (inf: nothing hit)
    correct: np.ndarray   # (V, H, W) bool: generated as a correct match


def dense_match_scene(n_views: int = 10, width: int = 560, height: int = 560, correct_frac: float = 0.7,
                      noise_px: float = 0.5, seed: int = 1006, f: float | None = None) -> DenseMatchWorkload:
    """A box-and-plane scene seen by one mapping camera and n_views covisible
    cameras (0.5-3 m away, looking at nearby targets).  For every pixel of the
    mapping image and every view: where the pixel's surface point is visible
    in the view (in the image, not occluded), with probability correct_frac
    the match is its true projection plus Gaussian noise (noise_px) with
    confidence U(0.3, 1]; every other match is a uniformly random pixel with
    confidence U(0, 0.6]."""
    rng = rng_for(seed)
    f = 0.8 * width if f is None else f
    K = (f, f, width / 2.0, height / 2.0)
    scene = make_scene(rng)
    ang = rng.uniform(0, 2 * np.pi)
    c0 = np.array([14.0 * np.cos(ang), 14.0 * np.sin(ang), 1.6])
    target = np.array([0.0, 0.0, 1.0]) + rng.normal(0, 1.0, 3)
    R0, t0 = look_at(c0, target)
    Rs, ts = [], []
    for _ in range(n_views):
        off = rng.normal(0, 1.0, 3)
        off *= rng.uniform(0.5, 3.0) / np.linalg.norm(off)
        off[2] = 0.3 * off[2]
        Rk, tk = look_at(c0 + off, target + rng.normal(0, 0.5, 3))
        Rs.append(Rk)
        ts.append(tk)
    d0 = render_depth(scene, R0, t0, K, width, height)
    fx, fy, cx, cy = K
    jj, ii = np.meshgrid(np.arange(width) + 0.5, np.arange(height) + 0.5)
    ok0 = np.isfinite(d0)
    dd = np.where(ok0, d0, 1.0)
    Xc = np.stack([(jj - cx) / fx * dd, (ii - cy) / fy * dd, dd], -1).reshape(-1, 3)
    Xw = (Xc - t0) @ R0  # R0^T (x_c - t0)
    V = n_views
    mu = np.empty((V, height, width), np.float32)
    mv = np.empty((V, height, width), np.float32)
    conf = np.empty((V, height, width), np.float32)
    correct = np.zeros((V, height, width), bool)
    for k in range(V):
        xk = Xw @ Rs[k].T + ts[k]
        zk = xk[:, 2]
        with np.errstate(divide="ignore", invalid="ignore"):
            uk = fx * xk[:, 0] / zk + cx
            vk = fy * xk[:, 1] / zk + cy
        vis = ok0.reshape(-1) & (zk > 0.1) & (uk >= 0) & (uk < width) & (vk >= 0) & (vk < height)
        dk = render_depth(scene, Rs[k], ts[k], K, width, height)
        ci = np.clip(np.floor(np.nan_to_num(uk)).astype(int), 0, width - 1)
        ri = np.clip(np.floor(np.nan_to_num(vk)).astype(int), 0, height - 1)
        vis &= np.abs(dk[ri, ci] - zk) < 0.02 * np.abs(zk)
        good = vis & (rng.random(vis.shape[0]) < correct_frac)
        n = vis.shape[0]
        u = np.where(good, uk + rng.normal(0, noise_px, n), rng.random(n) * width)
        v = np.where(good, vk + rng.normal(0, noise_px, n), rng.random(n) * height)
        c = np.where(good, 1.0 - 0.7 * rng.random(n), 0.6 * rng.random(n))
        mu[k] = u.reshape(height, width)
        mv[k] = v.reshape(height, width)
        conf[k] = c.reshape(height, width)
        correct[k] = good.reshape(height, width)
    pose = lambda R, t: np.concatenate([R.reshape(9), t])
    return DenseMatchWorkload(K, pose(R0, t0), np.tile(np.array(K), (V, 1)), np.stack([pose(R, t) for R, t in zip(Rs, ts)]),
                              mu, mv, conf, np.where(ok0, d0, np.inf), correct)


# ---------------------------------------------------------------------------
# Multi-camera rig queries (generalised absolute pose workload).
# ---------------------------------------------------------------------------

def _yaw(deg: float) -> np.ndarray:
    a = np.radians(deg)
    return np.array([[np.cos(a), 0.0, np.sin(a)], [0.0, 1.0, 0.0], [-np.sin(a), 0.0, np.cos(a)]])


def head_rig(n_cams: int = 4, K=(380.0, 380.0, 320.0, 240.0)):
    """A head-mounted rig: cameras yawed -80, -20, 20, 80 degrees (first
    n_cams of them), centres about 10 cm apart.  Returns a list of
    (K, cam_from_rig 12-vector)."""
    yaws = [-80.0, -20.0, 20.0, 80.0, -140.0, 140.0, 0.0, 180.0][:n_cams]
    rig = []
    for k, y in enumerate(yaws):
        Rc = _yaw(y).T                  # cam_from_rig rotation: the camera looks along yaw y
        centre = np.array([0.05 * np.sin(np.radians(y)), -0.02 * (k % 2), 0.05 * np.cos(np.radians(y))])
        tc = -Rc @ centre
        rig.append((tuple(K), np.concatenate([Rc.reshape(9), tc])))
    return rig


@dataclass
class RigQuery:
    u: np.ndarray
    v: np.ndarray
    X: np.ndarray
    Y: np.ndarray
    Z: np.ndarray
    w: np.ndarray | None
    cam: np.ndarray            # int32 camera of each correspondence (grouped: non-decreasing)
    rig: list                  # [(K, cam_from_rig)]
    R: np.ndarray              # rig_from_world
    t: np.ndarray
    is_inlier: np.ndarray

    @property
    def n(self) -> int:
        return int(self.u.shape[0])

    def corr(self) -> dict:
        return dict(u=self.u, v=self.v, X=self.X, Y=self.Y, Z=self.Z, w=self.w, cam=self.cam)

    def cam_start(self) -> np.ndarray:
        return np.searchsorted(self.cam, np.arange(len(self.rig) + 1)).astype(np.int64)


def make_rig_query(seed: int, n: int, inlier_ratio: float, sigma_px: float, n_cams: int = 4,
                   width: int = DEFAULT_W, height: int = DEFAULT_H, zmin: float = 2.0, zmax: float = 20.0,
                   tmax: float = 5.0, weights: str = "ones") -> RigQuery:
    """A rig query: random rig_from_world pose; the correspondences split evenly
    over the cameras (grouped by camera), in each camera inliers seen through
    the true pose with Gaussian pixel noise and outliers with a uniform pixel
    and an independent point from that camera's frustum."""
    rng = rng_for(seed)
    rig = head_rig(n_cams)
    R = random_rotation(rng)
    t = random_translation(rng, tmax)
    us, vs, Xs, cams, inls = [], [], [], [], []
    for c, (K, T) in enumerate(rig):
        Rc, tc = T[:9].reshape(3, 3), T[9:]
        nc = n // n_cams + (1 if c < n % n_cams else 0)
        n_in = int(round(nc * inlier_ratio))
        n_out = nc - n_in
        px, py, Xc = _frustum_points(rng, n_in, K, width, height, zmin, zmax)
        Xr = (Xc - tc) @ Rc                # rig frame
        Xw_in = (Xr - t) @ R               # world
        ou = rng.random(n_out) * width
        ov = rng.random(n_out) * height
        _, _, Xc_o = _frustum_points(rng, n_out, K, width, height, zmin, zmax)
        Xw_out = ((Xc_o - tc) @ Rc - t) @ R
        u = np.concatenate([px + rng.standard_normal(n_in) * sigma_px, ou])
        v = np.concatenate([py + rng.standard_normal(n_in) * sigma_px, ov])
        X = np.concatenate([Xw_in, Xw_out])
        inl = np.concatenate([np.ones(n_in, bool), np.zeros(n_out, bool)])
        perm = rng.permutation(nc)
        us.append(u[perm]); vs.append(v[perm]); Xs.append(X[perm]); inls.append(inl[perm])
        cams.append(np.full(nc, c, np.int32))
    f = lambda a: np.ascontiguousarray(np.concatenate(a) if isinstance(a, list) else a, np.float32)
    Xw = np.concatenate(Xs)
    w = None
    if weights != "ones":
        w = np.maximum((0.05 + 0.95 * rng.random(n)).astype(np.float32), np.float32(0.0500001))
    return RigQuery(f(us), f(vs), f(Xw[:, 0]), f(Xw[:, 1]), f(Xw[:, 2]), w, np.concatenate(cams), rig, R, t,
                    np.concatenate(inls))
