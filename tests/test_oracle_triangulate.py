"""Pins of the oracle's mapping-time depth estimation (Sec. 3.3 "Depth
Estimation by Dense Matching": one depth hypothesis per match, all tried,
most inliers at a 2 degree angular threshold wins, confidence-weighted
refinement of the squared angular errors, depths with more than 3 inliers
kept).

Pins: the closed-form hypothesis is the minimiser of the match's angular error
(numerical minimisation in numpy/scipy); exact rays give the exact depth;
rays that diverge give none; the angle is the plain arccos angle; the
refinement is scipy's minimiser of the same weighted cost; a noise-free scene
gives the rendered depth at every pixel seen by at least 4 views; the
confidence filter (>= 0.05) and the min-inlier rule cut exactly where they
should; ties go to the lowest view index; wrong matches do not move the depth."""
import math

import numpy as np
import pytest
from scipy.optimize import minimize_scalar

from paper_2601_04185_amd import synth


def _angle_np(C0, r0, l, Ck, rk):
    a = C0 + l * r0 - Ck
    return math.atan2(np.linalg.norm(np.cross(a, rk)), np.dot(a, rk))


def _angle_acos(C0, r0, l, Ck, rk):
    a = C0 + l * r0 - Ck
    c = np.dot(a, rk) / (np.linalg.norm(a) * np.linalg.norm(rk))
    return math.acos(max(-1.0, min(1.0, c)))


def _random_pair(rng, miss=0.0):
    """Reference ray (C0, r0 with unit z in a random camera frame) and an
    observation of X = C0 + l r0 from Ck, rotated off by about `miss` rad."""
    C0 = rng.normal(0, 2, 3)
    R = synth.random_rotation(rng)
    r0 = R.T @ np.array([rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5), 1.0])
    l = rng.uniform(2, 30)
    X = C0 + l * r0
    Ck = C0 + rng.normal(0, 1.5, 3)
    d = X - Ck
    d /= np.linalg.norm(d)
    if miss:
        n = np.cross(d, rng.normal(size=3))
        n /= np.linalg.norm(n)
        d = d * math.cos(miss) + n * math.sin(miss)
    return C0, r0, l, Ck, d


def test_angle_is_arccos_angle(orc):
    rng = np.random.default_rng(1)
    for _ in range(200):
        C0, r0, l, Ck, rk = _random_pair(rng, miss=rng.uniform(0.01, 1.0))
        lt = l * rng.uniform(0.5, 1.5)
        # arccos of the normalised dot product is accurate away from 0 and pi
        assert abs(orc.tri_angle(C0, r0, lt, Ck, rk) - _angle_acos(C0, r0, lt, Ck, rk)) < 1e-9


def test_exact_rays_give_exact_depth(orc):
    rng = np.random.default_rng(2)
    for _ in range(200):
        C0, r0, l, Ck, rk = _random_pair(rng)
        h = orc.tri_hypothesis(C0, r0, Ck, rk)
        assert h is not None and abs(h - l) <= 1e-9 * l
        assert orc.tri_angle(C0, r0, h, Ck, rk) < 1e-9


def test_hypothesis_minimises_the_angle(orc):
    rng = np.random.default_rng(3)
    n_checked = 0
    for _ in range(300):
        C0, r0, l, Ck, rk = _random_pair(rng, miss=rng.uniform(1e-4, 0.05))
        h = orc.tri_hypothesis(C0, r0, Ck, rk)
        f = lambda x: _angle_np(C0, r0, x, Ck, rk)
        grid = np.geomspace(0.05, 500.0, 4000)
        a = C0[None, :] + grid[:, None] * r0[None, :] - Ck[None, :]
        ang = np.arctan2(np.linalg.norm(np.cross(a, rk[None, :]), axis=1), a @ rk)
        g = grid[int(np.argmin(ang))]
        res = minimize_scalar(f, bounds=(g / 1.01, g * 1.01), method="bounded", options=dict(xatol=1e-12))
        if res.x <= 0.05 * 1.01 or res.x >= 500 / 1.01:
            continue
        n_checked += 1
        assert h is not None
        assert f(h) <= res.fun + 1e-12
        assert abs(h - res.x) <= 1e-5 * res.x
    assert n_checked > 250


def test_diverging_rays_give_no_hypothesis(orc):
    rng = np.random.default_rng(4)
    for _ in range(100):
        C0, r0, l, Ck, rk = _random_pair(rng)
        # the observation looks away from every point of the reference ray
        assert orc.tri_hypothesis(C0, r0, Ck, -rk) is None
    # parallel rays: no finite minimum
    assert orc.tri_hypothesis(np.zeros(3), np.array([0, 0, 1.0]), np.array([1.0, 0, 0]),
                              np.array([0, 0, 1.0])) is None


def test_refine_is_scipy_minimiser(orc):
    rng = np.random.default_rng(5)
    for _ in range(25):
        C0, r0, l, _, _ = _random_pair(rng)
        X = C0 + l * r0
        n = int(rng.integers(4, 12))
        Cs, rs = [], []
        for _k in range(n):
            Ck = C0 + rng.normal(0, 1.5, 3)
            d = X - Ck
            d /= np.linalg.norm(d)
            nrm = np.cross(d, rng.normal(size=3))
            nrm /= np.linalg.norm(nrm)
            miss = rng.uniform(0, 0.02)
            Cs.append(Ck)
            rs.append(d * math.cos(miss) + nrm * math.sin(miss))
        w = rng.uniform(0.05, 1.0, n)
        cost = lambda x: sum(w[k] * _angle_np(C0, r0, x, Cs[k], rs[k]) ** 2 for k in range(n))
        lr = orc.tri_refine(C0, r0, l * 1.02, Cs, rs, w)
        grid = np.linspace(0.7 * l, 1.4 * l, 701)
        gi = int(np.argmin([cost(x) for x in grid]))
        res = minimize_scalar(cost, bracket=(grid[gi - 1], grid[gi], grid[gi + 1]), method="brent", tol=1e-12)
        assert cost(lr) <= res.fun * (1 + 1e-12) + 1e-20
        # a minimum on both sides, at scipy's minimiser
        e = cost(lr)
        assert cost(lr * (1 + 1e-6)) >= e and cost(lr * (1 - 1e-6)) >= e
        assert abs(lr - res.x) <= 1e-6 * l


@pytest.fixture(scope="module")
def clean_scene():
    return synth.dense_match_scene(n_views=8, width=96, height=72, correct_frac=1.0, noise_px=0.0, seed=21)


def test_noise_free_scene_gives_rendered_depth(orc, clean_scene):
    w = clean_scene
    r = orc.triangulate(w.K0, w.T0, w.Ks, w.Ts, w.mu, w.mv, w.conf)
    seen = w.correct.sum(0)
    ok = r["depth"] > 0
    # every pixel seen by >= 4 views is kept, at the rendered depth (float32 pixels: ~1e-7)
    assert np.all(ok[seen >= 4])
    # where the inlier set is exactly the views that see the point, the depth
    # is the rendered one; a random match falling within 2 degrees (one more
    # inlier) is rare
    exact = (seen >= 4) & (r["inliers"] == seen)
    assert exact.sum() >= 0.99 * (seen >= 4).sum()
    rel = np.abs(r["depth"][exact] / w.depth_true[exact] - 1)
    assert rel.max() < 1e-5 and np.median(rel) < 1e-7
    # a kept pixel has at least 4 inliers, and the winning match is the lowest view seeing the point
    assert np.all(r["inliers"][ok] >= 4)
    first = np.argmax(w.correct, axis=0)
    m = seen >= 4
    assert np.mean(r["best_view"][m] == first[m]) > 0.99


def test_min_inliers_and_confidence_filter(orc, clean_scene):
    w = clean_scene
    seen = w.correct.sum(0)
    i, j = np.argwhere(seen >= 6)[0]
    vis = np.flatnonzero(w.correct[:, i, j])
    conf = w.conf.copy()
    conf[:, i, j] = 0.0
    conf[vis[:4], i, j] = np.float32(0.05)          # exactly at the threshold: used
    r = orc.triangulate(w.K0, w.T0, w.Ks, w.Ts, w.mu, w.mv, conf)
    assert r["inliers"][i, j] == 4 and r["depth"][i, j] > 0
    conf[vis[3], i, j] = np.nextafter(np.float32(0.05), np.float32(0))   # just below: ignored
    r = orc.triangulate(w.K0, w.T0, w.Ks, w.Ts, w.mu, w.mv, conf)
    assert r["inliers"][i, j] == 3 and r["depth"][i, j] == 0
    r = orc.triangulate(w.K0, w.T0, w.Ks, w.Ts, w.mu, w.mv, conf, min_inliers=3)
    assert r["depth"][i, j] > 0


def test_angle_threshold_is_strict_and_counts(orc, clean_scene):
    """At the exact depth, an observation off by 1.9 degrees is an inlier and
    one off by 2.1 is not; a hypothesis counts exactly the observations whose
    angle is below the threshold."""
    rng = np.random.default_rng(8)
    C0, r0, l, Ck, rk = _random_pair(rng)
    X = C0 + l * r0
    for deg, inside in ((1.9, True), (2.1, False), (1.999, True), (2.001, False)):
        d = X - Ck
        d /= np.linalg.norm(d)
        n = np.cross(d, r0)
        n /= np.linalg.norm(n)          # off the epipolar plane
        rot = d * math.cos(math.radians(deg)) + n * math.sin(math.radians(deg))
        assert (orc.tri_angle(C0, r0, l, Ck, rot) < math.radians(2.0)) == inside


def test_wrong_matches_do_not_move_the_depth(orc):
    w = synth.dense_match_scene(n_views=10, width=96, height=72, correct_frac=0.6, noise_px=0.0, seed=22)
    r = orc.triangulate(w.K0, w.T0, w.Ks, w.Ts, w.mu, w.mv, w.conf)
    m = (w.correct.sum(0) >= 4) & (r["depth"] > 0)
    assert m.mean() > 0.3
    rel = np.abs(r["depth"][m] / w.depth_true[m] - 1)
    assert np.median(rel) < 1e-6 and np.mean(rel < 1e-4) > 0.98


def test_reported_cost_and_curvature(orc):
    """The reported refinement cost is sum w angle^2 over the winning
    hypothesis' inliers at the kept depth (numpy), and the reported second
    derivative is positive there (a minimum)."""
    w = synth.dense_match_scene(n_views=6, width=40, height=30, correct_frac=0.8, noise_px=0.5, seed=23)
    r = orc.triangulate(w.K0, w.T0, w.Ks, w.Ts, w.mu, w.mv, w.conf)
    T0 = np.asarray(w.T0)
    R0, t0 = T0[:9].reshape(3, 3), T0[9:]
    C0 = -R0.T @ t0
    K0 = w.K0
    checked = 0
    for i, j in np.argwhere(r["depth"] > 0)[:40]:
        r0 = R0.T @ np.array([(j + 0.5 - K0[2]) / K0[0], (i + 0.5 - K0[3]) / K0[1], 1.0])
        rays, cents, ws = [], [], []
        for k in range(len(w.Ks)):
            if not (w.conf[k, i, j] >= np.float32(0.05)):
                continue
            Kk, Tk = w.Ks[k], np.asarray(w.Ts[k])
            Rk, tk = Tk[:9].reshape(3, 3), Tk[9:]
            d = Rk.T @ np.array([(float(w.mu[k, i, j]) - Kk[2]) / Kk[0], (float(w.mv[k, i, j]) - Kk[3]) / Kk[1], 1.0])
            rays.append(d / np.linalg.norm(d))
            cents.append(-Rk.T @ tk)
            ws.append(float(w.conf[k, i, j]))
        hv = int(r["best_view"][i, j])
        used = [k for k in range(len(w.Ks)) if w.conf[k, i, j] >= np.float32(0.05)]
        h = orc.tri_hypothesis(C0, r0, cents[used.index(hv)], rays[used.index(hv)])
        inl = [m for m in range(len(rays)) if _angle_np(C0, r0, h, cents[m], rays[m]) < math.radians(2.0)]
        assert len(inl) == r["inliers"][i, j]
        l = r["depth"][i, j]
        cost = sum(ws[m] * _angle_np(C0, r0, l, cents[m], rays[m]) ** 2 for m in inl)
        assert abs(cost - r["cost"][i, j]) <= 1e-9 * cost + 1e-18
        assert r["curv"][i, j] > 0
        checked += 1
    assert checked >= 20
