"""Pins of the oracle's multi-camera rig path (generalised absolute pose; the
appendix on LaMAR HoloLens rig queries, with the LO-RANSAC of Sec. 3.3).

Pins: the generalised P3P recovers the true rig pose from exact rays, every
solution satisfies the three distance equations and puts the rays through the
world points (checked in numpy), its solution count matches an independent
multi-start Newton search of the same equations, and with one camera at the
rig origin it returns exactly the single-camera P3P solutions (Grunert's
formulation); rig scoring, local optimisation and refinement with one
identity camera reduce to the single-camera oracle; the local optimisation's
fixed point is scipy's least-squares optimum over its inlier set with the rig
camera model written in numpy; the Cauchy refinement is scipy's minimiser of
the same cost; the whole LO-RANSAC recovers a noise-free rig pose and, in
exhaustive mode on a tiny input, returns the brute-force best triple."""
import math

import numpy as np
import pytest
from scipy.optimize import least_squares, minimize
from scipy.spatial.transform import Rotation

from conftest import rot_angle
from paper_2601_04185_amd import synth


def _rig_rays(q, idx):
    o, f = np.zeros((3, 3)), np.zeros((3, 3))
    for k, i in enumerate(idx):
        K, T = q.rig[q.cam[i]]
        Rc, tc = T[:9].reshape(3, 3), T[9:]
        d = np.array([(float(q.u[i]) - K[2]) / K[0], (float(q.v[i]) - K[3]) / K[1], 1.0])
        o[k] = -Rc.T @ tc
        f[k] = Rc.T @ d
    X = np.stack([q.X[idx], q.Y[idx], q.Z[idx]], 1).astype(np.float64)
    return o, f, X


class _Triple:
    def __init__(self, R, t):
        self.R, self.t = R, t


def _exact_rig_triple(rng, n_cams=4):
    """Three float64 world points seen by random cameras of the head rig at a
    random rig pose, and their exact rays (rig frame)."""
    rig = synth.head_rig(n_cams)
    R = synth.random_rotation(rng)
    t = synth.random_translation(rng, 5.0)
    o, f, X = np.zeros((3, 3)), np.zeros((3, 3)), np.zeros((3, 3))
    for k in range(3):
        K, T = rig[int(rng.integers(n_cams))]
        Rc, tc = T[:9].reshape(3, 3), T[9:]
        px, py, z = rng.uniform(0, 640), rng.uniform(0, 480), rng.uniform(2, 20)
        xc = np.array([(px - K[2]) / K[0] * z, (py - K[3]) / K[1] * z, z])
        xr = Rc.T @ (xc - tc)
        X[k] = R.T @ (xr - t)
        o[k] = -Rc.T @ tc
        f[k] = Rc.T @ (xc / z)
    return _Triple(R, t), (o, f, X)


def test_gp3p_recovers_true_pose_and_satisfies_equations(orc):
    rng = np.random.default_rng(0)
    found = 0
    for _ in range(200):
        q, (o, f, X) = _exact_rig_triple(rng)
        sols, dep, ill = orc.gp3p(o, f, X)
        fn = f / np.linalg.norm(f, axis=1, keepdims=True)
        for (R, t), l in zip(sols, dep):
            assert np.abs(R.T @ R - np.eye(3)).max() < 1e-9 and abs(np.linalg.det(R) - 1) < 1e-9
            P = o + l[:, None] * fn
            # the three distances and the rays through the world points
            for a, b in ((0, 1), (0, 2), (1, 2)):
                assert abs(np.linalg.norm(P[a] - P[b]) - np.linalg.norm(X[a] - X[b])) < 1e-7
            np.testing.assert_allclose(X @ R.T + t, P, atol=1e-6)
        errs = [rot_angle(R, q.R) + np.linalg.norm(t - q.t) for R, t in sols]
        if not ill:
            assert min(errs) < 1e-8
            found += 1
    assert found > 180


def _newton_all(o, f, X, rng, starts=400):
    """Every positive solution of the three distance equations reached by
    Newton's method from random starting depths (independent of the oracle)."""
    fn = f / np.linalg.norm(f, axis=1, keepdims=True)
    d2 = [np.sum((X[a] - X[b]) ** 2) for a, b in ((0, 1), (0, 2), (1, 2))]
    pairs = ((0, 1), (0, 2), (1, 2))

    def F(l):
        P = o + l[:, None] * fn
        return np.array([np.sum((P[a] - P[b]) ** 2) - d2[e] for e, (a, b) in enumerate(pairs)])

    def J(l):
        P = o + l[:, None] * fn
        M = np.zeros((3, 3))
        for e, (a, b) in enumerate(pairs):
            v = P[a] - P[b]
            M[e, a] = 2 * v @ fn[a]
            M[e, b] = -2 * v @ fn[b]
        return M

    scale = math.sqrt(max(d2))
    out = []
    for _ in range(starts):
        l = rng.uniform(0.01, 40.0, 3) * scale
        for _ in range(100):
            try:
                step = np.linalg.solve(J(l), F(l))
            except np.linalg.LinAlgError:
                break
            l = l - step
            if np.abs(step).max() < 1e-13 * (1 + np.abs(l).max()):
                break
        if np.all(l > 0) and np.abs(F(l)).max() < 1e-8 * sum(d2):
            if not any(np.abs(l - m).max() < 1e-6 * (1 + np.abs(l).max()) for m in out):
                out.append(l)
    return out


def test_gp3p_solution_count_matches_multistart_newton(orc):
    rng = np.random.default_rng(1)
    checked = 0
    for _ in range(20):
        _, (o, f, X) = _exact_rig_triple(rng)
        sols, dep, ill = orc.gp3p(o, f, X)
        if ill:
            continue
        ref = _newton_all(o, f, X, rng)
        assert len(sols) == len(ref), (len(sols), len(ref))
        for l in ref:
            assert np.min(np.abs(dep - l).max(axis=1)) < 1e-6 * (1 + np.abs(l).max())
        checked += 1
    assert checked >= 17


def test_gp3p_single_central_camera_equals_p3p(orc):
    """One camera at the rig origin: the generalised problem is the central
    P3P problem; the oracle's P3P (Grunert) is an independent formulation."""
    rng = np.random.default_rng(2)
    K = (500.0, 500.0, 320.0, 240.0)
    checked = 0
    for _ in range(200):
        q = synth.make_query(int(rng.integers(1 << 30)), 30, 1.0, 0.0)
        idx = rng.choice(q.n, 3, replace=False)
        uv = np.stack([q.u[idx], q.v[idx]], 1).astype(np.float64)
        X = np.stack([q.X[idx], q.Y[idx], q.Z[idx]], 1).astype(np.float64)
        p3, ill3 = orc.p3p(uv, X, K)
        f = np.stack([(uv[:, 0] - K[2]) / K[0], (uv[:, 1] - K[3]) / K[1], np.ones(3)], 1)
        g, _, illg = orc.gp3p(np.zeros((3, 3)), f, X)
        if ill3 or illg:
            continue
        checked += 1
        assert len(g) == len(p3)
        for (Ra, ta), (Rb, tb) in zip(g, p3):   # both in canonical order (depth of point 0, then 1)
            assert rot_angle(Ra, Rb) < 1e-8 and np.linalg.norm(ta - tb) < 1e-8 * (1 + np.linalg.norm(tb))
    assert checked > 150


def _identity_rig(K):
    return [(K, np.concatenate([np.eye(3).reshape(9), np.zeros(3)]))]


def test_one_identity_camera_reduces_to_single_camera(orc):
    q = synth.make_query(31, 1500, 0.4, 1.0, weights="conf")
    corr = dict(q.corr(), cam=np.zeros(q.n, np.int32))
    rig = _identity_rig(q.K)
    rng = np.random.default_rng(3)
    poses = []
    for _ in range(20):
        w = rng.normal(0, 0.01, 3)
        R = Rotation.from_rotvec(w).as_matrix() @ q.R
        poses.append(np.concatenate([R.reshape(9), q.t + rng.normal(0, 0.02, 3)]))
    poses = np.stack(poses)
    c1, m1 = orc.score(poses, q.corr(), q.K, 4.0)
    c2, m2 = orc.rig_score(poses, corr, rig, 4.0)
    np.testing.assert_array_equal(c1, c2)
    np.testing.assert_allclose(m1, m2, rtol=1e-12)
    Ra, ta = orc.lo(poses[0], q.corr(), q.K, 4.0, 10)[:2]
    b = orc.rig_lo(poses[0], corr, rig, 4.0, 10)
    np.testing.assert_allclose(np.concatenate([Ra.reshape(9), ta]), b["pose"], atol=1e-10)
    Ra, ta = orc.refine(poses[0], q.corr(), q.K, 4.0, 2.0, 10)[:2]
    b = orc.rig_refine(poses[0], corr, rig, 4.0, 2.0, 10)
    np.testing.assert_allclose(np.concatenate([Ra.reshape(9), ta]), b["pose"], atol=1e-10)


def _rig_residuals(params, q, sel):
    """numpy rig camera model: pixel residuals of the selected points at the
    pose (rotation vector, translation) -- independent of the oracle."""
    R = Rotation.from_rotvec(params[:3]).as_matrix()
    t = params[3:]
    out = []
    for c, (K, T) in enumerate(q.rig):
        m = sel & (q.cam == c)
        if not m.any():
            continue
        Rc, tc = T[:9].reshape(3, 3), T[9:]
        X = np.stack([q.X[m], q.Y[m], q.Z[m]], 1).astype(np.float64)
        xc = (X @ R.T + t) @ Rc.T + tc
        w = np.sqrt(q.w[m].astype(np.float64)) if q.w is not None else 1.0
        out.append(w * (K[0] * xc[:, 0] / xc[:, 2] + K[2] - q.u[m]))
        out.append(w * (K[1] * xc[:, 1] / xc[:, 2] + K[3] - q.v[m]))
    return np.concatenate(out)


def test_rig_lo_fixed_point_is_scipy_least_squares(orc):
    q = synth.make_rig_query(32, 2000, 0.5, 1.0, weights="conf")
    rng = np.random.default_rng(4)
    R0 = Rotation.from_rotvec(rng.normal(0, 0.003, 3)).as_matrix() @ q.R
    t0 = q.t + rng.normal(0, 0.01, 3)
    res = orc.rig_lo(np.concatenate([R0.reshape(9), t0]), q.corr(), q.rig, 4.0, 50)
    R, t = res["pose"][:9].reshape(3, 3), res["pose"][9:]
    # inlier set at the fixed point, then scipy on that fixed set
    sel = np.zeros(q.n, bool)
    r = _rig_residuals(np.concatenate([Rotation.from_matrix(R).as_rotvec(), t]), q, np.ones(q.n, bool))
    order = np.concatenate([np.flatnonzero(q.cam == c) for c in range(len(q.rig))])
    nres = r.reshape(-1)
    # residual pairs come camera by camera: rebuild per-point squared errors in that order
    per = []
    k = 0
    for c in range(len(q.rig)):
        m = np.flatnonzero(q.cam == c)
        du, dv = nres[k:k + len(m)], nres[k + len(m):k + 2 * len(m)]
        k += 2 * len(m)
        w = q.w[m].astype(np.float64)
        per.append((m, (du ** 2 + dv ** 2) / w))
    for m, e in per:
        sel[m] = e < 16.0
    assert sel.sum() == res["count"]
    ls = least_squares(_rig_residuals, np.concatenate([Rotation.from_matrix(R).as_rotvec(), t]), args=(q, sel),
                       xtol=1e-15, ftol=1e-15, gtol=1e-15)
    assert rot_angle(Rotation.from_rotvec(ls.x[:3]).as_matrix(), R) < 1e-9
    assert np.linalg.norm(ls.x[3:] - t) < 1e-8
    assert rot_angle(R, q.R) < math.radians(0.05)


def test_rig_refine_is_scipy_cauchy_minimiser(orc):
    q = synth.make_rig_query(33, 1200, 0.6, 1.0, weights="conf")
    start = np.concatenate([q.R.reshape(9), q.t])
    tau, s = 4.0, 2.0
    res = orc.rig_refine(start, q.corr(), q.rig, tau, s, 100)
    full = np.ones(q.n, bool)
    x0 = np.concatenate([Rotation.from_matrix(q.R).as_rotvec(), q.t])
    r0 = _rig_residuals(x0, q, full)
    # inlier set at the start pose (tau), per point in camera order
    sel = np.zeros(q.n, bool)
    k = 0
    for c in range(len(q.rig)):
        m = np.flatnonzero(q.cam == c)
        du, dv = r0[k:k + len(m)], r0[k + len(m):k + 2 * len(m)]
        k += 2 * len(m)
        sel[m] = (du ** 2 + dv ** 2) / q.w[m] < tau * tau
    assert sel.sum() == res["n_inliers"]

    def cost(x):
        r = _rig_residuals(x, q, sel)
        out, k = 0.0, 0
        for c in range(len(q.rig)):
            m = np.flatnonzero(sel & (q.cam == c))
            du, dv = r[k:k + len(m)], r[k + len(m):k + 2 * len(m)]
            k += 2 * len(m)
            w = q.w[m].astype(np.float64)
            out += np.sum(w * s * s * np.log1p((du ** 2 + dv ** 2) / w / (s * s)))
        return out

    mn = minimize(cost, x0, method="BFGS", options=dict(gtol=1e-10, maxiter=2000))
    R = res["pose"][:9].reshape(3, 3)
    assert cost(np.concatenate([Rotation.from_matrix(R).as_rotvec(), res["pose"][9:]])) <= mn.fun * (1 + 1e-9)
    assert rot_angle(Rotation.from_rotvec(mn.x[:3]).as_matrix(), R) < 1e-6
    assert np.linalg.norm(mn.x[3:] - res["pose"][9:]) < 1e-5


def test_rig_lo_ransac_noise_free_recovers_pose(orc):
    q = synth.make_rig_query(34, 800, 0.5, 0.0)
    r = orc.rig_lo_ransac(q.corr(), q.rig, threshold_px=4.0, fixed_samples=256, batch=256, lo_top_k=2)
    assert r["status"] == 0
    assert rot_angle(r["R"], q.R) < 1e-8 and np.linalg.norm(r["t"] - q.t) < 1e-7
    np.testing.assert_array_equal(r["mask"].astype(bool), q.is_inlier)


def test_rig_exhaustive_equals_brute_force(orc):
    q = synth.make_rig_query(35, 16, 0.6, 0.5)
    n = q.n
    import itertools
    best = None
    for idx in itertools.combinations(range(n), 3):
        a, b, c = idx
        h = math.comb(a, 1) + math.comb(b, 2) + math.comb(c, 3)   # colex rank of the sample
        o, f, X = _rig_rays(q, list(idx))
        sols, _, _ = orc.gp3p(o, f, X)
        if not sols:
            continue
        P = np.stack([np.concatenate([R.reshape(9), t]) for R, t in sols])
        cnt, ms = orc.rig_score(P, q.corr(), q.rig, 4.0)
        for j in range(len(sols)):
            key = (ms[j], -cnt[j], h, j)
            if best is None or key < best:
                best = key
    total = n * (n - 1) * (n - 2) // 6
    r = orc.rig_lo_ransac(q.corr(), q.rig, threshold_px=4.0, fixed_samples=total, batch=total, exhaustive=1,
                          lo_top_k=1, lo_iters=0, final_iters=0)
    assert (r["best_h"], r["best_j"]) == (best[2], best[3])
    assert abs(r["best_msac"] - best[0]) <= 1e-9 * best[0]
