"""Pins of the oracle's local optimisation (Gauss-Newton on the truncated
cost, started from each new best; Sec. 3.3 "Pose Estimation") and of its final
refinement (Cauchy-loss IRLS over every inlier, confidence-weighted; same
section).

Pins: the gradient and Gauss-Newton matrix against central finite differences
of the cost under the same left update; convergence to the ground truth on
noise-free data; the fixed point against scipy.optimize.least_squares (plain
and Cauchy loss) on the same point set; monotone cost; the run's ends (a
cost-raising or shorter-than-1e-10 step, the cap) retold from the oracle's
pieces."""
import numpy as np
import pytest
from scipy.optimize import least_squares, minimize
from scipy.spatial.transform import Rotation

from conftest import rot_angle
from paper_2601_04185_amd import synth


def _perturb(R, t, rng, ang=0.02, dt=0.05):
    w = rng.standard_normal(3)
    w *= ang / np.linalg.norm(w)
    return Rotation.from_rotvec(w).as_matrix() @ R, t + rng.standard_normal(3) * dt


def test_gradient_and_gn_matrix_finite_differences(orc):
    q = synth.make_query(11, 400, 1.0, 0.0)
    rng = np.random.default_rng(0)
    R0, t0 = _perturb(q.R, q.t, rng, 1e-3, 1e-3)
    tau = 1e6  # every point an inlier: the cost is the plain weighted sum of squares
    cost, H, g, cnt = orc.normal_equations((R0, t0), q.corr(), q.K, tau)
    assert cnt == 400

    def cost_at(d):
        return orc.normal_equations(orc.pose_update((R0, t0), d), q.corr(), q.K, tau)[0]

    h = 1e-6
    num_g = np.zeros(6)
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        num_g[k] = (cost_at(e) - cost_at(-e)) / (2 * h)
    # d(cost)/d(delta) = 2 g
    np.testing.assert_allclose(num_g, 2 * g, rtol=1e-5, atol=1e-6 * np.abs(g).max())
    # at a zero-residual pose the Hessian of the cost/2 equals J^T J
    cost_t, H_t, g_t, _ = orc.normal_equations((q.R, q.t), q.corr(), q.K, tau)

    def grad_at(d):
        return orc.normal_equations(orc.pose_update((q.R, q.t), d), q.corr(), q.K, tau)[2]

    num_H = np.zeros((6, 6))
    for k in range(6):
        e = np.zeros(6)
        e[k] = 1e-6
        num_H[:, k] = (grad_at(e) - grad_at(-e)) / 2e-6
    np.testing.assert_allclose(num_H, H_t, rtol=2e-4, atol=1e-4 * np.abs(H_t).max())


def test_lo_converges_noise_free(orc):
    q = synth.make_query(12, 1500, 0.5, 0.0)
    rng = np.random.default_rng(1)
    R0, t0 = _perturb(q.R, q.t, rng, 0.01, 0.02)
    R, t, cost, cnt, acc = orc.lo((R0, t0), q.corr(), q.K, 4.0, iters=10)
    assert acc >= 3
    assert rot_angle(R, q.R) < 1e-7 and np.linalg.norm(t - q.t) < 1e-6
    assert cnt >= q.is_inlier.sum()


def _reproj_vec(params, corr, K, sqrt_w):
    R = Rotation.from_rotvec(params[:3]).as_matrix()
    t = params[3:]
    X = np.stack([corr["X"], corr["Y"], corr["Z"]], 1).astype(np.float64)
    xc = X @ R.T + t
    fx, fy, cx, cy = K
    du = fx * xc[:, 0] / xc[:, 2] + cx - corr["u"].astype(np.float64)
    dv = fy * xc[:, 1] / xc[:, 2] + cy - corr["v"].astype(np.float64)
    return du, dv


def test_lo_fixed_point_matches_scipy_lsq(orc):
    q = synth.make_query(13, 3000, 0.4, 1.0)
    rng = np.random.default_rng(2)
    R0, t0 = _perturb(q.R, q.t, rng, 0.002, 0.01)
    R, t, cost, cnt, acc = orc.lo((R0, t0), q.corr(), q.K, 4.0, iters=30)
    # the inlier set at the result, held fixed: the LO pose is its least-squares optimum
    cnt_chk, _ = orc.score([(R, t)], q.corr(), q.K, 4.0)
    X = np.stack([q.X, q.Y, q.Z], 1).astype(np.float64)
    xc = X @ R.T + t
    du = 500 * xc[:, 0] / xc[:, 2] + 320 - q.u
    dv = 500 * xc[:, 1] / xc[:, 2] + 240 - q.v
    inl = (xc[:, 2] > 0) & (du * du + dv * dv < 16.0)
    sub = {k: np.asarray(v)[inl] for k, v in q.corr().items() if v is not None}

    def f(p):
        a, b = _reproj_vec(p, sub, q.K, None)
        return np.concatenate([a, b])

    p0 = np.concatenate([Rotation.from_matrix(R0).as_rotvec(), t0])
    res = least_squares(f, p0, xtol=1e-15, ftol=1e-15, gtol=1e-15, method="lm")
    Rs = Rotation.from_rotvec(res.x[:3]).as_matrix()
    assert rot_angle(R, Rs) < 1e-9 and np.linalg.norm(t - res.x[3:]) < 1e-8
    assert cnt == cnt_chk[0] == inl.sum()


def test_lo_cost_non_increasing(orc):
    q = synth.make_query(14, 2000, 0.3, 1.0)
    rng = np.random.default_rng(3)
    R0, t0 = _perturb(q.R, q.t, rng, 0.05, 0.2)
    c0 = orc.score([(R0, t0)], q.corr(), q.K, 4.0)[1][0]
    prev = c0
    for it in range(1, 8):
        _, _, cost, _, _ = orc.lo((R0, t0), q.corr(), q.K, 4.0, iters=it)
        assert cost <= prev + 1e-9 * abs(prev)
        prev = cost


def test_lo_run_ends_as_read(orc):
    """The run's control flow, retold from the oracle's own pieces (normal
    equations, left update) with a numpy solve: a step is taken only if it
    is at least 1e-10 long and does not raise the cost; the run ends at the
    first step that fails either test, or at the cap (never reached here: 50)."""
    ends = []
    for seed, n, eps, sigma in ((15, 2500, 0.4, 1.0), (16, 1200, 0.6, 0.0), (17, 4000, 0.2, 1.5)):
        q = synth.make_query(seed, n, eps, sigma)
        rng = np.random.default_rng(seed)
        R0, t0 = _perturb(q.R, q.t, rng, 0.01, 0.03)
        R, t, cost, cnt, acc = orc.lo((R0, t0), q.corr(), q.K, 4.0, iters=50)
        cur = (R0, t0)
        c_cur, H, g, _ = orc.normal_equations(cur, q.corr(), q.K, 4.0)
        taken, end = 0, "cap"
        for _ in range(50):
            d = np.linalg.solve(H, -g)
            if d @ d < 1e-20:
                end = "short step"
                break
            cand = orc.pose_update(cur, d)
            c_new, H2, g2, _ = orc.normal_equations(cand, q.corr(), q.K, 4.0)
            if not c_new <= c_cur:
                end = "cost rise"
                break
            cur, c_cur, H, g = cand, c_new, H2, g2
            taken += 1
        assert acc == taken < 50, (seed, acc, taken)
        assert rot_angle(R, cur[0]) < 1e-12 and np.linalg.norm(t - cur[1]) < 1e-11
        ends.append(end)
    assert "short step" in ends and "cap" not in ends, ends


def test_refine_cauchy_matches_scipy(orc):
    q = synth.make_query(15, 2500, 0.5, 1.0)
    rng = np.random.default_rng(4)
    R0, t0 = _perturb(q.R, q.t, rng, 0.001, 0.005)
    tau, s = 4.0, 2.0
    R, t, cost, ninl, acc = orc.refine((R0, t0), q.corr(), q.K, tau, s, iters=40)
    X = np.stack([q.X, q.Y, q.Z], 1).astype(np.float64)
    xc = X @ R0.T + t0
    du = 500 * xc[:, 0] / xc[:, 2] + 320 - q.u
    dv = 500 * xc[:, 1] / xc[:, 2] + 240 - q.v
    inl = (xc[:, 2] > 0) & (du * du + dv * dv < tau * tau)
    assert ninl == inl.sum()
    sub = {k: np.asarray(v)[inl] for k, v in q.corr().items() if v is not None}

    def cauchy_cost(p):
        a, b = _reproj_vec(p, sub, q.K, None)
        return float(np.sum(s * s * np.log1p((a * a + b * b) / (s * s))))

    p0 = np.concatenate([Rotation.from_matrix(R0).as_rotvec(), t0])
    res = minimize(cauchy_cost, p0, method="BFGS", options=dict(gtol=1e-9, maxiter=2000))
    Rs = Rotation.from_rotvec(res.x[:3]).as_matrix()
    # same minimum: the oracle's cost is not above the library optimiser's, and the poses agree
    assert cost <= res.fun * (1 + 1e-12)
    assert abs(cost - res.fun) < 1e-9 * cost
    assert rot_angle(R, Rs) < 1e-6 and np.linalg.norm(t - res.x[3:]) < 1e-5


def test_refine_large_scale_is_weighted_lsq(orc):
    q = synth.make_query(16, 2000, 0.5, 1.0, weights="conf")
    rng = np.random.default_rng(5)
    R0, t0 = _perturb(q.R, q.t, rng, 0.001, 0.005)
    R, t, cost, ninl, acc = orc.refine((R0, t0), q.corr(), q.K, 4.0, 1e5, iters=40)
    X = np.stack([q.X, q.Y, q.Z], 1).astype(np.float64)
    xc = X @ R0.T + t0
    du = 500 * xc[:, 0] / xc[:, 2] + 320 - q.u
    dv = 500 * xc[:, 1] / xc[:, 2] + 240 - q.v
    inl = (xc[:, 2] > 0) & (du * du + dv * dv < 16.0)
    sub = {k: np.asarray(v)[inl] for k, v in q.corr().items() if v is not None}
    sw = np.sqrt(sub["w"].astype(np.float64))

    def f(p):
        a, b = _reproj_vec(p, sub, q.K, None)
        return np.concatenate([sw * a, sw * b])

    p0 = np.concatenate([Rotation.from_matrix(R0).as_rotvec(), t0])
    res = least_squares(f, p0, xtol=1e-15, ftol=1e-15, gtol=1e-15, method="lm")
    Rs = Rotation.from_rotvec(res.x[:3]).as_matrix()
    assert rot_angle(R, Rs) < 1e-8 and np.linalg.norm(t - res.x[3:]) < 1e-7


def test_refine_is_more_robust_than_lsq(orc):
    """Gross errors inside the fixed set move the Cauchy estimate less than the
    least-squares one (noise-free data, 5 % of observations shifted by 3 px)."""
    q = synth.make_query(17, 600, 1.0, 0.0)
    corr = {k: (None if v is None else np.array(v, copy=True)) for k, v in q.corr().items()}
    corr["u"][:30] += 3.0
    Rc, tc, _, nc, _ = orc.refine((q.R, q.t), corr, q.K, 4.0, 0.5, iters=30)
    Rl, tl, _, nl, _ = orc.refine((q.R, q.t), corr, q.K, 4.0, 1e6, iters=30)
    assert nc == nl == 600
    assert np.linalg.norm(tc - q.t) < 0.2 * np.linalg.norm(tl - q.t)
    assert rot_angle(Rc, q.R) < 0.2 * rot_angle(Rl, q.R)
