"""Pins of the oracle's hypothesis scoring (Sec. 3.3: each match adds its
confidence times its squared reprojection error capped at the threshold, every hypothesis
against every scored correspondence).  Constructed points with exactly known
pixel residuals fix the threshold's strictness, cheirality and weighting."""
import numpy as np

from paper_2601_04185_amd import synth

K = (500.0, 500.0, 320.0, 240.0)
I3 = (np.eye(3), np.zeros(3))


def _pts(rows):
    a = np.asarray(rows, np.float64)
    d = dict(u=a[:, 0], v=a[:, 1], X=a[:, 2], Y=a[:, 3], Z=a[:, 4])
    d["w"] = a[:, 5] if a.shape[1] > 5 else None
    return d


def test_threshold_strict_and_exact_residuals(orc):
    # identity pose; X = (1, 0, 2) projects exactly to (570, 240)
    rows = [
        [570.0 - 4.0, 240.0, 1.0, 0.0, 2.0],   # r = 4 = tau  -> outlier (strict)
        [570.0 - 3.5, 240.0, 1.0, 0.0, 2.0],   # r = 3.5      -> inlier, r^2 = 12.25
        [570.0, 240.0 + 3.0, 1.0, 0.0, 2.0],   # r = 3        -> inlier, 9
        [570.0 + 3.0, 244.0, 1.0, 0.0, 2.0],   # r = 5        -> outlier
        [570.0, 240.0, -1.0, 0.0, -2.0],       # same ray behind the camera -> outlier
        [320.0, 240.0, 0.0, 0.0, 0.0],         # on the camera centre (z = 0) -> outlier
    ]
    cnt, ms = orc.score([I3], _pts(rows), K, 4.0)
    assert cnt[0] == 2
    assert ms[0] == 12.25 + 9.0 + 4 * 16.0


def test_weights(orc):
    rows = [
        [570.0 - 3.5, 240.0, 1.0, 0.0, 2.0, 0.5],
        [570.0, 243.0, 1.0, 0.0, 2.0, 0.25],
        [0.0, 0.0, 1.0, 0.0, 2.0, 2.0],
    ]
    cnt, ms = orc.score([I3], _pts(rows), K, 4.0)
    assert cnt[0] == 2
    assert ms[0] == 0.5 * 12.25 + 0.25 * 9.0 + 2.0 * 16.0


def test_translation_and_rotation_enter(orc):
    # rotate 90 deg about z: (x, y, z) -> (-y, x, z); then shift by t
    Rz = np.array([[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]])
    t = np.array([0.5, 0.0, 1.0])
    X = np.array([0.0, -1.0, 1.0])          # R X + t = (1.5, 0, 2) -> (695, 240)
    rows = [[695.0, 240.0 + 1.0, *X]]
    cnt, ms = orc.score([(Rz, t)], _pts(rows), K, 2.0)
    assert cnt[0] == 1 and ms[0] == 1.0


def test_true_pose_counts_all_noise_free_inliers(orc):
    q = synth.make_query(5, 3000, 0.3, 0.0)
    cnt, ms = orc.score([(q.R, q.t)], q.corr(), q.K, 1.0)
    assert cnt[0] >= q.is_inlier.sum()
    # inliers sit at float32 rounding distance from their projection
    assert ms[0] <= (cnt[0] - q.is_inlier.sum()) * 1.0 + q.is_inlier.sum() * 1e-6 + (3000 - cnt[0]) * 1.0 + 1e-9
    assert ms[0] >= (3000 - cnt[0]) * 1.0


def test_band_brackets_exact_count(orc):
    q = synth.make_query(6, 4000, 0.4, 1.0)
    rng = np.random.default_rng(0)
    poses = [(q.R, q.t)] + [(synth.random_rotation(rng), synth.random_translation(rng, 5)) for _ in range(8)]
    cnt, _ = orc.score(poses, q.corr(), q.K, 4.0)
    lo, hi, eb = orc.score_band(poses, q.corr(), q.K, 4.0, band_abs=1e-5, with_f32=True)
    assert np.all(lo <= cnt) and np.all(cnt <= hi)
    lo64, hi64, _ = orc.score_band(poses, q.corr(), q.K, 4.0, band_abs=1e-5, with_f32=False)
    assert np.all(lo <= lo64) and np.all(hi64 <= hi)
    # the float32 band is thin: a handful of residuals at most
    assert np.all(hi - lo <= 3)


# ---------------------------------------------------------------------------
# The float32 ambiguity band, pinned against an independent float32 evaluation
# of the division-free inlier test (rows of K[R|t] rounded to float32 with the
# first two divided by tau, three fused multiply-adds per row, u' = u * (1/tau),
# du' = a' - u' w and dv' by fused multiply-adds, e' = du'^2 + dv'^2, inlier iff
# e' < w |w|).  numpy has no float32 fma: a*b of two float32 values is exact in
# float64, so round(a*b + c) through float64 then float32 is the fused result
# except for a rare double-rounding tie.
# ---------------------------------------------------------------------------
_F32 = np.float32


def _fma32(a, b, c):
    return (a.astype(np.float64) * b.astype(np.float64) + c.astype(np.float64)).astype(_F32)


def _f32_test(R, t, K, tau, u, v, X):
    """float32 distance sqrt(e'/(w|w|)) tau the test acts on, its decision, and w."""
    fx, fy, cx, cy = K
    M = np.zeros((3, 4))
    M[0, :3] = fx * R[0] + cx * R[2]
    M[1, :3] = fy * R[1] + cy * R[2]
    M[2, :3] = R[2]
    M[0, 3], M[1, 3], M[2, 3] = fx * t[0] + cx * t[2], fy * t[1] + cy * t[2], t[2]
    p0, p1, p2 = (M[0] * (1.0 / tau)).astype(_F32), (M[1] * (1.0 / tau)).astype(_F32), M[2].astype(_F32)
    it = _F32(1.0 / tau)
    uu, vv = (u * it).astype(_F32), (v * it).astype(_F32)
    x, y, z = X[:, 0], X[:, 1], X[:, 2]
    one = np.ones(len(u), _F32)
    row = lambda p: _fma32(p[2] * one, z, _fma32(p[1] * one, y, _fma32(p[0] * one, x, p[3] * one)))
    a, b, w = row(p0), row(p1), row(p2)
    du, dv = _fma32(-uu, w, a), _fma32(-vv, w, b)
    e = _fma32(dv, dv, (du * du).astype(_F32))
    tt = (w * np.abs(w)).astype(_F32)
    with np.errstate(divide="ignore", invalid="ignore"):
        r32 = tau * np.sqrt(e.astype(np.float64) / tt.astype(np.float64))
    return r32, e < tt, w


def _near_threshold_query(rng, n, K, tau, rel=2e-5):
    """Frustum points (depth 2-20 m, |t| <= 5 m) whose observation sits within
    `rel` of tau from the true projection, in a random direction."""
    R = synth.random_rotation(rng)
    t = synth.random_translation(rng, 5.0)
    px, py, Xc = synth._frustum_points(rng, n, K, 640, 480, 2.0, 20.0)
    Xw = (Xc - t) @ R
    th = rng.random(n) * 2 * np.pi
    rr = tau * (1 + (rng.random(n) * 2 - 1) * rel)
    u = (px + rr * np.cos(th)).astype(_F32)
    v = (py + rr * np.sin(th)).astype(_F32)
    X = np.ascontiguousarray(Xw, _F32)
    corr = dict(u=u, v=v, X=X[:, 0].copy(), Y=X[:, 1].copy(), Z=X[:, 2].copy(), w=None)
    return R, t, corr, X


def test_f32_band_covers_and_is_tight(orc):
    """120,000 residuals within 2e-5 relative of the threshold: every float32
    decision that differs from the exact one lies inside the band, the float32
    distance error never exceeds the band, and the largest error reaches at
    least a fifth of its band (the bound is not several times too wide)."""
    K, tau = (500.0, 500.0, 320.0, 240.0), 4.0
    rng = np.random.default_rng(11)
    worst, flips = 0.0, 0
    for _ in range(60):
        R, t, corr, X = _near_threshold_query(rng, 2000, K, tau)
        r, beta = orc.residual_band((R, t), corr, K, tau, band_abs=0.0, with_f32=True)
        r32, inl32, _ = _f32_test(R, t, K, tau, corr["u"], corr["v"], X)
        ok = np.isfinite(r)
        assert ok.mean() > 0.99 and np.all(np.isfinite(beta[ok]))
        exact = r[ok] < tau
        flip = inl32[ok] != exact
        flips += int(flip.sum())
        assert np.all(np.abs(r[ok][flip] - tau) < beta[ok][flip])
        err = np.abs(r32[ok] - r[ok])
        assert np.all(err <= beta[ok])
        worst = max(worst, float(np.max(err / beta[ok])))
    assert flips > 1000          # the sample does exercise the threshold
    assert 0.2 <= worst <= 1.0, worst


def test_f32_band_brackets_float32_counts(orc):
    """Per candidate, the float32 inlier count of the same test lies in the
    oracle's [count_lo, count_hi] (near-threshold residuals plus a scene)."""
    K, tau = (500.0, 500.0, 320.0, 240.0), 4.0
    rng = np.random.default_rng(12)
    for _ in range(8):
        R, t, corr, X = _near_threshold_query(rng, 15000, K, tau, rel=2e-3)
        poses = [(R, t)] + [(R, t + rng.normal(0, 1e-4, 3)) for _ in range(3)]
        lo, hi, _ = orc.score_band(poses, corr, K, tau, band_abs=0.0, with_f32=True)
        cnt, _ = orc.score(poses, corr, K, tau)
        for p, (Rp, tp) in enumerate(poses):
            _, inl32, w = _f32_test(Rp, tp, K, tau, corr["u"], corr["v"], X)
            c32 = int(np.sum(inl32 & (w > 0)))
            assert lo[p] <= c32 <= hi[p], (p, lo[p], c32, hi[p])
            assert lo[p] <= cnt[p] <= hi[p]
            assert 0 < hi[p] - lo[p] < 0.25 * len(X)  # the band is thin against the 8e-3 px spread


def test_f32_band_width_matches_its_closed_form(orc):
    """The band of one residual, recomputed from its derivation in numpy."""
    K, tau = (500.0, 500.0, 320.0, 240.0), 6.0
    rng = np.random.default_rng(13)
    R, t, corr, X = _near_threshold_query(rng, 500, K, tau)
    r, beta = orc.residual_band((R, t), corr, K, tau, band_abs=0.0, with_f32=True)
    fx, fy, cx, cy = K
    P = np.zeros((3, 4))
    P[0, :3], P[1, :3], P[2, :3] = fx * R[0] + cx * R[2], fy * R[1] + cy * R[2], R[2]
    P[:, 3] = [fx * t[0] + cx * t[2], fy * t[1] + cy * t[2], t[2]]
    Xt = np.concatenate([X.astype(np.float64), np.ones((len(X), 1))], 1)
    A, B, W = (np.abs(Xt * P[k]).sum(1) for k in range(3))
    z = Xt @ P[2]
    uq = 2.0 ** -24
    u1 = 1.001 * uq
    g3, g4 = 3 * uq / (1 - 3 * uq), 4 * uq / (1 - 4 * uq)
    au, av = np.abs(corr["u"].astype(np.float64)), np.abs(corr["v"].astype(np.float64))
    k = g4 * W / z
    Pa = g4 * A + g3 * au * (z + g4 * W) + g4 * au * W
    Pb = g4 * B + g3 * av * (z + g4 * W) + g4 * av * W
    xc = X.astype(np.float64) @ R.T + t
    d = np.hypot(fx * xc[:, 0] / xc[:, 2] + cx - corr["u"], fy * xc[:, 1] / xc[:, 2] + cy - corr["v"])
    ref = (1.5 * u1 * d + ((1 + uq) * np.hypot(Pa, Pb) / z + uq * d + k * d) / (1 - k)) / (1 - 1.5 * u1)
    ok = np.isfinite(r)
    np.testing.assert_allclose(beta[ok], ref[ok], rtol=1e-12)
    # the exact distance is the textbook pinhole reprojection
    np.testing.assert_allclose(r[ok], d[ok], rtol=1e-12)
