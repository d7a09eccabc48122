"""Pins of the oracle's hypothesis scoring (Sec. 3.3: truncated squared
reprojection error weighted by the matching confidence, every hypothesis
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
