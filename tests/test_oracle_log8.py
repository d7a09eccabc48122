"""Pins of the oracle's 8-bit log-depth codes (Sec. 3.3 "Data Compression":
depth clipped to [0.25, 128] m and quantised in log space with 256 levels;
Sec. 4.3 "Depth Quantization": the relative quantisation error stays below
1.4 %) and of lifting through code maps.

Reading: code 0 marks a pixel without depth, codes 1..255 are the levels
0.25 * 512^((c - 1) / 254) with both range ends as levels, and a depth is
encoded to its nearest level in log depth.

Pins: the range ends are levels; consecutive levels have the constant ratio
512^(1/254); every level encodes to itself; no level lies closer in log depth
than the chosen one; the largest relative error over a dense sweep of the range
attains the closed form exp(ln 512 / 508) - 1 = 1.2356 % and stays below the
paper's 1.4 %; clipping and invalid depths; lifting a constant code map puts
every point at the decoded depth on its database ray; lifting codes agrees
with lifting the float32 decoded map."""
import math

import numpy as np

from paper_2601_04185_amd import synth

STEP = math.log(512.0) / 254.0          # log-depth spacing of the levels
MAX_REL = math.expm1(STEP / 2.0)        # worst relative error of nearest-level rounding


def _levels(orc):
    return np.array([orc.log8_decode(c) for c in range(256)])


def test_range_ends_and_invalid_code(orc):
    lv = _levels(orc)
    assert lv[0] == 0.0
    assert lv[1] == 0.25
    assert abs(lv[255] - 128.0) <= 1e-13 * 128.0


def test_levels_are_geometric(orc):
    lv = _levels(orc)[1:]
    ratio = lv[1:] / lv[:-1]
    np.testing.assert_allclose(ratio, math.exp(STEP), rtol=1e-13)
    assert np.all(np.diff(lv) > 0)


def test_every_level_encodes_to_itself(orc):
    lv = _levels(orc)
    codes = orc.log8_encode(lv[1:].astype(np.float32))
    np.testing.assert_array_equal(codes, np.arange(1, 256, dtype=np.uint8))


def test_nearest_level_in_log_depth(orc):
    rng = np.random.default_rng(7)
    d = np.exp(rng.uniform(math.log(0.25), math.log(128.0), 200_000)).astype(np.float32)
    c = orc.log8_encode(d).astype(np.int64)
    assert c.min() >= 1 and c.max() <= 255
    lv = _levels(orc)
    ld = np.log(d.astype(np.float64))
    own = np.abs(np.log(lv[c]) - ld)
    for nb in (c - 1, c + 1):
        ok = (nb >= 1) & (nb <= 255)
        other = np.abs(np.log(lv[nb[ok]]) - ld[ok])
        assert np.all(own[ok] <= other + 1e-12)
    assert own.max() <= STEP / 2 + 1e-12


def test_max_relative_error_closed_form_below_paper_bound(orc):
    d = np.geomspace(0.25, 128.0, 2_000_001).astype(np.float32)
    c = orc.log8_encode(d)
    rel = np.abs(_levels(orc)[c] / d.astype(np.float64) - 1.0)
    assert rel.max() <= MAX_REL + 1e-7          # float32 inputs: 6e-8 slack
    assert rel.max() >= 0.999 * MAX_REL         # the sweep reaches the worst case
    assert MAX_REL < 0.014                      # the paper's bound
    assert abs(MAX_REL - 0.012356) < 1e-6


def test_clipping_and_invalid_depths(orc):
    d = np.array([0.01, 0.2499, 0.25, 128.0, 128.5, 1e4, 0.0, -1.0, np.nan, np.inf, -np.inf], np.float32)
    c = orc.log8_encode(d)
    np.testing.assert_array_equal(c, [1, 1, 1, 255, 255, 255, 0, 0, 0, 0, 0])


def test_monotone_encoding(orc):
    d = np.sort(np.random.default_rng(3).uniform(0.0, 200.0, 100_000)).astype(np.float32)
    c = orc.log8_encode(d).astype(np.int64)
    c = c[d > 0]
    assert np.all(np.diff(c) >= 0)


Kc = (500.0, 480.0, 321.0, 239.0)


def _scene(H=40, W=56, nv=2, seed=11):
    poses = np.zeros((nv, 12))
    rng = np.random.default_rng(seed)
    for k in range(nv):
        poses[k, :9] = synth.random_rotation(rng).reshape(9)
        poses[k, 9:] = synth.random_translation(rng, 3.0)
    return np.tile(np.array(Kc), (nv, 1)), poses


def _matches(n, H, W, nv, seed):
    rng = np.random.default_rng(seed)
    return dict(q_u=rng.uniform(0, 640, n).astype(np.float32), q_v=rng.uniform(0, 480, n).astype(np.float32),
                db_u=rng.uniform(0.0, W, n).astype(np.float32), db_v=rng.uniform(0.0, H, n).astype(np.float32),
                conf=rng.uniform(0.0, 1.0, n).astype(np.float32), view=rng.integers(0, nv, n).astype(np.int32))


def test_constant_code_map_lifts_to_decoded_depth(orc):
    H, W, nv = 40, 56, 2
    cams, poses = _scene(H, W, nv)
    codes = np.empty((nv, H, W), np.uint8)
    codes[0], codes[1] = 77, 201
    m = _matches(3000, H, W, nv, 5)
    res = orc.lift(m, codes, cams, poses)
    assert len(res["src"]) > 1000
    for k, code in ((0, 77), (1, 201)):
        sel = m["view"][res["src"]] == k
        R, t = poses[k, :9].reshape(3, 3), poses[k, 9:]
        X = np.stack([res["X"][sel], res["Y"][sel], res["Z"][sel]], 1)
        xc = X @ R.T + t
        np.testing.assert_allclose(xc[:, 2], orc.log8_decode(code), rtol=1e-12)
        du = m["db_u"][res["src"]][sel].astype(np.float64)
        np.testing.assert_allclose(Kc[0] * xc[:, 0] / xc[:, 2] + Kc[2], du, atol=1e-9)


def test_code_zero_taps_drop_the_match(orc):
    H, W, nv = 40, 56, 1
    cams, poses = _scene(H, W, nv)
    codes = np.full((nv, H, W), 120, np.uint8)
    codes[0, 10, 20] = 0
    # a bilinear footprint with (row 10, col 20) as one of its four taps
    m = dict(q_u=np.zeros(3, np.float32), q_v=np.zeros(3, np.float32),
             db_u=np.array([20.9, 21.2, 30.0], np.float32), db_v=np.array([10.9, 11.2, 30.0], np.float32),
             conf=np.full(3, 0.9, np.float32), view=np.zeros(3, np.int32))
    res = orc.lift(m, codes, cams, poses)
    np.testing.assert_array_equal(res["src"], [2])
    res_int = orc.lift(m, codes, cams, poses, subpixel=False)   # texels (10, 20), (11, 21), (30, 30)
    np.testing.assert_array_equal(res_int["src"], [1, 2])


def test_codes_agree_with_float_lift_of_decoded_maps(orc):
    H, W, nv = 40, 56, 3
    cams, poses = _scene(H, W, nv, seed=4)
    rng = np.random.default_rng(9)
    codes = rng.integers(0, 256, (nv, H, W)).astype(np.uint8)
    codes[rng.random((nv, H, W)) < 0.9] = 150 + rng.integers(0, 5, 1)[0]
    codes[rng.random((nv, H, W)) < 0.03] = 0
    dec = _levels(orc)[codes].astype(np.float32)
    m = _matches(5000, H, W, nv, 12)
    a = orc.lift(m, codes, cams, poses)
    b = orc.lift(m, dec, cams, poses)
    np.testing.assert_array_equal(a["src"], b["src"])
    for k in ("X", "Y", "Z"):
        np.testing.assert_allclose(a[k], b[k], rtol=2e-7, atol=2e-6)
