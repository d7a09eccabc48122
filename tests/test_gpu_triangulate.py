"""Mapping-time depth by 1-DoF triangulation on the GPU (Sec. 3.3 "Depth
Estimation by Dense Matching") against the float64 oracle.

Bar: on every pixel whose angular tests all lie farther than 1e-9 rad from the
threshold (the oracle flags the others), the inlier count is equal and the
depth is the oracle's within one float32 ulp (the output is float32) plus
1e-9 relative plus the depth change that moves the refinement cost by a
relative 1e-12 at the oracle's minimum, sqrt(2e-12 E / E'') with E and E''
the oracle's cost and its second derivative: both refine to a Newton step
below 1e-12 l, so on a well-conditioned minimum they agree to float32, and on
a flat one any depth within that distance is an equally good minimiser in
float64.  Runs with fewer than 4 required inliers (below the paper's "more
than 3") can keep a pixel whose winning set is one to three nearly parallel
rays, whose cost is flat over an unbounded depth range: there depths beyond
1e4 m only have to be far on both sides; with 4 required inliers no pixel is
excused.  Flagged pixels are rare.  Integer outputs (inliers, kept or not) are
exact on unflagged pixels; codes are the oracle encoder's codes of the oracle
depth wherever the float32 depths agree."""
import numpy as np
import pytest

from paper_2601_04185_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import torch
    import paper_2601_04185_amd as pk
    assert torch.cuda.is_available()
    return pk


@pytest.fixture(scope="module")
def ctx(pk):
    return pk.Context(0)


def _run(pk, ctx, w, **kw):
    import torch
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    g = pk.imloc_triangulate_depth(ctx, w.K0, w.T0, w.Ks, w.Ts, dev(w.mu), dev(w.mv), dev(w.conf), **kw)
    return {k: v.cpu().numpy() for k, v in g.items()}


def _check(g, r, max_flagged=0.01, min_inliers=4):
    amb = r["ambiguous"]
    assert amb.mean() <= max_flagged
    ok = ~amb
    np.testing.assert_array_equal(g["inliers"][ok], r["inliers"][ok])
    ref = r["depth"].astype(np.float32).astype(np.float64)
    got = g["depth"].astype(np.float64)
    flat = np.sqrt(2e-12 * r["cost"] / np.maximum(r["curv"], 1e-300))
    tol = 1.01 * np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64) + 1e-9 * np.abs(r["depth"]) + flat
    # with fewer than 4 required inliers, a winning set of nearly parallel rays
    # leaves the depth undetermined beyond 1e4 m: both sides only have to agree
    # that it is far
    far = (r["depth"] > 1e4) if min_inliers < 4 else np.zeros_like(amb)
    assert np.all(got[ok & far] > 1e3)
    bad = ok & ~far & ~(np.abs(got - r["depth"]) <= tol)
    assert not bad.any(), list(zip(got[bad][:5], r["depth"][bad][:5], tol[bad][:5], r["inliers"][bad][:5]))
    assert np.array_equal(got[ok] > 0, r["depth"][ok] > 0)


def test_parity_noisy_scene(pk, ctx, orc):
    w = synth.dense_match_scene(n_views=10, width=96, height=72, correct_frac=0.7, noise_px=0.5, seed=31)
    g = _run(pk, ctx, w)
    r = orc.triangulate(w.K0, w.T0, w.Ks, w.Ts, w.mu, w.mv, w.conf)
    _check(g, r)
    assert (g["depth"] > 0).mean() > 0.3


@pytest.mark.parametrize("V,H,W", [(1, 23, 37), (3, 23, 37), (8, 31, 17), (9, 31, 17), (16, 19, 41), (17, 19, 41),
                                   (21, 13, 17), (24, 13, 17), (27, 9, 11), (32, 11, 13)])
def test_parity_view_counts_and_ragged_sizes(pk, ctx, orc, V, H, W):
    w = synth.dense_match_scene(n_views=V, width=W, height=H, correct_frac=0.8, noise_px=0.3, seed=40 + V,
                                f=0.8 * 96)
    for mi in (4, 1, 3):
        g = _run(pk, ctx, w, min_inliers=mi)
        r = orc.triangulate(w.K0, w.T0, w.Ks, w.Ts, w.mu, w.mv, w.conf, min_inliers=mi)
        _check(g, r, max_flagged=0.05, min_inliers=mi)


def test_noise_free_scene(pk, ctx, orc):
    w = synth.dense_match_scene(n_views=8, width=96, height=72, correct_frac=1.0, noise_px=0.0, seed=21)
    g = _run(pk, ctx, w)
    r = orc.triangulate(w.K0, w.T0, w.Ks, w.Ts, w.mu, w.mv, w.conf)
    _check(g, r)
    seen = w.correct.sum(0)
    exact = (seen >= 4) & (r["inliers"] == seen)
    rel = np.abs(g["depth"][exact] / w.depth_true[exact] - 1)
    assert np.median(rel) < 1e-7 and rel.max() < 1e-5


def test_codes_output(pk, ctx, orc):
    w = synth.dense_match_scene(n_views=6, width=64, height=48, correct_frac=0.8, noise_px=0.5, seed=33)
    g = _run(pk, ctx, w, want_codes=True)
    r = orc.triangulate(w.K0, w.T0, w.Ks, w.Ts, w.mu, w.mv, w.conf)
    ref32 = r["depth"].astype(np.float32)
    same = (g["depth"] == ref32) & ~r["ambiguous"]
    assert same.mean() > 0.9
    np.testing.assert_array_equal(g["codes"][same], orc.log8_encode(ref32)[same])


def test_edge_cases(pk, ctx, orc):
    import torch
    w = synth.dense_match_scene(n_views=5, width=40, height=30, correct_frac=0.9, noise_px=0.2, seed=34)
    conf = w.conf.copy()
    conf[:, :10, :] = 0.01                       # rows without a usable match
    mu = w.mu.copy()
    mu[2, 10:20, :] = np.nan                      # a view without coordinates
    conf[1, 20:, :] = np.float32(0.05)            # exactly at the threshold: used
    w2 = synth.DenseMatchWorkload(w.K0, w.T0, w.Ks, w.Ts, mu, w.mv, conf, w.depth_true, w.correct)
    g = _run(pk, ctx, w2)
    r = orc.triangulate(w2.K0, w2.T0, w2.Ks, w2.Ts, mu, w2.mv, conf)
    _check(g, r)
    assert np.all(g["depth"][:10] == 0) and np.all(g["inliers"][:10] == 0)
    # argument errors
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    for V in (0, 33):
        shape = (max(V, 1), 4, 4)
        z = dev(np.zeros(shape, np.float32))
        with pytest.raises(Exception):
            pk.imloc_triangulate_depth(ctx, w.K0, w.T0, np.tile(w.K0, (V, 1)), np.zeros((V, 12)), z[:V], z[:V], z[:V])
    with pytest.raises(Exception):
        pk.imloc_triangulate_depth(ctx, w.K0, w.T0, w.Ks, w.Ts, dev(w.mu), dev(w.mv), dev(w.conf), angle_deg=0.0)


def test_full_size_mapping_image(pk, ctx, orc):
    """The 560 x 560 mapping image with 10 covisible views."""
    w = synth.dense_match_scene(n_views=10, width=560, height=560, seed=1006)
    g = _run(pk, ctx, w)
    r = orc.triangulate(w.K0, w.T0, w.Ks, w.Ts, w.mu, w.mv, w.conf)
    _check(g, r, max_flagged=0.001)
    fin = np.isfinite(w.depth_true)
    ok = g["depth"] > 0
    # every surface pixel with at least 4 correct matches (the generator's own
    # record) is kept: those have 4 inliers at the true depth
    seen4 = w.correct.sum(0) >= 4
    assert ok[fin & seen4].mean() > 0.99
    rel = np.abs(g["depth"][ok & fin] / w.depth_true[ok & fin] - 1)
    assert np.median(rel) < 0.01
