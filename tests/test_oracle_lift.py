"""Pins of the oracle's 2D-2D -> 2D-3D lifting (Sec. 3.3 "Query Time Matching
and 2D-3D Lifting": bilinear depth at sub-pixel database coordinates, plain
lookup otherwise, keep matches with valid depth and confidence above 0.05).

Pins: lifted points project back to the database pixel at the interpolated
depth; bilinear interpolation is exact for depth affine in the pixel grid;
integer lookup hits the stored texel; each validity rule drops exactly the
matches it should; order is stable."""
import numpy as np
import pytest

from paper_2601_04185_amd import synth

Kc = (500.0, 480.0, 321.0, 239.0)


def _view_pose(seed):
    rng = np.random.default_rng(seed)
    return synth.random_rotation(rng), synth.random_translation(rng, 3.0)


def _setup(depth_fn, H=48, W=64, nv=2):
    ii, jj = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    depth = np.stack([depth_fn(ii, jj, k) for k in range(nv)]).astype(np.float32)
    poses = np.zeros((nv, 12))
    for k in range(nv):
        R, t = _view_pose(100 + k)
        poses[k, :9], poses[k, 9:] = R.reshape(9), t
    cams = np.tile(np.array(Kc), (nv, 1))
    return depth, cams, poses


def _matches(du, dv, view, conf=None):
    n = len(du)
    return dict(q_u=np.arange(n, dtype=np.float32), q_v=np.arange(n, dtype=np.float32) * 0.5,
                db_u=np.asarray(du, np.float32), db_v=np.asarray(dv, np.float32),
                conf=np.full(n, 0.9, np.float32) if conf is None else np.asarray(conf, np.float32),
                view=np.asarray(view, np.int32))


def _reproject(res, poses, k):
    R, t = poses[k, :9].reshape(3, 3), poses[k, 9:]
    X = np.stack([res["X"], res["Y"], res["Z"]], 1)
    xc = X @ R.T + t
    return Kc[0] * xc[:, 0] / xc[:, 2] + Kc[2], Kc[1] * xc[:, 1] / xc[:, 2] + Kc[3], xc[:, 2]


def test_affine_depth_bilinear_exact_and_reprojects(orc):
    a, b, c = 5.0, 0.03, -0.02
    depth, cams, poses = _setup(lambda i, j, k: a + k + b * j + c * i)
    rng = np.random.default_rng(0)
    n = 500
    du = rng.uniform(0.5, 63.5 - 1e-3, n)
    dv = rng.uniform(0.5, 47.5 - 1e-3, n)
    view = rng.integers(0, 2, n)
    m = _matches(du, dv, view)
    res = orc.lift(m, depth, cams, poses, subpixel=True)
    assert len(res["src"]) == n
    for k in range(2):
        sel = m["view"][res["src"]] == k
        sub = {kk: v[sel] for kk, v in res.items()}
        pu, pv, z = _reproject(sub, poses, k)
        dus, dvs = m["db_u"][res["src"]][sel].astype(float), m["db_v"][res["src"]][sel].astype(float)
        np.testing.assert_allclose(pu, dus, atol=1e-9)
        np.testing.assert_allclose(pv, dvs, atol=1e-9)
        # depth affine in index coordinates x = u - 0.5, y = v - 0.5
        np.testing.assert_allclose(z, a + k + b * (dus - 0.5) + c * (dvs - 0.5), rtol=1e-6)
    np.testing.assert_array_equal(res["u"], m["q_u"][res["src"]])
    np.testing.assert_array_equal(res["w"], m["conf"][res["src"]].astype(np.float64))


def test_integer_lookup_hits_texel(orc):
    depth, cams, poses = _setup(lambda i, j, k: 2.0 + 0.1 * i + 0.01 * j + 3 * k)
    rng = np.random.default_rng(1)
    cols, rows = rng.integers(0, 64, 300), rng.integers(0, 48, 300)
    frac = rng.uniform(0, 0.999, (2, 300))
    m = _matches(cols + frac[0], rows + frac[1], rng.integers(0, 2, 300))
    res = orc.lift(m, depth, cams, poses, subpixel=False)
    assert len(res["src"]) == 300
    for k in range(2):
        sel = m["view"][res["src"]] == k
        _, _, z = _reproject({kk: v[sel] for kk, v in res.items()}, poses, k)
        src = res["src"][sel]
        np.testing.assert_allclose(z, depth[k, rows[src], cols[src]], rtol=1e-9)


def test_validity_rules(orc):
    H, W = 48, 64
    base = lambda i, j, k: 4.0 + 0 * i
    depth, cams, poses = _setup(base, H, W)
    depth[0, 10, 20] = 0.0
    depth[0, 20, 30] = np.nan
    depth[0, 30, 40] = np.inf
    depth[0, 40, 50] = -1.0
    cases = [  # (db_u, db_v, view, conf, kept)
        (5.0, 5.0, 0, 0.9, True),
        (5.0, 5.0, 0, np.float32(0.05), False),                           # conf must exceed 0.05
        (5.0, 5.0, 0, np.nextafter(np.float32(0.05), np.float32(1)), True),
        (20.5 + 0.3, 10.5 + 0.3, 0, 0.9, False),   # tap (10, 20) is zero
        (20.5 - 0.3, 10.5 - 0.3, 0, 0.9, False),   # tap (10, 20) as the far corner
        (30.6, 20.6, 0, 0.9, False),                # NaN tap
        (40.6, 30.6, 0, 0.9, False),                # inf tap
        (50.6, 40.6, 0, 0.9, False),                # negative tap
        (0.5, 0.5, 0, 0.9, True),                   # footprint starts at (0, 0)
        (0.49, 5.0, 0, 0.9, False),                 # footprint leaves on the left
        (W - 0.5, 5.0, 0, 0.9, False),              # right tap column W is outside
        (W - 0.51, H - 0.51, 0, 0.9, True),
        (5.0, H - 0.5, 0, 0.9, False),
        (5.0, 5.0, 2, 0.9, False),                  # view out of range
        (5.0, 5.0, -1, 0.9, False),
        (np.nan, 5.0, 0, 0.9, False),
        (5.0, np.inf, 0, 0.9, False),
        (22.6, 10.6, 0, 0.9, True),                 # taps (10..11, 22..23) are fine
        (22.6, 10.6, 1, 0.9, True),                 # view 1 has no holes
        (20.6, 10.6, 1, 0.9, True),
    ]
    m = _matches([c[0] for c in cases], [c[1] for c in cases], [c[2] for c in cases], [c[3] for c in cases])
    res = orc.lift(m, depth, cams, poses, subpixel=True)
    kept = [i for i, c in enumerate(cases) if c[4]]
    assert res["src"].tolist() == kept
    # integer lookup: only the addressed texel matters
    cases_i = [(20.2, 10.7, 0, False), (21.2, 10.7, 0, True), (63.99, 47.99, 0, True), (64.0, 5.0, 0, False),
               (-0.01, 5.0, 0, False), (30.0, 20.0, 0, False), (31.0, 20.0, 0, True)]
    m = _matches([c[0] for c in cases_i], [c[1] for c in cases_i], [c[2] for c in cases_i])
    res = orc.lift(m, depth, cams, poses, subpixel=False)
    assert res["src"].tolist() == [i for i, c in enumerate(cases_i) if c[3]]


def test_rendered_scene_correct_matches_reproject(orc):
    wl = synth.config4_lift_scene(n_views=3, per_view=600, seed=77)
    res = orc.lift(wl.matches, wl.depth, wl.cams, wl.poses, subpixel=True)
    src = res["src"]
    assert np.all(np.diff(src) > 0)
    corr = wl.correct[src]
    X = np.stack([res["X"], res["Y"], res["Z"]], 1)
    xc = X @ wl.R.T + wl.t
    fx, fy, cx, cy = wl.K_query
    e = np.hypot(fx * xc[:, 0] / xc[:, 2] + cx - res["u"], fy * xc[:, 1] / xc[:, 2] + cy - res["v"])
    # a correct match is within 1 px in the database image; its lift lands within a few px in the query
    assert np.median(e[corr]) < 2.0
    assert np.median(e[~corr]) > 20.0
    assert corr.sum() > 0.8 * wl.correct.sum()
