"""8-bit log-depth code maps on the GPU (Sec. 3.3 "Data Compression") against
the float64 oracle: the encoder bit-exact (an integer result), lifting through
code maps with the same kept matches (bit-exact source indices) and world
points within one float32 ulp, then lifting + RANSAC on code maps against the
oracle and the ground truth."""
import numpy as np
import pytest

from conftest import pose_close, rot_angle
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


def _specials():
    return np.array([0.0, -0.0, -1.0, np.nan, np.inf, -np.inf, 1e-30, 0.01, 0.2499, 0.25, 0.2500001, 127.99, 128.0,
                     128.01, 1e30, 3.4e38], np.float32)


@pytest.mark.parametrize("n", [1, 3, 4, 5, 1023, 250_001])
def test_encode_bit_exact(pk, ctx, orc, n):
    import torch
    rng = np.random.default_rng(n)
    d = np.exp(rng.uniform(np.log(0.05), np.log(400.0), n)).astype(np.float32)
    sp = _specials()
    d[: min(n, len(sp))] = sp[: min(n, len(sp))]
    got = pk.imloc_depth_encode_log8(ctx, torch.from_numpy(d).cuda()).cpu().numpy()
    np.testing.assert_array_equal(got, orc.log8_encode(d))


def test_encode_unaligned_and_levels(pk, ctx, orc):
    import torch
    lv = np.array([orc.log8_decode(c) for c in range(1, 256)], np.float32)
    base = torch.from_numpy(np.concatenate([[1.0], lv]).astype(np.float32)).cuda()
    got = pk.imloc_depth_encode_log8(ctx, base[1:]).cpu().numpy()   # a view 4 bytes off alignment
    np.testing.assert_array_equal(got, np.arange(1, 256, dtype=np.uint8))


def _check_lift(g, ref):
    assert g["n"] == len(ref["src"])
    np.testing.assert_array_equal(g["src"].cpu().numpy(), ref["src"])
    for k in ("u", "v", "w"):
        np.testing.assert_array_equal(g[k].cpu().numpy(), ref[k].astype(np.float32))
    for k in ("X", "Y", "Z"):
        a = g[k].cpu().numpy().astype(np.float64)
        b = ref[k]
        assert np.all(np.abs(a - b) <= 1.01 * np.spacing(np.abs(b).astype(np.float32)).astype(np.float64) + 1e-12)


def test_lift_log8_parity_scene(pk, ctx, orc):
    import torch
    wl = synth.config4_lift_scene(n_views=4, per_view=3000, seed=141)
    codes = orc.log8_encode(wl.depth)
    m = {k: torch.from_numpy(v).cuda() for k, v in wl.matches.items()}
    dc = torch.from_numpy(codes).cuda()
    for sub in (True, False):
        _check_lift(pk.imloc_lift(ctx, m, dc, wl.cams, wl.poses, subpixel=sub),
                    orc.lift(wl.matches, codes, wl.cams, wl.poses, subpixel=sub))


def test_lift_log8_edge_cases(pk, ctx, orc):
    import torch
    H, W = 40, 56
    codes = np.full((2, H, W), 130, np.uint8)
    codes[0, 10, 20] = 0
    codes[0, 20, 30] = 1
    codes[0, 30, 40] = 255
    codes[1] = np.arange(H * W, dtype=np.int64).reshape(H, W) % 256
    pts = [(20.9, 10.9, 0), (21.2, 11.2, 0), (30.6, 20.6, 0), (40.6, 30.6, 0), (0.5, 0.5, 0), (0.49, 3.0, 0),
           (W - 0.5, 3.0, 0), (W - 0.51, H - 0.51, 0), (3.0, H - 0.5, 0), (7.3, 9.9, 1), (1.7, 33.2, 1),
           (44.4, 2.2, 1), (5.0, 5.0, 2)]
    n = len(pts)
    mt = dict(q_u=np.arange(n, dtype=np.float32), q_v=np.arange(n, dtype=np.float32),
              db_u=np.array([p[0] for p in pts], np.float32), db_v=np.array([p[1] for p in pts], np.float32),
              conf=np.full(n, 0.9, np.float32), view=np.array([p[2] for p in pts], np.int32))
    cams = np.tile(np.array((500.0, 500.0, 320.0, 240.0)), (2, 1))
    poses = np.zeros((2, 12))
    poses[:, [0, 4, 8]] = 1.0
    m = {k: torch.from_numpy(v).cuda() for k, v in mt.items()}
    dc = torch.from_numpy(codes).cuda()
    for sub in (True, False):
        _check_lift(pk.imloc_lift(ctx, m, dc, cams, poses, subpixel=sub),
                    orc.lift(mt, codes, cams, poses, subpixel=sub))


def test_log8_lift_then_ransac(pk, ctx, orc):
    """Code maps encoded on the GPU, lifted, then LO-RANSAC: the pose matches
    the oracle on the oracle's own codes and lift, and the ground truth."""
    import torch
    wl = synth.config4_lift_scene(n_views=5, per_view=4000, seed=151)
    codes = orc.log8_encode(wl.depth)
    dc = pk.imloc_depth_encode_log8(ctx, torch.from_numpy(wl.depth).cuda())
    np.testing.assert_array_equal(dc.cpu().numpy(), codes)
    m = {k: torch.from_numpy(v).cuda() for k, v in wl.matches.items()}
    g = pk.imloc_lift(ctx, m, dc, wl.cams, wl.poses)
    ref_l = orc.lift(wl.matches, codes, wl.cams, wl.poses)
    corr = {k: g[k] for k in ("u", "v", "X", "Y", "Z", "w")}
    prm = pk.make_params(threshold_px=4.0, batch=1024, min_iters=1024, max_iters=20000, confidence=0.999)
    rc, R, t, st = pk.imloc_lo_ransac_pnp(ctx, corr, wl.K_query, prm)
    ref = orc.lo_ransac_pnp({k: ref_l[k] for k in ("u", "v", "X", "Y", "Z", "w")}, wl.K_query, threshold_px=4.0,
                            batch=1024, min_iters=1024, max_iters=20000, confidence=0.999)
    assert rc == 0 and ref["status"] == 0
    assert pose_close(R, t, ref["R"], ref["t"])[0]
    assert np.degrees(rot_angle(R, wl.R)) < 2.0 and np.linalg.norm(t - wl.t) < 0.25
