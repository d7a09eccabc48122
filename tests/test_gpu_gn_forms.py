"""The Gauss-Newton runs (local optimisation and final refinement) have two
launch forms: fused (one launch per iteration; every workgroup of a problem
re-reduces the previous partial sums) and split (an evaluation launch and a
decision launch per iteration).  Both sum the same 512-point chunk partials in
the same order, so every output must be bitwise the same in either form, and
the automatic choice must match both."""
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


def _starts(q, k, seed):
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(seed)
    P = []
    for _ in range(k):
        R = Rotation.from_rotvec(rng.normal(0, 0.01, 3)).as_matrix() @ q.R
        P.append(np.concatenate([R.reshape(9), q.t + rng.normal(0, 0.05, 3)]))
    return np.stack(P)


@pytest.mark.parametrize("n", [1, 511, 512, 513, 5000, 50000])
def test_stage_calls_identical_in_both_forms(pk, n):
    import torch
    q = synth.make_query(900 + n % 97, n, 0.4, 1.0, weights="conf")
    d = pk.to_device(q)
    start = torch.from_numpy(_starts(q, 8, n)).cuda()
    out = {}
    for mode in (1, 2, 0):
        ctx = pk.Context(0)
        ctx.set_gn_mode(mode)
        lo = pk.imloc_local_optimize(ctx, d, q.K, start, 4.0, iters=10)
        ref = pk.imloc_refine(ctx, d, q.K, start[0].contiguous(), 4.0, 2.0, iters=10)
        out[mode] = [t.cpu().numpy() for t in lo] + [t.cpu().numpy() for t in ref]
    for mode in (2, 0):
        for a, b in zip(out[1], out[mode]):
            assert np.array_equal(a, b), mode


def test_ransac_identical_in_both_forms(pk):
    """Also the inlier mask: the fused form writes it in the launch that ends
    the final refinement, the split form with the mask kernel."""
    import torch
    q = synth.make_query(911, 30000, 0.3, 1.0, weights="conf")
    prm = pk.make_params(threshold_px=4.0, fixed_samples=2048, batch=1024, lo_top_k=8)
    res, masks = {}, {}
    for mode in (1, 2):
        ctx = pk.Context(0)
        ctx.set_gn_mode(mode)
        mask = torch.full((q.n,), 7, dtype=torch.uint8, device="cuda")
        res[mode] = pk.imloc_lo_ransac_pnp(ctx, pk.to_device(q), q.K, prm, mask=mask)
        masks[mode] = mask.cpu().numpy()
    (rc1, R1, t1, s1), (rc2, R2, t2, s2) = res[1], res[2]
    assert rc1 == rc2 == 0
    assert np.array_equal(R1, R2) and np.array_equal(t1, t2)
    for key in ("samples", "best_count", "full_count", "lo_runs", "best_h", "best_j", "best_msac", "final_cost"):
        assert s1[key] == s2[key], key
    assert np.array_equal(masks[1], masks[2]) and set(np.unique(masks[1])) <= {0, 1}
    assert int(masks[1].sum()) == s1["full_count"]


def test_mask_of_a_query_without_pose(pk):
    """A query that cannot sample (two points) finishes without a pose; both
    forms leave an all-zero mask and a zero inlier count."""
    import torch
    q = synth.make_query(912, 2, 0.5, 1.0)
    prm = pk.make_params(threshold_px=4.0, fixed_samples=64)
    for mode in (1, 2):
        ctx = pk.Context(0)
        ctx.set_gn_mode(mode)
        mask = torch.full((q.n,), 7, dtype=torch.uint8, device="cuda")
        rc, R, t, st = pk.imloc_lo_ransac_pnp(ctx, pk.to_device(q), q.K, prm, mask=mask)
        assert rc == pk.IMLOC_NO_POSE and st["full_count"] == 0
        assert np.all(mask.cpu().numpy() == 0)


def test_batch_identical_in_both_forms(pk):
    qs = [synth.make_query(920 + i, n, e, 1.0) for i, (n, e) in enumerate([(4000, 0.4), (70000, 0.2), (900, 0.5),
                                                                            (25000, 0.3)])]
    P = [pk.make_params(threshold_px=4.0, fixed_samples=1024, batch=1024, query_id=i) for i in range(len(qs))]
    res = {}
    for mode in (1, 2, 0):
        ctx = pk.Context(0)
        ctx.set_gn_mode(mode)
        res[mode] = pk.imloc_lo_ransac_pnp_batch(ctx, [pk.to_device(q) for q in qs], [q.K for q in qs], P)
    for mode in (2, 0):
        for i in range(len(qs)):
            assert res[mode][0][i] == res[1][0][i]
            assert np.array_equal(res[mode][1][i][0], res[1][1][i][0]), (mode, i)
            assert np.array_equal(res[mode][1][i][1], res[1][1][i][1]), (mode, i)
            assert res[mode][2][i]["final_cost"] == res[1][2][i]["final_cost"]
            assert res[mode][2][i]["full_count"] == res[1][2][i]["full_count"]


def test_invalid_mode(pk):
    ctx = pk.Context(0)
    for bad in (-1, 3):
        with pytest.raises(Exception):
            ctx.set_gn_mode(bad)
