"""The batched pipeline: a query's result is the same alone and in a mix of
queries of uneven sizes (bitwise: same Philox counters, integer-accumulated
scores, fixed-order float64 reductions), and does not depend on the launch
shape of the scoring kernel."""
import numpy as np
import pytest

from conftest import pose_close
from paper_2601_04185_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pk():
    import torch
    import paper_2601_04185_amd as pk
    assert torch.cuda.is_available()
    return pk


def _mix():
    specs = [  # (n, eps, sigma, weights, params)
        (3000, 0.4, 1.0, "ones", dict(fixed_samples=2048, batch=1024)),
        (20000, 0.15, 1.0, "conf", dict(confidence=0.999, batch=1024, min_iters=1024, max_iters=8192)),
        (600, 0.6, 1.0, "ones", dict(fixed_samples=512, batch=512, lo_top_k=1)),
        (12000, 0.3, 1.5, "ones", dict(fixed_samples=1024, batch=1024, max_score_points=2500)),
        (2, 0.5, 1.0, "ones", dict(fixed_samples=64)),
        (45000, 0.25, 1.0, "ones", dict(confidence=0.9999, batch=1024, min_iters=1024, max_iters=6000)),
    ]
    qs, prms = [], []
    for i, (n, e, s, w, kw) in enumerate(specs):
        qs.append(synth.make_query(300 + i, n, e, s, weights=w))
        prms.append(dict(threshold_px=4.0, query_id=i, **kw))
    return qs, prms


def test_alone_equals_in_mix(pk):
    ctx = pk.Context(0)
    qs, prms = _mix()
    P = [pk.make_params(**p) for p in prms]
    alone = [pk.imloc_lo_ransac_pnp(ctx, pk.to_device(q), q.K, p) for q, p in zip(qs, P)]
    status, poses, stats = pk.imloc_lo_ransac_pnp_batch(ctx, [pk.to_device(q) for q in qs], [q.K for q in qs], P)
    for i in range(len(qs)):
        rc, R, t, st = alone[i]
        assert status[i] == rc
        assert np.array_equal(poses[i][0], R) and np.array_equal(poses[i][1], t), i
        for key in ("samples", "candidates", "best_count", "full_count", "batches", "lo_runs", "best_h", "best_j",
                    "best_msac", "final_cost", "inlier_residuals"):
            assert stats[i][key] == st[key], (i, key)
    assert status[4] == pk.IMLOC_NO_POSE


def test_mix_matches_oracle(pk, orc):
    ctx = pk.Context(0)
    qs, prms = _mix()
    P = [pk.make_params(**p) for p in prms]
    status, poses, stats = pk.imloc_lo_ransac_pnp_batch(ctx, [pk.to_device(q) for q in qs], [q.K for q in qs], P)
    for i, (q, p) in enumerate(zip(qs, prms)):
        ref = orc.lo_ransac_pnp(q.corr(), q.K, **p)
        assert status[i] == ref["status"]
        if ref["status"] == 0:
            ok, ang, dt = pose_close(poses[i][0], poses[i][1], ref["R"], ref["t"])
            assert ok, (i, ang, dt)
            assert stats[i]["samples"] == ref["samples"]


def test_packed_batch_and_array_results_equal_lists(pk):
    """BatchQueries (descriptors packed once) with array results gives the
    list form's results, call after call."""
    ctx = pk.Context(0)
    qs, prms = _mix()
    P = [pk.make_params(**p) for p in prms]
    ds = [pk.to_device(q) for q in qs]
    status, poses, stats = pk.imloc_lo_ransac_pnp_batch(ctx, ds, [q.K for q in qs], P)
    b = pk.BatchQueries(ds, [q.K for q in qs], P)
    for _ in range(2):
        st_a, po_a, sa = pk.imloc_lo_ransac_pnp_batch(ctx, b, arrays=True)
        assert st_a.tolist() == list(status)
        for i in range(len(qs)):
            assert np.array_equal(po_a[i, :9].reshape(3, 3), poses[i][0])
            assert np.array_equal(po_a[i, 9:], poses[i][1])
            for k, v in stats[i].items():
                assert sa[i][k] == v, (i, k)


def test_tuning_does_not_change_results(pk):
    q = synth.make_query(400, 30000, 0.3, 1.0)
    d = pk.to_device(q)
    prm = pk.make_params(threshold_px=4.0, fixed_samples=3000, batch=3000)
    ref = None
    for ct, wg, pts in [(32, 64, 2048), (64, 2048, 512), (128, 517, 4096), (64, 1, 1024), (0, 4096, 2048),
                        (0, 4096, 512), (0, 0, 2048), (128, 0, 1024), (64, 100000, 4096)]:
        ctx = pk.Context(0)
        ctx.set_score_tuning(ct, wg)
        ctx.set_score_points(pts)
        rc, R, t, st = pk.imloc_lo_ransac_pnp(ctx, d, q.K, prm)
        cur = (R.tobytes(), t.tobytes(), st["best_msac"], st["inlier_residuals"], st["candidates"])
        if ref is None:
            ref = cur
        assert cur == ref, (ct, wg, pts)


def test_graph_replays_match_eager(pk):
    """A captured batch graph, replayed several times with eager work and
    synchronisation in between, and with new inputs of the same shapes, gives
    the eager results every time."""
    import torch
    eager = pk.Context(0)
    graph = pk.Context(0, graphs=True)
    shapes = [(3000, 0.4), (9000, 0.2), (700, 0.6)]
    P = [pk.make_params(threshold_px=4.0, fixed_samples=1024, batch=512, query_id=i) for i in range(3)]
    for rep in range(4):
        seed = 500 + (rep % 2) * 10  # alternate between two data sets of the same shapes
        qs = [synth.make_query(seed + i, n, e, 1.0) for i, (n, e) in enumerate(shapes)]
        ds = [pk.to_device(q) for q in qs]
        ref = pk.imloc_lo_ransac_pnp_batch(eager, ds, [q.K for q in qs], P)
        got = pk.imloc_lo_ransac_pnp_batch(graph, ds, [q.K for q in qs], P)
        torch.cuda.synchronize()
        for i in range(3):
            assert got[0][i] == ref[0][i]
            assert np.array_equal(got[1][i][0], ref[1][i][0]) and np.array_equal(got[1][i][1], ref[1][i][1])
            assert got[2][i]["best_msac"] == ref[2][i]["best_msac"]
            assert got[2][i]["inlier_residuals"] == ref[2][i]["inlier_residuals"]
    captures, launches = graph.graph_counters()
    assert captures == 1 and launches == 4
