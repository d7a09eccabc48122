"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times, on sampled outputs the oracle computes one by one.

- The 256-query batch (correspondences uniform in [5,000, 80,000], inlier
  ratios in [10 %, 60 %], 4,096 samples each, LO on the top 8), run as one
  fused call replayed as a captured graph with the autotuner's shape (128
  candidates x 2,048 correspondences per item, 8,192 workgroups): every query
  reports a pose with a rotation matrix and 4,096 samples; the smallest, the
  largest and three more queries match the float64 oracle within the
  end-to-end tolerance (1e-3 deg, 1e-4 relative translation), with the same
  candidate count and the final inlier count within 2 (float32 scoring ranks
  candidates of nearly equal cost in its own rounding, so the winning (h, j)
  may differ from the oracle's; the float64 configuration checks it).
- Lifting of 20 views x 8,000 matches: the kept set and source indices equal
  the oracle's, the lifted points within 1.01 float32 ulp.
- Beyond the workloads: a query of 2,000,000 correspondences against the
  oracle, and one fused call of 1,500 small queries against the same queries
  run alone.
"""
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


def test_batch256_full_size_sampled_against_oracle(pk, orc):
    qs = synth.config3_batch(256)
    ds = [pk.to_device(q) for q in qs]
    prms = [dict(threshold_px=4.0, fixed_samples=4096, batch=4096, lo_top_k=8, query_id=i) for i in range(len(qs))]
    ctx = pk.Context(0, graphs=True)
    ctx.set_score_tuning(128, 8192)
    ctx.set_score_points(2048)
    batch = pk.BatchQueries(ds, [q.K for q in qs], [pk.make_params(**p) for p in prms])
    for _ in range(2):  # captured, then replayed
        status, poses, stats = pk.imloc_lo_ransac_pnp_batch(ctx, batch, arrays=True)
    assert ctx.graph_counters()[1] >= 1
    assert np.all(status == 0)
    assert np.all(stats["samples"] == 4096)
    R = poses[:, :9].reshape(-1, 3, 3)
    assert np.abs(np.einsum("nji,njk->nik", R, R) - np.eye(3)).max() < 1e-12
    assert np.abs(np.linalg.det(R) - 1).max() < 1e-12
    ns = np.array([q.n for q in qs])
    sample = sorted({int(np.argmin(ns)), int(np.argmax(ns)), 0, 101, 255})
    for i in sample:
        ref = orc.lo_ransac_pnp(qs[i].corr(), qs[i].K, **prms[i])
        assert ref["status"] == 0
        ok, ang, dt = pose_close(R[i], poses[i, 9:], ref["R"], ref["t"])
        assert ok, (i, ang, dt)
        assert int(stats[i]["candidates"]) == ref["candidates"], i
        assert abs(int(stats[i]["full_count"]) - ref["full_count"]) <= 2, i


def test_lift_full_size_against_oracle(pk, orc):
    import torch
    wl = synth.config4_lift_scene()
    m = {k: torch.from_numpy(v).cuda() for k, v in wl.matches.items()}
    depth = torch.from_numpy(wl.depth).cuda()
    assert depth.shape == (20, 480, 640) and m["q_u"].numel() == 160000
    ctx = pk.Context(0)
    g = pk.imloc_lift(ctx, m, depth, wl.cams, wl.poses)
    ref = orc.lift(wl.matches, wl.depth, wl.cams, wl.poses)
    assert g["n"] == len(ref["src"])
    np.testing.assert_array_equal(g["src"].cpu().numpy(), ref["src"])
    for k in ("u", "v", "w"):
        np.testing.assert_array_equal(g[k].cpu().numpy(), ref[k].astype(np.float32))
    for k in ("X", "Y", "Z"):
        a = g[k].cpu().numpy().astype(np.float64)
        b = ref[k]
        assert np.all(np.abs(a - b) <= 1.01 * np.spacing(np.abs(b).astype(np.float32)).astype(np.float64) + 1e-12)


def test_query_ten_times_the_largest_workload_against_oracle(pk, orc):
    """One query of 2,000,000 correspondences (ten times the largest query of
    the serving workload), 1,024 samples, LO on the top 8: the whole pipeline
    against the float64 oracle."""
    import torch
    q = synth.make_query(77, 2_000_000, 0.3, 1.0)
    d = pk.to_device(q)
    kw = dict(threshold_px=4.0, fixed_samples=1024, batch=1024, lo_top_k=8)
    ctx = pk.Context(0)
    mask = torch.empty(q.n, dtype=torch.uint8, device="cuda")
    rc, R, t, st = pk.imloc_lo_ransac_pnp(ctx, d, q.K, pk.make_params(**kw), mask=mask)
    ref = orc.lo_ransac_pnp(q.corr(), q.K, **kw)
    assert rc == 0 and ref["status"] == 0
    ok, ang, dt = pose_close(R, t, ref["R"], ref["t"])
    assert ok, (ang, dt)
    assert st["candidates"] == ref["candidates"]
    assert st["residuals"] == ref["candidates"] * q.n
    assert abs(st["full_count"] - ref["full_count"]) <= 4
    assert int((mask.cpu().numpy() != ref["mask"]).sum()) <= 4


def test_batch_of_many_small_queries_equals_alone(pk):
    """1,500 queries of 6 to 400 correspondences in one fused call (the work
    list's per-thread query segments, ragged candidate tiles, tiny chunks): every
    result equals the query run alone, bit for bit, on a sample."""
    rng = np.random.default_rng(5)
    nq = 1500
    ns = rng.integers(6, 401, nq)
    qs = [synth.make_query(9000 + i, int(ns[i]), float(rng.uniform(0.3, 0.8)), 1.0) for i in range(nq)]
    ds = [pk.to_device(q) for q in qs]
    P = [pk.make_params(threshold_px=4.0, fixed_samples=64, batch=64, lo_top_k=2, query_id=i) for i in range(nq)]
    ctx = pk.Context(0)
    status, poses, stats = pk.imloc_lo_ransac_pnp_batch(ctx, pk.BatchQueries(ds, [q.K for q in qs], P), arrays=True)
    assert np.all((status == 0) | (status == pk.IMLOC_NO_POSE))
    assert np.mean(status == 0) > 0.9
    alone = pk.Context(0)
    for i in list(range(0, nq, 97)) + [nq - 1]:
        rc, R, t, st = pk.imloc_lo_ransac_pnp(alone, ds[i], qs[i].K, P[i])
        assert rc == status[i], i
        assert np.array_equal(R.reshape(9), poses[i, :9]) and np.array_equal(t, poses[i, 9:]), i
        assert st["candidates"] == stats[i]["candidates"] and st["best_count"] == stats[i]["best_count"], i
