"""GPU path (through the C ABI) against the FP64 oracle, stage by stage and
end to end.  Tolerances:
  - sampling: bit-exact triples;
  - P3P: same solution count where the oracle does not flag the triple as
    ill-conditioned, poses within 1e-9 rad / 1e-9 relative translation;
  - scoring: the inlier count lies within the oracle's ambiguity band (1e-5 px,
    widened to the float32 evaluation bound for float32 scoring); MSAC within
    the band's bound plus float32 summation error;
  - local optimisation / refinement (float64 on both sides): poses within
    1e-9 rad / 1e-8 m;
  - final poses: 1e-3 deg and 1e-4 relative translation (floor 1 m)."""
import numpy as np
import pytest

from conftest import pose_close, rot_angle
from paper_2601_04185_amd import synth

pytestmark = pytest.mark.gpu

K1 = (500.0, 500.0, 320.0, 240.0)


@pytest.fixture(scope="module")
def pk():
    import torch
    import paper_2601_04185_amd as pk
    assert torch.cuda.is_available()
    return pk


@pytest.fixture(scope="module")
def ctx(pk):
    return pk.Context(0)


def _dev(q):
    import paper_2601_04185_amd as pk
    return pk.to_device(q)


def _poses_tensor(poses):
    import torch
    import oracle
    a = np.stack([oracle.pose_array(R, t) for R, t in poses])
    return torch.from_numpy(a).cuda()


# ---------------------------------------------------------------- sampling --
@pytest.mark.parametrize("n", [3, 7, 2000, 50000])
@pytest.mark.parametrize("h0", [0, 123456])
def test_sample_triples_bit_exact(pk, ctx, orc, n, h0):
    q = synth.make_query(50 + n, n, 0.5, 1.0)
    d = _dev(q)
    out = pk.imloc_sample_p3p(ctx, d, q.K, seed=7, query_id=3, h0=h0, count=1500, want_triples=True)
    tri = out["triples"].cpu().numpy()
    for s in range(1500):
        ok, idx = orc.sample_triple(7, 3, h0 + s, n)
        assert list(tri[s]) == (list(idx) if ok else [-1, -1, -1]), s


def test_exhaustive_triples_bit_exact(pk, ctx, orc):
    q = synth.make_query(60, 15, 0.5, 1.0)
    out = pk.imloc_sample_p3p(ctx, _dev(q), q.K, 0, 0, 0, 460, exhaustive=1, want_triples=True)
    tri = out["triples"].cpu().numpy()
    for h in range(460):
        ok, idx = orc.unrank_triple(h, 15)
        assert list(tri[h]) == (list(idx) if ok else [-1, -1, -1])


# --------------------------------------------------------------------- P3P --
def _gpu_candidates(pk, ctx, q, h0, count, seed=0, qid=0):
    out = pk.imloc_sample_p3p(ctx, _dev(q), q.K, seed, qid, h0, count)
    P = out["poses"].cpu().numpy()
    H = out["h"].cpu().numpy()
    J = out["j"].cpu().numpy()
    by = {}
    for k in range(len(H)):
        by.setdefault(int(H[k]), {})[int(J[k])] = (P[k, :9].reshape(3, 3), P[k, 9:])
    return by


def test_p3p_parity(pk, ctx, orc):
    q = synth.config1_single_small()
    by = _gpu_candidates(pk, ctx, q, 0, 2048)
    checked = mismatched_ill = 0
    for h in range(2048):
        ok, idx = orc.sample_triple(0, 0, h, q.n)
        assert ok
        uv = np.stack([q.u[idx], q.v[idx]], 1).astype(np.float64)
        Xw = np.stack([q.X[idx], q.Y[idx], q.Z[idx]], 1).astype(np.float64)
        sols, ill = orc.p3p(uv, Xw, q.K)
        g = by.get(h, {})
        if ill:
            mismatched_ill += len(g) != len(sols)
            continue
        assert len(g) == len(sols), (h, len(g), len(sols))
        for j, (R, t) in enumerate(sols):
            Rg, tg = g[j]
            assert rot_angle(Rg, R) < 1e-9, (h, j)
            assert np.linalg.norm(tg - t) < 1e-9 * max(1.0, np.linalg.norm(t)), (h, j)
        checked += 1
    assert checked > 1800


def test_p3p_true_pose_noise_free(pk, ctx, orc):
    q = synth.make_query(61, 600, 1.0, 0.0)
    by = _gpu_candidates(pk, ctx, q, 0, 600)
    hits = 0
    for h, g in by.items():
        best = min(rot_angle(R, q.R) for R, _ in g.values())
        hits += best < 1e-4  # float32-rounded inputs: a three-point solve is ~1e-6 relative
        for R, t in g.values():
            assert np.abs(R.T @ R - np.eye(3)).max() < 1e-12 and abs(np.linalg.det(R) - 1) < 1e-12
    assert hits >= 0.99 * len(by) and len(by) > 590


# ----------------------------------------------------------------- scoring --
def _oracle_pose_set(orc, q, count=300, seed=0):
    rng = np.random.default_rng(seed)
    poses = [(q.R, q.t)]
    for h in range(count):
        ok, idx = orc.sample_triple(seed, 0, h, q.n)
        uv = np.stack([q.u[idx], q.v[idx]], 1).astype(np.float64)
        Xw = np.stack([q.X[idx], q.Y[idx], q.Z[idx]], 1).astype(np.float64)
        poses += orc.p3p(uv, Xw, q.K)[0]
    poses += [(synth.random_rotation(rng), synth.random_translation(rng, 5)) for _ in range(17)]
    return poses


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("n,weights", [(2000, "ones"), (1, "ones"), (65, "conf"), (4097, "conf"), (70001, "ones")])
def test_score_parity(pk, ctx, orc, precision, n, weights):
    q = synth.make_query(70 + n, n, 0.4, 1.0, weights=weights)
    poses = _oracle_pose_set(orc, q, count=150 if n > 10000 else 300)
    tau = 4.0
    cnt, ms = pk.imloc_score(ctx, _dev(q), q.K, _poses_tensor(poses), tau, precision)
    cnt, ms = cnt.cpu().numpy(), ms.cpu().numpy()
    lo, hi, eb = orc.score_band(poses, q.corr(), q.K, tau, band_abs=1e-5, with_f32=(precision == 0))
    ocnt, oms = orc.score(poses, q.corr(), q.K, tau)
    assert np.all(cnt >= lo) and np.all(cnt <= hi)
    if precision == 1:
        assert np.mean(cnt == ocnt) > 0.99
        tol = eb + 1e-11 * oms
    else:
        tol = eb + tau * tau * 2e-5 * hi + 1e-6 * oms
    assert np.all(np.abs(ms - oms) <= tol + 1e-9)


@pytest.mark.parametrize("n", [700, 4097, 70001])
def test_score_tiles_give_identical_scores(pk, orc, n):
    """The scoring kernel's tiling (candidates and correspondences per work
    item, workgroups) changes no score: every per-candidate count and
    truncated cost is bitwise the same for every shape, and inside the
    oracle's band."""
    q = synth.make_query(170 + n, n, 0.4, 1.0, weights="conf")
    poses = _oracle_pose_set(orc, q, count=130)
    lo, hi, _ = orc.score_band(poses, q.corr(), q.K, 4.0, band_abs=1e-5, with_f32=True)
    ref = None
    for ct, wg, pts in [(128, 2048, 2048), (32, 300, 512), (64, 1024, 1024), (128, 4096, 4096), (32, 7, 4096),
                        (64, 513, 512), (0, 0, 2048), (32, 0, 512)]:
        c = pk.Context(0)
        c.set_score_tuning(ct, wg)
        c.set_score_points(pts)
        assert c.score_points() == pts
        cnt, ms = pk.imloc_score(c, _dev(q), q.K, _poses_tensor(poses), 4.0, 0)
        cur = (cnt.cpu().numpy(), ms.cpu().numpy())
        assert np.all(cur[0] >= lo) and np.all(cur[0] <= hi), (ct, wg, pts)
        if ref is None:
            ref = cur
        np.testing.assert_array_equal(cur[0], ref[0])
        np.testing.assert_array_equal(cur[1], ref[1])


def test_score_points_rejects_other_values(pk):
    c = pk.Context(0)
    for bad in (0, 256, 768, 3000, 8192, -1):
        with pytest.raises(pk.ImlocError):
            c.set_score_points(bad)
    assert c.score_points() == 2048


def test_score_tuning_rejects_other_values(pk):
    c = pk.Context(0)
    assert c.score_tuning() == (0, 0)  # both picked per round
    for ct, wg in ((16, 0), (256, 0), (128, -1), (64, (1 << 20) + 1)):
        with pytest.raises(pk.ImlocError):
            c.set_score_tuning(ct, wg)
    assert c.score_tuning() == (0, 0)
    c.set_score_tuning(64, 1 << 20)
    assert c.score_tuning() == (64, 1 << 20)


def test_score_ragged_candidate_counts(pk, ctx, orc):
    q = synth.make_query(80, 3000, 0.3, 1.0)
    allp = _oracle_pose_set(orc, q, count=60)
    for npz in (1, 31, 32, 33, 64, 65):
        poses = allp[:npz]
        cnt, ms = pk.imloc_score(ctx, _dev(q), q.K, _poses_tensor(poses), 4.0, 0)
        lo, hi, _ = orc.score_band(poses, q.corr(), q.K, 4.0)
        c = cnt.cpu().numpy()
        assert len(c) == npz and np.all(c >= lo) and np.all(c <= hi)


@pytest.mark.parametrize("precision", [0, 1])
def test_score_non_finite_and_behind_camera(pk, ctx, orc, precision):
    """Correspondences with NaN or infinite coordinates never count as
    inliers, and points behind a candidate's camera cost tau^2 (Sec. 3.3,
    truncated reprojection cost): both sides on the same inputs."""
    import dataclasses
    q = synth.make_query(95, 4100, 0.4, 1.0)
    rng = np.random.default_rng(95)
    u, v, X, Y, Z = (a.copy() for a in (q.u, q.v, q.X, q.Y, q.Z))
    bad = rng.choice(q.n, 120, replace=False)
    u[bad[:30]] = np.nan
    v[bad[30:60]] = np.inf
    X[bad[60:90]] = np.nan
    Z[bad[90:]] = -np.inf
    # 300 inliers moved behind the true camera (reflected through its centre)
    C = -q.R.T @ q.t
    back = rng.choice(np.flatnonzero(q.is_inlier), 300, replace=False)
    P = np.stack([X[back], Y[back], Z[back]], 1).astype(np.float64)
    P = C + (C - P)
    X[back], Y[back], Z[back] = (P[:, c].astype(np.float32) for c in range(3))
    q2 = dataclasses.replace(q, u=u, v=v, X=X, Y=Y, Z=Z)
    poses = _oracle_pose_set(orc, q, count=100)
    tau = 4.0
    cnt, ms = pk.imloc_score(ctx, _dev(q2), q2.K, _poses_tensor(poses), tau, precision)
    cnt, ms = cnt.cpu().numpy(), ms.cpu().numpy()
    lo, hi, eb = orc.score_band(poses, q2.corr(), q2.K, tau, band_abs=1e-5, with_f32=(precision == 0))
    ocnt, oms = orc.score(poses, q2.corr(), q2.K, tau)
    assert np.all(cnt >= lo) and np.all(cnt <= hi)
    assert np.all(np.isfinite(ms))
    tol = eb + (1e-11 * oms if precision == 1 else tau * tau * 2e-5 * hi + 1e-6 * oms)
    assert np.all(np.abs(ms - oms) <= tol + 1e-9)


# ---------------------------------------------------- LO and refinement ----
def test_local_optimize_parity(pk, ctx, orc):
    import torch
    q = synth.make_query(90, 5000, 0.35, 1.0, weights="conf")
    rng = np.random.default_rng(0)
    from scipy.spatial.transform import Rotation
    starts = []
    for k in range(6):
        w = rng.standard_normal(3)
        w *= 0.01 * (k + 1) / np.linalg.norm(w)
        starts.append((Rotation.from_rotvec(w).as_matrix() @ q.R, q.t + rng.standard_normal(3) * 0.05 * (k + 1)))
    out, cost, cnt = pk.imloc_local_optimize(ctx, _dev(q), q.K, _poses_tensor(starts), 4.0, 10)
    out, cost, cnt = out.cpu().numpy(), cost.cpu().numpy(), cnt.cpu().numpy()
    for k, s in enumerate(starts):
        R, t, c, n_in, acc = orc.lo(s, q.corr(), q.K, 4.0, 10)
        assert rot_angle(out[k, :9].reshape(3, 3), R) < 1e-9
        assert np.linalg.norm(out[k, 9:] - t) < 1e-8
        assert abs(cost[k] - c) <= 1e-9 * c
        assert abs(int(cnt[k]) - n_in) <= 1


def test_refine_parity(pk, ctx, orc):
    import torch
    q = synth.make_query(91, 8000, 0.5, 1.0, weights="conf")
    start = (q.R, q.t + np.array([0.01, -0.02, 0.01]))
    st = torch.from_numpy(orc.pose_array(*start)).cuda()
    mask = torch.empty(q.n, dtype=torch.uint8, device="cuda")
    out, cost = pk.imloc_refine(ctx, _dev(q), q.K, st, 4.0, 2.0, 10, mask=mask)
    R, t, c, ninl, acc = orc.refine(start, q.corr(), q.K, 4.0, 2.0, 10)
    o = out.cpu().numpy()
    assert rot_angle(o[:9].reshape(3, 3), R) < 1e-9 and np.linalg.norm(o[9:] - t) < 1e-8
    assert abs(cost.item() - c) <= 1e-9 * c
    cnt, _ = orc.score([(R, t)], q.corr(), q.K, 4.0)
    assert abs(int(mask.sum().item()) - int(cnt[0])) <= 1


# ------------------------------------------------------------- end to end --
def _run_both(pk, ctx, orc, q, **kw):
    import torch
    prm = pk.make_params(**kw)
    mask = torch.empty(max(q.n, 1), dtype=torch.uint8, device="cuda")
    rc, R, t, st = pk.imloc_lo_ransac_pnp(ctx, _dev(q), q.K, prm, mask=mask)
    okw = {k: v for k, v in kw.items() if k != "precision"}
    ref = orc.lo_ransac_pnp(q.corr(), q.K, **okw)
    return rc, R, t, st, mask[:q.n].cpu().numpy(), ref


def test_ransac_config1_fp64(pk, ctx, orc):
    q = synth.config1_single_small()
    rc, R, t, st, mask, ref = _run_both(pk, ctx, orc, q, threshold_px=4.0, fixed_samples=1024, batch=1024,
                                        lo_top_k=1, precision=1)
    assert rc == 0 and ref["status"] == 0
    ok, ang, dt = pose_close(R, t, ref["R"], ref["t"])
    assert ok, (ang, dt)
    assert st["samples"] == ref["samples"] == 1024
    assert st["candidates"] == ref["candidates"]
    assert (st["best_h"], st["best_j"]) == (ref["best_h"], ref["best_j"])
    assert st["best_count"] == ref["best_count"]
    assert abs(st["best_msac"] - ref["best_msac"]) <= 1e-9 * ref["best_msac"]
    assert np.sum(mask != ref["mask"]) <= 1
    assert np.abs(R.T @ R - np.eye(3)).max() < 1e-12 and abs(np.linalg.det(R) - 1) < 1e-12


def test_ransac_config2_full_size_fp32(pk, ctx, orc):
    q = synth.config2_single_large()
    rc, R, t, st, mask, ref = _run_both(pk, ctx, orc, q, threshold_px=6.0, fixed_samples=10000, batch=10000,
                                        lo_top_k=8, precision=0)
    assert rc == 0 and ref["status"] == 0
    ok, ang, dt = pose_close(R, t, ref["R"], ref["t"])
    assert ok, (ang, dt)
    assert st["candidates"] == ref["candidates"]
    assert abs(st["full_count"] - ref["full_count"]) <= 2
    assert np.sum(mask != ref["mask"]) <= 2
    # and the ground truth is recovered at the paper's finest recall threshold
    assert np.degrees(rot_angle(R, q.R)) < 2.0 and np.linalg.norm(t - q.t) < 0.25


@pytest.mark.parametrize("eps,conf", [(0.6, 0.999), (0.15, 0.999), (0.08, 0.9999)])
def test_ransac_adaptive_stopping(pk, ctx, orc, eps, conf):
    q = synth.make_query(100 + int(eps * 100), 4000, eps, 1.0)
    rc, R, t, st, mask, ref = _run_both(pk, ctx, orc, q, threshold_px=4.0, batch=1024, min_iters=1024,
                                        max_iters=20000, confidence=conf, lo_top_k=4)
    assert rc == 0
    assert st["samples"] == ref["samples"] and st["batches"] == ref["batches"]
    assert pose_close(R, t, ref["R"], ref["t"])[0]


def test_ransac_subsample_and_weights(pk, ctx, orc):
    q = synth.make_query(110, 12000, 0.3, 1.0, weights="conf")
    rc, R, t, st, mask, ref = _run_both(pk, ctx, orc, q, threshold_px=4.0, fixed_samples=2048, batch=1024,
                                        max_score_points=3000, lo_top_k=8)
    assert rc == 0
    assert st["residuals"] == ref["residuals"] == st["candidates"] * 3000
    assert pose_close(R, t, ref["R"], ref["t"])[0]


def test_ransac_paper_mode(pk, ctx, orc):
    """The paper's own settings (Sec. 3.3 "Pose Estimation"): stride subsample
    to at most 10,000 scoring points, batches of 1,000 minimal sets, local
    optimisation of a new best, stop at 100,000 samples or once the
    probability that an all-inlier sample was never drawn falls under 1e-4, confidence-weighted costs, final
    Cauchy refinement over the full set."""
    q = synth.make_query(120, 50000, 0.25, 1.5, weights="conf", n_views=10)
    rc, R, t, st, mask, ref = _run_both(pk, ctx, orc, q, threshold_px=6.0, batch=1000, min_iters=1000,
                                        max_iters=100000, confidence=0.9999, max_score_points=10000, lo_top_k=1)
    assert rc == 0 and ref["status"] == 0
    assert st["samples"] == ref["samples"] and st["batches"] == ref["batches"]
    assert st["residuals"] == ref["residuals"] == st["candidates"] * 10000
    assert pose_close(R, t, ref["R"], ref["t"])[0]
    assert np.degrees(rot_angle(R, q.R)) < 2.0 and np.linalg.norm(t - q.t) < 0.25
    # the library's own paper settings run the same query to the same result
    rc2, R2, t2, st2 = pk.imloc_lo_ransac_pnp(ctx, _dev(q), q.K, pk.paper_params(6.0))
    assert rc2 == 0 and st2["samples"] == st["samples"] and st2["best_h"] == st["best_h"]
    assert np.array_equal(R2, R) and np.array_equal(t2, t)


@pytest.mark.parametrize("n", [0, 1, 2])
def test_ransac_too_few_points(pk, ctx, orc, n):
    import torch
    d = {k: torch.zeros(max(n, 1), dtype=torch.float32, device="cuda")[:n] for k in ("u", "v", "X", "Y", "Z")}
    d["w"] = None
    prm = pk.make_params(fixed_samples=64)
    rc, R, t, st = pk.imloc_lo_ransac_pnp(ctx, d, K1, prm)
    assert rc == pk.IMLOC_NO_POSE and np.array_equal(R, np.eye(3)) and not t.any()


def test_invalid_arguments(pk, ctx):
    q = synth.make_query(120, 100, 0.5, 1.0)
    with pytest.raises(pk.ImlocError):
        pk.imloc_lo_ransac_pnp(ctx, _dev(q), (0.0, 500.0, 320.0, 240.0), pk.make_params(fixed_samples=8))
    with pytest.raises(pk.ImlocError):
        pk.imloc_lo_ransac_pnp(ctx, _dev(q), K1, pk.make_params(threshold_px=-1.0, fixed_samples=8))


def test_batch_equals_single(pk, ctx):
    qs = [synth.make_query(130 + i, n, e, 1.0) for i, (n, e) in enumerate([(3000, 0.4), (9000, 0.2), (500, 0.6)])]
    prms = [pk.make_params(threshold_px=4.0, fixed_samples=2048, query_id=i) for i in range(3)]
    singles = [pk.imloc_lo_ransac_pnp(ctx, _dev(q), q.K, p) for q, p in zip(qs, prms)]
    status, poses, stats = pk.imloc_lo_ransac_pnp_batch(ctx, [_dev(q) for q in qs], [q.K for q in qs], prms)
    for i in range(3):
        assert status[i] == singles[i][0] == 0
        assert np.array_equal(poses[i][0], singles[i][1]) and np.array_equal(poses[i][1], singles[i][2])


# ------------------------------------------------------------------- lift --
def test_lift_parity_scene(pk, ctx, orc):
    import torch
    wl = synth.config4_lift_scene(n_views=4, per_view=3000, seed=140)
    m = {k: torch.from_numpy(v).cuda() for k, v in wl.matches.items()}
    depth = torch.from_numpy(wl.depth).cuda()
    for sub in (True, False):
        g = pk.imloc_lift(ctx, m, depth, wl.cams, wl.poses, subpixel=sub)
        ref = orc.lift(wl.matches, wl.depth, wl.cams, wl.poses, subpixel=sub)
        assert g["n"] == len(ref["src"])
        np.testing.assert_array_equal(g["src"].cpu().numpy(), ref["src"])
        for k in ("u", "v", "w"):
            np.testing.assert_array_equal(g[k].cpu().numpy(), ref[k].astype(np.float32))
        for k in ("X", "Y", "Z"):
            a = g[k].cpu().numpy().astype(np.float64)
            b = ref[k]
            assert np.all(np.abs(a - b) <= 1.01 * np.spacing(np.abs(b).astype(np.float32)).astype(np.float64) + 1e-12)


def test_lift_edge_cases(pk, ctx, orc):
    import torch
    H, W = 48, 64
    depth = np.full((2, H, W), 4.0, np.float32)
    depth[0, 10, 20] = 0.0
    depth[0, 20, 30] = np.nan
    depth[0, 30, 40] = np.inf
    depth[0, 40, 50] = -1.0
    cases = [(5.0, 5.0, 0, 0.9), (5.0, 5.0, 0, np.float32(0.05)),
             (5.0, 5.0, 0, np.nextafter(np.float32(0.05), np.float32(1))), (20.8, 10.8, 0, 0.9),
             (20.2, 10.2, 0, 0.9), (30.6, 20.6, 0, 0.9), (40.6, 30.6, 0, 0.9), (50.6, 40.6, 0, 0.9),
             (0.5, 0.5, 0, 0.9), (0.49, 5.0, 0, 0.9), (W - 0.5, 5.0, 0, 0.9), (W - 0.51, H - 0.51, 0, 0.9),
             (5.0, H - 0.5, 0, 0.9), (5.0, 5.0, 2, 0.9), (5.0, 5.0, -1, 0.9), (np.nan, 5.0, 0, 0.9),
             (5.0, np.inf, 0, 0.9), (22.6, 10.6, 1, 0.9)]
    n = len(cases)
    mt = dict(q_u=np.arange(n, dtype=np.float32), q_v=np.arange(n, dtype=np.float32),
              db_u=np.array([c[0] for c in cases], np.float32), db_v=np.array([c[1] for c in cases], np.float32),
              conf=np.array([c[3] for c in cases], np.float32), view=np.array([c[2] for c in cases], np.int32))
    cams = np.tile(np.array(K1), (2, 1))
    poses = np.zeros((2, 12))
    poses[:, [0, 4, 8]] = 1.0
    m = {k: torch.from_numpy(v).cuda() for k, v in mt.items()}
    for sub in (True, False):
        g = pk.imloc_lift(ctx, m, torch.from_numpy(depth).cuda(), cams, poses, subpixel=sub)
        ref = orc.lift(mt, depth, cams, poses, subpixel=sub)
        np.testing.assert_array_equal(g["src"].cpu().numpy(), ref["src"])
    # empty input and a capacity smaller than the kept count
    e = {k: v[:0] for k, v in m.items()}
    assert pk.imloc_lift(ctx, e, torch.from_numpy(depth).cuda(), cams, poses)["n"] == 0
    g = pk.imloc_lift(ctx, m, torch.from_numpy(depth).cuda(), cams, poses, capacity=2)
    ref = orc.lift(mt, depth, cams, poses)
    assert g["n"] == len(ref["src"]) and g["src"].cpu().numpy().tolist() == ref["src"][:2].tolist()


def test_lift_then_ransac_end_to_end(pk, ctx, orc):
    import torch
    wl = synth.config4_lift_scene(n_views=5, per_view=4000, seed=150)
    m = {k: torch.from_numpy(v).cuda() for k, v in wl.matches.items()}
    g = pk.imloc_lift(ctx, m, torch.from_numpy(wl.depth).cuda(), wl.cams, wl.poses)
    ref_l = orc.lift(wl.matches, wl.depth, wl.cams, wl.poses)
    corr = {k: g[k] for k in ("u", "v", "X", "Y", "Z", "w")}
    prm = pk.make_params(threshold_px=4.0, batch=1024, min_iters=1024, max_iters=20000, confidence=0.999)
    rc, R, t, st = pk.imloc_lo_ransac_pnp(ctx, corr, wl.K_query, prm)
    ref = orc.lo_ransac_pnp({k: ref_l[k] for k in ("u", "v", "X", "Y", "Z", "w")}, wl.K_query, threshold_px=4.0,
                            batch=1024, min_iters=1024, max_iters=20000, confidence=0.999)
    assert rc == 0 and ref["status"] == 0
    assert pose_close(R, t, ref["R"], ref["t"])[0]
    assert np.degrees(rot_angle(R, wl.R)) < 2.0 and np.linalg.norm(t - wl.t) < 0.25
