"""The loop's top-k choice of local-optimisation starts (Sec. 3.3 "Pose
Estimation"), through imloc_select_top_k, against a host sort of the same
keys: the truncated cost and inlier count that imloc_score returns for the
same poses on the GPU (the selection only orders them).  The order is a
strict total order (cost, then the larger count, then the pose index), so the
chosen indices must match exactly; exact copies of poses force equal costs
and counts, so the index decides.  Sizes span one to sixteen selection
workgroups and both selection paths (k <= 8 in one launch, k > 8 by rounds)."""
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


@pytest.fixture(scope="module")
def scene(pk):
    q = synth.make_query(4242, 4000, 0.3, 1.0)
    return q, pk.to_device(q)


def _rodrigues(w):
    th = float(np.linalg.norm(w))
    if th == 0.0:
        return np.eye(3)
    k = w / th
    Kx = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + np.sin(th) * Kx + (1 - np.cos(th)) * Kx @ Kx


def _poses(q, count, seed):
    """Perturbations of the true pose over four decades, then exact copies of
    some poses (several of the best ones among them) at other indices."""
    rng = np.random.default_rng(seed)
    out = np.zeros((count, 12))
    for i in range(count):
        s = 10.0 ** rng.uniform(-4.0, 0.0)
        R = _rodrigues(rng.normal(size=3) * s) @ q.R
        t = q.t + rng.normal(size=3) * 2.0 * s
        out[i, :9] = R.ravel()
        out[i, 9:] = t
    if count >= 8:
        src = rng.integers(0, count, size=count // 8)
        dst = rng.integers(0, count, size=count // 8)
        out[dst] = out[src]
    return out


def _expected(cnt, ms, k, gate):
    idx = [i for i in range(len(ms)) if ms[i] < gate]
    idx.sort(key=lambda i: (ms[i], -int(cnt[i]), i))
    return np.array(idx[:k], dtype=np.int64)


def _check(pk, ctx, q, d, poses, k, gate=float("inf")):
    import torch
    P = torch.tensor(poses, dtype=torch.float64, device="cuda")
    cnt, ms = pk.imloc_score(ctx, d, q.K, P, 4.0)
    sel = pk.imloc_select_top_k(ctx, d, q.K, P, 4.0, k, gate)
    want = _expected(cnt.cpu().numpy(), ms.cpu().numpy(), k, gate)
    np.testing.assert_array_equal(sel.cpu().numpy().astype(np.int64), want)
    return cnt.cpu().numpy(), ms.cpu().numpy(), want


@pytest.mark.parametrize("count,k", [(20000, 8), (20000, 1), (20000, 3), (20000, 20), (20000, 32),
                                     (3000, 8), (1025, 8), (5, 8), (9, 12)])
def test_select_matches_host_sort(pk, ctx, scene, count, k):
    q, d = scene
    _check(pk, ctx, q, d, _poses(q, count, 100 + count + k), k)


def test_select_ties_decided_by_index(pk, ctx, scene):
    """The best pose copied to 40 scattered indices: equal costs and counts
    over several waves and workgroups, so the pose index orders them."""
    q, d = scene
    poses = _poses(q, 6000, 7)
    cnt, ms, _ = _check(pk, ctx, q, d, poses, 1)
    best = int(np.lexsort((np.arange(len(ms)), -cnt, ms))[0])
    rng = np.random.default_rng(8)
    dst = rng.choice(len(poses), size=40, replace=False)
    poses[dst] = poses[best]
    for k in (8, 32):
        _, ms2, want = _check(pk, ctx, q, d, poses, k)
        assert len(set(ms2[want].tolist())) < len(want)  # the top k holds tied costs


def test_select_gate(pk, ctx, scene):
    q, d = scene
    poses = _poses(q, 5000, 11)
    cnt, ms, _ = _check(pk, ctx, q, d, poses, 8)
    srt = np.sort(ms)
    for gate in (srt[5], srt[0], float(srt[0]) - 1.0, float(np.nextafter(srt[3], np.inf))):
        _check(pk, ctx, q, d, poses, 8, gate)
        _check(pk, ctx, q, d, poses, 20, gate)


def test_select_no_poses(pk, ctx, scene):
    import torch
    q, d = scene
    sel = pk.imloc_select_top_k(ctx, d, q.K, torch.zeros((0, 12), dtype=torch.float64, device="cuda"), 4.0, 4)
    assert sel.numel() == 0


def test_select_invalid_arguments(pk, ctx, scene):
    import torch
    q, d = scene
    P = torch.tensor(_poses(q, 16, 3), dtype=torch.float64, device="cuda")
    for k in (0, 33):
        with pytest.raises(pk.ImlocError):
            pk.imloc_select_top_k(ctx, d, q.K, P, 4.0, k)
    with pytest.raises(pk.ImlocError):
        pk.imloc_select_top_k(ctx, d, q.K, P, 4.0, 4, float("nan"))
