"""Pins of the oracle's P3P (Sec. 3.3 names a P3P minimal solver; Sec. 1 cites
the Haralick et al. review, whose Grunert formulation the oracle uses).

Pins: exact triples from a known pose give the true pose among the solutions;
every solution reprojects its three points; the number of real solutions
equals an independent brute-force count of the roots of the law-of-cosines
system along a one-parameter scan; rotation invariants."""
import numpy as np
import pytest

from conftest import rot_angle
from paper_2601_04185_amd import synth

K = (500.0, 500.0, 320.0, 240.0)


def _exact_triple(rng):
    R = synth.random_rotation(rng)
    t = synth.random_translation(rng, 5.0)
    px, py = rng.random(3) * 640, rng.random(3) * 480
    z = rng.uniform(2, 20, 3)
    Xc = np.stack([(px - 320) / 500 * z, (py - 240) / 500 * z, z], 1)
    return R, t, np.stack([px, py], 1), (Xc - t) @ R


def test_true_pose_recovered_and_reprojects(orc):
    rng = np.random.default_rng(0)
    hist = np.zeros(5, int)
    for _ in range(1500):
        R, t, uv, Xw = _exact_triple(rng)
        sols, ill = orc.p3p(uv, Xw, K)
        assert 1 <= len(sols) <= 4
        hist[len(sols)] += 1
        best = min(rot_angle(Rs, R) for Rs, _ in sols)
        assert best < 1e-9
        for Rs, ts in sols:
            assert np.abs(Rs.T @ Rs - np.eye(3)).max() < 1e-12
            assert abs(np.linalg.det(Rs) - 1.0) < 1e-12
            xc = Xw @ Rs.T + ts
            assert (xc[:, 2] > 0).all()
            e = np.hypot(500 * xc[:, 0] / xc[:, 2] + 320 - uv[:, 0], 500 * xc[:, 1] / xc[:, 2] + 240 - uv[:, 1])
            assert e.max() < (1e-6 if ill else 1e-9)
    assert hist[2:].sum() > 0.3 * hist.sum()  # multiple solutions do occur


def _bruteforce_count(uv, Xw, ngrid=200001):
    """Count positive solutions of the law-of-cosines system by scanning s1.

    s2 and s3 follow from the c- and b-equations as the roots of quadratics
    (two branches each); the remaining a-equation residual changes sign at
    every solution along each branch pair."""
    j = np.stack([(uv[:, 0] - 320) / 500, (uv[:, 1] - 240) / 500, np.ones(3)], 1)
    j /= np.linalg.norm(j, axis=1, keepdims=True)
    a2 = np.sum((Xw[1] - Xw[2]) ** 2)
    b2 = np.sum((Xw[0] - Xw[2]) ** 2)
    c2 = np.sum((Xw[0] - Xw[1]) ** 2)
    ca, cb, cg = j[1] @ j[2], j[0] @ j[2], j[0] @ j[1]
    smax = min(np.sqrt(c2 / (1 - cg * cg)), np.sqrt(b2 / (1 - cb * cb)))
    s1 = np.linspace(smax * 1e-9, smax * (1 - 1e-12), ngrid)
    roots, near = 0, False
    disc2 = np.sqrt(np.maximum(c2 - s1 * s1 * (1 - cg * cg), 0.0))
    disc3 = np.sqrt(np.maximum(b2 - s1 * s1 * (1 - cb * cb), 0.0))
    for sg2 in (1, -1):
        for sg3 in (1, -1):
            s2 = s1 * cg + sg2 * disc2
            s3 = s1 * cb + sg3 * disc3
            f = s2 * s2 + s3 * s3 - 2 * s2 * s3 * ca - a2
            ok = (s2 > 0) & (s3 > 0)
            sgn = np.sign(f)
            ch = (sgn[:-1] * sgn[1:] < 0) & ok[:-1] & ok[1:]
            roots += int(ch.sum())
            # a local minimum of |f| close to zero without a sign change, or a
            # sign change at a branch end, makes the scan count unreliable
            af = np.abs(f) / max(a2, 1e-300)
            same = (sgn[:-2] == sgn[1:-1]) & (sgn[1:-1] == sgn[2:])
            loc = (af[1:-1] <= af[:-2]) & (af[1:-1] <= af[2:]) & ok[1:-1] & same
            if np.any(af[1:-1][loc] < 1e-4):
                near = True
            if ok[-1] and abs(f[-1]) / a2 < 1e-2:
                near = True
    return roots, near


def test_solution_count_matches_bruteforce(orc):
    rng = np.random.default_rng(1)
    checked = 0
    for trial in range(600):
        if trial % 2 == 0:
            _, _, uv, Xw = _exact_triple(rng)
        else:  # arbitrary triples: 0-4 solutions
            uv = np.stack([rng.random(3) * 640, rng.random(3) * 480], 1)
            Xw = rng.uniform(-10, 10, (3, 3))
        sols, ill = orc.p3p(uv, Xw, K)
        nb, near = _bruteforce_count(uv, Xw)
        if ill or near:
            continue
        assert len(sols) == nb, (trial, len(sols), nb)
        checked += 1
    assert checked > 450


def test_solutions_satisfy_distances(orc):
    rng = np.random.default_rng(2)
    for _ in range(200):
        uv = np.stack([rng.random(3) * 640, rng.random(3) * 480], 1)
        Xw = rng.uniform(-10, 10, (3, 3))
        sols, ill = orc.p3p(uv, Xw, K)
        for Rs, ts in sols:
            xc = Xw @ Rs.T + ts
            for a, b in ((0, 1), (0, 2), (1, 2)):
                assert abs(np.linalg.norm(xc[a] - xc[b]) - np.linalg.norm(Xw[a] - Xw[b])) < 1e-9 * 20
            # each camera point lies on its bearing
            j = np.stack([(uv[:, 0] - 320) / 500, (uv[:, 1] - 240) / 500, np.ones(3)], 1)
            j /= np.linalg.norm(j, axis=1, keepdims=True)
            cosang = np.sum(xc * j, 1) / np.linalg.norm(xc, axis=1)
            assert np.all(cosang > 1 - 1e-12)


def test_canonical_order(orc):
    rng = np.random.default_rng(3)
    for _ in range(300):
        _, _, uv, Xw = _exact_triple(rng)
        sols, _ = orc.p3p(uv, Xw, K)
        z = [((Rs @ Xw[0] + ts)[2], (Rs @ Xw[1] + ts)[2]) for Rs, ts in sols]
        assert z == sorted(z)


def test_degenerate_triples(orc):
    uv = np.array([[100.0, 100.0], [200.0, 150.0], [300.0, 200.0]])
    collinear = np.array([[0.0, 0.0, 5.0], [1.0, 0.0, 5.0], [2.0, 0.0, 5.0]])
    sols, ill = orc.p3p(uv, collinear, K)
    assert sols == [] and ill
    repeated = np.array([[0.0, 0.0, 5.0], [0.0, 0.0, 5.0], [2.0, 0.0, 5.0]])
    sols, ill = orc.p3p(uv, repeated, K)
    assert sols == [] and ill
