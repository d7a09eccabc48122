"""Pins of the oracle's minimal sampling (Sec. 3.3: batches of minimal sets,
drawn here from a counter-based Philox4x64-10 stream) against the Philox
publication's known-answer vectors and numpy's independent Philox."""
import itertools
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x64_10_kat.txt")
MASK = (1 << 64) - 1


def _numpy_block(ctr, key):
    """numpy's Philox increments its 256-bit counter before each block, so a
    generator started at ctr - 1 emits the block of ctr first."""
    c = [int(x) for x in ctr]
    # decrement the 256-bit counter by one (little-endian words)
    for i in range(4):
        if c[i] > 0:
            c[i] -= 1
            break
        c[i] = MASK
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(c, dtype=np.uint64))
    return bg.random_raw(4).astype(np.uint64)


def test_philox_known_answers(orc):
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = orc.philox(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_philox_matches_numpy(orc):
    rng = np.random.default_rng(7)
    for _ in range(200):
        ctr = [int(x) for x in rng.integers(0, 2 ** 63, size=4, dtype=np.int64)]
        key = [int(x) for x in rng.integers(0, 2 ** 63, size=2, dtype=np.int64)]
        ctr[0] += 1  # keep the decrement inside word 0 for most draws
        assert np.array_equal(orc.philox(ctr, key), _numpy_block(ctr, key))
    # small counters as used by the sampler: (h, query, attempt, 0)
    for h, q, a in [(0, 0, 0), (1, 0, 0), (1023, 5, 3), (99999, 255, 15)]:
        assert np.array_equal(orc.philox([h, q, a, 0], [0, 0]), _numpy_block([h, q, a, 0], [0, 0]))


def _triple_from_numpy(seed, qid, h, n):
    for attempt in range(16):
        w = _numpy_block([h, qid, attempt, 0], [seed, 0])
        idx = [(int(x) * n) >> 64 for x in w[:3]]
        if len(set(idx)) == 3:
            return True, idx
    return False, [-1, -1, -1]


@pytest.mark.parametrize("n", [3, 4, 7, 2000, 50000, 200000])
def test_sample_triple_matches_numpy_philox(orc, n):
    for h in list(range(64)) + [1023, 4095, 9999, 99999]:
        ok, idx = orc.sample_triple(0, 3, h, n)
        ok2, idx2 = _triple_from_numpy(0, 3, h, n)
        assert ok == ok2 and list(idx) == idx2
        if ok:
            assert len(set(idx.tolist())) == 3 and min(idx) >= 0 and max(idx) < n


def test_sample_triple_degenerate(orc):
    for n in (0, 1, 2):
        ok, idx = orc.sample_triple(0, 0, 5, n)
        assert not ok and list(idx) == [-1, -1, -1]


def test_sample_uniformity(orc):
    """Each index is (close to) uniform: chi-square over 16 bins, 6,000 samples."""
    n = 16
    counts = np.zeros(n)
    for h in range(6000):
        ok, idx = orc.sample_triple(11, 0, h, n)
        assert ok
        counts[idx] += 1
    exp = counts.sum() / n
    chi2 = ((counts - exp) ** 2 / exp).sum()
    assert chi2 < 45.0  # 15 dof, p ~ 1e-4


@pytest.mark.parametrize("n", [3, 4, 5, 9, 13])
def test_unrank_is_bijection(orc, n):
    got = []
    for h in range(len(list(itertools.combinations(range(n), 3)))):
        ok, idx = orc.unrank_triple(h, n)
        assert ok and idx[0] < idx[1] < idx[2] < n
        got.append(tuple(idx.tolist()))
    assert sorted(got) == sorted(itertools.combinations(range(n), 3))
    assert len(set(got)) == len(got)
    ok, _ = orc.unrank_triple(len(got), n)
    assert not ok


def test_unrank_colex_order(orc):
    # colexicographic: ordered by the largest element, then the middle, then the smallest
    seq = [tuple(orc.unrank_triple(h, 8)[1].tolist()) for h in range(56)]
    assert seq == sorted(seq, key=lambda t: (t[2], t[1], t[0]))
