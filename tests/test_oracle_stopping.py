"""Pins of the stopping rule (Sec. 3.3 "Pose Estimation": a 100K-sample cap
and the standard RANSAC confidence bound, read for minimal sets of 3).

The defining property: k is the smallest sample count with
(1 - eps^3)^k <= 1 - confidence, i.e. the chance that none of k samples is
all-inlier is at most 1 - confidence."""
import math

import pytest


@pytest.mark.parametrize("conf", [0.999, 0.9999])
@pytest.mark.parametrize("eps", [0.6, 0.5, 0.4, 0.3, 0.25, 0.1, 0.05])
def test_smallest_k_with_miss_probability_below_bound(orc, conf, eps):
    k = orc.required_samples(eps, conf, 10 ** 9)
    miss = lambda kk: (1.0 - eps ** 3) ** kk
    assert miss(k) <= (1.0 - conf) * (1 + 1e-12)
    assert miss(k - 1) > (1.0 - conf) * (1 - 1e-12)


def test_extremes(orc):
    assert orc.required_samples(0.0, 0.9999, 100000) == 100000
    assert orc.required_samples(1.0, 0.9999, 100000) == 0
    assert orc.required_samples(1e-6, 0.9999, 100000) == 100000  # capped
    assert orc.required_samples(0.05, 0.9999, 50000) == 50000


def test_monotone_in_eps(orc):
    ks = [orc.required_samples(e / 100, 0.999, 10 ** 9) for e in range(2, 100)]
    assert all(a >= b for a, b in zip(ks, ks[1:]))
