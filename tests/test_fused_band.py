"""The error bound behind the FP64 fused-square filter of the grid-row
kernel (CPU only).

The kernel sums squared differences with fused multiply-adds and decides a
pair directly only when that sum F lies outside eps^2 (1 +- 2^-45); inside,
the predicate's own left-to-right sum S decides. That is exact as long as
|F - S| <= 2 gamma_d / (1 - gamma_d) F (gamma_d = d u / (1 - d u),
u = 2^-53, the standard bound for a sum of d non-negative rounded terms,
Higham, Accuracy and Stability of Numerical Algorithms, Section 4.2) and
that bound is below 2^-45. Here both sums are computed independently of the
kernel: S with Python doubles, F with exact rationals rounded once per
step.
"""
from __future__ import annotations

import numpy as np
import pytest

from tests._helpers import fused_square_sum, ordered_square_sum, straddling_points

U = 2.0 ** -53
BAND = 2.0 ** -45


def _bound(d):
    g = d * U / (1 - d * U)
    return 2 * g / (1 - g)


@pytest.mark.parametrize("d", range(1, 9))
def test_fused_and_ordered_sums_within_bound(d):
    g = np.random.default_rng(100 + d)
    worst = 0.0
    for _ in range(1500):
        dv = [float(t) for t in g.normal(size=d) * 10.0 ** g.uniform(-3, 3, size=d)]
        S = ordered_square_sum(dv)
        F = fused_square_sum(dv)
        assert abs(F - S) <= _bound(d) * F, (dv, S, F)
        worst = max(worst, abs(F - S) / F)
    assert _bound(d) * 15 <= BAND  # at least 15 times the bound up to d = 8
    assert worst <= _bound(d)


@pytest.mark.parametrize("d", [3, 6, 8])
def test_straddling_pairs_fall_in_the_band(d):
    """Every pair the two sums decide differently has F within the band, so
    the kernel re-decides it with S."""
    eps = 0.7
    eps2 = eps * eps
    pts, found = straddling_points(d, eps, 20, seed=d)
    assert found == 20
    for a in range(0, 2 * found, 2):
        dv = [float(t) for t in pts[a] - pts[a + 1]]
        S, F = ordered_square_sum(dv), fused_square_sum(dv)
        assert (S <= eps2) != (F <= eps2)
        assert eps2 * (1 - BAND) <= F <= eps2 * (1 + BAND)


def test_fused_sum_differs_from_ordered_sum():
    """The two sums are not the same function (else the filter would test
    nothing): a small case where they differ."""
    g = np.random.default_rng(7)
    diff = 0
    for _ in range(500):
        dv = [float(t) for t in g.normal(size=4)]
        diff += ordered_square_sum(dv) != fused_square_sum(dv)
    assert diff > 0
