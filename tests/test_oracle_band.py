"""Pins for the FP32 pre-test bound of the band oracle (CPU only).

The bound is checked empirically: over random pairs and pairs placed at the
eps boundary, the FP32 squared distance (numpy float32 arithmetic) never
strays from the exact squared distance (long double) by more than Delta(E),
and every pair the thresholds classify without re-decision agrees with the
FP64 definition.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import band
from paper_1803_04120_amd import datagen


def _pairs_near(pts, eps, m, seed):
    """m random pairs whose distance is near eps (both sides of it)."""
    g = np.random.default_rng(seed)
    n, d = pts.shape
    i = g.integers(0, n, size=m)
    direction = g.standard_normal((m, d))
    direction /= np.linalg.norm(direction, axis=1, keepdims=True)
    r = eps * (1.0 + g.uniform(-1e-3, 1e-3, size=m))
    r[: m // 4] = eps  # exactly at eps (up to rounding of the offset)
    q = pts[i] + direction * r[:, None]
    return i, q


@pytest.mark.parametrize("kind,d,eps", [("uniform", 2, 0.04), ("uniform", 2, 0.2),
                                        ("uniform", 3, 0.9142), ("uniform", 6, 13.0564),
                                        ("clustered", 2, 0.0909), ("clustered", 3, 0.491)])
def test_fp32_error_within_bound(kind, d, eps):
    pts = datagen.make(kind, 20000, d, seed=3)
    i, q = _pairs_near(pts, eps, 40000, seed=d)
    allp = np.concatenate([pts, q], axis=0)
    j = np.arange(pts.shape[0], allp.shape[0])
    s, X = band.shift_and_extent(allp)
    tau = band.tau_of(X)
    y = band.fp32_copy(allp, s)
    S = band.s32(y, i, j).astype(np.longdouble)
    E = band.exact_sq(allp, i, j)
    bound = np.array([band.delta(float(e), d, tau) for e in E])
    err = np.abs(S - E).astype(np.float64)
    assert np.all(err <= bound)
    # the bound is not vacuous: it is within a few hundred times the worst error seen
    assert bound.max() < 1e3 * max(err.max(), 1e-300) or err.max() == 0.0


@pytest.mark.parametrize("kind,d,eps", [("uniform", 2, 0.2), ("uniform", 4, 2.8661),
                                        ("clustered", 3, 0.491)])
def test_thresholds_agree_with_fp64(kind, d, eps):
    pts = datagen.make(kind, 20000, d, seed=9)
    i, q = _pairs_near(pts, eps, 60000, seed=10 + d)
    allp = np.concatenate([pts, q], axis=0)
    j = np.arange(pts.shape[0], allp.shape[0])
    s, X = band.shift_and_extent(allp)
    th = band.thresholds(eps, d, X)
    assert th is not None
    lo, hi = th
    eps2 = eps * eps
    assert float(lo) < eps2 < float(hi)
    S = band.s32(band.fp32_copy(allp, s), i, j)
    acc = np.zeros(i.shape[0])
    for k in range(d):
        t = allp[i, k] - allp[j, k]
        acc = acc + t * t
    in64 = acc <= eps2
    assert np.all(in64[S < lo])
    assert not np.any(in64[S > hi])
    band_frac = np.mean((S >= lo) & (S <= hi))
    assert 0.0 < band_frac < 0.5  # these pairs were placed at the boundary on purpose


def test_unusable_when_eps_tiny():
    assert band.thresholds(1e-6, 3, 1e3) is None
    assert band.thresholds(1.0, 3, 1e3) is not None
