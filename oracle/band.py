"""Oracle for the FP32 pre-test with an FP64 re-decision band.

TEST INFRASTRUCTURE ONLY; shares no code with the HIP implementation.

The paper computes distances in FP64 only (Section VI-B). The FP32 pre-test
is an addition of this implementation; it must leave the pair set of the FP64
definition unchanged. This module states the error bound that makes that so
and emulates the FP32 evaluation with numpy float32 arithmetic so tests can
check the bound empirically.

Setup: shift s_j (the bounding-box centre), y = fl32(fl64(x - s)),
X = max_j max_i |x_ij - s_j|, tau = X * 2^-24 * (1 + 2^-28) + 2^-126 (the
last term covers FP32 underflow of y). For two points, S is the FP32
evaluation of the squared distance on their y copies (same order as the FP64
form), E the exact real squared distance of their x, d2 the FP64 value.
With u32 = 2^-24, u64 = 2^-53 and gamma(k, u) = k u / (1 - k u):

  |S - E|  <= Delta(E) = 4 tau sqrt(d E) + 4 d tau^2
                         + gamma(d+2, u32) (sqrt(E) + 2 tau sqrt(d))^2
                         + (2d + 2) 2^-126
  |d2 - E| <= gamma(d+2, u64) E

Thresholds: E_a = eps2 / (1 + g64), E_r = eps2 / (1 - g64),
lo = round_down_fp32(E_a - 2 Delta(E_a)), hi = round_up_fp32(E_r + 2 Delta(E_r)).
S < lo implies d2 <= eps2; S > hi implies d2 > eps2; anything in [lo, hi]
is decided by the FP64 definition. The argument needs E - Delta(E) to grow
with E above E_a, which holds when eps >> tau sqrt(d); below
eps < 64 tau sqrt(d) the pre-test is not used.
"""
from __future__ import annotations

import math

import numpy as np

U32 = 2.0 ** -24
U64 = 2.0 ** -53
TINY32 = 2.0 ** -126


def gamma(k: int, u: float) -> float:
    return k * u / (1.0 - k * u)


def shift_and_extent(points):
    x = np.asarray(points, dtype=np.float64)
    mins, maxs = x.min(axis=0), x.max(axis=0)
    s = (mins + maxs) * 0.5
    X = float(np.max(np.abs(x - s))) if x.size else 0.0
    return s, X


def tau_of(X: float) -> float:
    return X * U32 * (1.0 + 2.0 ** -28) + TINY32


def delta(E: float, d: int, tau: float) -> float:
    rE = math.sqrt(max(E, 0.0))
    return (4.0 * tau * math.sqrt(d * E) + 4.0 * d * tau * tau
            + gamma(d + 2, U32) * (rE + 2.0 * tau * math.sqrt(d)) ** 2
            + (2 * d + 2) * TINY32)


def usable(eps: float, d: int, tau: float) -> bool:
    return eps >= 64.0 * tau * math.sqrt(d)


def thresholds(eps: float, d: int, X: float):
    """(lo, hi) as float32 values, or None when the pre-test is not usable."""
    tau = tau_of(X)
    if not usable(eps, d, tau):
        return None
    eps2 = eps * eps
    g64 = gamma(d + 2, U64)
    Ea = eps2 / (1.0 + g64)
    Er = eps2 / (1.0 - g64)
    lo = Ea - 2.0 * delta(Ea, d, tau)
    hi = Er + 2.0 * delta(Er, d, tau)
    lo32 = np.float32(lo)
    if float(lo32) > lo:
        lo32 = np.nextafter(lo32, np.float32(-np.inf))
    hi32 = np.float32(hi)
    if float(hi32) < hi:
        hi32 = np.nextafter(hi32, np.float32(np.inf))
    return lo32, hi32


def fp32_copy(points, s) -> np.ndarray:
    x = np.asarray(points, dtype=np.float64)
    return (x - s).astype(np.float32)


def s32(y: np.ndarray, i, j) -> np.ndarray:
    """FP32 squared distance between rows i and j of the shifted copy (numpy
    float32 arithmetic, dimension order 0..d-1, each operation rounded)."""
    acc = np.zeros(np.broadcast(np.asarray(i), np.asarray(j)).shape, dtype=np.float32)
    for k in range(y.shape[1]):
        t = (y[i, k] - y[j, k]).astype(np.float32)
        acc = (acc + (t * t).astype(np.float32)).astype(np.float32)
    return acc


def exact_sq(points, i, j) -> np.ndarray:
    """Squared distance with 64-bit-mantissa long doubles (exact to far
    below the FP32 band) for error-bound checks."""
    x = np.asarray(points, dtype=np.float64).astype(np.longdouble)
    acc = np.zeros(np.broadcast(np.asarray(i), np.asarray(j)).shape, dtype=np.longdouble)
    for k in range(x.shape[1]):
        t = x[i, k] - x[j, k]
        acc = acc + t * t
    return acc
