"""Seeded synthetic point sets shaped like the paper's workloads.

This module only draws coordinates. It holds none of the join's arithmetic
(no distances, no grid), so both the HIP path and the CPU oracle can be fed
from it without sharing any of the method.

Workload shapes (Section VI-A, Table "datasets"):
  * ``uniform``: coordinates independent per dimension, FP64, uniform in
    [0, 100]^d -- the paper's synthetic "Syn" sets.
  * ``clustered``: stands in for the skew of the paper's real SW-/SDSS-
    datasets, which are not available here: 10% uniform background in
    [0, 100]^d plus 90% drawn from 64 isotropic Gaussians whose centres are
    uniform in [0, 100]^d, sigma ~ U[0.5, 5], mixture weights
    Dirichlet(0.5 * 1_64), per-cluster counts multinomial.

All generators use numpy's PCG64 with an explicit seed and return a
C-contiguous (n, d) float64 array (row-major, one point per row).
"""
from __future__ import annotations

import numpy as np

BOX = 100.0


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def uniform(n: int, d: int, seed: int, box: float = BOX) -> np.ndarray:
    """n points uniform in [0, box]^d (float64, row-major)."""
    g = rng(seed)
    return np.ascontiguousarray(g.uniform(0.0, box, size=(int(n), int(d))))


def clustered(n: int, d: int, seed: int, n_clusters: int = 64,
              background: float = 0.10, sigma_lo: float = 0.5,
              sigma_hi: float = 5.0, alpha: float = 0.5,
              box: float = BOX) -> np.ndarray:
    """Gaussian-mixture points plus a uniform background (float64, row-major).

    The rows are shuffled so that original ids carry no spatial order.
    """
    g = rng(seed)
    n = int(n)
    n_bg = int(round(background * n))
    n_cl = n - n_bg
    centres = g.uniform(0.0, box, size=(n_clusters, d))
    sigmas = g.uniform(sigma_lo, sigma_hi, size=n_clusters)
    weights = g.dirichlet(np.full(n_clusters, alpha))
    counts = g.multinomial(n_cl, weights)
    parts = [g.uniform(0.0, box, size=(n_bg, d))]
    for c in range(n_clusters):
        if counts[c]:
            parts.append(centres[c] + sigmas[c] * g.standard_normal((counts[c], d)))
    pts = np.concatenate(parts, axis=0)
    g.shuffle(pts, axis=0)
    return np.ascontiguousarray(pts)


def lattice(k: int, d: int, spacing: float = 1.0, origin: float = 0.0) -> np.ndarray:
    """All points of the k^d integer lattice scaled by ``spacing`` (row-major)."""
    axes = [np.arange(k, dtype=np.float64) * spacing + origin for _ in range(d)]
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.ascontiguousarray(np.stack([m.ravel() for m in mesh], axis=1))


def make(kind: str, n: int, d: int, seed: int) -> np.ndarray:
    if kind == "uniform":
        return uniform(n, d, seed)
    if kind == "clustered":
        return clustered(n, d, seed)
    raise ValueError(f"unknown point distribution {kind!r}")


def poisson_arrivals(count: int, rate_per_s: float, seed: int) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of the given rate."""
    g = rng(seed)
    return np.cumsum(g.exponential(1.0 / rate_per_s, size=int(count)))


def serving_requests(count: int, seed: int, n_lo: float = 1e3, n_hi: float = 2e6,
                     d_choices=(2, 3, 4, 5, 6), k_lo: float = 4.0, k_hi: float = 128.0):
    """Request descriptors for the serving stream: sizes, dimension, kind,
    target neighbour count and a per-request point seed.

    n is log-uniform in [n_lo, n_hi], d uniform over ``d_choices``, the
    distribution is uniform or clustered with equal odds, and the target mean
    neighbour count k is log-uniform in [k_lo, k_hi].
    """
    g = rng(seed)
    out = []
    for r in range(int(count)):
        n = int(round(np.exp(g.uniform(np.log(n_lo), np.log(n_hi)))))
        d = int(g.choice(np.asarray(d_choices)))
        kind = "uniform" if g.uniform() < 0.5 else "clustered"
        k = float(np.exp(g.uniform(np.log(k_lo), np.log(k_hi))))
        out.append({"id": r, "n": n, "d": d, "kind": kind, "k": k,
                    "seed": int(g.integers(1, 2**31 - 1))})
    return out
