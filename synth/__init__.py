"""Seeded synthetic point-set generators (shared by tests, bench and oracle scripts).

This module holds no arithmetic of the method: it only draws point clouds.
All sets are float32, C-contiguous, ``n x D`` row-major.  Every draw is
deterministic in ``seed`` and independent of the number of threads used:
rows are generated in fixed chunks of ``CHUNK`` rows, each chunk from its own
PCG64 stream keyed by ``SeedSequence(seed, spawn_key=(tag, chunk))``.

Workload laws (the paper's public datasets are not available; these stand in
for its clustered embeddings, physics vectors and random clouds):

``gauss_outliers``  A ~ N(0, I); B ~ N(shift * 1, I); ``floor(frac * nB)``
                    uniformly chosen rows of B replaced by points uniform on
                    the sphere of radius ``radius`` about the origin.
``mixture``         K isotropic Gaussian clusters: centres ~ N(0, cs^2 I);
                    B's centres are A's plus N(0, bs^2 I); labels uniform;
                    within-cluster N(0, sigma^2 I); optional row L2
                    normalisation; optional replacement of ``frac`` of the
                    rows of each set by multivariate Student-t(nu) outliers
                    around their cluster centre.
``t_mixture``       like ``mixture`` but every point is centre + t(nu) noise.
``shells``          the same random directions at radius r1 (A) and r2 (B),
                    B row-permuted: a closed-form test case.
``uniform_clouds``  A ~ U[0,1]^D, B ~ U[0,1]^D + offset (every coordinate).
``batch_sizes``     per-pair (nA, nB, D) for many uneven pairs.
"""

from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

CHUNK = 16384

__all__ = [
    "CHUNK", "rng", "gauss_outliers", "mixture", "t_mixture", "shells",
    "uniform_clouds", "batch_sizes", "batch_pair", "workload",
]


def rng(seed: int, *key: int) -> np.random.Generator:
    """PCG64 generator for ``(seed, key...)``."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(int(seed), spawn_key=tuple(int(k) for k in key))))


def _threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _chunked(n: int, D: int, fill, tag: int, seed: int) -> np.ndarray:
    """Allocate ``n x D`` float32 and fill chunk c with ``fill(g, rows, out)``."""
    out = np.empty((n, D), dtype=np.float32)
    nchunks = (n + CHUNK - 1) // CHUNK

    def work(c):
        lo = c * CHUNK
        hi = min(n, lo + CHUNK)
        fill(rng(seed, tag, c), hi - lo, out[lo:hi])

    if nchunks <= 1:
        for c in range(nchunks):
            work(c)
    else:
        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(work, range(nchunks)))
    return out


def gauss_outliers(nA: int, nB: int, D: int, seed: int, shift: float = 0.5,
                   outlier_frac: float = 0.01, radius: float = 6.0):
    """Two Gaussians with a shifted mean, plus outliers on a sphere in B."""
    def fa(g, r, o):
        o[:] = g.standard_normal((r, D), dtype=np.float32)

    def fb(g, r, o):
        o[:] = g.standard_normal((r, D), dtype=np.float32) + np.float32(shift)

    A = _chunked(nA, D, fa, 1, seed)
    B = _chunked(nB, D, fb, 2, seed)
    n_out = int(math.floor(outlier_frac * nB + 1e-9))
    if n_out > 0:
        g = rng(seed, 3)
        rows = g.choice(nB, size=n_out, replace=False)
        v = g.standard_normal((n_out, D))
        v *= radius / np.linalg.norm(v, axis=1, keepdims=True)
        B[rows] = v.astype(np.float32)
    return A, B


def _centres(seed: int, K: int, D: int, centre_std: float, b_centre_std: float):
    g = rng(seed, 10)
    cA = (centre_std * g.standard_normal((K, D))).astype(np.float32)
    cB = (cA + b_centre_std * g.standard_normal((K, D))).astype(np.float32)
    return cA, cB


def mixture(nA: int, nB: int, D: int, seed: int, K: int = 64,
            centre_std: float = 2.0, b_centre_std: float = 0.5,
            sigma: float = 1.0, normalize: bool = False,
            outlier_frac: float = 0.0, nu: float = 3.0, centre_seed: int | None = None):
    """Gaussian-cluster mixture pair, optionally with Student-t outliers.
    ``centre_seed`` (default: ``seed``) fixes the cluster centres, so that
    several pairs can be drawn from one distribution."""
    cA, cB = _centres(seed if centre_seed is None else centre_seed, K, D, centre_std, b_centre_std)

    def make(centres):
        def f(g, r, o):
            lab = g.integers(0, K, size=r)
            o[:] = centres[lab] + np.float32(sigma) * g.standard_normal((r, D), dtype=np.float32)
            if normalize:
                o /= np.linalg.norm(o, axis=1, keepdims=True)
        return f

    A = _chunked(nA, D, make(cA), 11, seed)
    B = _chunked(nB, D, make(cB), 12, seed)
    if outlier_frac > 0:
        for tag, X, C in ((13, A, cA), (14, B, cB)):
            n = X.shape[0]
            n_out = int(math.floor(outlier_frac * n + 1e-9))
            if n_out == 0:
                continue
            g = rng(seed, tag)
            rows = g.choice(n, size=n_out, replace=False)
            lab = g.integers(0, K, size=n_out)
            z = g.standard_normal((n_out, D))
            w = g.chisquare(nu, size=(n_out, 1))
            X[rows] = (C[lab] + sigma * z * np.sqrt(nu / w)).astype(np.float32)
    return A, B


def t_mixture(nA: int, nB: int, D: int, seed: int, K: int = 128,
              centre_std: float = 2.0, b_centre_std: float = 0.5,
              sigma: float = 1.0, nu: float = 3.0, centre_seed: int | None = None):
    """Mixture where every point is its centre plus multivariate t(nu) noise
    (``centre_seed`` as in ``mixture``)."""
    cA, cB = _centres(seed if centre_seed is None else centre_seed, K, D, centre_std, b_centre_std)

    def make(centres):
        def f(g, r, o):
            lab = g.integers(0, K, size=r)
            z = g.standard_normal((r, D), dtype=np.float32)
            w = g.chisquare(nu, size=(r, 1)).astype(np.float32)
            o[:] = centres[lab] + np.float32(sigma) * z * np.sqrt(np.float32(nu) / w)
        return f

    return _chunked(nA, D, make(cA), 21, seed), _chunked(nB, D, make(cB), 22, seed)


def shells(n: int, D: int, seed: int, r1: float = 1.0, r2: float = 2.0):
    """A = r1 * g/|g|, B = r2 * (same rows, permuted).  H = |r2 - r1|."""
    g = rng(seed, 30)
    v = g.standard_normal((n, D))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    A = (r1 * v).astype(np.float32)
    perm = g.permutation(n)
    B = (np.float64(r2) / np.float64(r1) * A.astype(np.float64)[perm]).astype(np.float32)
    return A, B


def uniform_clouds(nA: int, nB: int, D: int, seed: int, offset: float = 0.1):
    """Random clouds: U[0,1]^D and U[0,1]^D + offset."""
    def fa(g, r, o):
        o[:] = g.random((r, D), dtype=np.float32)

    def fb(g, r, o):
        o[:] = g.random((r, D), dtype=np.float32) + np.float32(offset)

    return _chunked(nA, D, fa, 41, seed), _chunked(nB, D, fb, 42, seed)


def batch_sizes(P: int, seed: int, lo: int = 256, hi: int = 65536,
                dims=(64, 128, 256)):
    """Per-pair sizes: nA, nB log-uniform in [lo, hi], D uniform over dims."""
    g = rng(seed, 50)
    nA = np.floor(np.exp(g.uniform(math.log(lo), math.log(hi), size=P))).astype(np.int64)
    nB = np.floor(np.exp(g.uniform(math.log(lo), math.log(hi), size=P))).astype(np.int64)
    D = np.asarray(dims)[g.integers(0, len(dims), size=P)].astype(np.int64)
    return np.clip(nA, lo, hi), np.clip(nB, lo, hi), D


def batch_pair(seed: int, i: int, nA: int, nB: int, D: int):
    """Pair i of a batch drawn with ``batch_sizes(P, seed)``: the
    ``gauss_outliers`` law at that pair's sizes, seed ``seed * 2^20 + i``."""
    return gauss_outliers(int(nA), int(nB), int(D), seed=(int(seed) << 20) + int(i))


def workload(name: str, seed: int = 0):
    """The named workloads with their full sizes.

    ``gauss5k``   5 000 x 5 000, D=32, Gaussian pair with sphere outliers;
                  centroid + 3 PCs, k = 100 per direction end.
    ``mix200k``   200 000 x 200 000, D=128, 64-cluster mixture, rows
                  normalised; centroid + 8 PCs, k = 1 000.
    ``heavy2m``   2 000 000 x 2 000 000, D=256, 128-cluster mixture with
                  0.1 % t(3) outliers; alpha = 0.01, m = 16.
    Returns ``(A, B, params)`` where params holds m and k (or alpha).
    """
    if name == "gauss5k":
        A, B = gauss_outliers(5000, 5000, 32, seed)
        return A, B, {"m": 3, "k": 100}
    if name == "mix200k":
        A, B = mixture(200_000, 200_000, 128, seed, K=64, normalize=True)
        return A, B, {"m": 8, "k": 1000}
    if name == "heavy2m":
        A, B = mixture(2_000_000, 2_000_000, 256, seed, K=128, outlier_frac=0.001)
        return A, B, {"m": 16, "alpha": 0.01}
    raise KeyError(name)
