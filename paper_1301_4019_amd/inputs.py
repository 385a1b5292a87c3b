"""Seeded synthetic inputs for the resampling step.

This module only generates data; it holds none of the resampling arithmetic,
and both the HIP path and the CPU oracle are fed from it.  The weight sets
follow the paper's experimental setup (section 3.1): x_i ~ N(0, 1) and a
Gaussian likelihood of an observation y, here unnormalised,
    w_i = exp(-(x_i - y)^2 / 2),
so that max w = 1; every resampler is invariant to a constant factor
(appendix E).  Values are computed in float64 and rounded once to the
requested dtype.  All draws come from numpy's Philox bit generator keyed by an
explicit seed, so every input is reproducible byte for byte.
"""
from __future__ import annotations

import math

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(int(seed)))


def weights(n: int, y: float, seed: int = 0, dtype=np.float32) -> np.ndarray:
    """Weight set of size n for observation y (section 3.1 of the paper)."""
    x = _rng(seed).standard_normal(int(n))
    w = np.exp(-0.5 * (x - float(y)) ** 2)
    return w.astype(dtype)


def expected_weight(y: float) -> float:
    """E[w] for the unnormalised weights above: 2^{-1/2} exp(-y^2/4)."""
    return 2.0 ** -0.5 * math.exp(-y * y / 4.0)


def expected_weight_sq(y: float) -> float:
    """E[w^2] for the unnormalised weights above: 3^{-1/2} exp(-y^2/3)."""
    return 3.0 ** -0.5 * math.exp(-y * y / 3.0)


def ragged_batch(n_filters: int = 4096, lo_log2: int = 8, hi_log2: int = 16, seed: int = 0,
                 dtype=np.float32):
    """Ragged batch: N_f = round(2^(lo + (hi-lo) v)), v ~ U[0,1); y_f ~ U[0,4].

    Returns (w_all, offsets[F+1] int64, y[F] float64).  Filter f's weights are
    w_all[offsets[f]:offsets[f+1]], drawn with weights(N_f, y_f, seed*1_000_003+f+1).
    """
    g = _rng(seed)
    v = g.random(n_filters)
    sizes = np.rint(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * v)).astype(np.int64)
    ys = g.uniform(0.0, 4.0, n_filters)
    offsets = np.zeros(n_filters + 1, dtype=np.int64)
    np.cumsum(sizes, out=offsets[1:])
    w_all = np.empty(int(offsets[-1]), dtype=dtype)
    for f in range(n_filters):
        w_all[offsets[f]:offsets[f + 1]] = weights(int(sizes[f]), float(ys[f]),
                                                   seed * 1_000_003 + f + 1, dtype)
    return w_all, offsets, ys


def ssm_data(T: int, phi: float = 0.9, q: float = 1.0, r: float = 0.5, seed: int = 0):
    """Synthetic trajectory of x_t = phi x_{t-1} + N(0,q^2), y_t = x_t + N(0,r^2).

    x_0 is drawn from the stationary law N(0, q^2 / (1 - phi^2)).  Returns
    (x[0..T], y[1..T]) as float64 arrays of length T+1 and T.
    """
    g = _rng(seed)
    x = np.empty(T + 1)
    x[0] = g.standard_normal() * q / math.sqrt(1.0 - phi * phi)
    for t in range(1, T + 1):
        x[t] = phi * x[t - 1] + q * g.standard_normal()
    y = x[1:] + r * g.standard_normal(T)
    return x, y
