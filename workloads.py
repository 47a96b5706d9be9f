"""Seeded synthetic path generators shared by the tests, the benchmark and the
oracle checks.

This module draws random paths and nothing else: it contains none of the
signature-kernel arithmetic, so that the GPU library and the CPU oracle can be
fed the very same float32 values without sharing any computation.  Every
generator returns float32 NumPy arrays (row-major ``[paths, points, channels]``
or a list of ``[points, channels]`` arrays for ragged batches) drawn from
NumPy's PCG64 with a fixed seed.

The shapes and distributions follow the paper's setting (piecewise-linear
interpolations of Brownian-like paths, Section 3.1.1 and its timing figure)
at the sizes of the five workloads this library is measured on:

1. ``single_pair``      two 32-point paths in R^2, increments N(0, 1/32), and a
                        straight-segment pair (2 points, each N(0, I_2)).
2. ``gram_batch``       128 x 128 paths of 256 points, 8 channels with
                        increments N(0, (0.3/16)^2) plus a time channel.
3. ``ragged_pairs``     4096 pairs, lengths uniform in [64, 1024], d = 16,
                        increment std 0.3/sqrt(L-1), rescaled so that
                        |<x_T - x_0, y_T - y_0>| <= 2.
4. ``mmd_paths``        64 Gaussian random walks (512 points, d = 4, std 0.05)
                        and 64 Ornstein-Uhlenbeck targets (theta 2, sigma 0.3,
                        dt 1/512).
5. ``corrector_pairs``  pairs of 256-point paths in R^8, std 0.3/16.
"""
from __future__ import annotations

import numpy as np

SEED_SINGLE = 14794
SEED_GRAM = 14795
SEED_RAGGED = 14796
SEED_MMD = 14797
SEED_CORRECTOR_TRAIN = 14798
SEED_CORRECTOR_EVAL = 14799


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def brownian(rng: np.random.Generator, n_paths: int, n_points: int, dim: int,
             std: float, start_zero: bool = True) -> np.ndarray:
    """Gaussian random walks: x_0 = 0 and i.i.d. N(0, std^2) increments."""
    inc = rng.normal(0.0, std, size=(n_paths, n_points - 1, dim))
    out = np.zeros((n_paths, n_points, dim), dtype=np.float64)
    out[:, 1:, :] = np.cumsum(inc, axis=1)
    if not start_zero:
        out += rng.normal(0.0, 1.0, size=(n_paths, 1, dim))
    return out.astype(np.float32)


def add_time_channel(paths: np.ndarray) -> np.ndarray:
    """Append t_i = i / (L-1) in [0, 1] as the last channel."""
    B, L, d = paths.shape
    t = (np.arange(L, dtype=np.float64) / (L - 1)).astype(np.float32)
    tt = np.broadcast_to(t[None, :, None], (B, L, 1))
    return np.ascontiguousarray(np.concatenate([paths, tt], axis=2), dtype=np.float32)


# 1 -------------------------------------------------------------------------
def single_pair(seed: int = SEED_SINGLE):
    """Returns (x, y, xs, ys): a 32-point R^2 pair with N(0, 1/32) increments
    starting at 0, and a straight-segment pair (2 points each, N(0, I_2))."""
    rng = _rng(seed)
    xy = brownian(rng, 2, 32, 2, np.sqrt(1.0 / 32.0))
    seg = rng.normal(0.0, 1.0, size=(2, 2, 2)).astype(np.float32)
    return xy[0], xy[1], seg[0], seg[1]


# 2 -------------------------------------------------------------------------
def gram_batch(seed: int = SEED_GRAM, n_x: int = 128, n_y: int = 128,
               n_points: int = 256, dim: int = 8):
    """X [n_x, L, dim+1], Y [n_y, L, dim+1]: increments N(0, (0.3/sqrt L)^2),
    start 0, time channel appended."""
    rng = _rng(seed)
    std = 0.3 / np.sqrt(n_points)
    X = brownian(rng, n_x, n_points, dim, std)
    Y = brownian(rng, n_y, n_points, dim, std)
    return add_time_channel(X), add_time_channel(Y)


# 3 -------------------------------------------------------------------------
def ragged_pairs(seed: int = SEED_RAGGED, n_pairs: int = 4096, lo: int = 64,
                 hi: int = 1024, dim: int = 16):
    """Lists xs, ys of [L, dim] float32 arrays with L ~ U{lo..hi} drawn
    independently for every path; increment std 0.3/sqrt(L-1).  If the
    endpoint displacements of a pair have |<x_T - x_0, y_T - y_0>| > 2, both
    paths are scaled by sqrt(2/|c|)."""
    rng = _rng(seed)
    xs, ys = [], []
    for _ in range(n_pairs):
        lx = int(rng.integers(lo, hi + 1))
        ly = int(rng.integers(lo, hi + 1))
        x = brownian(rng, 1, lx, dim, 0.3 / np.sqrt(lx - 1))[0].astype(np.float64)
        y = brownian(rng, 1, ly, dim, 0.3 / np.sqrt(ly - 1))[0].astype(np.float64)
        c = float(np.dot(x[-1] - x[0], y[-1] - y[0]))
        if abs(c) > 2.0:
            s = np.sqrt(2.0 / abs(c))
            x *= s
            y *= s
        xs.append(x.astype(np.float32))
        ys.append(y.astype(np.float32))
    return xs, ys


# 4 -------------------------------------------------------------------------
def ornstein_uhlenbeck(rng: np.random.Generator, n_paths: int, n_points: int,
                       dim: int, theta: float, sigma: float, dt: float) -> np.ndarray:
    """Exact OU transition X <- X e^{-theta dt} + sigma sqrt((1 - e^{-2 theta dt})
    / (2 theta)) xi, X_0 = 0, channels independent."""
    a = np.exp(-theta * dt)
    s = sigma * np.sqrt((1.0 - np.exp(-2.0 * theta * dt)) / (2.0 * theta))
    out = np.zeros((n_paths, n_points, dim), dtype=np.float64)
    for i in range(1, n_points):
        out[:, i] = out[:, i - 1] * a + s * rng.normal(size=(n_paths, dim))
    return out.astype(np.float32)


def mmd_paths(seed: int = SEED_MMD, n: int = 64, n_points: int = 512, dim: int = 4):
    """(X, Y): X are the generated paths (the trainable parameters, initialised
    as Gaussian random walks with std 0.05), Y the OU targets."""
    rng = _rng(seed)
    X = brownian(rng, n, n_points, dim, 0.05)
    Y = ornstein_uhlenbeck(rng, n, n_points, dim, theta=2.0, sigma=0.3,
                           dt=1.0 / n_points)
    return X, Y


# 5 -------------------------------------------------------------------------
def corrector_pairs(seed: int, n_pairs: int, n_points: int = 256, dim: int = 8):
    """(X, Y) [n_pairs, n_points, dim]: independent pairs, std 0.3/sqrt(L)."""
    rng = _rng(seed)
    std = 0.3 / np.sqrt(n_points)
    X = brownian(rng, n_pairs, n_points, dim, std)
    Y = brownian(rng, n_pairs, n_points, dim, std)
    return X, Y


def random_paths(seed: int, n_paths: int, n_points: int, dim: int,
                 std: float = 0.3) -> np.ndarray:
    """Generic small random walks used by unit tests."""
    return brownian(_rng(seed), n_paths, n_points, dim, std / np.sqrt(max(n_points - 1, 1)))


def ragged_lengths(seed: int, n: int, lo: int, hi: int) -> np.ndarray:
    return _rng(seed).integers(lo, hi + 1, size=n)


# 6 -------------------------------------------------------------------------
SEED_FIG3 = 14800


def fig3_pairs(n_points: int, dim: int, n_pairs: int = 5, seed: int = SEED_FIG3):
    """(X, Y) [n_pairs, n_points, dim]: Brownian motion on [0, 1] sampled at
    n_points equally spaced times, start 0, each channel with variance 1/dim
    at time 1 (increments N(0, 1 / (dim (n_points - 1)))), so that |x_1|^2 has
    mean 1 for every dim -- the inputs of the Figure 3 protocol."""
    rng = _rng(seed + 1000 * dim + n_points)
    std = 1.0 / np.sqrt(dim * (n_points - 1))
    X = brownian(rng, n_pairs, n_points, dim, std)
    Y = brownian(rng, n_pairs, n_points, dim, std)
    return X, Y


# 7 -------------------------------------------------------------------------
SEED_FBM = 14801


def fbm_paths(seed: int = SEED_FBM, n_paths: int = 30, n_points: int = 100,
              hursts=(0.2, 0.5, 0.8)):
    """(paths [n_paths, n_points, 2], hurst [n_paths]): fractional Brownian
    motion on t_i = i / (n_points - 1), B(0) = 0, with a Hurst exponent drawn
    uniformly from `hursts` per path, sampled exactly through the Cholesky
    factor of its covariance 0.5 (s^{2H} + t^{2H} - |t - s|^{2H}); channel 0
    is the time t, channel 1 the fBM."""
    rng = _rng(seed)
    t = np.linspace(0.0, 1.0, n_points)
    H = rng.choice(np.asarray(hursts, dtype=np.float64), size=n_paths)
    out = np.zeros((n_paths, n_points, 2), dtype=np.float64)
    out[:, :, 0] = t
    s, u = np.meshgrid(t[1:], t[1:], indexing="ij")
    for i in range(n_paths):
        h2 = 2.0 * H[i]
        cov = 0.5 * (s ** h2 + u ** h2 - np.abs(s - u) ** h2)
        L = np.linalg.cholesky(cov)
        out[i, 1:, 1] = L @ rng.normal(size=n_points - 1)
    return out.astype(np.float32), H
