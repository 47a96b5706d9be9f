"""FP64 oracle of the moments-matching reduction of a discrete measure on
paths (Section "Moments-matching reduction algorithm for the support of a
discrete measure on paths").

TEST INFRASTRUCTURE ONLY (see the package docstring).

For a measure mu = sum_i alpha_i delta_{x_i} and the signature-kernel Gram
K[i][j] = k(x_i, x_j), the reduced weights beta minimise eq. (min_lasso),
    f(beta) = L(beta) + lam ||beta||_1,   L(beta) = (alpha - beta)^T K (alpha - beta),
by the proximal-gradient iteration of eq. (fixed_point):
    beta^{k+1} = A_t(beta^k - gamma grad L(beta^k)),   grad L(beta) = 2 K (beta - alpha),
with A_t the soft-thresholding operator of the same section.  Reading: the
printed iteration thresholds at the step gamma; the fixed point that
characterises a minimiser of L + lam ||.||_1 thresholds at t = gamma lam
(the proximal operator of gamma lam ||.||_1), which is what is computed here.
The step defaults to 1 / Lip with Lip = 2 lambda_max(K), the Lipschitz
constant of grad L.
"""
from __future__ import annotations

import numpy as np


def soft_threshold(v, t: float) -> np.ndarray:
    """A_t(v)_i = v_i - t if v_i > t, 0 if |v_i| <= t, v_i + t if v_i < -t."""
    v = np.asarray(v, dtype=np.float64)
    out = np.zeros_like(v)
    out[v > t] = v[v > t] - t
    out[v < -t] = v[v < -t] + t
    return out


def objective(K, alpha, beta, lam: float) -> float:
    """f(beta) = (alpha - beta)^T K (alpha - beta) + lam ||beta||_1."""
    K = np.asarray(K, dtype=np.float64)
    d = np.asarray(alpha, np.float64) - np.asarray(beta, np.float64)
    return float(d @ K @ d + lam * np.abs(beta).sum())


def gradient(K, alpha, beta) -> np.ndarray:
    """grad L(beta) = 2 K (beta - alpha) (K symmetric)."""
    K = np.asarray(K, dtype=np.float64)
    return 2.0 * K @ (np.asarray(beta, np.float64) - np.asarray(alpha, np.float64))


def lipschitz(K) -> float:
    """2 lambda_max(K) (the largest eigenvalue of the symmetric Gram)."""
    K = np.asarray(K, dtype=np.float64)
    return 2.0 * float(np.linalg.eigvalsh(0.5 * (K + K.T)).max())


def ista(K, alpha, lam: float, iters: int, step: float | None = None, beta0=None):
    """(beta after `iters` iterations from beta0 (default alpha), objective
    before each iteration and after the last) -- eq. (fixed_point) iterated."""
    alpha = np.asarray(alpha, np.float64)
    gamma = 1.0 / lipschitz(K) if step is None else float(step)
    beta = alpha.copy() if beta0 is None else np.asarray(beta0, np.float64).copy()
    losses = []
    for _ in range(iters):
        losses.append(objective(K, alpha, beta, lam))
        beta = soft_threshold(beta - gamma * gradient(K, alpha, beta), gamma * lam)
    losses.append(objective(K, alpha, beta, lam))
    return beta, np.array(losses)


def lambda_max(K, alpha) -> float:
    """The smallest penalty at which beta = 0 is a minimiser:
    max_i |grad L(0)_i| = 2 max_i |(K alpha)_i|."""
    return float(np.abs(gradient(K, alpha, np.zeros_like(np.asarray(alpha, np.float64)))).max())


def ista_support(K, alpha, support: int, iters: int, rounds: int):
    """Penalty by bisection on [0, lambda_max] so that ista's weights have
    `support` non-zeros: each round runs `iters` iterations from the previous
    round's weights; more non-zeros than wanted raises the lower end, else the
    upper end.  Returns (beta, lam) of the last round whose support size
    equals `support` (else of the last round)."""
    lo, hi = 0.0, lambda_max(K, alpha)
    beta = np.asarray(alpha, np.float64).copy()
    best = None
    for _ in range(rounds):
        lam = 0.5 * (lo + hi)
        beta, _ = ista(K, alpha, lam, iters, beta0=beta)
        nnz = int(np.count_nonzero(beta))
        if nnz == support:
            best = (beta.copy(), lam)
        if nnz > support:
            lo = lam
        else:
            hi = lam
    return best if best is not None else (beta, lam)
