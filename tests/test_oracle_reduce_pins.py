"""Pins of the reduced-measure oracle (Section "Moments-matching reduction
algorithm ...", eqs. (min_lasso) and (fixed_point)): closed forms, an
independent bound-constrained quasi-Newton solve of the same convex problem,
the optimality (KKT) conditions, monotone descent, and the support size on
the signature Gram of the fBM ensemble."""
import numpy as np
import pytest
from scipy.optimize import minimize

import oracle
import workloads
from oracle import reduced_measure as rm


def spd(seed, n, cond=20.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    ev = np.geomspace(1.0, cond, n)
    return (Q * ev) @ Q.T


def test_soft_threshold_definition():
    got = rm.soft_threshold([3.0, 0.5, -2.0, -1.0, 1.0, 0.0], 1.0)
    assert np.array_equal(got, [2.0, 0.0, -1.0, 0.0, 0.0, 0.0])


def test_identity_gram_is_one_soft_threshold():
    # K = I: min |alpha - beta|^2 + lam |beta|_1 is soft(alpha, lam / 2), and
    # one step of length 1 / Lip = 1 / 2 from any start lands on it
    alpha = np.array([0.5, -0.2, 0.05, 1.0, -0.7])
    lam = 0.3
    beta, _ = rm.ista(np.eye(5), alpha, lam, 1, beta0=np.zeros(5))
    assert np.allclose(beta, rm.soft_threshold(alpha, lam / 2), atol=1e-15)
    beta20, _ = rm.ista(np.eye(5), alpha, lam, 20)
    assert np.allclose(beta20, rm.soft_threshold(alpha, lam / 2), atol=1e-15)


def test_zero_penalty_recovers_alpha():
    K = spd(1, 12, cond=5.0)
    alpha = np.full(12, 1.0 / 12)
    beta, losses = rm.ista(K, alpha, 0.0, 400, beta0=np.zeros(12))
    assert np.abs(beta - alpha).max() < 1e-10 and losses[-1] < 1e-18


def split_solve(K, alpha, lam):
    """The same problem with beta = p - q, p, q >= 0 (smooth, bounded),
    by L-BFGS-B: an independent solver of eq. (min_lasso)."""
    n = len(alpha)

    def f(z):
        p, q = z[:n], z[n:]
        d = alpha - (p - q)
        g = -2.0 * K @ d
        return d @ K @ d + lam * z.sum(), np.concatenate([g + lam, -g + lam])

    z0 = np.concatenate([np.maximum(alpha, 0), np.maximum(-alpha, 0)])
    r = minimize(f, z0, jac=True, method="L-BFGS-B", bounds=[(0, None)] * (2 * n),
                 options={"ftol": 1e-15, "gtol": 1e-12, "maxiter": 20000})
    return r.x[:n] - r.x[n:]


@pytest.mark.parametrize("seed,lam", [(2, 0.02), (3, 0.1), (4, 0.005)])
def test_matches_an_independent_solver_and_kkt(seed, lam):
    K = spd(seed, 15)
    alpha = np.random.default_rng(seed).dirichlet(np.ones(15))
    beta, losses = rm.ista(K, alpha, lam, 20000)
    ref = split_solve(K, alpha, lam)
    assert abs(rm.objective(K, alpha, beta, lam) - rm.objective(K, alpha, ref, lam)) < 1e-10
    assert np.abs(beta - ref).max() < 1e-5
    g = rm.gradient(K, alpha, beta)
    nz = beta != 0
    assert np.abs(g[nz] + lam * np.sign(beta[nz])).max() < 1e-8
    assert np.all(np.abs(g[~nz]) <= lam + 1e-8)
    assert np.all(np.diff(losses) <= 1e-15)  # non-increasing with step 1 / Lip


def test_penalty_at_lambda_max_gives_the_empty_support():
    K = spd(5, 10)
    alpha = np.full(10, 0.1)
    lm = rm.lambda_max(K, alpha)
    beta, _ = rm.ista(K, alpha, 1.001 * lm, 5000)
    assert np.all(beta == 0.0)
    beta2, _ = rm.ista(K, alpha, 0.9 * lm, 5000)
    assert np.count_nonzero(beta2) > 0


def test_support_of_six_on_the_fbm_ensemble():
    # 50-point paths at dyadic order 6: the rough (H = 0.2) members need a fine
    # grid before the discrete Gram is close to positive semi-definite (its
    # negative eigenvalues shrink fourfold per order, -0.013 here)
    P, H = workloads.fbm_paths(n_points=50)
    K = oracle.gram(P.astype(np.float64), P.astype(np.float64), 6)
    assert np.linalg.eigvalsh(K)[0] > -0.02
    alpha = np.full(30, 1.0 / 30)
    beta, lam = rm.ista_support(K, alpha, 6, 3000, 40)
    assert np.count_nonzero(beta) == 6
    g = rm.gradient(K, alpha, beta)
    nz = beta != 0
    assert np.abs(g[nz] + lam * np.sign(beta[nz])).max() < 1e-6
    assert np.all(np.abs(g[~nz]) <= lam * (1 + 1e-6))
