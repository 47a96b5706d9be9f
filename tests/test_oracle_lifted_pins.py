"""Pins of the static-kernel lift in the oracle (eq. (PDE_lifted) and the
finite-difference form after it), each against something other than the lift
itself: the plain solver on explicit feature paths, closed forms, limits of the
bandwidth and invariances of the RBF kernel."""
import math

import numpy as np
import pytest

import oracle


def rand_path(seed, L, d, scale=0.3):
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.normal(0.0, scale / math.sqrt(L), size=(L, d)), axis=0)


def rel(a, b):
    return abs(a - b) / max(1.0, abs(b))


@pytest.mark.parametrize("scheme", ["explicit", "implicit"])
@pytest.mark.parametrize("lam", [0, 1, 2])
def test_coefficient_solver_equals_path_solvers(lam, scheme):
    # driven by the increment Gram, the coefficient solver is the plain scheme
    x, y = rand_path(1, 13, 3, 2.0), rand_path(2, 9, 3, 2.0)
    v = oracle.solve_coef(oracle.increment_gram(x, y), lam, scheme)
    ref = oracle.solve_implicit(x, y, lam) if scheme == "implicit" else oracle.solve(x, y, lam)
    assert v == ref


@pytest.mark.parametrize("lam", [0, 2])
def test_linear_static_kernel_is_the_plain_kernel(lam):
    x, y = rand_path(3, 17, 4, 3.0), rand_path(4, 11, 4, 3.0)
    c = oracle.lifted_coefficients(x, y, oracle.LINEAR)
    g = oracle.increment_gram(x, y)
    assert np.abs(c - g).max() <= 1e-13 * (1 + np.abs(x).max() * np.abs(y).max())
    assert rel(oracle.solve_lifted(x, y, lam, oracle.LINEAR), oracle.solve(x, y, lam)) < 1e-12


def test_asymmetric_pairing_follows_the_row_path():
    # kappa(a, b) = <A a, b>: phi(a) = A a, psi(b) = b; A not symmetric, so a
    # transposed operand or swapped node index would change the value
    rng = np.random.default_rng(5)
    A = rng.normal(size=(3, 3))
    x, y = rand_path(6, 12, 3, 2.0), rand_path(7, 15, 3, 2.0)
    v = oracle.solve_lifted(x, y, 1, lambda P, Q: (P @ A.T) @ Q.T)
    assert rel(v, oracle.solve(x @ A.T, y, 1)) < 1e-12
    assert rel(v, oracle.solve(x @ A, y, 1)) > 1e-6


@pytest.mark.parametrize("lam", [0, 1])
def test_polynomial_kernel_is_the_kernel_of_its_feature_paths(lam):
    # <a,b> + <a,b>^2 = <phi(a), phi(b)> with phi(a) = (a, a (x) a)
    x, y = rand_path(8, 10, 3, 3.0), rand_path(9, 14, 3, 3.0)

    def phi(P):
        return np.concatenate([P, np.einsum("li,lj->lij", P, P).reshape(len(P), -1)], axis=1)

    def kap(P, Q):
        G = P @ Q.T
        return G + G * G

    v = oracle.solve_lifted(x, y, lam, kap)
    assert rel(v, oracle.solve(phi(x), phi(y), lam)) < 1e-12


@pytest.mark.parametrize("a,b,sigma", [(1.0, 1.0, 1.0), (0.5, -2.0, 0.7), (3.0, 2.0, 2.5),
                                       (-1.0, 0.25, 0.3)])
def test_rbf_one_cell_closed_form(a, b, sigma):
    # one cell at order 0: coefficient G = k(a,b) - k(0,b) - k(a,0) + k(0,0);
    # explicit: 1 + G; implicit: (1 + 3G/4) / (1 - G/4)
    k = lambda u, v: math.exp(-(u - v) ** 2 / (2 * sigma ** 2))  # noqa: E731
    G = k(a, b) - k(0, b) - k(a, 0) + k(0, 0)
    x, y = np.array([[0.0], [a]]), np.array([[0.0], [b]])
    assert rel(oracle.solve_lifted(x, y, 0, oracle.rbf(sigma)), 1 + G) < 1e-15
    assert rel(oracle.solve_lifted(x, y, 0, oracle.rbf(sigma), "implicit"),
               (1 + 0.75 * G) / (1 - 0.25 * G)) < 1e-15


def test_rbf_large_bandwidth_tends_to_the_plain_kernel():
    # sigma^2 exp(-|a-b|^2 / 2 sigma^2) = sigma^2 - |a|^2/2 - |b|^2/2 + <a,b> + O(1/sigma^2);
    # the second difference keeps only <dx, dy> + O(1/sigma^2)
    x, y = rand_path(10, 9, 2, 3.0), rand_path(11, 12, 2, 3.0)
    ref = oracle.solve(x, y, 1)

    def err(sigma):
        kap = lambda P, Q: sigma ** 2 * oracle.static_kernel_matrix(P, Q, oracle.rbf(sigma))  # noqa
        return abs(oracle.solve_lifted(x, y, 1, kap) - ref)

    e = [err(s) for s in (32.0, 64.0, 128.0)]
    assert e[2] < 2e-3 * abs(ref)
    for r in (e[0] / e[1], e[1] / e[2]):
        assert 3.7 < r < 4.3


@pytest.mark.parametrize("lam", [0, 1])
def test_rbf_small_bandwidth_is_the_simplex_path(lam):
    # sigma far below every node distance: kappa(x_i, x_j) = [i == j], the lift
    # of x sends its nodes to orthonormal vectors e_0, e_1, ...; so k(x, x) is
    # the plain kernel of the identity-matrix path, and k(x, y) = 1 when no
    # node of y is near a node of x
    x = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0], [0.0, 2.0], [2.0, 2.0]])
    y = x + np.array([0.5, 0.25])
    s = oracle.rbf(1e-3)
    eye = np.eye(len(x))
    assert rel(oracle.solve_lifted(x, x, lam, s), oracle.solve(eye, eye, lam)) < 1e-13
    assert oracle.solve_lifted(x, y, lam, s) == 1.0


def test_rbf_invariances():
    x, y = rand_path(12, 14, 3, 4.0), rand_path(13, 11, 3, 4.0)
    s = oracle.rbf(0.5)
    v = oracle.solve_lifted(x, y, 1, s)
    shift = np.array([3.0, -1.0, 0.5])
    assert rel(oracle.solve_lifted(x + shift, y + shift, 1, s), v) < 1e-12
    Q, _ = np.linalg.qr(np.random.default_rng(14).normal(size=(3, 3)))
    assert rel(oracle.solve_lifted(x @ Q, y @ Q, 1, s), v) < 1e-12
    assert rel(oracle.solve_lifted(y, x, 1, s), v) < 1e-12
    # a repeated node is a stationary segment: zero coefficients, same value
    xr = np.concatenate([x[:5], x[4:5], x[5:]], axis=0)
    assert rel(oracle.solve_lifted(xr, y, 1, s), v) < 1e-13
    assert rel(oracle.solve_lifted(xr, y, 0, s), oracle.solve_lifted(x, y, 0, s)) < 1e-13


def test_batches_match_single_solves():
    X = np.stack([rand_path(20 + i, 9, 2, 2.0) for i in range(4)])
    Y = np.stack([rand_path(30 + i, 7, 2, 2.0) for i in range(3)])
    K = oracle.lifted_rbf_gram(X, Y, 1, 0.8)
    for a in range(4):
        for b in range(3):
            assert K[a, b] == oracle.solve_lifted(X[a], Y[b], 1, oracle.rbf(0.8))
    P = oracle.lifted_rbf_pairs(list(X[:3]), [Y[0], Y[1], Y[2][:4]], 2, 0.8, "implicit")
    assert P[2] == oracle.solve_lifted(X[2], Y[2][:4], 2, oracle.rbf(0.8), "implicit")
