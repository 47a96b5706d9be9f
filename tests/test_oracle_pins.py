"""Pins for the FP64 oracle, each against something other than the oracle itself.

A plausible mistake in the oracle (a dropped term, a wrong sign, a transposed
operand, a wrong refinement scale, a wrong adjoint index) fails at least one of
these:

* hand-expanded values of the scheme (golden fixtures, exact dyadic rationals);
* the closed form of theorem (simple_Goursat_sol) / eq. (bessel_series) for
  straight segments, cross-checked with SciPy's Bessel routines;
* the second-order convergence of theorem (error);
* brute-force truncated signatures through Chen's identity (definition
  (signature), truncated signature, inner product of Section 2);
* invariances that hold for the discrete scheme or for its limit;
* the local error bound of theorem (local_error);
* finite differences of the forward solve for the discrete adjoint.
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest
import scipy.special as sp

import oracle
import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def seg_pair(c: float, d: int = 2):
    a = np.zeros((2, d))
    b = np.zeros((2, d))
    a[1, 0] = 1.0
    b[1, 0] = c
    return a, b


# ---------------------------------------------------------------------------
# Hand values (exact in binary floating point)
# ---------------------------------------------------------------------------
def _read_rows(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_straight_segment_hand_values():
    rows = _read_rows("straight_segment_hand_values.txt")
    assert len(rows) >= 8
    for c, lam, num, den in rows:
        x, y = seg_pair(float(Fraction(c)))
        want = Fraction(int(num), int(den))
        got = oracle.solve(x, y, int(lam))
        assert got == float(want), (c, lam, got, want)


def test_one_by_two_grid_hand_values():
    for r in _read_rows("one_by_two_grid.txt"):
        ax, ay, b1x, b1y, b2x, b2y, want = map(float, r)
        x = np.array([[0, 0], [ax, ay]])
        y = np.array([[0, 0], [b1x, b1y], [b1x + b2x, b1y + b2y]])
        assert oracle.solve(x, y, 0) == want
        # the same value with the roles of x and y exchanged
        assert oracle.solve(y, x, 0) == want


# ---------------------------------------------------------------------------
# Closed form for straight segments (Appendix A) and convergence order
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("c", [1.0, -1.0, 2.0, 0.3, -2.5])
def test_closed_form_series_matches_scipy(c):
    # eq. (bessel_series) with n = 0 versus library Bessel functions
    want = sp.i0(2 * math.sqrt(c)) if c >= 0 else sp.j0(2 * math.sqrt(-c))
    assert abs(oracle.straight_segment_kernel(c) - want) < 1e-13 * max(1.0, abs(want))
    # and the n = 1 series against I1 (used by the gradient pin below)
    if c > 0:
        z = math.sqrt(c)
        assert abs(oracle.bessel_series(1, z) - sp.i1(2 * z)) < 1e-13 * sp.i1(2 * z)


@pytest.mark.parametrize("c", [1.0, -1.0, 2.0, 0.3])
def test_limit_is_riemann_function(c):
    x, y = seg_pair(c)
    v6, v7 = oracle.solve(x, y, 6), oracle.solve(x, y, 7)
    exact = oracle.straight_segment_kernel(c)
    assert abs(oracle.richardson(v6, v7) - exact) < 2e-8
    assert abs(v7 - exact) < 1e-4 * max(1.0, abs(exact))


def test_paper_values_I0_J0():
    # I0(2) and J0(2): c = +1 and c = -1
    assert abs(oracle.straight_segment_kernel(1.0) - 2.279585302336067) < 1e-12
    assert abs(oracle.straight_segment_kernel(-1.0) - 0.2238907791412357) < 1e-12


@pytest.mark.parametrize("c", [1.0, 2.0, -1.0])
def test_second_order_convergence_straight(c):
    # theorem (error): sup error <= K / 4^lambda; the ratio tends to 4
    x, y = seg_pair(c)
    exact = oracle.straight_segment_kernel(c)
    errs = [oracle.solve(x, y, lam) - exact for lam in range(3, 8)]
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    for r in ratios:
        assert 3.8 < r < 4.2, ratios


def test_second_order_convergence_random_pair():
    x, y, _, _ = workloads.single_pair()
    x = x[:9].astype(np.float64)
    y = y[:7].astype(np.float64)
    v = [oracle.solve(x, y, lam) for lam in range(2, 8)]
    diffs = [v[i + 1] - v[i] for i in range(len(v) - 1)]
    ratios = [diffs[i] / diffs[i + 1] for i in range(len(diffs) - 1)]
    assert all(3.7 < r < 4.3 for r in ratios[1:]), ratios


def test_local_error_bound_single_cell():
    # theorem (local_error), eq. (error_estimate_1) with boundary data 1
    for c in [0.05, 0.2, 0.5, 1.0, -0.3, -1.0]:
        x, y = seg_pair(c)
        err = abs(oracle.straight_segment_kernel(c) - oracle.solve(x, y, 0))
        assert err <= oracle.local_error_bound_boundary_one(c) + 1e-15, (c, err)


@pytest.mark.parametrize("c", [0.5, 1.0, -1.0])
def test_local_error_bound_equals_bessel_values(c):
    # The bound is |c| sup_{z between 0 and c} |I1(2 sqrt z) / sqrt z - 1|.  The
    # series has positive coefficients and is increasing on [-1, inf), so the
    # supremum sits at z = c: I1(2 sqrt c) / sqrt c - 1 for c > 0 and
    # J1(2 sqrt |c|) / sqrt |c| - 1 for c < 0 (SciPy's Bessel routines).  A
    # looser or tighter bound than the theorem's fails here.
    r = math.sqrt(abs(c))
    f = (sp.iv(1, 2 * r) if c > 0 else sp.jv(1, 2 * r)) / r - 1.0
    want = abs(c) * abs(f)
    assert abs(oracle.local_error_bound_boundary_one(c) - want) <= 1e-14 * want, c
    # hand value at c = 1: I1(2) - 1
    if c == 1.0:
        assert abs(oracle.local_error_bound_boundary_one(c) - 0.590636854637329) < 1e-14


def test_truncation_tail_bound_is_exact_for_parallel_segments():
    # For x = [0, a] and y = [0, t a] (t > 0), <S^k(x), S^k(y)> = <a, t a>^k / (k!)^2
    # and |x|_1 |y|_1 = <a, t a>: the bound of the factorial decay and
    # Cauchy-Schwarz is attained.  The tail is summed by brute force from the
    # truncated signatures (levels N+1 .. N+11; the levels above add < 1e-19).
    a = np.array([0.6, -1.1])
    x = np.array([np.zeros(2), a])
    y = np.array([np.zeros(2), 1.3 * a])
    N, top = 3, 14
    sx = oracle.truncated_signature(x, top)
    sy = oracle.truncated_signature(y, top)
    exact = sum(float(np.sum(sx[k] * sy[k])) for k in range(N + 1, top + 1))
    bound = oracle.truncation_tail_bound(x, y, N)
    assert abs(bound - exact) <= 1e-13 * exact, (bound, exact)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_truncation_tail_bound_holds_on_random_paths(seed):
    # the exact levels above N (brute force) stay below the bound, and the bound
    # is not vacuous: within a factor 10^4 of the level-(N+1) term here
    rng = np.random.default_rng(seed)
    x = np.cumsum(rng.normal(0, 0.5, size=(4, 2)), axis=0)
    y = np.cumsum(rng.normal(0, 0.5, size=(3, 2)), axis=0)
    N, top = 2, 10
    sx = oracle.truncated_signature(x, top)
    sy = oracle.truncated_signature(y, top)
    levels = [float(np.sum(sx[k] * sy[k])) for k in range(N + 1, top + 1)]
    bound = oracle.truncation_tail_bound(x, y, N)
    assert sum(abs(v) for v in levels) <= bound
    assert bound <= 1e4 * max(abs(levels[0]), 1e-300)


# ---------------------------------------------------------------------------
# Brute-force signatures (definition (signature), Chen's identity)
# ---------------------------------------------------------------------------
def test_chen_single_segment_is_tensor_exponential():
    # level-2 signature of a straight segment v is v (x) v / 2, and of two
    # segments v, w is v(x)v/2 + v(x)w + w(x)w/2 (Chen)
    v = np.array([0.3, -0.2, 0.5])
    w = np.array([-0.1, 0.4, 0.2])
    s = oracle.truncated_signature(np.array([np.zeros(3), v, v + w]), 3)
    assert np.allclose(s[1], v + w, atol=1e-15)
    want2 = np.outer(v, v) / 2 + np.outer(v, w) + np.outer(w, w) / 2
    assert np.allclose(s[2], want2, atol=1e-15)


@pytest.mark.parametrize("d,lx,ly,seed", [(2, 5, 4, 1), (3, 5, 4, 2), (3, 4, 6, 3)])
def test_bruteforce_truncated_signature_kernel(d, lx, ly, seed):
    rng = np.random.default_rng(seed)
    x = np.cumsum(rng.normal(0, 0.3, size=(lx, d)), axis=0)
    y = np.cumsum(rng.normal(0, 0.3, size=(ly, d)), axis=0)
    N = 12
    tail = oracle.truncation_tail_bound(x, y, N)
    assert tail < 1e-12
    brute = oracle.signature_kernel_truncated(x, y, N)
    pde = oracle.richardson(oracle.solve(x, y, 6), oracle.solve(x, y, 7))
    assert abs(brute - pde) < 1e-9 * max(1.0, abs(brute)), (brute, pde)


# ---------------------------------------------------------------------------
# Increment Gram against a library product
# ---------------------------------------------------------------------------
def test_increment_gram_matches_matmul():
    rng = np.random.default_rng(7)
    x = rng.normal(size=(13, 5))
    y = rng.normal(size=(9, 5))
    g = oracle.increment_gram(x, y)
    want = np.diff(x, axis=0) @ np.diff(y, axis=0).T
    assert g.shape == (12, 8)
    assert np.allclose(g, want, rtol=1e-14, atol=1e-14)


# ---------------------------------------------------------------------------
# Invariants
# ---------------------------------------------------------------------------
def _rand_pair(seed, lx=12, ly=9, d=3, s=0.3):
    rng = np.random.default_rng(seed)
    x = np.cumsum(rng.normal(0, s, size=(lx, d)), axis=0)
    y = np.cumsum(rng.normal(0, s, size=(ly, d)), axis=0)
    return x, y


@pytest.mark.parametrize("lam", [0, 1, 2])
def test_symmetry_bitwise(lam):
    # <S(x), S(y)> = <S(y), S(x)>; the scheme is symmetric cell by cell
    x, y = _rand_pair(11)
    assert oracle.solve(x, y, lam) == oracle.solve(y, x, lam)
    g = oracle.solve_grid(x, y, lam)
    gt = oracle.solve_grid(y, x, lam)
    assert np.array_equal(g, gt.T)


@pytest.mark.parametrize("lam", [0, 2])
def test_translation_and_rotation(lam):
    x, y = _rand_pair(12)
    v = oracle.solve(x, y, lam)
    assert abs(oracle.solve(x + 3.0, y - 1.5, lam) - v) < 1e-13 * abs(v)
    q, _ = np.linalg.qr(np.random.default_rng(5).normal(size=(3, 3)))
    assert abs(oracle.solve(x @ q, y @ q, lam) - v) < 1e-12 * abs(v)


def test_boundary_and_degenerate_paths():
    x, y = _rand_pair(13)
    assert oracle.solve(x[:1], y, 2) == 1.0
    assert oracle.solve(x, y[:1], 0) == 1.0
    const = np.repeat(x[:1], 6, axis=0)
    assert oracle.solve(const, y, 1) == 1.0
    g = oracle.solve_grid(x, y, 1)
    assert np.all(g[0, :] == 1.0) and np.all(g[:, 0] == 1.0)


@pytest.mark.parametrize("lam", [0, 1])
def test_duplicate_point_is_invisible(lam):
    # a zero increment is a constant reparametrisation piece: zero coefficient rows
    x, y = _rand_pair(14)
    xd = np.insert(x, 5, x[5], axis=0)
    v = oracle.solve(x, y, lam)
    assert abs(oracle.solve(xd, y, lam) - v) < 1e-14 * abs(v)


@pytest.mark.parametrize("lam", [0, 1, 2])
def test_midpoint_subdivision_equals_next_dyadic_order(lam):
    # definition (fintite_diff) + the refinement remark: halving every segment
    # of both paths and solving at lambda reproduces P_{lambda+1}
    x, y = _rand_pair(15, lx=7, ly=6)

    def halve(p):
        out = [p[0]]
        for i in range(len(p) - 1):
            out += [(p[i] + p[i + 1]) / 2, p[i + 1]]
        return np.array(out)

    v1 = oracle.solve(x, y, lam + 1)
    v2 = oracle.solve(halve(x), halve(y), lam)
    assert abs(v1 - v2) < 1e-13 * abs(v1)


def test_reparametrisation_invariance_in_the_limit():
    # S(x o phi) = S(x): inserting a point on a segment (at 1/3) changes the
    # grid but not the limit
    x, y = _rand_pair(16, lx=5, ly=4)
    xr = np.insert(x, 2, x[1] + (x[2] - x[1]) / 3.0, axis=0)
    a = oracle.richardson(oracle.solve(x, y, 6), oracle.solve(x, y, 7))
    b = oracle.richardson(oracle.solve(xr, y, 6), oracle.solve(xr, y, 7))
    assert abs(a - b) < 1e-8 * abs(a)
    assert abs(oracle.solve(x, y, 2) - oracle.solve(xr, y, 2)) > 1e-9  # grids differ


def test_tree_like_retracing_in_the_limit():
    # appending a segment and its reversal leaves the signature unchanged
    x, y = _rand_pair(17, lx=5, ly=4)
    a_seg = np.array([0.2, -0.3, 0.1])
    xt = np.vstack([x, x[-1] + a_seg, x[-1]])
    a = oracle.richardson(oracle.solve(x, y, 6), oracle.solve(x, y, 7))
    b = oracle.richardson(oracle.solve(xt, y, 6), oracle.solve(xt, y, 7))
    assert abs(a - b) < 1e-8 * abs(a)


# ---------------------------------------------------------------------------
# Batches are the single-pair solver applied pair by pair
# ---------------------------------------------------------------------------
def test_batch_entry_points_match_single_solves():
    rng = np.random.default_rng(21)
    xs = [np.cumsum(rng.normal(0, 0.2, size=(L, 3)), 0) for L in (5, 9, 1, 7)]
    ys = [np.cumsum(rng.normal(0, 0.2, size=(L, 3)), 0) for L in (6, 2, 8, 1)]
    out = oracle.pairs(xs, ys, 1)
    for k in range(4):
        assert out[k] == oracle.solve(xs[k], ys[k], 1)
    K = oracle.gram(xs, ys, 1)
    for a in range(4):
        for b in range(4):
            assert K[a, b] == oracle.solve(xs[a], ys[b], 1)


# ---------------------------------------------------------------------------
# Discrete adjoint
# ---------------------------------------------------------------------------
def _fd_grad(x, y, lam, h=1e-4):
    gx = np.zeros_like(x)
    gy = np.zeros_like(y)
    for arr, g in ((x, gx), (y, gy)):
        for idx in np.ndindex(arr.shape):
            old = arr[idx]
            arr[idx] = old + h
            fp = oracle.solve(x, y, lam)
            arr[idx] = old - h
            fm = oracle.solve(x, y, lam)
            arr[idx] = old
            g[idx] = (fp - fm) / (2 * h)
    return gx, gy


@pytest.mark.parametrize("lam", [0, 1, 2])
def test_adjoint_matches_central_differences(lam):
    x, y = _rand_pair(31, lx=6, ly=5, d=2, s=0.4)
    v, gx, gy = oracle.solve_grad(x, y, lam)
    assert v == oracle.solve(x, y, lam)
    fx, fy = _fd_grad(x.copy(), y.copy(), lam)
    scale = max(np.abs(fx).max(), np.abs(fy).max())
    assert np.abs(gx - fx).max() < 1e-7 * scale
    assert np.abs(gy - fy).max() < 1e-7 * scale


def test_adjoint_translation_and_swap():
    x, y = _rand_pair(32, lx=8, ly=6)
    _, gx, gy = oracle.solve_grad(x, y, 1)
    # k depends on increments only, so the gradient sums to zero over points
    assert np.abs(gx.sum(axis=0)).max() < 1e-13
    assert np.abs(gy.sum(axis=0)).max() < 1e-13
    _, hy, hx = oracle.solve_grad(y, x, 1)
    assert np.allclose(gx, hx, rtol=1e-13, atol=1e-15)
    assert np.allclose(gy, hy, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("c", [0.7, 1.5])
def test_adjoint_limit_straight_segment(c):
    # d/dc sum c^k/(k!)^2 = I1(2 sqrt c)/sqrt c (eq. (bessel_identity_1)), so
    # d k / d a = b I1(2 sqrt c)/sqrt c for the segment endpoint a
    b = np.array([0.6, 0.0])
    a = np.array([c / 0.6, 0.0])
    x = np.array([[0.0, 0.0], a])
    y = np.array([[0.0, 0.0], b])
    _, g6, _ = oracle.solve_grad(x, y, 6)
    _, g7, _ = oracle.solve_grad(x, y, 7)
    lim = oracle.richardson(g6[1, 0], g7[1, 0])
    want = b[0] * oracle.bessel_series(1, math.sqrt(c)) / math.sqrt(c)
    assert abs(lim - want) < 1e-7 * abs(want)


def test_gram_backward_matches_finite_differences():
    rng = np.random.default_rng(41)
    X = np.cumsum(rng.normal(0, 0.3, size=(3, 5, 2)), axis=1)
    Y = np.cumsum(rng.normal(0, 0.3, size=(2, 4, 2)), axis=1)
    dK = rng.normal(size=(3, 2))
    dX, dY = oracle.gram_backward(X, Y, dK, 1)

    def f(X, Y):
        return float(np.sum(dK * oracle.gram(X, Y, 1)))

    h = 1e-5
    for arr, g in ((X, dX), (Y, dY)):
        for idx in np.ndindex(arr.shape):
            old = arr[idx]
            arr[idx] = old + h
            fp = f(X, Y)
            arr[idx] = old - h
            fm = f(X, Y)
            arr[idx] = old
            assert abs((fp - fm) / (2 * h) - g[idx]) < 1e-7 * max(1.0, abs(g[idx]))


def test_mmd2_unbiased_definition_and_weights():
    rng = np.random.default_rng(51)
    X = np.cumsum(rng.normal(0, 0.3, size=(4, 6, 2)), axis=1)
    Y = np.cumsum(rng.normal(0, 0.3, size=(3, 6, 2)), axis=1)
    Kxx, Kyy, Kxy = oracle.gram(X, X, 0), oracle.gram(Y, Y, 0), oracle.gram(X, Y, 0)
    # direct double loop of the U-statistic
    n, m = 4, 3
    want = sum(Kxx[i, j] for i in range(n) for j in range(n) if i != j) / (n * (n - 1))
    want += sum(Kyy[i, j] for i in range(m) for j in range(m) if i != j) / (m * (m - 1))
    want -= 2 * Kxy.sum() / (n * m)
    assert abs(oracle.mmd2_unbiased(Kxx, Kyy, Kxy) - want) < 1e-14
    wxx, wyy, wxy = oracle.mmd2_weights(n, m)
    assert abs(np.sum(wxx * Kxx) + np.sum(wyy * Kyy) + np.sum(wxy * Kxy) - want) < 1e-14


# ---------------------------------------------------------------------------
# Implicit scheme (remark after eq. explicit_finite_diff)
# ---------------------------------------------------------------------------
def _implicit_golden():
    rows = []
    for line in open(os.path.join(GOLDEN, "implicit_one_cell.txt")):
        if line.strip() and not line.startswith("#"):
            c, num, den = line.split()
            rows.append((float(c), int(num) / int(den)))
    return rows


def straight(a, b):
    x = np.array([np.zeros_like(a), a])
    y = np.array([np.zeros_like(b), b])
    return x, y


@pytest.mark.parametrize("c,expected", _implicit_golden())
def test_implicit_one_cell_closed_form(c, expected):
    # c = <a, b> with a = (c, 0), b = (1, 0)
    x, y = straight(np.array([c, 0.0]), np.array([1.0, 0.0]))
    assert abs(oracle.solve_implicit(x, y, 0) - expected) <= 1e-15 * max(1, abs(expected))


def test_implicit_matches_bessel_series_to_second_order():
    # one cell: (1 + 3c/4)/(1 - c/4) = 1 + c + c^2/4 + c^3/16 + ...; the exact
    # kernel sum c^k/(k!)^2 = 1 + c + c^2/4 + c^3/36 + ...: they differ at c^3
    for c in (1e-2, -1e-2, 3e-3):
        x, y = straight(np.array([c, 0.0]), np.array([1.0, 0.0]))
        diff = oracle.solve_implicit(x, y, 0) - oracle.straight_segment_kernel(c)
        assert abs(diff - c ** 3 * (1 / 16 - 1 / 36)) <= 2 * abs(c) ** 4


def test_implicit_converges_second_order_to_the_explicit_limit():
    rng = np.random.default_rng(5)
    x = np.cumsum(rng.normal(size=(6, 3)) * 0.5, axis=0)
    y = np.cumsum(rng.normal(size=(5, 3)) * 0.5, axis=0)
    lim = oracle.richardson(oracle.solve(x, y, 6), oracle.solve(x, y, 7))
    errs = [abs(oracle.solve_implicit(x, y, lam) - lim) for lam in range(1, 6)]
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(3.5 < r < 4.5 for r in ratios[1:]), ratios


def test_implicit_invariants():
    rng = np.random.default_rng(6)
    x = np.cumsum(rng.normal(size=(7, 2)) * 0.4, axis=0)
    y = np.cumsum(rng.normal(size=(4, 2)) * 0.4, axis=0)
    k = oracle.solve_implicit(x, y, 2)
    assert abs(oracle.solve_implicit(y, x, 2) - k) <= 1e-13
    assert abs(oracle.solve_implicit(x + 3.0, y - 1.0, 2) - k) <= 1e-12
    assert oracle.solve_implicit(x[:1], y, 1) == 1.0
    g = oracle.solve_implicit(x, y, 1, grid=True)
    assert g.shape == (13, 7) and np.all(g[0] == 1.0) and np.all(g[:, 0] == 1.0)
    # the cell relation holds at every cell of the grid (the solve, checked
    # against its defining equation rather than its own rearrangement)
    c = oracle.increment_gram(x, y) / 4.0
    for i in range(12):
        for j in range(6):
            inc = c[i >> 1, j >> 1]
            lhs = g[i + 1, j + 1]
            rhs = g[i + 1, j] + g[i, j + 1] - g[i, j] + 0.25 * inc * (
                g[i, j] + g[i + 1, j] + g[i, j + 1] + g[i + 1, j + 1])
            assert abs(lhs - rhs) <= 1e-14 * max(1, abs(lhs))
    xs = [x, y, x[:3]]
    ys = [y, x, y[:2]]
    assert np.allclose(oracle.pairs_implicit(xs, ys, 1),
                       [oracle.solve_implicit(a, b, 1) for a, b in zip(xs, ys)], rtol=0, atol=0)
