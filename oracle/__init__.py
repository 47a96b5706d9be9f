"""FP64 CPU oracle for the PDE signature kernel (arXiv 2006.14794).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_2006_14794_amd``) never imports it, and the two share no code: the
only thing both sides consume is the seeded synthetic inputs of
``workloads.py``, which contain none of the method's arithmetic.

Contents
--------
* ``libsko.so`` (built from ``sko.c``): the explicit scheme of eq.
  (explicit_finite_diff), Section 3.1, on the dyadic grid P_lambda of definition
  (fintite_diff), in IEEE double, plus its discrete adjoint and OpenMP loops over
  the pairs of a batch or a Gram matrix; and the implicit scheme of the remark
  after that equation (all four corners in the cell quadrature), solved for the
  new corner cell by cell.
* Pure-Python / NumPy pieces used to pin the solver:
  - ``bessel_series``: I_n(2z) = z^n sum_k z^{2k} / (k! (n+k)!), eq.
    (bessel_series), Appendix A.  With theorem (simple_Goursat_sol) the exact
    signature kernel of two straight segments with <a, b> = c is
    R(1, 1) = sum_k c^k / (k!)^2.
  - ``truncated_signature`` / ``signature_kernel_truncated``: definition
    (signature), the truncation of eq. (truncated_signature), Chen's identity
    (the remark on multiplicative functionals in the rough-path appendix) and
    the inner product of definition 2.1 (Section 2).
  - ``mmd2_unbiased``: the unbiased MMD estimator mentioned at the end of
    Section 3.1.1 (U-statistic, diagonal terms excluded).
* The static-kernel lift (eq. (PDE_lifted) and its finite-difference form):
  ``static_kernel_matrix`` (RBF, linear or any callable kernel),
  ``lifted_coefficients`` (its second difference over each coarse cell),
  ``solve_coef`` (either scheme driven by a given coefficient matrix),
  ``solve_lifted`` and the OpenMP batches ``lifted_rbf_pairs`` /
  ``lifted_rbf_gram``.
* ``reduced_measure``: the moments-matching reduction of a discrete measure on
  paths (eqs. (min_lasso), (fixed_point)): soft-thresholding, proximal
  gradient, and the penalty that gives a chosen support size.

Every function here is pinned by ``tests/test_oracle_pins.py`` against
something other than itself (hand-derived values, closed forms, library
routines, brute force, invariants).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsko.so")
_SRC_PATH = os.path.join(_HERE, "sko.c")
_lib = None


def build(force: bool = True) -> str:
    """Compile sko.c into libsko.so with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
               "-o", tmp, _SRC_PATH, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC_PATH)):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int64)
    i64, i32 = ctypes.c_int64, ctypes.c_int32
    lib.sko_increment_gram.argtypes = [dp, i64, dp, i64, i32, dp]
    lib.sko_increment_gram.restype = None
    lib.sko_solve.argtypes = [dp, i64, dp, i64, i32, i32, dp]
    lib.sko_solve.restype = ctypes.c_double
    lib.sko_solve_grad.argtypes = [dp, i64, dp, i64, i32, i32, dp, dp]
    lib.sko_solve_grad.restype = ctypes.c_double
    lib.sko_pairs.argtypes = [dp, ip, dp, ip, i64, i32, i32, dp, ctypes.c_int]
    lib.sko_pairs.restype = None
    lib.sko_gram.argtypes = [dp, ip, i64, dp, ip, i64, i32, i32, dp, ctypes.c_int]
    lib.sko_gram.restype = None
    lib.sko_gram_backward.argtypes = [dp, ip, i64, dp, ip, i64, i32, i32, dp, dp, dp,
                                      ctypes.c_int]
    lib.sko_gram_backward.restype = None
    lib.sko_solve_implicit.argtypes = [dp, i64, dp, i64, i32, i32, dp]
    lib.sko_solve_implicit.restype = ctypes.c_double
    lib.sko_pairs_implicit.argtypes = [dp, ip, dp, ip, i64, i32, i32, dp, ctypes.c_int]
    lib.sko_pairs_implicit.restype = None
    lib.sko_static_rbf.argtypes = [dp, i64, dp, i64, i32, ctypes.c_double, dp]
    lib.sko_static_rbf.restype = None
    lib.sko_static_linear.argtypes = [dp, i64, dp, i64, i32, dp]
    lib.sko_static_linear.restype = None
    lib.sko_lifted_coefficients.argtypes = [dp, i64, i64, dp]
    lib.sko_lifted_coefficients.restype = None
    lib.sko_solve_coef.argtypes = [dp, i64, i64, i32, i32, dp]
    lib.sko_solve_coef.restype = ctypes.c_double
    lib.sko_lifted_rbf_batch.argtypes = [dp, ip, i64, dp, ip, i64, i32, i32, ctypes.c_double,
                                         i32, i32, dp, ctypes.c_int]
    lib.sko_lifted_rbf_batch.restype = None
    lib.sko_max_threads.argtypes = []
    lib.sko_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _path(a) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if a.ndim == 1:
        a = a.reshape(-1, 1)
    assert a.ndim == 2 and a.shape[0] >= 1
    return a


def max_threads() -> int:
    return int(_load().sko_max_threads())


# ---------------------------------------------------------------------------
# Single pairs
# ---------------------------------------------------------------------------
def increment_gram(x, y) -> np.ndarray:
    """G0[p, q] = <x_{p+1} - x_p, y_{q+1} - y_q> (Section 3.1), FP64."""
    x, y = _path(x), _path(y)
    assert x.shape[1] == y.shape[1]
    m, n = x.shape[0] - 1, y.shape[0] - 1
    g = np.zeros((max(m, 0), max(n, 0)), dtype=np.float64)
    if m > 0 and n > 0:
        _load().sko_increment_gram(_dptr(x), x.shape[0], _dptr(y), y.shape[0],
                                   x.shape[1], _dptr(g))
    return g


def solve(x, y, dyadic_order: int = 0) -> float:
    """Terminal value k_hat(s_M, t_N) of the explicit scheme on P_lambda."""
    x, y = _path(x), _path(y)
    assert x.shape[1] == y.shape[1] and dyadic_order >= 0
    return float(_load().sko_solve(_dptr(x), x.shape[0], _dptr(y), y.shape[0],
                                   x.shape[1], int(dyadic_order), None))


def solve_implicit(x, y, dyadic_order: int = 0, grid: bool = False):
    """Terminal value (or all nodes with grid=True) of the implicit scheme of
    the remark after eq. (explicit_finite_diff), on P_lambda."""
    x, y = _path(x), _path(y)
    assert x.shape[1] == y.shape[1] and dyadic_order >= 0
    M = (x.shape[0] - 1) << dyadic_order
    N = (y.shape[0] - 1) << dyadic_order
    g = np.empty((M + 1, N + 1), dtype=np.float64) if grid else None
    v = _load().sko_solve_implicit(_dptr(x), x.shape[0], _dptr(y), y.shape[0], x.shape[1],
                                   int(dyadic_order), _dptr(g) if grid else None)
    return g if grid else float(v)


def pairs_implicit(xs, ys, dyadic_order: int = 0, nthreads: int = 0) -> np.ndarray:
    """Independent pairs with the implicit scheme (OpenMP over pairs)."""
    xf, xo, d = _pack(xs)
    yf, yo, d2 = _pack(ys)
    assert d == d2 and len(xo) == len(yo)
    n = len(xo) - 1
    out = np.empty(n, dtype=np.float64)
    _load().sko_pairs_implicit(_dptr(xf), _iptr(xo), _dptr(yf), _iptr(yo), n, d,
                               int(dyadic_order), _dptr(out), int(nthreads))
    return out


def solve_grid(x, y, dyadic_order: int = 0) -> np.ndarray:
    """All nodes of the explicit scheme on P_lambda, shape (M+1, N+1)."""
    x, y = _path(x), _path(y)
    M = (x.shape[0] - 1) << dyadic_order
    N = (y.shape[0] - 1) << dyadic_order
    grid = np.empty((M + 1, N + 1), dtype=np.float64)
    _load().sko_solve(_dptr(x), x.shape[0], _dptr(y), y.shape[0], x.shape[1],
                      int(dyadic_order), _dptr(grid))
    return grid


def solve_grad(x, y, dyadic_order: int = 0):
    """(k_hat, d k_hat / d x [lx, d], d k_hat / d y [ly, d]) -- discrete adjoint."""
    x, y = _path(x), _path(y)
    gx = np.zeros_like(x)
    gy = np.zeros_like(y)
    v = _load().sko_solve_grad(_dptr(x), x.shape[0], _dptr(y), y.shape[0],
                               x.shape[1], int(dyadic_order), _dptr(gx), _dptr(gy))
    return float(v), gx, gy


# ---------------------------------------------------------------------------
# Batches (ragged paths given as a list of [L_k, d] arrays, or a [B, L, d] array)
# ---------------------------------------------------------------------------
def _pack(paths) -> tuple[np.ndarray, np.ndarray, int]:
    if isinstance(paths, np.ndarray) and paths.ndim == 3:
        B, L, d = paths.shape
        flat = np.ascontiguousarray(paths.reshape(B * L, d), dtype=np.float64)
        off = np.arange(B + 1, dtype=np.int64) * L
        return flat, off, d
    arrs = [_path(p) for p in paths]
    d = arrs[0].shape[1]
    off = np.zeros(len(arrs) + 1, dtype=np.int64)
    off[1:] = np.cumsum([a.shape[0] for a in arrs])
    flat = np.ascontiguousarray(np.concatenate(arrs, axis=0), dtype=np.float64)
    return flat, off, d


def pairs(xs, ys, dyadic_order: int = 0, nthreads: int = 0) -> np.ndarray:
    """out[k] = k_hat(x_k, y_k) for independent pairs (OpenMP over pairs)."""
    xf, xo, d = _pack(xs)
    yf, yo, d2 = _pack(ys)
    assert d == d2 and len(xo) == len(yo)
    n = len(xo) - 1
    out = np.empty(n, dtype=np.float64)
    _load().sko_pairs(_dptr(xf), _iptr(xo), _dptr(yf), _iptr(yo), n, d,
                      int(dyadic_order), _dptr(out), int(nthreads))
    return out


def gram(X, Y, dyadic_order: int = 0, nthreads: int = 0) -> np.ndarray:
    """K[a, b] = k_hat(X_a, Y_b) (OpenMP over pairs)."""
    xf, xo, d = _pack(X)
    yf, yo, d2 = _pack(Y)
    assert d == d2
    nx, ny = len(xo) - 1, len(yo) - 1
    K = np.empty((nx, ny), dtype=np.float64)
    _load().sko_gram(_dptr(xf), _iptr(xo), nx, _dptr(yf), _iptr(yo), ny, d,
                     int(dyadic_order), _dptr(K), int(nthreads))
    return K


def gram_backward(X, Y, dK, dyadic_order: int = 0, nthreads: int = 0):
    """(dX, dY): sum_b dK[a,b] grad_{X_a} k(X_a,Y_b) and the Y counterpart.

    Returned with the packed (ragged) layout [total points, d]; for [B, L, d]
    inputs they are reshaped back to [B, L, d]."""
    xf, xo, d = _pack(X)
    yf, yo, _ = _pack(Y)
    nx, ny = len(xo) - 1, len(yo) - 1
    dK = np.ascontiguousarray(np.asarray(dK, dtype=np.float64).reshape(nx, ny))
    dX = np.zeros_like(xf)
    dY = np.zeros_like(yf)
    _load().sko_gram_backward(_dptr(xf), _iptr(xo), nx, _dptr(yf), _iptr(yo), ny, d,
                              int(dyadic_order), _dptr(dK), _dptr(dX), _dptr(dY),
                              int(nthreads))
    if isinstance(X, np.ndarray) and X.ndim == 3:
        dX = dX.reshape(X.shape)
    if isinstance(Y, np.ndarray) and Y.ndim == 3:
        dY = dY.reshape(Y.shape)
    return dX, dY


# ---------------------------------------------------------------------------
# Signature-kernel MMD (end of Section 3.1.1: an unbiased estimator)
# ---------------------------------------------------------------------------
def mmd2_unbiased(Kxx: np.ndarray, Kyy: np.ndarray, Kxy: np.ndarray) -> float:
    """U-statistic MMD^2: mean of off-diagonal Kxx + mean of off-diagonal Kyy
    - 2 mean of Kxy."""
    n, m = Kxx.shape[0], Kyy.shape[0]
    sxx = (Kxx.sum() - np.trace(Kxx)) / (n * (n - 1))
    syy = (Kyy.sum() - np.trace(Kyy)) / (m * (m - 1))
    sxy = Kxy.sum() / (n * m)
    return float(sxx + syy - 2.0 * sxy)


def mmd2_weights(n: int, m: int):
    """d MMD^2 / d K for the three Gram blocks (Kxx, Kyy, Kxy)."""
    wxx = np.full((n, n), 1.0 / (n * (n - 1)))
    np.fill_diagonal(wxx, 0.0)
    wyy = np.full((m, m), 1.0 / (m * (m - 1)))
    np.fill_diagonal(wyy, 0.0)
    wxy = np.full((n, m), -2.0 / (n * m))
    return wxx, wyy, wxy


# ---------------------------------------------------------------------------
# Closed forms (Appendix A)
# ---------------------------------------------------------------------------
def bessel_series(n: int, z: float, terms: int = 80) -> float:
    """I_n(2z) by the series of eq. (bessel_series), summed in double."""
    s = 0.0
    for k in range(terms):
        s += z ** (2 * k) / (math.factorial(k) * math.factorial(n + k))
    return s * z ** n


def straight_segment_kernel(c: float, terms: int = 80) -> float:
    """Exact signature kernel of two straight segments with <a, b> = c.

    Theorem (simple_Goursat_sol) with boundary data 1 gives k = R(1, 1), and the
    series of eq. (bessel_series) with n = 0 turns R into sum_k c^k / (k!)^2,
    which is real for either sign of c (I_0(2 sqrt c) for c > 0, J_0(2 sqrt|c|)
    for c < 0)."""
    s = 0.0
    for k in range(terms):
        s += c ** k / (math.factorial(k) ** 2)
    return s


def richardson(v_coarse: float, v_fine: float, order: int = 2) -> float:
    """Eliminate the leading 2^{-order * lambda} error term of theorem (error)."""
    r = 2.0 ** order
    return (r * v_fine - v_coarse) / (r - 1.0)


# ---------------------------------------------------------------------------
# Brute-force truncated signatures (definition (signature), Chen's identity)
# ---------------------------------------------------------------------------
def _tensor_exp(v: np.ndarray, N: int) -> list[np.ndarray]:
    """exp(v) in T^N(R^d): level k is v^{(x)k} / k!  (signature of a straight
    segment with increment v)."""
    levels = [np.ones(())]
    cur = np.ones(())
    for k in range(1, N + 1):
        cur = np.multiply.outer(cur, v) / k
        levels.append(cur)
    return levels


def _tensor_mul(a: list[np.ndarray], b: list[np.ndarray], N: int) -> list[np.ndarray]:
    """Product of eq. (tensor_product) truncated at level N:
    c_k = sum_i a_i (x) b_{k-i}."""
    out = []
    for k in range(N + 1):
        acc = None
        for i in range(k + 1):
            term = np.multiply.outer(a[i], b[k - i])
            acc = term if acc is None else acc + term
        out.append(acc)
    return out


def truncated_signature(path, N: int) -> list[np.ndarray]:
    """S^N of a piecewise-linear path: the ordered product of exp(increments)
    (Chen's identity for multiplicative functionals)."""
    path = _path(path)
    d = path.shape[1]
    sig = [np.ones(())] + [np.zeros((d,) * k) for k in range(1, N + 1)]
    for p in range(path.shape[0] - 1):
        sig = _tensor_mul(sig, _tensor_exp(path[p + 1] - path[p], N), N)
    return sig


def signature_kernel_truncated(x, y, N: int) -> float:
    """sum_{k<=N} <S^k(x), S^k(y)> with the inner product of Section 2
    (product of coordinate inner products on basis tensors)."""
    sx = truncated_signature(x, N)
    sy = truncated_signature(y, N)
    return float(sum(np.sum(a * b) for a, b in zip(sx, sy)))


def truncation_tail_bound(x, y, N: int) -> float:
    """Bound on the levels above N: by the factorial decay (eq.
    (factorial_decay), with the 1-variation of a piecewise-linear path) and
    Cauchy-Schwarz, |<S^k(x), S^k(y)>| <= (|x|_1 |y|_1)^k / (k!)^2."""
    x, y = _path(x), _path(y)
    lx = float(np.sum(np.linalg.norm(np.diff(x, axis=0), axis=1)))
    ly = float(np.sum(np.linalg.norm(np.diff(y, axis=0), axis=1)))
    r = lx * ly
    return sum(r ** k / math.factorial(k) ** 2 for k in range(N + 1, N + 60))


def local_error_bound_boundary_one(c: float) -> float:
    """Right-hand side of eq. (error_estimate_1) of theorem (local_error) for
    one cell with C3 * area = c and boundary data identically 1 (so the
    1-variation terms vanish): |c| * 2 / 2 * sup_{z in [0,c]} |I1(2 sqrt z)/sqrt z - 1|.
    I1(2 sqrt z) / sqrt z = sum_k z^k / (k! (k+1)!) (eq. (bessel_series), n=1)."""
    zs = np.linspace(0.0, c, 201)
    def f(z):
        return sum(z ** k / (math.factorial(k) * math.factorial(k + 1)) for k in range(40)) - 1.0
    sup = max(abs(f(float(z))) for z in zs)
    return abs(c) * sup


# ---------------------------------------------------------------------------
# Static-kernel lift (eq. (PDE_lifted) and the finite-difference form after it)
# ---------------------------------------------------------------------------
def rbf(sigma: float) -> dict:
    """The Gaussian static kernel exp(-|a - b|^2 / (2 sigma^2))."""
    assert sigma > 0
    return {"kind": "rbf", "sigma": float(sigma)}


LINEAR = {"kind": "linear"}


def static_kernel_matrix(x, y, kernel) -> np.ndarray:
    """kappa(x_i, y_j) over all node pairs, shape (lx, ly).  ``kernel`` is
    ``rbf(sigma)``, ``LINEAR``, or a callable (A [lx, d], B [ly, d]) -> matrix."""
    x, y = _path(x), _path(y)
    assert x.shape[1] == y.shape[1]
    if callable(kernel):
        return np.ascontiguousarray(np.asarray(kernel(x, y), dtype=np.float64))
    k = np.empty((x.shape[0], y.shape[0]), dtype=np.float64)
    if kernel["kind"] == "rbf":
        _load().sko_static_rbf(_dptr(x), x.shape[0], _dptr(y), y.shape[0], x.shape[1],
                               kernel["sigma"], _dptr(k))
    elif kernel["kind"] == "linear":
        _load().sko_static_linear(_dptr(x), x.shape[0], _dptr(y), y.shape[0], x.shape[1],
                                  _dptr(k))
    else:
        raise ValueError(kernel)
    return k


def lifted_coefficients(x, y, kernel) -> np.ndarray:
    """Coarse coefficients of the lifted scheme: the second difference of the
    static-kernel matrix over each cell, shape (lx - 1, ly - 1)."""
    k = static_kernel_matrix(x, y, kernel)
    lx, ly = k.shape
    c = np.zeros((max(lx - 1, 0), max(ly - 1, 0)), dtype=np.float64)
    if lx > 1 and ly > 1:
        _load().sko_lifted_coefficients(_dptr(k), lx, ly, _dptr(c))
    return c


def solve_coef(coef, dyadic_order: int = 0, scheme: str = "explicit", grid: bool = False):
    """Either scheme on P_lambda driven by a coarse coefficient matrix [m, n]."""
    coef = np.ascontiguousarray(np.asarray(coef, dtype=np.float64))
    m, n = coef.shape
    M, N = m << dyadic_order, n << dyadic_order
    g = np.empty((M + 1, N + 1), dtype=np.float64) if grid else None
    v = _load().sko_solve_coef(_dptr(coef) if coef.size else None, m, n, int(dyadic_order),
                               1 if scheme == "implicit" else 0, _dptr(g) if grid else None)
    return g if grid else float(v)


def solve_lifted(x, y, dyadic_order: int = 0, kernel=None, scheme: str = "explicit",
                 grid: bool = False):
    """The lifted signature kernel of one pair (default kernel: RBF, sigma 1)."""
    kernel = rbf(1.0) if kernel is None else kernel
    return solve_coef(lifted_coefficients(x, y, kernel), dyadic_order, scheme, grid)


def _lifted_rbf_batch(X, Y, dyadic_order, sigma, scheme, gram, nthreads):
    xf, xo, d = _pack(X)
    yf, yo, d2 = _pack(Y)
    assert d == d2 and sigma > 0
    nx, ny = len(xo) - 1, len(yo) - 1
    if not gram:
        assert nx == ny
    out = np.empty((nx, ny) if gram else (nx,), dtype=np.float64)
    _load().sko_lifted_rbf_batch(_dptr(xf), _iptr(xo), nx, _dptr(yf), _iptr(yo), ny, d,
                                 int(dyadic_order), float(sigma),
                                 1 if scheme == "implicit" else 0, 1 if gram else 0,
                                 _dptr(out), int(nthreads))
    return out


def lifted_rbf_pairs(xs, ys, dyadic_order: int = 0, sigma: float = 1.0,
                     scheme: str = "explicit", nthreads: int = 0) -> np.ndarray:
    """RBF-lifted kernels of independent pairs (OpenMP over pairs)."""
    return _lifted_rbf_batch(xs, ys, dyadic_order, sigma, scheme, False, nthreads)


def lifted_rbf_gram(X, Y, dyadic_order: int = 0, sigma: float = 1.0,
                    scheme: str = "explicit", nthreads: int = 0) -> np.ndarray:
    """RBF-lifted Gram matrix K[a, b] = k(X_a, Y_b) (OpenMP over pairs)."""
    return _lifted_rbf_batch(X, Y, dyadic_order, sigma, scheme, True, nthreads)
