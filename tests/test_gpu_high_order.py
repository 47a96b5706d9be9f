"""Dyadic orders beyond the compiled sweeps (lambda > 3): the batch is split
into 2^(lambda - 3) equal sub-increments per segment and swept at order 3,
which gives exactly the fine cells and coefficients of P_lambda (definition
(fintite_diff) and the remark after eq. (explicit_finite_diff)).  Checked
against the FP64 oracle on P_lambda itself: pairs, Gram runs, tall grids
through row bands, ragged batches, symmetric Grams, the implicit scheme, the
Gram backward and the MMD with its gradient."""
import numpy as np
import pytest
import torch

import oracle
import paper_2006_14794_amd as sk
import workloads
from conftest import grad_close
from paper_2006_14794_amd import RaggedPaths

pytestmark = pytest.mark.gpu
TOL = 1e-6


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sk.load()


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def f64(a):
    return np.asarray(a, dtype=np.float64)


def mixed_err(got, ref):
    return np.abs(np.asarray(got, np.float64) - ref) / np.maximum(1.0, np.abs(ref))


@pytest.mark.parametrize("lam,L,d", [(4, 12, 2), (5, 12, 3), (6, 6, 4), (7, 4, 9)])
def test_pairs(lam, L, d):
    # unit-scale paths: the float32 increment inner products (relative error
    # about d 2^-24 per coarse cell) keep the kernel within the bound
    X = workloads.random_paths(300 + lam, 9, L, d, std=1.0)
    Y = workloads.random_paths(310 + lam, 9, L + 3, d, std=1.0)
    got = sk.sigkernel_pair(cuda(X), cuda(Y), lam).cpu().numpy()
    assert mixed_err(got, oracle.pairs(f64(X), f64(Y), lam)).max() <= TOL


def test_gram_runs_and_tall_bands():
    # one-wave Gram at order 4 with several pairs per wave
    # 33600 pairs: the default path scale, as in the plain parity tests (the
    # float32-coefficient tail grows with the number of pairs and their scale)
    X = workloads.random_paths(320, 48, 9, 3)
    Y = workloads.random_paths(321, 700, 9, 3)
    K = sk.sigkernel_gram(cuda(X), cuda(Y), 4).cpu().numpy()
    assert mixed_err(K, oracle.gram(f64(X), f64(Y), 4)).max() <= TOL
    # 39 * 2^6 = 2496 fine rows: beyond one wave, through the persistent pair kernel
    Xt = workloads.random_paths(322, 2, 40, 2, std=1.0)
    Yt = workloads.random_paths(323, 3, 10, 2, std=1.0)
    Kt = sk.sigkernel_gram(cuda(Xt), cuda(Yt), 6).cpu().numpy()
    assert mixed_err(Kt, oracle.gram(f64(Xt), f64(Yt), 6)).max() <= TOL


def fp32_increment_gram(x, y):
    """The coarse coefficients as the GPU forms them: float32 increments and
    float32 FMA inner products over the channels in order (the product of two
    floats is exact in double; the sum is rounded once to float)."""
    dx = (np.asarray(x[1:], np.float32) - np.asarray(x[:-1], np.float32)).astype(np.float64)
    dy = (np.asarray(y[1:], np.float32) - np.asarray(y[:-1], np.float32)).astype(np.float64)
    G = np.zeros((len(dx), len(dy)), np.float32)
    for k in range(dx.shape[1]):
        G = (np.multiply.outer(dx[:, k], dy[:, k]) + G.astype(np.float64)).astype(np.float32)
    return G.astype(np.float64)


@pytest.mark.parametrize("lam", [4, 6])
def test_refinement_is_exact_given_the_float32_coefficients(lam):
    # with the coefficients rounded as on the GPU, the oracle's double sweep on
    # P_lambda reproduces the refined GPU sweep to the float32 output rounding:
    # the split into sub-increments adds no error of its own
    X = workloads.random_paths(370 + lam, 6, 10, 3, std=1.5)
    Y = workloads.random_paths(380 + lam, 6, 8, 3, std=1.5)
    got = sk.sigkernel_pair(cuda(X), cuda(Y), lam).cpu().numpy()
    ref = np.array([oracle.solve_coef(fp32_increment_gram(X[i], Y[i]), lam) for i in range(6)])
    assert mixed_err(got, ref).max() <= 2e-7


def test_ragged_and_degenerate_paths():
    lens_x = [1, 2, 13, 7, 30]
    lens_y = [9, 17, 1, 2, 11]
    xs = [workloads.random_paths(330 + i, 1, L, 2, std=1.0)[0] for i, L in enumerate(lens_x)]
    ys = [workloads.random_paths(340 + i, 1, L, 2, std=1.0)[0] for i, L in enumerate(lens_y)]
    X, Y = RaggedPaths.from_list(xs, "cuda"), RaggedPaths.from_list(ys, "cuda")
    got = sk.sigkernel_pair(X, Y, 5).cpu().numpy()
    ref = oracle.pairs([f64(a) for a in xs], [f64(b) for b in ys], 5)
    assert mixed_err(got, ref).max() <= TOL
    assert got[0] == 1.0 and got[2] == 1.0
    G = sk.sigkernel_gram(X, Y, 4).cpu().numpy()
    assert mixed_err(G, oracle.gram([f64(a) for a in xs], [f64(b) for b in ys], 4)).max() <= TOL
    # a path breaking the declared length bound: NaN for its pairs only
    X.max_len = 20
    bad = sk.sigkernel_pair(X, Y, 4).cpu().numpy()
    assert np.isnan(bad[4]) and np.all(np.isfinite(bad[:4]))


def test_symmetric_gram_and_implicit_scheme():
    X = workloads.random_paths(350, 7, 15, 3)
    Xt = cuda(X)
    full = oracle.gram(f64(X), f64(X), 4)
    sym = sk.sigkernel_gram(Xt, None, 4, symmetric=True, no_diag=True).cpu().numpy()
    np.fill_diagonal(full, 0.0)
    assert mixed_err(sym, full).max() <= TOL
    imp = sk.sigkernel_pair(Xt, Xt.flip(0).contiguous(), 5, scheme="implicit").cpu().numpy()
    ref = oracle.pairs_implicit(f64(X), f64(X[::-1]), 5)
    assert mixed_err(imp, ref).max() <= TOL


def test_gram_backward_and_mmd():
    X = workloads.random_paths(360, 3, 12, 3, std=1.0)
    Y = workloads.random_paths(361, 4, 10, 3, std=1.0)
    dK = np.random.default_rng(5).normal(size=(3, 4)).astype(np.float32)
    gx, gy = sk.sigkernel_gram_backward(cuda(X), cuda(Y), cuda(dK), 4)
    rx, ry = oracle.gram_backward(f64(X), f64(Y), dK.astype(np.float64), 4)
    grad_close(gx.cpu().numpy(), rx, "dX order 4")
    grad_close(gy.cpu().numpy(), ry, "dY order 4")
    A = workloads.random_paths(362, 5, 14, 2)
    B = workloads.random_paths(363, 4, 11, 2)
    val, dA = sk.sigkernel_mmd2(cuda(A), cuda(B), 4, grad=True)
    Ad, Bd = f64(A), f64(B)
    ref = oracle.mmd2_unbiased(oracle.gram(Ad, Ad, 4), oracle.gram(Bd, Bd, 4),
                               oracle.gram(Ad, Bd, 4))
    assert abs(val.item() - ref) <= 1e-6 * max(1.0, abs(ref)) + 1e-7
    wxx, _, wxy = oracle.mmd2_weights(5, 4)
    g1, g2 = oracle.gram_backward(Ad, Ad, wxx, 4)
    g3, _ = oracle.gram_backward(Ad, Bd, wxy, 4)
    rx = g1 + g2 + g3
    grad_close(dA.cpu().numpy(), rx, "MMD dX order 4")
