"""Unbiased signature-kernel MMD^2 (value and gradient in X) on the GPU against
the FP64 oracle, and -- at the full size of the MMD workload (64 random walks
of 512 points in R^4 vs 64 Ornstein-Uhlenbeck targets, dyadic order 1) --
against central finite differences (h = 1e-4, FP64) of the oracle's MMD^2 on
sampled coordinates."""
import numpy as np
import pytest
import torch

import oracle
import paper_2006_14794_amd as sk
import workloads
from conftest import grad_close
from paper_2006_14794_amd import RaggedPaths

pytestmark = pytest.mark.gpu


def cuda(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32).cuda()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sk.load()


def oracle_mmd2(X, Y, lam):
    X = X.astype(np.float64)
    Y = Y.astype(np.float64)
    Kxx, Kyy, Kxy = oracle.gram(X, X, lam), oracle.gram(Y, Y, lam), oracle.gram(X, Y, lam)
    return oracle.mmd2_unbiased(Kxx, Kyy, Kxy)


@pytest.mark.parametrize("lam", [0, 1, 2])
def test_mmd2_value_and_gradient_small(lam):
    X = workloads.random_paths(11, 5, 20, 3)
    Y = workloads.random_paths(12, 4, 17, 3)
    val, dX = sk.sigkernel_mmd2(cuda(X), cuda(Y), lam, grad=True)
    ref = oracle_mmd2(X, Y, lam)
    assert abs(val.item() - ref) <= 1e-6 * max(1.0, abs(ref)) + 1e-7
    n, m = 5, 4
    wxx, _, wxy = oracle.mmd2_weights(n, m)
    gxx, gxx2 = oracle.gram_backward(X.astype(np.float64), X.astype(np.float64), wxx, lam)
    gxy, _ = oracle.gram_backward(X.astype(np.float64), Y.astype(np.float64), wxy, lam)
    rx = gxx + gxx2 + gxy
    grad_close(dX.cpu().numpy(), rx, f"MMD dX lam{lam}")


@pytest.mark.parametrize("lam", [1, 2])
def test_mmd2_ragged_value_and_gradient(lam):
    # uneven lengths with a one-point path on each side; dX is [total, d]
    lx, ly = [12, 1, 30, 7, 19], [9, 22, 1, 14]
    xs = [workloads.random_paths(70 + i, 1, L, 3)[0] for i, L in enumerate(lx)]
    ys = [workloads.random_paths(80 + i, 1, L, 3)[0] for i, L in enumerate(ly)]
    X, Y = RaggedPaths.from_list(xs, "cuda"), RaggedPaths.from_list(ys, "cuda")
    val, dX = sk.sigkernel_mmd2(X, Y, lam, grad=True)
    val_only, _ = sk.sigkernel_mmd2(X, Y, lam)
    xd = [x.astype(np.float64) for x in xs]
    yd = [y.astype(np.float64) for y in ys]
    Kxx, Kyy, Kxy = oracle.gram(xd, xd, lam), oracle.gram(yd, yd, lam), oracle.gram(xd, yd, lam)
    ref = oracle.mmd2_unbiased(Kxx, Kyy, Kxy)
    assert abs(val.item() - ref) <= 1e-6 * max(1.0, abs(ref)) + 1e-7
    assert val.item() == val_only.item()
    wxx, _, wxy = oracle.mmd2_weights(len(xs), len(ys))
    g1, g2 = oracle.gram_backward(xd, xd, wxx, lam)
    g3, _ = oracle.gram_backward(xd, yd, wxy, lam)
    assert dX.shape == (sum(lx), 3)
    grad_close(dX.cpu().numpy(), g1 + g2 + g3, f"MMD ragged dX lam{lam}")


def test_mmd2_autograd_and_value_only_path():
    X = workloads.random_paths(13, 6, 12, 2)
    Y = workloads.random_paths(14, 6, 12, 2)
    Xt = cuda(X).requires_grad_(True)
    loss = sk.mmd2(Xt, cuda(Y), 1)
    (3.0 * loss).backward()
    _, dX = sk.sigkernel_mmd2(cuda(X), cuda(Y), 1, grad=True)
    assert torch.allclose(Xt.grad, 3.0 * dX)
    val, none = sk.sigkernel_mmd2(cuda(X), cuda(Y), 1)
    assert none is None and abs(val.item() - loss.item()) == 0.0


def test_mmd2_full_size_value_and_fd_gradient():
    X, Y = workloads.mmd_paths()
    val, dX = sk.sigkernel_mmd2(cuda(X), cuda(Y), 1, grad=True)
    Xd, Yd = X.astype(np.float64), Y.astype(np.float64)
    n, m = X.shape[0], Y.shape[0]
    # value: the full oracle estimator
    ref = oracle_mmd2(X, Y, 1)
    assert abs(val.item() - ref) <= 1e-5 * max(1.0, abs(ref)) + 1e-6
    # gradient on sampled coordinates: only path a's Gram row moves, so the
    # oracle solves 2 x (n - 1 + m) pairs per difference
    rng = np.random.default_rng(0)
    gpu = dX.cpu().numpy()
    h = 1e-4  # central differences in FP64: truncation ~1e-8 relative here
    worst = 0.0
    for _ in range(8):
        a, i, c = int(rng.integers(n)), int(rng.integers(1, 512)), int(rng.integers(4))
        others = [b for b in range(n) if b != a]

        def row_terms(xa):
            kxx = oracle.pairs([xa] * len(others), [Xd[b] for b in others], 1)
            kxy = oracle.pairs([xa] * m, [Yd[b] for b in range(m)], 1)
            return 2.0 * kxx.sum() / (n * (n - 1)) - 2.0 * kxy.sum() / (n * m)

        xp = Xd[a].copy()
        xp[i, c] += h
        xm = Xd[a].copy()
        xm[i, c] -= h
        fd = (row_terms(xp) - row_terms(xm)) / (2 * h)
        err = abs(gpu[a, i, c] - fd) / np.abs(gpu).max()
        worst = max(worst, err)
        assert err <= 1e-5, (a, i, c, err)
    print(f"GRADERR MMD full-size FD abs {worst:.3e}")


@pytest.mark.parametrize("lam,L", [(0, 30), (2, 25), (4, 9), (1, 1)])
def test_mmd2_value_same_with_and_without_gradient(lam, L):
    """With the gradient, Kxx and Kxy come from the gradient launches' forward
    passes (paths of at least two points) instead of separate Gram calls: the
    same cells in the same order, so the value is bitwise the same."""
    X = workloads.random_paths(15 + lam, 7, L, 3)
    Y = workloads.random_paths(16 + lam, 5, L + (L > 1), 3)
    val_g, dX = sk.sigkernel_mmd2(cuda(X), cuda(Y), lam, grad=True)
    val, _ = sk.sigkernel_mmd2(cuda(X), cuda(Y), lam)
    assert val_g.item() == val.item()
    if L == 1:
        assert val.item() == 0.0 and not dX.abs().any()
    else:
        assert abs(val.item() - oracle_mmd2(X, Y, lam)) <= 1e-6
