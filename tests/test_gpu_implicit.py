"""The implicit scheme (remark after eq. explicit_finite_diff) on the GPU
against the FP64 oracle's implicit solve: independent pairs (uniform and
ragged), Gram batches streamed in runs, symmetric Grams, and the banded pair
kernel for tall grids."""
import numpy as np
import pytest
import torch

import oracle
import paper_2006_14794_amd as sk
import workloads
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


def mixed_err(got, ref):
    return np.abs(np.asarray(got, np.float64) - ref) / np.maximum(1.0, np.abs(ref))


def test_straight_segments_closed_form():
    # one cell at order 0: (1 + 3c/4) / (1 - c/4) with c = <a, b>
    cs = np.array([1.0, -1.0, 2.0, 0.5, -2.0], np.float32)
    X = np.zeros((5, 2, 2), np.float32)
    Y = np.zeros((5, 2, 2), np.float32)
    X[:, 1, 0] = cs
    Y[:, 1, 0] = 1.0
    got = sk.sigkernel_pair(cuda(X), cuda(Y), 0, scheme="implicit").cpu().numpy()
    ref = (1 + 0.75 * cs.astype(np.float64)) / (1 - 0.25 * cs.astype(np.float64))
    assert mixed_err(got, ref).max() <= 1e-7


@pytest.mark.parametrize("lam,L,d", [(0, 64, 2), (1, 129, 5), (2, 100, 9), (3, 40, 16)])
def test_uniform_pairs(lam, L, d):
    X = workloads.random_paths(40 + lam, 21, L, d)
    Y = workloads.random_paths(50 + lam, 21, L - 7, d)
    got = sk.sigkernel_pair(cuda(X), cuda(Y), lam, scheme="implicit").cpu().numpy()
    ref = oracle.pairs_implicit(X.astype(np.float64), Y.astype(np.float64), lam)
    assert mixed_err(got, ref).max() <= TOL
    # and it differs from the explicit scheme by the scheme's own error
    expl = sk.sigkernel_pair(cuda(X), cuda(Y), lam).cpu().numpy()
    assert np.abs(expl - got).max() > 0


def test_ragged_pairs_and_gram():
    lens = workloads.ragged_lengths(61, 30, 1, 300)
    xs = [workloads.random_paths(600 + i, 1, int(n), 4)[0] for i, n in enumerate(lens)]
    ys = [workloads.random_paths(700 + i, 1, int(n), 4)[0] for i, n in enumerate(lens[::-1])]
    X, Y = RaggedPaths.from_list(xs, "cuda"), RaggedPaths.from_list(ys, "cuda")
    xd = [a.astype(np.float64) for a in xs]
    yd = [b.astype(np.float64) for b in ys]
    got = sk.sigkernel_pair(X, Y, 2, scheme="implicit").cpu().numpy()
    assert mixed_err(got, oracle.pairs_implicit(xd, yd, 2)).max() <= TOL
    G = sk.sigkernel_gram(X, Y, 1, scheme="implicit").cpu().numpy()
    ref = np.array([[oracle.solve_implicit(a, b, 1) for b in yd] for a in xd])
    assert mixed_err(G, ref).max() <= TOL


@pytest.mark.parametrize("symmetric", [False, True])
def test_gram_runs_and_symmetric(symmetric):
    X = workloads.random_paths(81, 17, 90, 6)
    Y = X if symmetric else workloads.random_paths(82, 23, 75, 6)
    K = sk.sigkernel_gram(cuda(X), None if symmetric else cuda(Y), 1, symmetric=symmetric,
                          no_diag=symmetric, scheme="implicit").cpu().numpy()
    ref = np.array([[oracle.solve_implicit(a, b, 1) for b in Y.astype(np.float64)]
                    for a in X.astype(np.float64)])
    if symmetric:
        np.fill_diagonal(ref, 0.0)
    assert mixed_err(K, ref).max() <= TOL


def test_tall_paths_through_row_bands():
    X = workloads.random_paths(91, 2, 2100, 3)
    Y = workloads.random_paths(92, 3, 40, 3)
    K = sk.sigkernel_gram(cuda(X), cuda(Y), 0, scheme="implicit").cpu().numpy()
    ref = np.array([[oracle.solve_implicit(a, b, 0) for b in Y.astype(np.float64)]
                    for a in X.astype(np.float64)])
    assert mixed_err(K, ref).max() <= TOL
