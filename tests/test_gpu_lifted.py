"""The RBF-lifted signature kernel (static-kernel lift of eq. (PDE_lifted),
Gaussian static kernel) on the GPU against the FP64 oracle.  The coefficient,
the static kernel and the sweep are all double on both sides; only the float32
output rounding separates them, hence the tight bound."""
import numpy as np
import pytest
import torch

import oracle
import paper_2006_14794_amd as sk
import workloads
from paper_2006_14794_amd import RaggedPaths

pytestmark = pytest.mark.gpu
TOL = 2e-7


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


@pytest.mark.parametrize("lam,L,d,sigma", [(0, 64, 2, 0.3), (1, 129, 5, 1.0), (2, 100, 9, 0.5),
                                           (3, 40, 16, 2.0), (1, 33, 3, 0.05), (0, 200, 4, 20.0)])
def test_pairs(lam, L, d, sigma):
    X = workloads.random_paths(140 + lam, 19, L, d, std=1.0)
    Y = workloads.random_paths(150 + lam, 19, L - 5, d, std=1.0)
    got = sk.sigkernel_pair_lifted(cuda(X), cuda(Y), lam, sigma=sigma).cpu().numpy()
    ref = oracle.lifted_rbf_pairs(f64(X), f64(Y), lam, sigma)
    assert mixed_err(got, ref).max() <= TOL


def test_implicit_scheme():
    X = workloads.random_paths(160, 13, 70, 3, std=1.0)
    Y = workloads.random_paths(161, 13, 90, 3, std=1.0)
    got = sk.sigkernel_pair_lifted(cuda(X), cuda(Y), 2, sigma=0.7, scheme="implicit")
    ref = oracle.lifted_rbf_pairs(f64(X), f64(Y), 2, 0.7, "implicit")
    assert mixed_err(got.cpu().numpy(), ref).max() <= TOL
    G = sk.sigkernel_gram_lifted(cuda(X[:5]), cuda(Y[:7]), 1, sigma=0.7, scheme="implicit")
    Gref = oracle.lifted_rbf_gram(f64(X[:5]), f64(Y[:7]), 1, 0.7, "implicit")
    assert mixed_err(G.cpu().numpy(), Gref).max() <= TOL


def test_gram_with_runs_of_pairs():
    # 64 x 1024 pairs: several pairs streamed back to back through each wave
    X = workloads.random_paths(170, 64, 12, 3, std=1.0)
    Y = workloads.random_paths(171, 1024, 12, 3, std=1.0)
    K = sk.sigkernel_gram_lifted(cuda(X), cuda(Y), 1, sigma=0.8).cpu().numpy()
    ref = oracle.lifted_rbf_gram(f64(X), f64(Y), 1, 0.8)
    assert mixed_err(K, ref).max() <= TOL


def test_symmetric_gram_and_no_diag():
    X = workloads.random_paths(180, 9, 50, 4, std=1.0)
    Xt = cuda(X)
    full = sk.sigkernel_gram_lifted(Xt, Xt, 1, sigma=0.6).cpu().numpy()
    assert mixed_err(full, oracle.lifted_rbf_gram(f64(X), f64(X), 1, 0.6)).max() <= TOL
    sym = sk.sigkernel_gram_lifted(Xt, None, 1, sigma=0.6, symmetric=True).cpu().numpy()
    assert np.array_equal(sym, sym.T)
    assert mixed_err(sym, full).max() <= TOL
    nd = sk.sigkernel_gram_lifted(Xt, None, 1, sigma=0.6, symmetric=True,
                                  no_diag=True).cpu().numpy()
    assert np.all(np.diag(nd) == 0.0)
    off = ~np.eye(9, dtype=bool)
    assert np.array_equal(nd[off], sym[off])


def test_ragged_batches():
    lens_x = [1, 2, 17, 60, 33, 5, 128]
    lens_y = [40, 1, 9, 61, 2, 90, 30]
    xs = [workloads.random_paths(190 + i, 1, L, 3, std=1.0)[0] for i, L in enumerate(lens_x)]
    ys = [workloads.random_paths(200 + i, 1, L, 3, std=1.0)[0] for i, L in enumerate(lens_y)]
    X, Y = RaggedPaths.from_list(xs, "cuda"), RaggedPaths.from_list(ys, "cuda")
    got = sk.sigkernel_pair_lifted(X, Y, 2, sigma=0.4).cpu().numpy()
    ref = oracle.lifted_rbf_pairs([f64(a) for a in xs], [f64(b) for b in ys], 2, 0.4)
    assert mixed_err(got, ref).max() <= TOL
    assert got[0] == 1.0 and got[1] == 1.0
    G = sk.sigkernel_gram_lifted(X, Y, 1, sigma=0.4).cpu().numpy()
    Gref = oracle.lifted_rbf_gram([f64(a) for a in xs], [f64(b) for b in ys], 1, 0.4)
    assert mixed_err(G, Gref).max() <= TOL


def test_ragged_contract_violation_gives_nan_for_that_pair_only():
    xs = [workloads.random_paths(210, 1, L, 2)[0] for L in (10, 30, 12)]
    ys = [workloads.random_paths(211, 1, L, 2)[0] for L in (11, 9, 13)]
    X = RaggedPaths.from_list(xs, "cuda")
    X.max_len = 20
    Y = RaggedPaths.from_list(ys, "cuda")
    got = sk.sigkernel_pair_lifted(X, Y, 1, sigma=0.5).cpu().numpy()
    assert np.isnan(got[1])
    ref = oracle.lifted_rbf_pairs([f64(a) for a in xs], [f64(b) for b in ys], 1, 0.5)
    assert mixed_err(got[[0, 2]], ref[[0, 2]]).max() <= TOL


def test_tallest_compiled_x_path():
    # 2048 fine rows: 32 rows per lane at order 0 with two channels
    X = workloads.random_paths(220, 2, 2049, 2, std=1.0)
    Y = workloads.random_paths(221, 3, 25, 2, std=1.0)
    K = sk.sigkernel_gram_lifted(cuda(X), cuda(Y), 0, sigma=0.3).cpu().numpy()
    assert mixed_err(K, oracle.lifted_rbf_gram(f64(X), f64(Y), 0, 0.3)).max() <= TOL
    with pytest.raises(sk.SigKernelError):
        sk.sigkernel_gram_lifted(cuda(X), cuda(Y), 1, sigma=0.3)


@pytest.mark.parametrize("L", [200, 256, 257])
def test_top_lane_node_when_the_grid_fills_the_wave(L):
    # a lane takes its top node's kernel value from the lane above; lane 0
    # evaluates it itself only when the x grid fills the wave exactly (257
    # points at order 1: 512 fine rows, 8 per lane), else it reuses its own
    # node 1 (both are x_0 above the grid)
    X = workloads.random_paths(240 + L, 2, L, 4)
    Y = workloads.random_paths(250 + L, 3, 90, 4)
    K = sk.sigkernel_gram_lifted(cuda(X), cuda(Y), 1, sigma=0.7).cpu().numpy()
    assert mixed_err(K, oracle.lifted_rbf_gram(f64(X), f64(Y), 1, 0.7)).max() <= TOL


def test_linear_static_kernel_is_the_plain_call():
    X = workloads.random_paths(230, 6, 40, 3)
    Y = workloads.random_paths(231, 5, 30, 3)
    a = sk.sigkernel_gram_lifted(cuda(X), cuda(Y), 1, kernel="linear").cpu().numpy()
    b = sk.sigkernel_gram(cuda(X), cuda(Y), 1).cpu().numpy()
    assert np.array_equal(a, b)


def test_headline_shape_sampled():
    # the Gram batch shape (128 x 128 pairs, 256 points, 8 channels + time,
    # order 1): sampled pairs against the oracle
    X, Y = workloads.gram_batch()
    K = sk.sigkernel_gram_lifted(cuda(X), cuda(Y), 1, sigma=0.5).cpu().numpy()
    rng = np.random.default_rng(7)
    idx = rng.choice(128 * 128, size=48, replace=False)
    xs = [f64(X[i // 128]) for i in idx]
    ys = [f64(Y[i % 128]) for i in idx]
    ref = oracle.lifted_rbf_pairs(xs, ys, 1, 0.5)
    assert mixed_err(K.reshape(-1)[idx], ref).max() <= TOL
    assert np.all(np.isfinite(K))


@pytest.mark.parametrize("n", [70, 180])
def test_symmetric_runs_equal_the_full_gram(n):
    # default run lengths of the upper-triangle launch at sizes where they
    # exceed one pair per run: bitwise the full launch's values
    X = cuda(workloads.random_paths(1200 + n, n, 20, 3, std=1.0))
    full = sk.sigkernel_gram_lifted(X, X, 1, sigma=0.6)
    sym = sk.sigkernel_gram_lifted(X, None, 1, sigma=0.6, symmetric=True)
    iu = torch.triu_indices(n, n, device=X.device)
    assert torch.equal(sym[iu[0], iu[1]], full[iu[0], iu[1]])
    assert torch.equal(sym, sym.T)
