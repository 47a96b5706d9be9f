"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same float32 inputs, at the same dyadic order.

Error metric (stated tolerance for the plain scheme at FP32 storage): a value
passes when |k_gpu - k_ref| / max(1, |k_ref|) <= tol.  The stated tolerance is
1e-5; the double-state sweep is held to 1e-6 here (its error is dominated by
the float32 increments and the float32 output rounding, about 1e-7).
"""
import os

import numpy as np
import pytest
import torch

import oracle
import paper_2006_14794_amd as sk
import workloads
from paper_2006_14794_amd import RaggedPaths

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
TOL = 1e-6


def mixed_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return np.abs(got - ref) / np.maximum(1.0, np.abs(ref))


def cuda(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32).cuda()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sk.load()


# ---------------------------------------------------------------------------
def test_straight_segment_hand_values_bitwise():
    from fractions import Fraction
    rows = []
    with open(os.path.join(GOLDEN, "straight_segment_hand_values.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(line.split())
    for c, lam, num, den in rows:
        c = float(Fraction(c))
        x = np.array([[[0.0, 0.0], [1.0, 0.0]]])
        y = np.array([[[0.0, 0.0], [c, 0.0]]])
        got = sk.sigkernel_pair(cuda(x), cuda(y), int(lam)).cpu().item()
        assert got == float(np.float32(int(num) / int(den))), (c, lam, got)


def test_single_pair_32_points_lambda0():
    x, y, xs, ys = workloads.single_pair()
    got = sk.sigkernel_pair(cuda(x[None]), cuda(y[None]), 0).cpu().numpy()
    ref = oracle.solve(x.astype(np.float64), y.astype(np.float64), 0)
    assert mixed_err(got[0], ref) <= 1e-5
    got = sk.sigkernel_pair(cuda(xs[None]), cuda(ys[None]), 0).cpu().numpy()
    ref = oracle.solve(xs.astype(np.float64), ys.astype(np.float64), 0)
    assert mixed_err(got[0], ref) <= 1e-5


@pytest.mark.parametrize("lam", [0, 1, 2, 3])
def test_gram_small_all_orders(lam):
    X, Y = workloads.gram_batch(seed=101, n_x=5, n_y=7, n_points=40, dim=3)
    got = sk.sigkernel_gram(cuda(X), cuda(Y), lam).cpu().numpy()
    ref = oracle.gram(X.astype(np.float64), Y.astype(np.float64), lam)
    assert mixed_err(got, ref).max() <= TOL


@pytest.mark.parametrize("d", [1, 2, 3, 5, 8, 9, 12, 13, 16])
def test_gram_every_padding_of_the_channel_dimension(d):
    X, Y = workloads.gram_batch(seed=200 + d, n_x=3, n_y=4, n_points=70, dim=d - 1)
    got = sk.sigkernel_gram(cuda(X), cuda(Y), 1).cpu().numpy()
    ref = oracle.gram(X.astype(np.float64), Y.astype(np.float64), 1)
    assert mixed_err(got, ref).max() <= TOL


def test_gram_several_tiles_and_ragged_tail():
    # x side: 64 lanes x R rows with a partial last lane; y side spans many steps
    X, Y = workloads.gram_batch(seed=303, n_x=3, n_y=3, n_points=150, dim=8)
    Y = Y[:, :97]
    got = sk.sigkernel_gram(cuda(X), cuda(Y), 1).cpu().numpy()
    ref = oracle.gram(X.astype(np.float64), Y.astype(np.float64), 1)
    assert mixed_err(got, ref).max() <= TOL


def test_row_capacity_limit_exactly_filled_and_exceeded():
    # M = 64 lanes x 32 rows exactly, then one coarse row more (a second band)
    for L in (1025, 1026):
        x = workloads.random_paths(7, 1, L, 4)
        y = workloads.random_paths(8, 1, L + 3, 4)
        got = sk.sigkernel_pair(cuda(x), cuda(y), 1).cpu().numpy()
        ref = oracle.solve(x[0].astype(np.float64), y[0].astype(np.float64), 1)
        assert mixed_err(got[0], ref) <= 1e-5


@pytest.mark.parametrize("lam", [0, 2])
def test_ragged_pairs_with_degenerate_lengths(lam):
    rng = np.random.default_rng(77)
    lens_x = [1, 2, 3, 17, 64, 65, 129, 5, 1, 200]
    lens_y = [4, 1, 2, 33, 63, 66, 2, 128, 1, 150]
    xs = [workloads.random_paths(1000 + i, 1, L, 6)[0] for i, L in enumerate(lens_x)]
    ys = [workloads.random_paths(2000 + i, 1, L, 6)[0] for i, L in enumerate(lens_y)]
    X = RaggedPaths.from_list(xs, "cuda")
    Y = RaggedPaths.from_list(ys, "cuda")
    got = sk.sigkernel_pair(X, Y, lam).cpu().numpy()
    ref = oracle.pairs([a.astype(np.float64) for a in xs], [b.astype(np.float64) for b in ys], lam)
    assert mixed_err(got, ref).max() <= TOL
    assert got[0] == 1.0 and got[1] == 1.0 and got[8] == 1.0
    # ragged Gram of the same batches
    G = sk.sigkernel_gram(X, Y, lam).cpu().numpy()
    Gref = oracle.gram([a.astype(np.float64) for a in xs], [b.astype(np.float64) for b in ys], lam)
    assert mixed_err(G, Gref).max() <= TOL


def test_ragged_contract_violation_gives_nan_for_that_pair_only():
    xs = [workloads.random_paths(1, 1, L, 3)[0] for L in (10, 30, 12)]
    ys = [workloads.random_paths(2, 1, L, 3)[0] for L in (11, 9, 13)]
    X = RaggedPaths.from_list(xs, "cuda")
    X.max_len = 20  # path 1 has 30 points: breaks the declared bound
    Y = RaggedPaths.from_list(ys, "cuda")
    got = sk.sigkernel_pair(X, Y, 1).cpu().numpy()
    assert np.isnan(got[1])
    ref = oracle.pairs([a.astype(np.float64) for a in xs], [b.astype(np.float64) for b in ys], 1)
    assert mixed_err(got[[0, 2]], ref[[0, 2]]).max() <= TOL


def test_ragged_offsets_beyond_the_points_buffer_give_nan():
    # The points buffer holds offsets[n] rows.  Path 1 below ends at row 22 of a
    # 20-row buffer (its length, 12, is within the declared bound and its end
    # within n * len): it must get NaN, not a read past the buffer; path 2 runs
    # backwards (NaN); path 0 is well formed.  Offsets that do not start at 0
    # break the contract for every path.
    pts = workloads.random_paths(31, 1, 20, 3)[0]
    X = RaggedPaths(cuda(pts), torch.tensor([0, 10, 22, 20], dtype=torch.int64,
                                            device="cuda"), 12)
    ys = [workloads.random_paths(32 + i, 1, L, 3)[0] for i, L in enumerate((9, 8, 7))]
    Y = RaggedPaths.from_list(ys, "cuda")
    got = sk.sigkernel_pair(X, Y, 1).cpu().numpy()
    assert np.isnan(got[1]) and np.isnan(got[2])
    ref = oracle.solve(pts[:10].astype(np.float64), ys[0].astype(np.float64), 1)
    assert mixed_err(got[0], ref) <= TOL
    X0 = RaggedPaths(cuda(workloads.random_paths(33, 1, 31, 3)[0]),
                     torch.tensor([1, 11, 21, 31], dtype=torch.int64, device="cuda"), 12)
    assert np.all(np.isnan(sk.sigkernel_pair(X0, Y, 1).cpu().numpy()))


def test_symmetric_gram_and_no_diag():
    X, _ = workloads.gram_batch(seed=404, n_x=6, n_y=1, n_points=50, dim=4)
    full = sk.sigkernel_gram(cuda(X), cuda(X), 1).cpu().numpy()
    Xt = cuda(X)
    sym = sk.sigkernel_gram(Xt, None, 1, symmetric=True).cpu().numpy()
    assert np.array_equal(sym, sym.T)
    assert mixed_err(sym, full).max() <= 1e-6
    nd = sk.sigkernel_gram(Xt, None, 1, symmetric=True, no_diag=True).cpu().numpy()
    assert np.all(np.diag(nd) == 0.0)
    off = ~np.eye(6, dtype=bool)
    assert np.array_equal(nd[off], sym[off])


@pytest.mark.parametrize("d", [3, 20])
def test_symmetric_no_diag_covers_pairs_without_cells(d):
    """One-point paths have nothing to sweep (value 1): without the diagonal
    their diagonal entries are 0 too, in uniform and ragged batches (d = 20
    runs the coefficient sweep)."""
    one = torch.ones((4, 1, d), device="cuda")
    nd = sk.sigkernel_gram(one, None, 1, symmetric=True, no_diag=True).cpu().numpy()
    assert np.array_equal(nd, 1.0 - np.eye(4, dtype=np.float32))
    lens = [1, 30, 1, 45, 2]
    xs = [workloads.random_paths(606 + i, 1, L, d)[0] for i, L in enumerate(lens)]
    X = RaggedPaths.from_list(xs, "cuda")
    nd = sk.sigkernel_gram(X, None, 1, symmetric=True, no_diag=True).cpu().numpy()
    ref = oracle.gram([x.astype(np.float64) for x in xs], [x.astype(np.float64) for x in xs], 1)
    np.fill_diagonal(ref, 0.0)
    assert np.all(np.diag(nd) == 0.0)
    # the float32 inner products' rounding grows with the channels
    assert mixed_err(nd, ref).max() <= TOL * max(1.0, np.sqrt(d / 16))


def test_nan_propagates_to_its_own_pairs_only():
    X, Y = workloads.gram_batch(seed=505, n_x=4, n_y=3, n_points=30, dim=2)
    clean = sk.sigkernel_gram(cuda(X), cuda(Y), 1).cpu().numpy()
    Xn = X.copy()
    Xn[2, 7, 1] = np.nan
    dirty = sk.sigkernel_gram(cuda(Xn), cuda(Y), 1).cpu().numpy()
    assert np.all(np.isnan(dirty[2]))
    keep = [0, 1, 3]
    assert np.array_equal(dirty[keep], clean[keep])


def test_empty_and_single_point_batches():
    X = torch.zeros((0, 5, 3), device="cuda")
    Y = torch.zeros((2, 5, 3), device="cuda")
    assert sk.sigkernel_gram(X, Y, 1).shape == (0, 2)
    one = torch.ones((3, 1, 3), device="cuda")
    G = sk.sigkernel_gram(one, Y + torch.arange(5, device="cuda")[None, :, None] * 0.1, 2)
    assert torch.all(G == 1.0)


@pytest.mark.parametrize("run", [1, 2, 3, 5, 7, 64])
def test_gram_streamed_runs_with_tail(run, monkeypatch):
    # several y paths streamed through one wave, including a partial last run
    monkeypatch.setenv("SIGKERNEL_GRAM_RUN", str(run))
    X, Y = workloads.gram_batch(seed=707, n_x=3, n_y=7, n_points=45, dim=5)
    got = sk.sigkernel_gram(cuda(X), cuda(Y), 1).cpu().numpy()
    ref = oracle.gram(X.astype(np.float64), Y.astype(np.float64), 1)
    assert mixed_err(got, ref).max() <= TOL
    sym = sk.sigkernel_gram(cuda(X), None, 2, symmetric=True, no_diag=True).cpu().numpy()
    refs = oracle.gram(X.astype(np.float64), X.astype(np.float64), 2)
    np.fill_diagonal(refs, 0.0)
    assert mixed_err(sym, refs).max() <= TOL
    assert np.all(np.diag(sym) == 0.0)


def test_repeated_calls_are_deterministic():
    X, Y = workloads.gram_batch(seed=606, n_x=8, n_y=8, n_points=64, dim=8)
    a = sk.sigkernel_gram(cuda(X), cuda(Y), 1)
    b = sk.sigkernel_gram(cuda(X), cuda(Y), 1)
    assert torch.equal(a, b)


# ---------------------------------------------------------------------------
# Full-size workload (128 x 128 Gram, 256 points, d = 8 + time, lambda = 1)
# in the launch configuration the benchmark times; sampled entries against
# the oracle (each oracle pair is 510 x 510 fine cells).
# ---------------------------------------------------------------------------
def test_full_size_gram_sampled():
    tol = 1e-5
    X, Y = workloads.gram_batch()
    got = sk.sigkernel_gram(cuda(X), cuda(Y), 1).cpu().numpy()
    assert np.all(np.isfinite(got))
    rng = np.random.default_rng(0)
    idx = rng.choice(128 * 128, size=48, replace=False)
    xs = [X[i // 128].astype(np.float64) for i in idx]
    ys = [Y[i % 128].astype(np.float64) for i in idx]
    ref = oracle.pairs(xs, ys, 1)
    err = mixed_err(got.reshape(-1)[idx], ref)
    assert err.max() <= tol, err.max()
