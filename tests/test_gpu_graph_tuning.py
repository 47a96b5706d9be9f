"""Batching row: hipGraph replay of whole library calls and launch tuning.

Graph replays are checked against eager calls on the same inputs after each
replay (with eager work and synchronisation between replays, and the inputs
rewritten in place so that every replay must re-read them); tunings are
checked to leave forward outputs bit-identical, and one replay and one tuned
result against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2006_14794_amd as sk
import workloads
from paper_2006_14794_amd import RaggedPaths, _lib

pytestmark = pytest.mark.gpu
TOL = 1e-6


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sk.load()


@pytest.fixture(autouse=True)
def _clean_table():
    sk.tune_clear()
    yield
    sk.tune_clear()


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def mixed_err(got, ref):
    return np.abs(np.asarray(got, np.float64) - ref) / np.maximum(1.0, np.abs(ref))


@pytest.mark.parametrize("symmetric", [False, True])
def test_gram_graph_replays_match_eager(symmetric):
    nx, ny, L, d, lam = 13, 17, 40, 5, 1
    X = cuda(workloads.random_paths(101, nx, L, d))
    Y = X if symmetric else cuda(workloads.random_paths(102, ny, L - 7, d))
    g, K = sk.capture_gram(X, None if symmetric else Y, lam, symmetric=symmetric)
    for i in range(4):
        # rewrite the inputs in place, run other eager work, then replay
        X.copy_(cuda(workloads.random_paths(200 + i, nx, L, d)))
        eager = sk.sigkernel_gram(X, None if symmetric else Y, lam, symmetric=symmetric)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(K, eager), f"replay {i}"
    ref = oracle.gram(X.cpu().double().numpy(), Y.cpu().double().numpy(), lam)
    assert mixed_err(K.cpu().numpy(), ref).max() <= TOL
    g.close()


def test_pair_graph_replays_reset_the_queue():
    # ragged pairs through the persistent kernel: every replay re-plans the
    # order and re-zeroes the queue counters inside the graph
    lens = workloads.ragged_lengths(7, 40, 2, 300)
    xs = [workloads.random_paths(300 + i, 1, int(n), 6)[0] for i, n in enumerate(lens)]
    ys = [workloads.random_paths(400 + i, 1, int(n), 6)[0] for i, n in enumerate(lens[::-1])]
    X, Y = RaggedPaths.from_list(xs, "cuda"), RaggedPaths.from_list(ys, "cuda")
    g, out = sk.capture_pair(X, Y, 2)
    for i in range(4):
        X.points.mul_(-0.5 if i % 2 else 1.25)
        eager = sk.sigkernel_pair(X, Y, 2)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), f"replay {i}"
    got_x = X.points.cpu().double().numpy()
    offs = X.offsets.cpu().numpy()
    xs_now = [got_x[offs[k]:offs[k + 1]] for k in range(len(xs))]
    ref = oracle.pairs(xs_now, [b.astype(np.float64) for b in ys], 2)
    assert mixed_err(out.cpu().numpy(), ref).max() <= TOL


def test_tall_gram_graph_through_pair_kernel():
    # x paths taller than one wave's strips take the banded pair kernel
    X = cuda(workloads.random_paths(501, 2, 2200, 3))
    Y = cuda(workloads.random_paths(502, 3, 50, 3))
    g, K = sk.capture_gram(X, Y, 0)
    for i in range(3):
        Y.mul_(0.9)
        eager = sk.sigkernel_gram(X, Y, 0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(K, eager), f"replay {i}"


def test_mmd2_graph_with_gradient():
    X = cuda(workloads.random_paths(601, 6, 33, 4, std=0.3))
    Y = cuda(workloads.random_paths(602, 5, 33, 4, std=0.3))
    g, val, dX = sk.capture_mmd2(X, Y, 1, grad=True)
    for i in range(3):
        X.mul_(1.0 + 0.05 * (i + 1))
        v_e, dX_e = sk.sigkernel_mmd2(X, Y, 1, grad=True)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(val, v_e) and torch.equal(dX, dX_e), f"replay {i}"


def test_autotune_gram_keeps_outputs_identical():
    X = cuda(workloads.random_paths(701, 24, 64, 9))
    Y = cuda(workloads.random_paths(702, 40, 64, 9))
    base = sk.sigkernel_gram(X, Y, 1)
    tune, ms = sk.autotune("gram", X, Y, 1)
    assert ms > 0 and 1 <= tune["run"] <= 40 and tune["waves_per_block"] in (1, 2, 4)
    assert sk.tune_get(sk.tune_key("gram", X, Y, 1)) == tune
    assert torch.equal(sk.sigkernel_gram(X, Y, 1), base)


@pytest.mark.parametrize("tune", [dict(run=1, waves_per_block=1), dict(run=3, waves_per_block=2),
                                  dict(run=7, waves_per_block=4), dict(run=64, waves_per_block=1)])
@pytest.mark.parametrize("symmetric", [False, True])
def test_manual_tunings_bit_identical(tune, symmetric):
    X = cuda(workloads.random_paths(801, 19, 50, 6))
    Y = X if symmetric else cuda(workloads.random_paths(802, 23, 45, 6))
    Yarg = None if symmetric else Y
    base = sk.sigkernel_gram(X, Yarg, 2, symmetric=symmetric, no_diag=symmetric)
    key = sk.tune_key("gram", X, Y, 2, _lib.SK_SYMMETRIC | _lib.SK_NO_DIAG if symmetric else 0)
    sk.tune_set(key, tune)
    got = sk.sigkernel_gram(X, Yarg, 2, symmetric=symmetric, no_diag=symmetric)
    assert torch.equal(got, base)
    ref = oracle.gram(X.cpu().double().numpy(), Y.cpu().double().numpy(), 2)
    if symmetric:
        np.fill_diagonal(ref, 0.0)
    assert mixed_err(got.cpu().numpy(), ref).max() <= TOL


def test_autotune_pairs_and_blocks_per_cu():
    lens = workloads.ragged_lengths(9, 64, 2, 500)
    xs = [workloads.random_paths(900 + i, 1, int(n), 8)[0] for i, n in enumerate(lens)]
    X = RaggedPaths.from_list(xs, "cuda")
    Y = RaggedPaths.from_list(xs[::-1], "cuda")
    base = sk.sigkernel_pair(X, Y, 1)
    tune, ms = sk.autotune("pair", X, Y, 1)
    assert ms > 0 and 0 <= tune["pair_blocks_per_cu"] <= 8
    assert torch.equal(sk.sigkernel_pair(X, Y, 1), base)
    for b in (1, 5):
        sk.tune_set(sk.tune_key("pair", X, Y, 1), dict(pair_blocks_per_cu=b))
        assert torch.equal(sk.sigkernel_pair(X, Y, 1), base)


def test_backward_with_tuned_run_matches():
    X = cuda(workloads.random_paths(1001, 10, 30, 4))
    Y = cuda(workloads.random_paths(1002, 14, 26, 4))
    dK = cuda(workloads.random_paths(1003, 1, 10, 14)[0])
    dX0, dY0 = sk.sigkernel_gram_backward(X, Y, dK, 1)
    sk.tune_set(sk.tune_key("gram_backward", X, Y, 1), dict(run=3, waves_per_block=2))
    dX1, dY1 = sk.sigkernel_gram_backward(X, Y, dK, 1)
    # the per-run partial sums associate differently: float32 rounding only
    for a, b in ((dX0, dX1), (dY0, dY1)):
        assert torch.allclose(a, b, rtol=1e-5, atol=1e-6 * float(b.abs().max()))


def test_autotune_refused_under_capture():
    import ctypes
    X = cuda(workloads.random_paths(1101, 4, 20, 3))
    lib = _lib.load()
    sx = sk.api._describe(X)
    out = torch.empty(16, dtype=torch.float32, device="cuda")
    nbytes = sk.workspace_bytes(_lib.SK_OP_GRAM, X, X, 1)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    best, ms, h = _lib.SkTune(), ctypes.c_float(), ctypes.c_void_p()
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    assert lib.sigkernel_graph_begin(s.cuda_stream) == 0
    st = lib.sigkernel_autotune(_lib.SK_OP_GRAM, ctypes.byref(sx), ctypes.byref(sx), 1, 0,
                                out.data_ptr(), ws.data_ptr(), nbytes, 2, s.cuda_stream,
                                ctypes.byref(best), ctypes.byref(ms))
    assert lib.sigkernel_graph_end(s.cuda_stream, ctypes.byref(h)) == 0
    assert st == _lib.SK_ERR_STATE
    assert lib.sigkernel_graph_destroy(h) == 0


@pytest.mark.parametrize("n", [33, 70, 129, 180, 260])
def test_default_runs_symmetric_equals_full(n):
    # the default run length follows a cost model of the busiest SIMD and so
    # changes with n (here 1, 3, 3, 9 and 12 pairs per run for the upper
    # triangle, more for the full square): the upper-triangle launch must give
    # the full launch's values bit for bit, mirrored, and the unbiased form
    # only a zero diagonal on top
    X = cuda(workloads.random_paths(1100 + n, n, 24, 3))
    full = sk.sigkernel_gram(X, X, 1)
    sym = sk.sigkernel_gram(X, None, 1, symmetric=True)
    iu = torch.triu_indices(n, n, device=X.device)
    assert torch.equal(sym[iu[0], iu[1]], full[iu[0], iu[1]])
    assert torch.equal(sym, sym.T)
    nd = sk.sigkernel_gram(X, None, 1, symmetric=True, no_diag=True)
    assert torch.all(torch.diagonal(nd) == 0)
    off = ~torch.eye(n, dtype=torch.bool, device=X.device)
    assert torch.equal(nd[off], sym[off])
    # a sample of entries against the oracle
    rng = np.random.default_rng(n)
    idx = rng.choice(n * n, size=12, replace=False)
    Xd = X.cpu().double().numpy()
    ref = oracle.pairs([Xd[i // n] for i in idx], [Xd[i % n] for i in idx], 1)
    assert mixed_err(sym.reshape(-1)[idx].cpu().numpy(), ref).max() <= TOL


@pytest.mark.parametrize("scheme", ["explicit", "implicit"])
def test_unbiased_symmetric_without_diagonal_sweeps(scheme):
    # the unbiased Gram's triangle leaves the diagonal out of its waves and
    # zeroes it separately: the off-diagonal values are the full launch's,
    # bit for bit, for uniform and ragged batches and both schemes
    n = 41
    X = cuda(workloads.random_paths(1300, n, 30, 4))
    full = sk.sigkernel_gram(X, X, 1, scheme=scheme)
    nd = sk.sigkernel_gram(X, None, 1, symmetric=True, no_diag=True, scheme=scheme)
    off = ~torch.eye(n, dtype=torch.bool, device=X.device)
    assert torch.equal(nd[off], full[off])
    assert torch.all(torch.diagonal(nd) == 0)
    lens = [1, 2, 17, 30, 9, 2, 25]
    xs = [workloads.random_paths(1310 + i, 1, L, 3)[0] for i, L in enumerate(lens)]
    R = RaggedPaths.from_list(xs, "cuda")
    fullr = sk.sigkernel_gram(R, R, 2, scheme=scheme)
    ndr = sk.sigkernel_gram(R, None, 2, symmetric=True, no_diag=True, scheme=scheme)
    offr = ~torch.eye(len(lens), dtype=torch.bool, device=X.device)
    assert torch.equal(ndr[offr], fullr[offr])
    assert torch.all(torch.diagonal(ndr) == 0)
    lifted_full = sk.sigkernel_gram_lifted(X, X, 1, sigma=0.7, scheme=scheme)
    lifted_nd = sk.sigkernel_gram_lifted(X, None, 1, sigma=0.7, symmetric=True, no_diag=True,
                                         scheme=scheme)
    assert torch.equal(lifted_nd[off], lifted_full[off])
    assert torch.all(torch.diagonal(lifted_nd) == 0)
