"""Pipelined row bands (pair_band_kernel): pairs whose grids need several
row bands are swept with every band of a pair at once, each band handing its
bottom row to the next through sentinel-filled slots.  Checked against the
FP64 oracle, and bitwise against the sequential bands (the tuning entry
pair_bands = 1, where each pair's bands run one after another in one wave):
the hand-over moves the same doubles, so the values must be identical."""
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


def f64(a):
    return np.asarray(a, dtype=np.float64)


def mixed_err(got, ref):
    return np.abs(np.asarray(got, np.float64) - ref) / np.maximum(1.0, np.abs(ref))


def sequential(X, Y, lam, **kw):
    """The same call with each pair's bands swept one after another in one
    wave (a tuning entry for the call's key, removed afterwards)."""
    Xt = X if isinstance(X, RaggedPaths) else cuda(X)
    Yt = Y if isinstance(Y, RaggedPaths) else cuda(Y)
    key = sk.tune_key("pair", Xt, Yt, lam)
    sk.tune_set(key, dict(pair_bands=1))
    try:
        return sk.sigkernel_pair(Xt, Yt, lam, **kw).cpu().numpy()
    finally:
        sk.tune_set(key, None)


@pytest.mark.parametrize("lam,L,d", [(3, 300, 2), (1, 1200, 3), (4, 1000, 2), (0, 2600, 2)])
def test_uniform_pairs(lam, L, d):
    X = workloads.random_paths(500 + lam, 4, L, d)
    Y = workloads.random_paths(510 + lam, 4, L + 17, d)
    got = sk.sigkernel_pair(cuda(X), cuda(Y), lam).cpu().numpy()
    assert mixed_err(got, oracle.pairs(f64(X), f64(Y), lam)).max() <= TOL
    assert np.array_equal(got, sequential(X, Y, lam))


def test_implicit_scheme():
    X = workloads.random_paths(520, 3, 700, 2)
    Y = workloads.random_paths(521, 3, 650, 2)
    got = sk.sigkernel_pair(cuda(X), cuda(Y), 3, scheme="implicit").cpu().numpy()
    assert mixed_err(got, oracle.pairs_implicit(f64(X), f64(Y), 3)).max() <= TOL
    assert np.array_equal(got, sequential(X, Y, 3, scheme="implicit"))


def test_ragged_mix_of_long_short_and_degenerate():
    lens_x = [900, 40, 1, 1300, 2, 700]
    lens_y = [1100, 50, 30, 800, 600, 1]
    xs = [workloads.random_paths(530 + i, 1, L, 2)[0] for i, L in enumerate(lens_x)]
    ys = [workloads.random_paths(540 + i, 1, L, 2)[0] for i, L in enumerate(lens_y)]
    X, Y = RaggedPaths.from_list(xs, "cuda"), RaggedPaths.from_list(ys, "cuda")
    got = sk.sigkernel_pair(X, Y, 2).cpu().numpy()
    ref = oracle.pairs([f64(a) for a in xs], [f64(b) for b in ys], 2)
    assert mixed_err(got, ref).max() <= TOL
    assert got[2] == 1.0 and got[5] == 1.0
    assert np.array_equal(got, sequential(X, Y, 2))


# d = 16 at dyadic order 2 runs full bands of 16 fine rows per lane (256
# increments on the rows); the top band takes 4, 8 or 16 rows per lane by the
# rows left over.  Shorter-path increments m around every switch: one band
# (64 | 65, 128 | 129, 256), two bands (257, 320 | 321, 384 | 385, 512) and
# three (600); half the pairs put the shorter path on y.
TOP_BAND_M = [64, 65, 128, 129, 256, 257, 320, 321, 384, 385, 512, 600]


def test_top_band_heights():
    xs, ys = [], []
    for i, m in enumerate(TOP_BAND_M):
        a = workloads.random_paths(560 + i, 1, m + 1, 16)[0]
        b = workloads.random_paths(580 + i, 1, m + 1 + 23 * (i % 3), 16)[0]
        xs.append(a if i % 2 == 0 else b)
        ys.append(b if i % 2 == 0 else a)
    X, Y = RaggedPaths.from_list(xs, "cuda"), RaggedPaths.from_list(ys, "cuda")
    got = sk.sigkernel_pair(X, Y, 2).cpu().numpy()
    ref = oracle.pairs([f64(a) for a in xs], [f64(b) for b in ys], 2)
    assert mixed_err(got, ref).max() <= TOL
    assert np.array_equal(got, sequential(X, Y, 2))


def test_more_pairs_than_one_scan_chunk():
    """1500 uniform pairs of two bands each: the band plan numbers the tasks
    over two 1024-pair chunks of its scan."""
    X = workloads.random_paths(570, 1500, 300, 2)
    Y = workloads.random_paths(571, 1500, 310, 2)
    got = sk.sigkernel_pair(cuda(X), cuda(Y), 3).cpu().numpy()
    idx = np.random.default_rng(572).choice(1500, 24, replace=False)
    ref = oracle.pairs(f64(X[idx]), f64(Y[idx]), 3)
    assert mixed_err(got[idx], ref).max() <= TOL
    assert np.array_equal(got, sequential(X, Y, 3))


def test_ragged_batch_across_scan_chunks():
    """1300 ragged pairs of one to three bands, short pairs and one-point
    paths among them."""
    rng = np.random.default_rng(580)
    lx = rng.integers(60, 700, 1300)
    ly = rng.integers(60, 700, 1300)
    lx[::97] = 1
    xs = [workloads.random_paths(581 + i, 1, int(L), 2)[0] for i, L in enumerate(lx)]
    ys = [workloads.random_paths(5000 + i, 1, int(L), 2)[0] for i, L in enumerate(ly)]
    X, Y = RaggedPaths.from_list(xs, "cuda"), RaggedPaths.from_list(ys, "cuda")
    got = sk.sigkernel_pair(X, Y, 3).cpu().numpy()
    idx = np.concatenate([np.arange(0, 1300, 97), rng.choice(1300, 16, replace=False)])
    ref = oracle.pairs([f64(xs[i]) for i in idx], [f64(ys[i]) for i in idx], 3)
    assert mixed_err(got[idx], ref).max() <= TOL
    assert np.all(got[::97] == 1.0)
    assert np.array_equal(got, sequential(X, Y, 3))


def test_tall_gram():
    X = workloads.random_paths(550, 2, 700, 2)
    Y = workloads.random_paths(551, 3, 800, 2)
    K = sk.sigkernel_gram(cuda(X), cuda(Y), 2).cpu().numpy()
    assert mixed_err(K, oracle.gram(f64(X), f64(Y), 2)).max() <= TOL


def test_graph_replays_refill_the_slots():
    X = workloads.random_paths(560, 3, 900, 2)
    Y = workloads.random_paths(561, 3, 850, 2)
    Xt, Yt = cuda(X), cuda(Y)
    eager = sk.sigkernel_pair(Xt, Yt, 2).cpu().numpy()
    graph, out = sk.capture_pair(Xt, Yt, 2)
    for i in range(3):
        graph.replay()
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy(), eager), i
        sk.sigkernel_pair(Xt[:1], Yt[:1], 0)  # other work between replays


def test_repeated_calls_with_pairs_without_cells():
    """Pairs without cells are single tasks at the end of the band queue.
    Written by one lane before the loop's continue, they once let a wave
    sweep an earlier band again with part of its lanes, corrupting the first
    pair's hand-over in some calls: every repeat must equal the sequential
    bands."""
    rng = np.random.default_rng(580)
    lx = rng.integers(60, 700, 1300)
    ly = rng.integers(60, 700, 1300)
    lx[::97] = 1
    xs = [workloads.random_paths(581 + i, 1, int(L), 2)[0] for i, L in enumerate(lx)]
    ys = [workloads.random_paths(5000 + i, 1, int(L), 2)[0] for i, L in enumerate(ly)]
    X, Y = RaggedPaths.from_list(xs, "cuda"), RaggedPaths.from_list(ys, "cuda")
    ref = sequential(X, Y, 3)
    for i in range(6):
        assert np.array_equal(sk.sigkernel_pair(X, Y, 3).cpu().numpy(), ref), i
