"""Pipelined row bands (pair_band_kernel): a few pairs whose grids need
several row bands are swept with every band of a pair at once, each band
handing its bottom row to the next through sentinel-filled slots.  Checked
against the FP64 oracle, and bitwise against the sequential bands (the same
pairs inside a batch too large for the pipeline, where each pair's bands run
one after another in one wave): the hand-over moves the same doubles, so the
values must be identical."""
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
    """The same pairs swept with sequential bands: padded with 300 copies of
    the last pair, beyond the pipeline's batch limit."""
    n = X.shape[0]
    Xb = np.concatenate([X, np.repeat(X[-1:], 300, 0)])
    Yb = np.concatenate([Y, np.repeat(Y[-1:], 300, 0)])
    return sk.sigkernel_pair(cuda(Xb), cuda(Yb), lam, **kw).cpu().numpy()[:n]


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
