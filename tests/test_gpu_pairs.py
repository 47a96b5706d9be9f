"""Independent pairs through the persistent, length-sorted launch
(sigkernel_pair): uneven lengths, the shorter path on the rows, row bands for
grids taller than one wave, two row classes; against the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2006_14794_amd as sk
import workloads
from paper_2006_14794_amd import RaggedPaths

pytestmark = pytest.mark.gpu
TOL = 1e-6


def mixed_err(got, ref):
    return np.abs(np.asarray(got, np.float64) - ref) / np.maximum(1.0, np.abs(ref))


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sk.load()


def run_pairs(xs, ys, lam):
    X = RaggedPaths.from_list(xs, "cuda")
    Y = RaggedPaths.from_list(ys, "cuda")
    return sk.sigkernel_pair(X, Y, lam).cpu().numpy()


@pytest.mark.parametrize("lam,d,lens", [
    (3, 16, [(300, 310), (20, 300), (301, 9)]),       # 2 bands of 64 x 32 rows
    (2, 16, [(600, 700), (700, 650), (257, 258)]),    # up to 3 bands of 64 x 16 rows
    (1, 4, [(1030, 1040), (1030, 12)]),                # bands at R = 32
    (0, 2, [(2, 2), (5, 3000), (3000, 5)]),           # one-segment rows, long columns
])
def test_row_bands_and_orientation(lam, d, lens):
    xs = [workloads.random_paths(10 + i, 1, a, d)[0] for i, (a, _) in enumerate(lens)]
    ys = [workloads.random_paths(20 + i, 1, b, d)[0] for i, (_, b) in enumerate(lens)]
    got = run_pairs(xs, ys, lam)
    ref = oracle.pairs([a.astype(np.float64) for a in xs], [b.astype(np.float64) for b in ys],
                       lam)
    assert mixed_err(got, ref).max() <= TOL


def test_swapped_pair_equals_unswapped():
    x = workloads.random_paths(31, 1, 200, 5)[0]
    y = workloads.random_paths(32, 1, 90, 5)[0]
    a = run_pairs([x], [y], 2)[0]
    b = run_pairs([y], [x], 2)[0]
    ref = oracle.solve(x.astype(np.float64), y.astype(np.float64), 2)
    assert mixed_err(a, ref) <= TOL and mixed_err(b, ref) <= TOL


def test_many_short_and_long_pairs_mixed_classes():
    rng = np.random.default_rng(3)
    lx = rng.integers(2, 400, size=300)
    ly = rng.integers(2, 400, size=300)
    xs = [workloads.random_paths(1000 + i, 1, int(L), 3)[0] for i, L in enumerate(lx)]
    ys = [workloads.random_paths(5000 + i, 1, int(L), 3)[0] for i, L in enumerate(ly)]
    got = run_pairs(xs, ys, 1)
    ref = oracle.pairs([a.astype(np.float64) for a in xs], [b.astype(np.float64) for b in ys], 1)
    assert mixed_err(got, ref).max() <= TOL
    # deterministic across calls (the queue order may differ, the values may not)
    assert np.array_equal(got, run_pairs(xs, ys, 1))


def test_ragged_workload_full_size_sampled():
    # 4096 pairs, lengths uniform in [64, 1024], d = 16, dyadic order 2: the
    # launch configuration of the ragged workload, sampled against the oracle
    xs, ys = workloads.ragged_pairs()
    got = run_pairs(xs, ys, 2)
    assert np.all(np.isfinite(got))
    cost = np.array([min(len(a), len(b)) * max(len(a), len(b)) for a, b in zip(xs, ys)])
    rng = np.random.default_rng(0)
    idx = list(np.argsort(cost)[-3:]) + list(np.argsort(cost)[:3]) + list(
        rng.choice(len(xs), 18, replace=False))
    ref = oracle.pairs([xs[i].astype(np.float64) for i in idx],
                       [ys[i].astype(np.float64) for i in idx], 2)
    err = mixed_err(got[idx], ref)
    assert err.max() <= 1e-5, err.max()


def test_gram_with_x_paths_taller_than_one_wave():
    # 64 lanes x 32 rows cannot hold 1100 segments at dyadic order 1: the Gram
    # goes through the persistent pair kernel with row bands
    X = workloads.random_paths(41, 3, 1101, 2)
    Y = workloads.random_paths(42, 2, 300, 2)
    got = sk.sigkernel_gram(torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda(), 1)
    ref = oracle.gram(X.astype(np.float64), Y.astype(np.float64), 1)
    assert mixed_err(got.cpu().numpy(), ref).max() <= TOL
    Xt = torch.from_numpy(X).cuda()
    sym = sk.sigkernel_gram(Xt, None, 1, symmetric=True, no_diag=True).cpu().numpy()
    refs = oracle.gram(X.astype(np.float64), X.astype(np.float64), 1)
    np.fill_diagonal(refs, 0.0)
    assert mixed_err(sym, refs).max() <= TOL and np.all(np.diag(sym) == 0)
