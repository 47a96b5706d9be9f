"""Batches wider than the fused sweeps (more than 16 channels): the coarse
increment Gram (Section 3.1) is formed on the matrix cores and the scheme of
eq. (explicit_finite_diff) is swept from it (coef.hip).  Checked against the
FP64 oracle: pairs at orders 0-3 and beyond, Gram runs, symmetric Grams,
ragged batches, the implicit scheme, 16-bit increments, and the 128 x 128
Gram batch shape at 64 channels."""
import numpy as np
import pytest
import torch

import oracle
import paper_2006_14794_amd as sk
import workloads
from paper_2006_14794_amd import RaggedPaths

pytestmark = pytest.mark.gpu
TOL = 1e-6


def tol(d):
    """The coefficients are float32 sums of d products (matrix-core
    accumulation): their rounding grows like sqrt(d) for random signs, so the
    16-channel bound of the fused sweeps scales by sqrt(d / 16)."""
    return TOL * max(1.0, (d / 16.0) ** 0.5)


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


@pytest.mark.parametrize("lam,L,d", [(0, 40, 17), (1, 33, 33), (2, 25, 100), (3, 20, 300),
                                     (1, 129, 20), (5, 9, 24)])
def test_pairs(lam, L, d):
    X = workloads.random_paths(400 + d, 11, L, d)
    Y = workloads.random_paths(410 + d, 11, L + 4, d)
    got = sk.sigkernel_pair(cuda(X), cuda(Y), lam).cpu().numpy()
    assert mixed_err(got, oracle.pairs(f64(X), f64(Y), lam)).max() <= tol(d)


def test_gram_runs_symmetric_and_implicit():
    # 40 x 1000 pairs: several pairs per wave share the coefficient stream
    X = workloads.random_paths(420, 40, 10, 20)
    Y = workloads.random_paths(421, 1000, 12, 20)
    K = sk.sigkernel_gram(cuda(X), cuda(Y), 1).cpu().numpy()
    assert mixed_err(K, oracle.gram(f64(X), f64(Y), 1)).max() <= tol(20)
    Z = workloads.random_paths(422, 9, 30, 40)
    Zt = cuda(Z)
    full = oracle.gram(f64(Z), f64(Z), 2)
    np.fill_diagonal(full, 0.0)
    sym = sk.sigkernel_gram(Zt, None, 2, symmetric=True, no_diag=True).cpu().numpy()
    assert np.array_equal(sym, sym.T)
    assert mixed_err(sym, full).max() <= tol(40)
    imp = sk.sigkernel_pair(Zt, Zt.flip(0).contiguous(), 1, scheme="implicit").cpu().numpy()
    assert mixed_err(imp, oracle.pairs_implicit(f64(Z), f64(Z[::-1]), 1)).max() <= tol(40)


def test_ragged_and_degenerate_paths():
    lens_x = [1, 2, 40, 17, 63]
    lens_y = [30, 45, 1, 2, 20]
    xs = [workloads.random_paths(430 + i, 1, L, 24)[0] for i, L in enumerate(lens_x)]
    ys = [workloads.random_paths(440 + i, 1, L, 24)[0] for i, L in enumerate(lens_y)]
    X, Y = RaggedPaths.from_list(xs, "cuda"), RaggedPaths.from_list(ys, "cuda")
    got = sk.sigkernel_pair(X, Y, 2).cpu().numpy()
    ref = oracle.pairs([f64(a) for a in xs], [f64(b) for b in ys], 2)
    assert mixed_err(got, ref).max() <= tol(24)
    assert got[0] == 1.0 and got[2] == 1.0
    G = sk.sigkernel_gram(X, Y, 4).cpu().numpy()
    Gref = oracle.gram([f64(a) for a in xs], [f64(b) for b in ys], 4)
    assert mixed_err(G, Gref).max() <= tol(24)
    X.max_len = 50  # path 4 (63 points) breaks the declared bound
    bad = sk.sigkernel_pair(X, Y, 1).cpu().numpy()
    assert np.isnan(bad[4]) and np.all(np.isfinite(bad[:4]))


def test_zero_channel_agrees_with_the_fused_sweep():
    # a 17th channel that is identically zero: the coefficient path must give
    # the fused 16-channel result up to float32 summation order
    X = workloads.random_paths(450, 6, 60, 16)
    Y = workloads.random_paths(451, 7, 50, 16)
    pad = lambda a: np.concatenate([a, np.zeros(a.shape[:-1] + (1,), a.dtype)], -1)  # noqa
    k16 = sk.sigkernel_gram(cuda(X), cuda(Y), 2).cpu().numpy()
    k17 = sk.sigkernel_gram(cuda(pad(X)), cuda(pad(Y)), 2).cpu().numpy()
    assert mixed_err(k17, k16.astype(np.float64)).max() <= 1e-6


def rounded_paths(P):
    """Paths whose float32 increments are those of P rounded to bfloat16."""
    inc = torch.from_numpy(np.diff(P.astype(np.float32), axis=-2)).to(torch.bfloat16)
    inc = inc.to(torch.float64).numpy()
    start = P[..., :1, :].astype(np.float64)
    return np.concatenate([start, start + np.cumsum(inc, axis=-2)], axis=-2)


def test_bf16_increments():
    X = workloads.random_paths(460, 5, 40, 48)
    Y = workloads.random_paths(461, 6, 35, 48)
    K = sk.sigkernel_gram(cuda(X), cuda(Y), 1, gram_precision="bf16").cpu().numpy()
    ref = oracle.gram(rounded_paths(X), rounded_paths(Y), 1)
    assert mixed_err(K, ref).max() <= tol(48)


def fp32_increment_gram(x, y):
    """Coarse coefficients with float32 increments and float32 FMA sums over
    the channels in order: the GPU's precision model (its matrix-core sums
    differ from this only in their rounding order)."""
    dx = (x[1:].astype(np.float32) - x[:-1].astype(np.float32)).astype(np.float64)
    dy = (y[1:].astype(np.float32) - y[:-1].astype(np.float32)).astype(np.float64)
    G = np.zeros((len(dx), len(dy)), np.float32)
    for k in range(dx.shape[1]):
        G = (np.multiply.outer(dx[:, k], dy[:, k]) + G.astype(np.float64)).astype(np.float32)
    return G.astype(np.float64)


def test_gram_batch_shape_at_64_channels_sampled():
    # The time channel adds the same product (1/255)^2 to every coefficient,
    # so its float32 rounding is systematic and the error against the double
    # oracle grows with the number of cells (about 2.4e-6 here, for float32
    # coefficients computed in any order).  The GPU must do no worse than
    # float32 coefficients swept in double, within the float32 output rounding.
    X, Y = workloads.gram_batch(seed=470, dim=63)  # 63 channels + time
    K = sk.sigkernel_gram(cuda(X), cuda(Y), 1).cpu().numpy()
    rng = np.random.default_rng(8)
    idx = rng.choice(128 * 128, size=32, replace=False)
    xs = [f64(X[i // 128]) for i in idx]
    ys = [f64(Y[i % 128]) for i in idx]
    ref = oracle.pairs(xs, ys, 1)
    model = np.array([oracle.solve_coef(fp32_increment_gram(x, y), 1) for x, y in zip(xs, ys)])
    got = K.reshape(-1)[idx].astype(np.float64)
    assert np.all(np.abs(got - ref) <= np.abs(model - ref) + 3e-7 * np.maximum(1.0, np.abs(ref)))
    assert mixed_err(got, model).max() <= 3e-7
    assert mixed_err(got, ref).max() <= 5e-6


def test_tall_wide_paths_are_rejected():
    X = workloads.random_paths(480, 2, 2100, 20)
    with pytest.raises(sk.SigKernelError):
        sk.sigkernel_gram(cuda(X), cuda(X[:, :50]), 0)
