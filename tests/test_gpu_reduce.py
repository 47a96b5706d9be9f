"""Reduced measures on the GPU (eqs. (min_lasso) and (fixed_point)) against
the FP64 oracle: the iterates and losses of the proximal-gradient iteration
for a fixed penalty, convergence to the minimiser of a strictly convex
instance, the support search on the 30-path fBM ensemble, and the end-to-end
path from the GPU signature Gram."""
import numpy as np
import pytest
import torch

import oracle
import paper_2006_14794_amd as sk
import workloads
from oracle import reduced_measure as rm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sk.load()


@pytest.fixture(scope="module")
def fbm_gram():
    P, H = workloads.fbm_paths(n_points=50)
    K = oracle.gram(P.astype(np.float64), P.astype(np.float64), 6).astype(np.float32)
    return P, H, K


def spd(seed, n, cond=20.0):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    return ((Q * np.geomspace(1.0, cond, n)) @ Q.T).astype(np.float32)


def test_fixed_penalty_iterates_and_losses(fbm_gram):
    _, _, K = fbm_gram
    K64 = K.astype(np.float64)
    alpha = np.full(30, np.float32(1.0 / 30)).astype(np.float64)
    step = 1.0 / rm.lipschitz(K64)
    lam = 2.0
    beta, loss, used = sk.reduced_measure(torch.from_numpy(K).cuda(), lam, 500, step=step)
    ref, ref_loss = rm.ista(K64, alpha, lam, 500, step=step)
    assert used.item() == step
    assert np.abs(beta.cpu().numpy() - ref).max() <= 1e-10
    assert np.array_equal(beta.cpu().numpy() == 0.0, ref == 0.0)
    assert np.abs(loss.cpu().numpy() - ref_loss).max() <= 1e-10 * np.abs(ref_loss).max()


@pytest.mark.parametrize("n", [1, 32, 33, 64])
def test_one_wave_sizes(n):
    # up to 64 atoms one wave holds K in registers (32 or 64 columns, zero
    # beyond n): iterates, losses and the power-iteration step of a fixed
    # penalty against the oracle
    K = spd(40 + n, n, cond=8.0)
    K64 = K.astype(np.float64)
    alpha = np.full(n, np.float32(1.0 / n)).astype(np.float64)
    lam = 1e-3
    beta, loss, used = sk.reduced_measure(torch.from_numpy(K).cuda(), lam, 200)
    lip = rm.lipschitz(K64)
    assert 0.9 / lip <= used.item() <= 1.0 / lip
    ref, ref_loss = rm.ista(K64, alpha, lam, 200, step=used.item())
    assert np.abs(beta.cpu().numpy() - ref).max() <= 1e-10
    assert np.abs(loss.cpu().numpy() - ref_loss).max() <= 1e-10 * np.abs(ref_loss).max()


def test_automatic_step_reaches_the_minimiser():
    K = spd(11, 200)
    K64 = K.astype(np.float64)
    alpha = np.full(200, np.float32(1.0 / 200)).astype(np.float64)
    lam = 0.002
    beta, loss, used = sk.reduced_measure(torch.from_numpy(K).cuda(), lam, 3000)
    # the power-iteration step stays below 1 / Lip (descent) and close to it
    lip = rm.lipschitz(K64)
    assert 0.9 / lip <= used.item() <= 1.0 / lip
    assert np.all(np.diff(loss.cpu().numpy()) <= 1e-14)
    ref, _ = rm.ista(K64, alpha, lam, 30000)
    assert np.abs(beta.cpu().numpy() - ref).max() <= 1e-7


def test_support_search_on_the_fbm_ensemble(fbm_gram):
    _, H, K = fbm_gram
    K64 = K.astype(np.float64)
    alpha = np.full(30, np.float32(1.0 / 30)).astype(np.float64)
    beta, lam, used = sk.reduced_measure_support(torch.from_numpy(K).cuda(), 6, 3000, 40)
    b = beta.cpu().numpy()
    lam = lam.item()
    assert np.count_nonzero(b) == 6
    g = rm.gradient(K64, alpha, b)
    nz = b != 0
    assert np.abs(g[nz] + lam * np.sign(b[nz])).max() < 1e-6
    assert np.all(np.abs(g[~nz]) <= lam * (1 + 1e-6))
    # The bisection's path is not unique: on this nearly singular Gram, 3000
    # iterations leave components at the threshold, where rounding decides
    # zero or not.  What is unique is the minimum of eq. (min_lasso) at the
    # penalty found: the GPU weights must attain it (long oracle run).
    _, ref_loss = rm.ista(K64, alpha, lam, 100000)
    assert rm.objective(K64, alpha, b, lam) <= ref_loss[-1] + 1e-6 * abs(ref_loss[-1])


def test_end_to_end_from_the_gpu_gram():
    P, H = workloads.fbm_paths(n_points=50)
    Pt = torch.from_numpy(P).cuda()
    K = sk.sigkernel_gram(Pt, None, 6, symmetric=True)
    beta, lam, _ = sk.reduced_measure_support(K, 6)
    b = beta.cpu().numpy()
    assert np.count_nonzero(b) == 6 and np.all(np.isfinite(b))
    Kr = oracle.gram(P.astype(np.float64), P.astype(np.float64), 6)
    assert np.abs(K.cpu().numpy() - Kr).max() <= 1e-5 * np.abs(Kr).max()


def test_largest_size():
    K = spd(12, 4096, cond=5.0)
    beta, loss, used = sk.reduced_measure(torch.from_numpy(K).cuda(), 1e-5, 5, step=0.05)
    alpha = np.full(4096, np.float32(1.0 / 4096)).astype(np.float64)
    ref, ref_loss = rm.ista(K.astype(np.float64), alpha, 1e-5, 5, step=0.05)
    assert np.abs(beta.cpu().numpy() - ref).max() <= 1e-12
    assert np.abs(loss.cpu().numpy() - ref_loss).max() <= 1e-10 * np.abs(ref_loss).max()
