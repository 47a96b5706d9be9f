"""Learned corrector on the GPU against its FP64 oracle (oracle/corrector.py)
and against the plain scheme (its fallback and judge).

* Integer-valued networks (inputs, weights, biases and upstream gradients
  small integers) make every bf16 rounding and every float32 sum exact, so
  all four layers, the head and every gradient must equal the oracle bit for
  bit: any index, tap, stride or layout slip shows.
* Realistic random networks compare within float32 accumulation tolerances
  (the bf16 rounding of a stored activation can flip by one unit where
  float32 and FP64 land on either side of a rounding midpoint: one bf16 unit
  per stored value, a chain tolerance downstream).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2006_14794_amd as sk
import workloads
from oracle import corrector as oc
from paper_2006_14794_amd import corrector as corr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    sk.load()


def cuda(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


BF16_ULP = 2.0 ** -7  # spacing of bf16 relative to the value (upper bound)


def split_acts(acts, n):
    """GPU activations (bf16, layer-major) -> list of NHWC float64 arrays."""
    a = acts.float().cpu().numpy().astype(np.float64)
    out, off = [], 0
    for ho in (32, 16, 8, 4):
        k = n * ho * ho * 32
        out.append(a[off:off + k].reshape(n, ho, ho, 32))
        off += k
    return out


def integer_net(seed, n):
    r = np.random.default_rng(seed)
    feats = r.integers(-1, 2, size=(n, 64, 64, 8)).astype(np.float32)
    parts = []
    for name, shape in oc.param_layout():
        if name[0] == "w":
            w = r.integers(-1, 2, size=shape) * (r.random(shape) < 0.015)
            parts.append(w.reshape(-1))
        else:
            parts.append(r.integers(0, 2, size=shape).reshape(-1))
    theta = np.concatenate(parts).astype(np.float32)
    dy = r.integers(-3, 4, size=(n, 2)).astype(np.float32)
    return feats, theta, dy


def test_param_count_and_layout():
    assert corr.param_count() == oc.n_params() == 31106
    assert corr.act_elems() == 32 * 32 * 32 + 16 * 16 * 32 + 8 * 8 * 32 + 4 * 4 * 32


@pytest.mark.parametrize("n", [1, 3])
def test_integer_network_bit_exact(n):
    feats, theta, dy = integer_net(7 + n, n)
    y_ref, cache = oc.network_forward(theta.astype(np.float64), feats)
    g_ref = oc.network_backward(theta.astype(np.float64), cache, dy.astype(np.float64))
    assert np.abs(y_ref).max() > 0 and np.abs(g_ref).max() > 0  # not a vacuous case
    # exactness of the case: every activation a bf16 integer, every sum < 2^24
    assert max(np.abs(a).max() for a in cache[0]) <= 256
    assert np.abs(g_ref).max() < 2 ** 24 and np.all(g_ref == np.round(g_ref))
    P = cuda(theta)
    F = cuda(feats, torch.bfloat16)
    acts, y = corr.forward(P, F)
    for l, a in enumerate(split_acts(acts, n)):
        assert np.array_equal(a, cache[0][l + 1]), f"layer {l + 1}"
    assert np.array_equal(y.cpu().numpy().astype(np.float64), y_ref)
    g = corr.backward(P, F, acts, cuda(dy))
    assert np.array_equal(g.cpu().numpy().astype(np.float64), g_ref)


def param_slices():
    off = 0
    for name, shape in oc.param_layout():
        k = int(np.prod(shape))
        yield name, slice(off, off + k)
        off += k


@pytest.mark.parametrize("n", [2, 37])
def test_random_network_forward_backward(n):
    r = np.random.default_rng(100 + n)
    feats = r.normal(size=(n, 64, 64, 8)).astype(np.float32)
    theta = corr.init_params(5 + n)
    theta[2304:2336] = r.normal(size=32) * 0.1  # nonzero biases
    dy = r.normal(size=(n, 2)).astype(np.float32)
    y_ref, cache = oc.network_forward(theta.astype(np.float64), feats)
    g_ref = oc.network_backward(theta.astype(np.float64), cache, dy.astype(np.float64))
    P, F = cuda(theta), cuda(feats, torch.bfloat16)
    acts, y = corr.forward(P, F)
    a1 = split_acts(acts, n)[0]
    # layer 1 sees the same bf16 operands on both sides; its stored output is
    # the bf16 rounding of a float32 sum: one bf16 unit
    ref1 = cache[0][1]
    assert np.all(np.abs(a1 - ref1) <= BF16_ULP * np.abs(ref1) + 1e-6 * np.abs(ref1).max())
    yg = y.cpu().numpy().astype(np.float64)
    assert np.abs(yg - y_ref).max() <= 2e-3 * np.abs(y_ref).max()
    g = corr.backward(P, F, acts, cuda(dy)).cpu().numpy().astype(np.float64)
    for name, sl in param_slices():
        rel = np.linalg.norm(g[sl] - g_ref[sl]) / max(np.linalg.norm(g_ref[sl]), 1e-30)
        assert rel <= 3e-3, (name, rel)


@pytest.mark.parametrize("lx,ly,d", [(256, 256, 8), (37, 50, 3), (2, 9, 1), (257, 100, 16)])
def test_features_match_oracle_grid(lx, ly, d):
    n = 3
    X = workloads.random_paths(200 + lx, n, lx, d)
    Y = workloads.random_paths(300 + ly, n, ly, d)
    r = np.random.default_rng(d)
    norm = np.concatenate([r.normal(size=8) * 0.01, 1.0 + r.random(8)]).astype(np.float32)
    f, k0 = corr.features(cuda(X), cuda(Y), cuda(norm))
    f = f.float().cpu().numpy().astype(np.float64)
    k0g = k0.cpu().numpy()
    for i in range(n):
        x, y = X[i].astype(np.float64), Y[i].astype(np.float64)
        K = oracle.solve_grid(x, y, 0)
        c = np.diff(x, axis=0) @ np.diff(y, axis=0).T
        ref = oc.normalise(oc.block_features(K, c), norm[:8], norm[8:])
        for ch in range(8):
            # float32 moments (relative to the channel's scale), then one bf16 unit
            scale = max(np.abs(ref[:, :, ch]).max(), 1e-6)
            tol = BF16_ULP * np.abs(ref[:, :, ch]) + 3e-5 * scale
            assert np.all(np.abs(f[i, :, :, ch] - ref[:, :, ch]) <= tol), (i, ch)
        assert abs(k0g[i] - K[-1, -1]) <= 1e-6 * max(1.0, abs(K[-1, -1]))
    # the order-0 value is the plain solve's, bit for bit
    assert torch.equal(k0, sk.sigkernel_pair(cuda(X), cuda(Y), 0))


def test_one_point_paths_features():
    X = workloads.random_paths(1, 2, 1, 4)
    Y = workloads.random_paths(2, 2, 30, 4)
    f, k0 = corr.features(cuda(X), cuda(Y))
    assert torch.all(k0 == 1.0)
    fr = f.float().cpu().numpy()
    assert np.all(fr[..., :6] == 0)
    P, Q = np.meshgrid(np.arange(64) / 63, np.arange(64) / 63, indexing="ij")
    assert np.array_equal(fr[0, ..., 6], oc.bf16_round(P)) and np.array_equal(fr[1, ..., 7],
                                                                            oc.bf16_round(Q))


def test_loss_matches_oracle():
    r = np.random.default_rng(3)
    n = 1000
    y = r.normal(size=(n, 2)).astype(np.float32)
    k0 = (1 + 0.1 * r.normal(size=n)).astype(np.float32)
    k3 = (k0 + 0.02 + 0.01 * r.normal(size=n)).astype(np.float32)
    tn = np.array([0.02, 0.01], np.float32)
    lv, dy = corr.loss(cuda(y), cuda(k3), cuda(k0), cuda(tn))
    t = (k3.astype(np.float64) - k0 - np.float64(tn[0])) / np.float64(tn[1])
    l_ref, dy_ref = oc.loss_and_grad(y.astype(np.float64), t)
    assert abs(float(lv.item()) - l_ref) <= 1e-5 * max(1.0, abs(l_ref))
    assert np.abs(dy.cpu().numpy() - dy_ref).max() <= 1e-5 * np.abs(dy_ref).max()


def test_adam_matches_oracle():
    r = np.random.default_rng(4)
    n = 5000
    p = r.normal(size=n).astype(np.float32)
    P, M, V = cuda(p), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    pr, mr, vr = p.astype(np.float64), np.zeros(n), np.zeros(n)
    for t in range(1, 4):
        g = r.normal(size=n).astype(np.float32)
        corr.adam_step(P, cuda(g), M, V, step, 1e-2)
        pr, mr, vr = oc.adam_step(pr, g.astype(np.float64), mr, vr, t, 1e-2)
    assert int(step.item()) == 3
    assert np.abs(P.cpu().numpy() - pr).max() <= 1e-6 * np.abs(pr).max()


@pytest.mark.parametrize("with_sub", [False, True])
def test_channel_stats_match_oracle(with_sub):
    r = np.random.default_rng(5)
    x = (r.normal(size=(100003, 5)) * [1, 2, 0.5, 3, 0] + [0, 1, -2, 5, 7]).astype(np.float32)
    sub = r.normal(size=x.shape).astype(np.float32) if with_sub else None
    mean, rstd = corr.channel_stats(cuda(x), 5, cuda(sub) if with_sub else None)
    v = x.astype(np.float64) - (sub if with_sub else 0)
    m_ref, r_ref = oc.channel_stats(v)
    assert np.allclose(mean.cpu().numpy(), m_ref, rtol=1e-6, atol=1e-6)
    assert np.allclose(rstd.cpu().numpy(), r_ref, rtol=1e-5)


def small_corrector(seed):
    theta = corr.init_params(seed)
    r = np.random.default_rng(seed)
    norm = np.concatenate([np.zeros(8), np.full(8, 1.0)]).astype(np.float32)
    norm[8:14] = [1e2, 1e4, 1e2, 1e-2, 1e4, 1e2]
    tn = np.array([0.015, 0.004], np.float32)
    return sk.Corrector(cuda(theta), cuda(norm), cuda(tn)), theta, norm, tn


def test_predict_without_fallback_matches_oracle_network():
    n = 5
    X, Y = workloads.corrector_pairs(11, n, n_points=65, dim=4)
    c, theta, norm, tn = small_corrector(12)
    out, err, fb = c.predict(cuda(X), cuda(Y), tol=1e30)
    assert int(fb.sum().item()) == 0
    feats = []
    k0 = []
    for i in range(n):
        x, y = X[i].astype(np.float64), Y[i].astype(np.float64)
        K = oracle.solve_grid(x, y, 0)
        c0 = np.diff(x, axis=0) @ np.diff(y, axis=0).T
        feats.append(oc.normalise(oc.block_features(K, c0), norm[:8], norm[8:]))
        k0.append(K[-1, -1])
    y_ref, _ = oc.network_forward(theta.astype(np.float64), np.array(feats))
    k_ref, e_ref, fb_ref = oc.decide(k0, y_ref, tn[0], tn[1], 3.0, 1e30)
    assert not fb_ref.any()
    assert np.abs(out.cpu().numpy() - k_ref).max() <= 1e-4 * np.abs(k_ref).max()
    assert np.allclose(err.cpu().numpy(), e_ref, rtol=5e-3)


@pytest.mark.parametrize("n", [70, 600])
def test_fused_predict_equals_layerwise_forward(n):
    # the on-chip network of predict and the layer-by-layer training forward
    # run the same instructions: with target_norm = (0, 1), k_hat - k0 is y0.
    # 600 pairs: the persistent workgroups (one per compute unit) take
    # several pairs each, the later ones from their prefetch registers
    X, Y = workloads.corrector_pairs(15, n, n_points=256, dim=8)
    Xc, Yc = cuda(X), cuda(Y)
    theta = corr.init_params(16)
    norm = np.concatenate([np.zeros(8), np.full(8, 1.0)]).astype(np.float32)
    norm[8:14] = [1e2, 1e4, 1e2, 1e-2, 1e4, 1e2]
    model = sk.Corrector(cuda(theta), cuda(norm), cuda(np.array([0.0, 1.0], np.float32)))
    out, err, fb = model.predict(Xc, Yc, tol=1e30)
    feats, k0 = corr.features(Xc, Yc, model.norm)
    _, y = corr.forward(model.params, feats)
    k0n = k0.cpu().numpy()
    yn = y.cpu().numpy()
    expect = k0n + np.float32(0.0) + np.float32(1.0) * yn[:, 0]
    got = out.cpu().numpy()
    assert np.all(np.abs(got - expect) <= 2 * np.spacing(np.abs(expect))), np.abs(got - expect).max()
    assert np.allclose(err.cpu().numpy(), np.exp(yn[:, 1].astype(np.float64)), rtol=1e-6)


def test_predict_fallback_is_the_plain_order3_solve():
    n = 300
    X, Y = workloads.corrector_pairs(13, n, n_points=96, dim=8)
    Xc, Yc = cuda(X), cuda(Y)
    c, *_ = small_corrector(14)
    plain = sk.sigkernel_pair(Xc, Yc, 3)
    out0, err0, fb0 = c.predict(Xc, Yc, tol=0.0)  # every pair falls back
    assert int(fb0.sum().item()) == n
    assert torch.equal(out0, plain)
    ref = oracle.pairs([a.astype(np.float64) for a in X[:6]], [b.astype(np.float64) for b in Y[:6]],
                       3)
    assert np.abs(out0.cpu().numpy()[:6] - ref).max() <= 1e-6 * max(1, np.abs(ref).max())
    k_inf, e_inf, fb_inf = c.predict(Xc, Yc, tol=1e30)
    assert int(fb_inf.sum().item()) == 0
    # a threshold in between: every pair is either its corrected value or the
    # plain solve, exactly as the predicted error decides
    tol = float(np.median(3.0 * e_inf.cpu().numpy() / np.abs(k_inf.cpu().numpy())))
    out, err, fb = c.predict(Xc, Yc, kappa=3.0, tol=tol)
    fbn = fb.cpu().numpy().astype(bool)
    assert 0 < fbn.sum() < n
    # accepted where kappa e <= tol |k_hat| (float32 products, as on the device)
    expect = ~(np.float32(3.0) * err.cpu().numpy() <= np.float32(tol) * np.abs(k_inf.cpu().numpy()))
    assert np.array_equal(fbn, expect)
    o = out.cpu().numpy()
    assert np.array_equal(o[fbn], plain.cpu().numpy()[fbn])
    assert np.array_equal(o[~fbn], k_inf.cpu().numpy()[~fbn])


def test_training_reduces_loss_and_error():
    # a short run on 8192 pairs: the loss falls and the corrected values beat
    # the order-0 values on held-out pairs
    n_train, n_test = 8192, 512
    X, Y = workloads.corrector_pairs(workloads.SEED_CORRECTOR_TRAIN, n_train)
    Xt, Yt = workloads.corrector_pairs(workloads.SEED_CORRECTOR_EVAL, n_test)
    Xc, Yc, Xtc, Ytc = cuda(X), cuda(Y), cuda(Xt), cuda(Yt)
    k3 = corr.order3_targets(Xc, Yc)
    logs = []
    model = corr.train(Xc, Yc, k3, epochs=4, batch=128, lr=2e-3, log_every=16,
                       log=logs.append)
    hist = [float(h.split(":")[1]) for h in model.meta["history"].split(";")]
    assert np.mean(hist[-3:]) < np.mean(hist[:2]) - 0.3, logs
    k3t = corr.order3_targets(Xtc, Ytc).cpu().numpy().astype(np.float64)
    k0t = sk.sigkernel_pair(Xtc, Ytc, 0).cpu().numpy().astype(np.float64)
    out, err, fb = model.predict(Xtc, Ytc, tol=1e30)
    e0 = np.abs(k0t - k3t) / np.abs(k3t)
    e1 = np.abs(out.cpu().numpy() - k3t) / np.abs(k3t)
    assert np.median(e1) < np.median(e0) / 4, (np.median(e1), np.median(e0))
