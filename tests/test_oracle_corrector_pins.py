"""Pins of the corrector's FP64 oracle (oracle/corrector.py) against things
other than itself: torch's bfloat16 conversion, torch's float64 convolution,
autograd and Adam, central finite differences, brute-force loops, and the
closed form sum of all coarse coefficients = <x_T - x_0, y_T - y_0>."""
import numpy as np
import pytest
import torch

import oracle
import workloads
from oracle import corrector as oc


def rng(seed):
    return np.random.default_rng(seed)


def test_bf16_rounding_matches_torch_including_ties():
    a = rng(1).normal(size=4096).astype(np.float32) * np.float32(3.7)
    # exact ties: low 16 bits 0x8000, both parities of the kept bit
    ties = (np.arange(64, dtype=np.uint32) << 16 | 0x3F808000).view(np.float32)
    x = np.concatenate([a, ties, -ties, np.float32([0.0, -0.0, 1e-30, 65504.0])])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(oc.bf16_round(x), ref)


def test_param_layout_size():
    sizes = [32 * 9 * 8 + 32] + [32 * 9 * 32 + 32] * 3 + [2 * 512 + 2]
    assert oc.n_params() == sum(sizes) == 31106


def torch_conv(x, w, b):
    """torch float64 conv2d (stride 2, pad 1) on NHWC / [Cout][3][3][Cin]."""
    xt = torch.from_numpy(x).permute(0, 3, 1, 2)
    wt = torch.from_numpy(w).permute(0, 3, 1, 2)
    return torch.nn.functional.conv2d(xt, wt, torch.from_numpy(b), stride=2, padding=1)


@pytest.mark.parametrize("h,cin", [(64, 8), (9, 32), (4, 3)])
def test_conv_forward_matches_torch(h, cin):
    r = rng(h + cin)
    x = r.normal(size=(2, h, h, cin)).astype(np.float32)
    w = r.normal(size=(5, 3, 3, cin)).astype(np.float32) * 0.2
    b = r.normal(size=5)
    got = oc.conv_forward(x, w, b)
    ref = torch_conv(oc.bf16_round(x), oc.bf16_round(w), b).permute(0, 2, 3, 1).numpy()
    assert got.shape == ((2, (h + 1) // 2, (h + 1) // 2, 5))
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


def test_conv_centre_tap_picks_even_positions():
    # output (ho, wo) sees input (2 ho - 1 + kh, 2 wo - 1 + kw): the centre tap
    # alone reads input (2 ho, 2 wo)
    x = np.arange(36, dtype=np.float32).reshape(1, 6, 6, 1)
    w = np.zeros((1, 3, 3, 1), np.float32)
    w[0, 1, 1, 0] = 1.0
    got = oc.conv_forward(x, w, np.zeros(1))[0, :, :, 0]
    assert np.array_equal(got, x[0, ::2, ::2, 0])
    w[:] = 0.0
    w[0, 0, 0, 0] = 1.0  # top-left tap: input (2 ho - 1, 2 wo - 1), zero outside
    got = oc.conv_forward(x, w, np.zeros(1))[0, :, :, 0]
    ref = np.zeros((3, 3))
    ref[1:, 1:] = x[0, 1:5:2, 1:5:2, 0]
    assert np.array_equal(got, ref)


def test_conv_backward_matches_autograd():
    r = rng(7)
    x = r.normal(size=(3, 10, 10, 6)).astype(np.float32)
    w = (r.normal(size=(4, 3, 3, 6)) * 0.3).astype(np.float32)
    b = r.normal(size=4)
    dpre = r.normal(size=(3, 5, 5, 4))
    dx, dw, db = oc.conv_backward(x, w, dpre)
    xt = torch.from_numpy(oc.bf16_round(x)).permute(0, 3, 1, 2).requires_grad_()
    wt = torch.from_numpy(oc.bf16_round(w)).permute(0, 3, 1, 2).requires_grad_()
    bt = torch.from_numpy(b).requires_grad_()
    y = torch.nn.functional.conv2d(xt, wt, bt, stride=2, padding=1)
    y.backward(torch.from_numpy(dpre).permute(0, 3, 1, 2))
    assert np.allclose(dx, xt.grad.permute(0, 2, 3, 1).numpy(), rtol=0, atol=1e-12)
    assert np.allclose(dw, wt.grad.permute(0, 2, 3, 1).numpy(), rtol=0, atol=1e-11)
    assert np.allclose(db, bt.grad.numpy(), rtol=0, atol=1e-12)


def small_theta(seed, scale=1.0):
    r = rng(seed)
    parts = []
    for name, shape in oc.param_layout():
        fan_in = int(np.prod(shape[1:])) if len(shape) > 1 else 1
        std = scale * np.sqrt(2.0 / fan_in) if name[0] == "w" else 0.05
        parts.append(r.normal(size=shape).reshape(-1) * std)
    return np.concatenate(parts).astype(np.float32).astype(np.float64)


def torch_network(theta, feats, rounding):
    """The same network assembled from torch modules (float64), bf16 rounding
    applied as a straight-through step on weights and layer inputs."""
    p = {k: torch.from_numpy(v.copy()).requires_grad_() for k, v in oc.unflatten(theta).items()}

    def rnd(t):
        if not rounding:
            return t
        r = torch.from_numpy(oc.bf16_round(t.detach().numpy()))
        return t + (r - t).detach()
    a = torch.from_numpy(feats).permute(0, 3, 1, 2)
    for i in range(4):
        w = rnd(p[f"w{i + 1}"].permute(0, 3, 1, 2))
        a = torch.relu(torch.nn.functional.conv2d(rnd(a), w, p[f"b{i + 1}"], stride=2, padding=1))
    flat = rnd(a.permute(0, 2, 3, 1).reshape(a.shape[0], -1))
    return flat @ p["wh"].T + p["bh"], p


def test_network_forward_backward_match_torch():
    feats = rng(3).normal(size=(3, 64, 64, 8)).astype(np.float32)
    theta = small_theta(4)
    y, cache = oc.network_forward(theta, feats)
    yt, p = torch_network(theta, feats.astype(np.float64), True)
    assert np.abs(y - yt.detach().numpy()).max() <= 1e-10 * np.abs(y).max()
    dy = rng(5).normal(size=y.shape)
    g = oc.network_backward(theta, cache, dy)
    yt.backward(torch.from_numpy(dy))
    gt = oc.flatten({k: v.grad.numpy() for k, v in p.items()})
    assert np.abs(g - gt).max() <= 1e-10 * np.abs(gt).max()


def test_network_gradient_by_finite_differences():
    # without rounding the network is piecewise smooth: central differences
    feats = rng(8).normal(size=(2, 64, 64, 8))
    theta = small_theta(9)
    dy = rng(10).normal(size=(2, 2))
    _, cache = oc.network_forward(theta, feats, rounding=False)
    g = oc.network_backward(theta, cache, dy)
    idx = rng(11).choice(theta.size, size=40, replace=False)
    idx = np.concatenate([idx, [0, 2304, 31104, 31105, 30079]])
    eps = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += eps
        tm[i] -= eps
        fd = (np.sum(dy * oc.network_forward(tp, feats, False)[0]) -
              np.sum(dy * oc.network_forward(tm, feats, False)[0])) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), i


def test_loss_and_gradient_match_autograd():
    r = rng(12)
    y = r.normal(size=(16, 2))
    t = r.normal(size=16)
    loss, dy = oc.loss_and_grad(y, t)
    yt = torch.from_numpy(y).requires_grad_()
    res = yt[:, 0] - torch.from_numpy(t)
    s = yt[:, 1]
    lt = (res ** 2 + 0.5 * res.detach() ** 2 * torch.exp(-2 * s) + s).mean()
    lt.backward()
    assert abs(loss - lt.item()) <= 1e-14
    assert np.allclose(dy, yt.grad.numpy(), rtol=1e-14, atol=1e-16)


def test_adam_matches_torch():
    r = rng(13)
    theta = r.normal(size=50)
    grads = [r.normal(size=50) for _ in range(3)]
    tt = torch.from_numpy(theta.copy()).requires_grad_()
    opt = torch.optim.Adam([tt], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(50)
    v = np.zeros(50)
    th = theta.copy()
    for k, g in enumerate(grads):
        th, m, v = oc.adam_step(th, g, m, v, k + 1, 3e-3)
        tt.grad = torch.from_numpy(g)
        opt.step()
    assert np.abs(th - tt.detach().numpy()).max() <= 1e-14


def brute_features(K, c):
    m, n = c.shape
    out = np.zeros((64, 64, 8))
    for p in range(m):
        for q in range(n):
            Cv, Av, Bv, cv = K[p][q], K[p + 1][q], K[p][q + 1], c[p][q]
            f = out[p // 4, q // 4]
            f[0] += cv
            f[1] += cv * cv * (Av + Bv) / 2
            f[2] += cv * (Av + Bv)
            f[3] += Cv - 1
            f[4] += cv * cv * Cv
            f[5] += cv * (Bv - Av)
    for P in range(64):
        for Q in range(64):
            out[P, Q, 6] = P / 63
            out[P, Q, 7] = Q / 63
    return out


@pytest.mark.parametrize("m,n", [(9, 13), (255, 255), (4, 1)])
def test_block_features_brute_force_and_closed_form(m, n):
    x = workloads.random_paths(20, 1, m + 1, 3)[0].astype(np.float64)
    y = workloads.random_paths(21, 1, n + 1, 3)[0].astype(np.float64)
    K = oracle.solve_grid(x, y, 0)
    c = np.diff(x, axis=0) @ np.diff(y, axis=0).T
    f = oc.block_features(K, c)
    if m * n < 1000:
        assert np.allclose(f, brute_features(K, c), rtol=1e-13, atol=1e-15)
    # channel 0 sums to <x_T - x_0, y_T - y_0>
    assert abs(f[:, :, 0].sum() - np.dot(x[-1] - x[0], y[-1] - y[0])) <= 1e-13
    assert np.all(f[(m + 3) // 4:, :, :6] == 0) and np.all(f[:, (n + 3) // 4:, :6] == 0)


def test_channel_stats():
    a = rng(14).normal(size=(100, 7, 3)) * [1.0, 2.0, 0.0] + [0.5, -1.0, 3.0]
    mean, rstd = oc.channel_stats(a)
    flat = a.reshape(-1, 3)
    assert np.allclose(mean, flat.mean(axis=0), rtol=1e-14, atol=1e-14)
    assert np.allclose(rstd[:2], 1 / flat[:, :2].std(axis=0), rtol=1e-12)
    assert rstd[2] == 1.0


def test_decide_hand_values():
    y = np.array([[0.5, np.log(1e-3)], [0.0, np.log(1e-5)], [-1.0, 0.0]])
    k_hat, err, fb = oc.decide([2.0, 0.1, 3.0], y, mu=0.01, sigma=0.02, kappa=3.0, tol=1e-3)
    assert np.allclose(k_hat, [2.0 + 0.01 + 0.01, 0.11, 3.0 + 0.01 - 0.02])
    assert np.allclose(err, [2e-5, 2e-7, 0.02])
    # 3 * 2e-5 = 6e-5 <= 2.02e-3: keep; 6e-7 <= 1e-3: keep; 0.06 > 2.99e-3: fall back
    assert list(fb) == [False, False, True]
