"""FP64 CPU oracle of the learned corrector (test infrastructure only).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: imported by ``tests/``
and never by the product path, with which it shares no code.

The paper has no learned component.  The corrector is this project's own: a
small convolutional network that maps what the explicit scheme of Section 3.1
computes at dyadic order 0 (the coarse increment inner products and the node
values of the order-0 grid) to the order-3 terminal value, with the plain
order-3 solve as its fallback and the judge of its error.  What is pinned here
is therefore not a passage of the paper but the network's own definition,
written out plainly:

* ``block_features``: eight channels per 4 x 4 block of coarse cells of the
  order-0 grid (cell (p, q) has corners C = K[p][q], A = K[p+1][q],
  B = K[p][q+1] and coefficient c = <x_{p+1} - x_p, y_{q+1} - y_q>):
    0: sum c            1: sum c^2 (A + B) / 2     2: sum c (A + B)
    3: sum (C - 1)      4: sum c^2 C               5: sum c (B - A)
    6: P / 63           7: Q / 63                  (block row / column)
  over the cells of block (P, Q) that lie in the grid (64 x 64 blocks; blocks
  and cells outside the grid contribute 0 to channels 0-5);
* ``conv_forward`` / ``conv_backward``: 3 x 3 convolution, stride 2, zero
  padding 1, NHWC activations and [Cout][3][3][Cin] weights, whose weights and
  input activations are rounded to bfloat16 (round to nearest even) before
  the products, as the matrix-core kernels consume them; products and sums
  are exact here (FP64).  The backward is the chain rule through the rounded
  operands (the rounding itself is passed straight through);
* ``network_forward`` / ``network_backward``: four such layers with ReLU
  (32 channels each), then a dense head 512 -> 2 whose input activations are
  rounded to bfloat16 like every layer's (its weights stay float32); the
  network therefore only ever reads bfloat16 activations, and the features
  it reads are ``bf16_round(normalise(block_features))``;
* ``loss_and_grad``: squared error of output 0 against the normalised target,
  plus the Gaussian negative log-likelihood of that (detached) residual under
  the predicted log-scale output 1;
* ``adam_step``: Adam with bias correction;
* ``decide``: corrected value k0 + mu + sigma * y0, predicted error
  sigma * exp(y1), fallback when kappa times that error exceeds
  tol * max(1, |k_hat|).
"""
from __future__ import annotations

import numpy as np

CIN = (8, 32, 32, 32)
COUT = 32
N_FEAT = 8
GRID_BLOCKS = 64  # feature map side: 64 blocks of 4 coarse cells


def param_layout():
    """[(name, shape)] of the flat parameter vector, in order."""
    out = []
    for i, cin in enumerate(CIN):
        out.append((f"w{i + 1}", (COUT, 3, 3, cin)))
        out.append((f"b{i + 1}", (COUT,)))
    out.append(("wh", (2, 4 * 4 * COUT)))
    out.append(("bh", (2,)))
    return out


def n_params() -> int:
    return int(sum(np.prod(s) for _, s in param_layout()))


def unflatten(theta: np.ndarray) -> dict:
    p, off = {}, 0
    for name, shape in param_layout():
        n = int(np.prod(shape))
        p[name] = np.asarray(theta[off:off + n], np.float64).reshape(shape)
        off += n
    return p


def flatten(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], np.float64).reshape(-1)
                           for name, _ in param_layout()])


def bf16_round(x) -> np.ndarray:
    """float32 -> nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = ((u + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


# ---- features --------------------------------------------------------------
def block_features(K: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Raw features [64, 64, 8] (NHWC) of one pair from its order-0 grid K
    ((m+1) x (n+1) nodes) and coarse coefficients c (m x n), m, n <= 256."""
    m, n = c.shape
    assert K.shape == (m + 1, n + 1) and m <= 256 and n <= 256
    C = K[:-1, :-1]
    A = K[1:, :-1]
    B = K[:-1, 1:]
    cell = np.stack([c, c * c * (A + B) / 2, c * (A + B), C - 1.0, c * c * C, c * (B - A)], -1)
    pad = np.zeros((256, 256, 6))
    pad[:m, :n] = cell
    out = np.zeros((GRID_BLOCKS, GRID_BLOCKS, N_FEAT))
    out[:, :, :6] = pad.reshape(64, 4, 64, 4, 6).sum(axis=(1, 3))
    P, Q = np.meshgrid(np.arange(64), np.arange(64), indexing="ij")
    out[:, :, 6] = P / 63.0
    out[:, :, 7] = Q / 63.0
    return out


def normalise(f: np.ndarray, mean, rstd) -> np.ndarray:
    return (f - np.asarray(mean, np.float64)) * np.asarray(rstd, np.float64)


def channel_stats(a: np.ndarray):
    """Per-channel (last axis) mean and 1 / standard deviation (population);
    a channel with zero variance gets 1."""
    a = np.asarray(a, np.float64).reshape(-1, a.shape[-1])
    mean = a.mean(axis=0)
    var = ((a - mean) ** 2).mean(axis=0)
    rstd = np.where(var > 0, 1.0 / np.sqrt(np.where(var > 0, var, 1.0)), 1.0)
    return mean, rstd


# ---- convolution -----------------------------------------------------------
def _padded(x):
    n, h, w, c = x.shape
    xp = np.zeros((n, h + 2, w + 2, c))
    xp[:, 1:h + 1, 1:w + 1] = x
    return xp


def _rnd(a, rounding):
    return bf16_round(a) if rounding else np.asarray(a, np.float64)


def conv_forward(x: np.ndarray, w: np.ndarray, b: np.ndarray, rounding: bool = True):
    """Pre-activation of one layer: x [N, H, W, Cin] -> [N, H/2, W/2, Cout].
    ``rounding=False`` skips the bfloat16 rounding (finite-difference pins)."""
    xr = _rnd(x, rounding)
    wr = _rnd(w, rounding)
    n, h, wd, _ = x.shape
    ho, wo = (h + 1) // 2, (wd + 1) // 2
    xp = _padded(xr)
    out = np.broadcast_to(np.asarray(b, np.float64), (n, ho, wo, w.shape[0])).copy()
    for kh in range(3):
        for kw in range(3):
            # input row 2 ho - 1 + kh is padded row 2 ho + kh
            patch = xp[:, kh:kh + 2 * ho:2, kw:kw + 2 * wo:2, :]
            out += np.tensordot(patch, wr[:, kh, kw, :], axes=([3], [1]))
    return out


def conv_backward(x: np.ndarray, w: np.ndarray, dpre: np.ndarray, need_dx: bool = True,
                  rounding: bool = True):
    """(dx, dw, db) of one layer given the gradient of its pre-activation."""
    xr = _rnd(x, rounding)
    wr = _rnd(w, rounding)
    n, h, wd, cin = x.shape
    ho, wo = dpre.shape[1], dpre.shape[2]
    xp = _padded(xr)
    dw = np.zeros(w.shape)
    dxp = np.zeros_like(xp)
    for kh in range(3):
        for kw in range(3):
            patch = xp[:, kh:kh + 2 * ho:2, kw:kw + 2 * wo:2, :]
            dw[:, kh, kw, :] = np.tensordot(dpre, patch, axes=([0, 1, 2], [0, 1, 2]))
            if need_dx:
                dxp[:, kh:kh + 2 * ho:2, kw:kw + 2 * wo:2, :] += np.tensordot(
                    dpre, wr[:, kh, kw, :], axes=([3], [0]))
    db = dpre.sum(axis=(0, 1, 2))
    dx = dxp[:, 1:h + 1, 1:wd + 1, :] if need_dx else None
    return dx, dw, db


# ---- network ---------------------------------------------------------------
def network_forward(theta: np.ndarray, feats: np.ndarray, rounding: bool = True):
    """(y [N, 2], cache): four conv + ReLU layers, then the dense head over
    the flattened [4, 4, 32] map (NHWC order)."""
    p = unflatten(theta)
    acts, pres = [np.asarray(feats, np.float64)], []
    for i in range(4):
        pre = conv_forward(acts[-1], p[f"w{i + 1}"], p[f"b{i + 1}"], rounding)
        pres.append(pre)
        acts.append(np.maximum(pre, 0.0))
    flat = _rnd(acts[-1].reshape(acts[-1].shape[0], -1), rounding)
    y = flat @ p["wh"].T + p["bh"]
    return y, (acts, pres, flat, rounding)


def network_backward(theta: np.ndarray, cache, dy: np.ndarray) -> np.ndarray:
    """Gradient of sum(dy * y) with respect to the flat parameters."""
    p = unflatten(theta)
    acts, pres, flat, rounding = cache
    g = {"wh": dy.T @ flat, "bh": dy.sum(axis=0)}
    da = (dy @ p["wh"]).reshape(acts[-1].shape)
    for i in range(3, -1, -1):
        dpre = da * (pres[i] > 0)
        dx, dw, db = conv_backward(acts[i], p[f"w{i + 1}"], dpre, i > 0, rounding)
        g[f"w{i + 1}"], g[f"b{i + 1}"] = dw, db
        da = dx
    return flatten(g)


def loss_and_grad(y: np.ndarray, target: np.ndarray):
    """(mean loss, dL/dy) with L_i = r^2 + (r_d^2 exp(-2 s) / 2 + s), r = y0 - t,
    s = y1 and r_d the residual with its gradient stopped."""
    y = np.asarray(y, np.float64)
    r = y[:, 0] - np.asarray(target, np.float64)
    s = y[:, 1]
    e = np.exp(-2.0 * s)
    n = y.shape[0]
    loss = float(np.mean(r * r + 0.5 * r * r * e + s))
    dy = np.stack([2.0 * r / n, (1.0 - r * r * e) / n], -1)
    return loss, dy


def adam_step(theta, grad, m, v, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (step t >= 1); returns new (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def decide(k0, y, mu: float, sigma: float, kappa: float, tol: float):
    """(k_hat, predicted error, fallback mask)."""
    y = np.asarray(y, np.float64)
    k_hat = np.asarray(k0, np.float64) + mu + sigma * y[:, 0]
    err = sigma * np.exp(y[:, 1])
    fallback = kappa * err > tol * np.maximum(1.0, np.abs(k_hat))
    return k_hat, err, fallback
