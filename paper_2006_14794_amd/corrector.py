"""Learned corrector: bindings and the training driver.

The network, its features, loss, gradients and optimiser all run in
libsigkernel's HIP kernels (``sigkernel_corrector_*``, ``sigkernel_adam_step``,
``sigkernel_channel_stats``); this module allocates device buffers, slices
batches (contiguous views, no copies) and loops over them.  The order-3
targets are the plain scheme itself (``sigkernel_pair`` at dyadic order 3),
which also serves as the fallback of :meth:`Corrector.predict`.

Random initial weights are drawn on the host from a seeded NumPy generator
and uploaded (He-normal weights, zero biases).
"""
from __future__ import annotations

import ctypes
import math
import time
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

from . import _lib
from .api import _describe, _stream_ptr, sigkernel_pair

# Fallback margin on the predicted error.  calibrate_kappa on 65536
# calibration pairs (seed 14797, disjoint from the training and held-out
# seeds) gives 3.75 for tol 1e-3 (10 % of the pairs fall back); the default
# takes the next quarter step.  An empirical margin, not a bound: the error
# head is a prediction.
KAPPA = 4.0

CIN = (8, 32, 32, 32)
COUT = 32
FEAT_FLOATS = 64 * 64 * 8


def param_count() -> int:
    return int(_lib.load().sigkernel_corrector_param_count())


def act_elems() -> int:
    return int(_lib.load().sigkernel_corrector_act_elems())


def init_params(seed: int) -> np.ndarray:
    """He-normal conv and head weights, zero biases (float32 host vector)."""
    rng = np.random.default_rng(seed)
    parts = []
    for cin in CIN:
        fan_in = 9 * cin
        parts.append(rng.normal(size=COUT * 9 * cin) * math.sqrt(2.0 / fan_in))
        parts.append(np.zeros(COUT))
    parts.append(rng.normal(size=2 * 512) * math.sqrt(1.0 / 512))
    parts.append(np.zeros(2))
    theta = np.concatenate(parts).astype(np.float32)
    assert theta.size == param_count()
    return theta


def _ptr(t: Optional[torch.Tensor]):
    return t.data_ptr() if t is not None else None


def _slice(X: torch.Tensor, a: int, b: int) -> torch.Tensor:
    return X[a:b]  # a contiguous view of a [n, L, d] contiguous tensor


def features(X: torch.Tensor, Y: torch.Tensor, norm: Optional[torch.Tensor] = None,
             feats: Optional[torch.Tensor] = None, k0: Optional[torch.Tensor] = None,
             workspace: Optional[torch.Tensor] = None):
    """(feats [n, 64, 64, 8] bf16, k0 [n]) of the pairs (X_k, Y_k)."""
    lib = _lib.load()
    n = int(X.shape[0])
    sx, sy = _describe(X), _describe(Y)
    if feats is None:
        feats = torch.empty((n, 64, 64, 8), dtype=torch.bfloat16, device=X.device)
    if k0 is None:
        k0 = torch.empty(n, dtype=torch.float32, device=X.device)
    nbytes = int(lib.sigkernel_workspace_bytes(_lib.SK_OP_CORRECTOR_FEATURES, ctypes.byref(sx),
                                               ctypes.byref(sy), 0, 0))
    ws = workspace if workspace is not None else torch.empty(max(nbytes, 256), dtype=torch.uint8,
                                                             device=X.device)
    _lib.check(lib.sigkernel_corrector_features(ctypes.byref(sx), ctypes.byref(sy), _ptr(norm),
                                                _ptr(feats), _ptr(k0), ws.data_ptr(), ws.numel(),
                                                _stream_ptr(X.device)),
               "sigkernel_corrector_features")
    return feats, k0


def forward(params: torch.Tensor, feats: torch.Tensor, acts: Optional[torch.Tensor] = None,
            y: Optional[torch.Tensor] = None):
    """(acts bf16, y [n, 2])."""
    n = int(feats.shape[0])
    dev = feats.device
    if acts is None:
        acts = torch.empty(n * act_elems(), dtype=torch.bfloat16, device=dev)
    if y is None:
        y = torch.empty((n, 2), dtype=torch.float32, device=dev)
    _lib.check(_lib.load().sigkernel_corrector_forward(params.data_ptr(), feats.data_ptr(), n,
                                                       acts.data_ptr(), y.data_ptr(),
                                                       _stream_ptr(dev)),
               "sigkernel_corrector_forward")
    return acts, y


def backward_workspace_bytes(n: int) -> int:
    lib = _lib.load()
    sx = _lib.SkPaths(None, None, int(n), 1, 1)
    return int(lib.sigkernel_workspace_bytes(_lib.SK_OP_CORRECTOR_BACKWARD, ctypes.byref(sx),
                                             ctypes.byref(sx), 0, 0))


def backward(params, feats, acts, dy, grads: Optional[torch.Tensor] = None,
             workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    n = int(feats.shape[0])
    dev = feats.device
    if grads is None:
        grads = torch.empty_like(params)
    if workspace is None:
        workspace = torch.empty(backward_workspace_bytes(n), dtype=torch.uint8, device=dev)
    _lib.check(_lib.load().sigkernel_corrector_backward(
        params.data_ptr(), feats.data_ptr(), acts.data_ptr(), dy.data_ptr(), n, grads.data_ptr(),
        workspace.data_ptr(), workspace.numel(), _stream_ptr(dev)), "sigkernel_corrector_backward")
    return grads


def loss(y, k_target, k0, target_norm, out_loss=None, dy=None):
    """(loss [1], dy [n, 2])."""
    n = int(y.shape[0])
    dev = y.device
    if out_loss is None:
        out_loss = torch.empty(1, dtype=torch.float32, device=dev)
    if dy is None:
        dy = torch.empty_like(y)
    _lib.check(_lib.load().sigkernel_corrector_loss(y.data_ptr(), k_target.data_ptr(),
                                                    k0.data_ptr(), target_norm.data_ptr(), n,
                                                    out_loss.data_ptr(), dy.data_ptr(),
                                                    _stream_ptr(dev)), "sigkernel_corrector_loss")
    return out_loss, dy


def adam_step(params, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    _lib.check(_lib.load().sigkernel_adam_step(params.data_ptr(), grads.data_ptr(), m.data_ptr(),
                                               v.data_ptr(), params.numel(), step.data_ptr(),
                                               float(lr), float(beta1), float(beta2), float(eps),
                                               _stream_ptr(params.device)), "sigkernel_adam_step")


def channel_stats(x: torch.Tensor, channels: int, sub: Optional[torch.Tensor] = None):
    """(mean [C], rstd [C]) over the rows of x viewed as [rows, C] (of x - sub)."""
    dev = x.device
    rows = x.numel() // channels
    mean = torch.empty(channels, dtype=torch.float32, device=dev)
    rstd = torch.empty(channels, dtype=torch.float32, device=dev)
    ws = torch.empty(_lib.SK_CHANNEL_STATS_WORKSPACE_BYTES, dtype=torch.uint8, device=dev)
    if x.dtype not in (torch.float32, torch.bfloat16):
        raise TypeError("channel_stats reads float32 or bfloat16")
    dt = 1 if x.dtype == torch.bfloat16 else 0
    _lib.check(_lib.load().sigkernel_channel_stats(x.data_ptr(), dt, _ptr(sub), rows, channels,
                                                   mean.data_ptr(), rstd.data_ptr(),
                                                   ws.data_ptr(), ws.numel(), _stream_ptr(dev)),
               "sigkernel_channel_stats")
    return mean, rstd


@dataclass
class Corrector:
    """Parameters and normalisation constants of a corrector (device tensors):
    params [P], norm [16] (feature mean and 1/std), target_norm [2] (mean and
    std of the order-3 minus order-0 difference)."""
    params: torch.Tensor
    norm: torch.Tensor
    target_norm: torch.Tensor
    meta: dict = field(default_factory=dict)

    # ---- persistence (plain arrays; no pickled objects) ----
    def save(self, path: str) -> None:
        np.savez(path, params=self.params.cpu().numpy(), norm=self.norm.cpu().numpy(),
                 target_norm=self.target_norm.cpu().numpy(),
                 meta_keys=np.array(list(self.meta.keys()), dtype=np.str_),
                 meta_vals=np.array([str(v) for v in self.meta.values()], dtype=np.str_))

    @staticmethod
    def load(path: str, device="cuda") -> "Corrector":
        with np.load(path, allow_pickle=False) as z:
            meta = dict(zip(z["meta_keys"].tolist(), z["meta_vals"].tolist()))
            return Corrector(torch.from_numpy(z["params"]).to(device),
                             torch.from_numpy(z["norm"]).to(device),
                             torch.from_numpy(z["target_norm"]).to(device), meta)

    def predict(self, X: torch.Tensor, Y: torch.Tensor, *, fallback_order: int = 3,
                kappa: float = KAPPA, tol: float = 1e-3, chunk: int = 16384):
        """(k_hat [n], predicted error [n], fallback [n] int32): corrected
        order-3 values; pairs other than those with kappa * error <= tol *
        |k_hat| get the plain solve at ``fallback_order`` on the device."""
        lib = _lib.load()
        n = int(X.shape[0])
        dev = X.device
        out = torch.empty(n, dtype=torch.float32, device=dev)
        err = torch.empty(n, dtype=torch.float32, device=dev)
        fb = torch.empty(n, dtype=torch.int32, device=dev)
        ws = None
        for a in range(0, n, chunk):
            b = min(n, a + chunk)
            Xa, Ya = _slice(X, a, b), _slice(Y, a, b)
            sx, sy = _describe(Xa), _describe(Ya)
            nbytes = int(lib.sigkernel_workspace_bytes(_lib.SK_OP_CORRECTOR_PREDICT,
                                                       ctypes.byref(sx), ctypes.byref(sy),
                                                       fallback_order, 0))
            if ws is None or ws.numel() < nbytes:
                ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
            _lib.check(lib.sigkernel_corrector_predict(
                ctypes.byref(sx), ctypes.byref(sy), int(fallback_order), self.params.data_ptr(),
                self.norm.data_ptr(), self.target_norm.data_ptr(), float(kappa), float(tol),
                out[a:b].data_ptr(), err[a:b].data_ptr(), fb[a:b].data_ptr(), ws.data_ptr(),
                ws.numel(), _stream_ptr(dev)), "sigkernel_corrector_predict")
        return out, err, fb


def calibrate_kappa(model: "Corrector", X: torch.Tensor, Y: torch.Tensor,
                    k_ref: torch.Tensor, tol: float = 1e-3, grid=None):
    """(kappa, fallback fraction, max accepted relative error): the smallest
    kappa of ``grid`` whose accepted pairs all have |k_hat - k_ref| <= tol
    |k_ref| (k_ref: the plain order-3 values of the pairs)."""
    raw, err, _ = model.predict(X, Y, tol=float("inf"), chunk=int(X.shape[0]))
    k = raw.double()
    rel = (k - k_ref.double()).abs() / k_ref.double().abs()
    grid = grid if grid is not None else [1.0 + 0.25 * i for i in range(37)]
    for kappa in grid:
        acc = kappa * err.double() <= tol * k.abs()
        worst = float(rel[acc].max()) if bool(acc.any()) else 0.0
        if worst <= tol:
            return kappa, float(1.0 - acc.double().mean()), worst
    return float("inf"), 1.0, 0.0


def order3_targets(X: torch.Tensor, Y: torch.Tensor, order: int = 3, chunk: int = 16384):
    """The plain scheme at ``order`` for every pair: the training targets."""
    out = torch.empty(int(X.shape[0]), dtype=torch.float32, device=X.device)
    for a in range(0, int(X.shape[0]), chunk):
        b = min(int(X.shape[0]), a + chunk)
        sigkernel_pair(_slice(X, a, b), _slice(Y, a, b), order, out=out[a:b])
    return out


def fit_normalisation(X, Y, k_target, n_stats: int = 4096):
    """Feature and target normalisation constants from the training pairs."""
    dev = X.device
    n = int(X.shape[0])
    ns = min(n, n_stats)
    feats, _ = features(_slice(X, 0, ns), _slice(Y, 0, ns))  # raw moments, bf16
    fmean, frstd = channel_stats(feats, 8)
    del feats
    k0 = torch.empty(n, dtype=torch.float32, device=dev)
    chunk = 4096
    fbuf = torch.empty((chunk, 64, 64, 8), dtype=torch.bfloat16, device=dev)
    for a in range(0, n, chunk):
        b = min(n, a + chunk)
        features(_slice(X, a, b), _slice(Y, a, b), None, fbuf[:b - a], k0[a:b])
    tmean, trstd = channel_stats(k_target, 1, sub=k0)
    # a handful of constants: assembled on the host, uploaded once
    norm = np.concatenate([fmean.cpu().numpy(), frstd.cpu().numpy()]).astype(np.float32)
    tnorm = np.array([float(tmean[0]), 1.0 / float(trstd[0])], np.float32)  # (mu, sigma)
    return torch.from_numpy(norm).to(dev), torch.from_numpy(tnorm).to(dev), k0


def train(X: torch.Tensor, Y: torch.Tensor, k_target: torch.Tensor, *, epochs: int = 10,
          batch: int = 256, lr: float = 2e-3, lr_final: float = 1e-4, seed: int = 0,
          log_every: int = 200, log=print, corrector: Optional[Corrector] = None) -> Corrector:
    """Train (or continue training) a corrector on pairs (X_k, Y_k) with
    targets k_target (the plain order-3 values) by Adam, cosine learning-rate
    decay, contiguous batches whose boundaries shift every epoch."""
    dev = X.device
    n = int(X.shape[0])
    if corrector is None:
        norm, tnorm, _ = fit_normalisation(X, Y, k_target)
        corrector = Corrector(torch.from_numpy(init_params(seed)).to(dev), norm, tnorm,
                              {"seed": seed})
    P = corrector.params.numel()
    grads = torch.empty(P, dtype=torch.float32, device=dev)
    m = torch.zeros(P, dtype=torch.float32, device=dev)
    v = torch.zeros(P, dtype=torch.float32, device=dev)
    step = torch.zeros(1, dtype=torch.int32, device=dev)
    feats = torch.empty((batch, 64, 64, 8), dtype=torch.bfloat16, device=dev)
    k0 = torch.empty(batch, dtype=torch.float32, device=dev)
    acts = torch.empty(batch * act_elems(), dtype=torch.bfloat16, device=dev)
    y = torch.empty((batch, 2), dtype=torch.float32, device=dev)
    dy = torch.empty((batch, 2), dtype=torch.float32, device=dev)
    lbuf = torch.empty(1, dtype=torch.float32, device=dev)
    sb = _describe(_slice(X, 0, min(n, batch)))
    fws = torch.empty(max(256, int(_lib.load().sigkernel_workspace_bytes(
        _lib.SK_OP_CORRECTOR_FEATURES, ctypes.byref(sb), ctypes.byref(sb), 0, 0))),
        dtype=torch.uint8, device=dev)
    bws = torch.empty(backward_workspace_bytes(batch), dtype=torch.uint8, device=dev)
    steps_per_epoch = max(1, n // batch)
    total = epochs * steps_per_epoch
    history = []
    t0 = time.time()
    it = 0
    for ep in range(epochs):
        shift = (ep * batch // max(epochs, 1)) % batch if n > batch else 0
        for s in range(steps_per_epoch):
            a = shift + s * batch
            b = min(n, a + batch)
            if b - a < batch:  # the shifted last batch wraps: skip it
                continue
            Xb, Yb = _slice(X, a, b), _slice(Y, a, b)
            features(Xb, Yb, corrector.norm, feats, k0, fws)
            forward(corrector.params, feats, acts, y)
            loss(y, k_target[a:b], k0, corrector.target_norm, lbuf, dy)
            backward(corrector.params, feats, acts, dy, grads, bws)
            frac = it / max(total - 1, 1)
            lr_t = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * frac))
            adam_step(corrector.params, grads, m, v, step, lr_t)
            it += 1
            if log_every and (it % log_every == 0 or it == total):
                lv = float(lbuf.item())
                history.append((it, lv))
                if log:
                    log(f"step {it}/{total} epoch {ep} loss {lv:.4f} lr {lr_t:.2e} "
                        f"{time.time() - t0:.1f}s")
    corrector.meta.update({"epochs": epochs, "batch": batch, "lr": lr, "pairs": n,
                           "steps": it, "train_seconds": round(time.time() - t0, 2)})
    corrector.meta["history"] = ";".join(f"{i}:{l:.5f}" for i, l in history)
    return corrector
