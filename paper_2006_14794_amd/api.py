"""Torch-facing wrappers of the C ABI (same names as the C entry points).

PyTorch supplies device memory and the current HIP stream; every step of the
computation runs in libsigkernel's HIP kernels.  Inputs are float32 CUDA (HIP)
tensors:

* a uniform batch is a contiguous ``[n_paths, len, dim]`` tensor;
* a ragged batch is a :class:`RaggedPaths` (``points [total, dim]``, device
  ``offsets [n_paths + 1]`` int64, and an upper bound ``max_len``).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Union

import torch

from . import _lib
from ._lib import SkPaths


@dataclass
class RaggedPaths:
    points: torch.Tensor   # [total, dim] float32, device
    offsets: torch.Tensor  # [n_paths + 1] int64, device
    max_len: int

    @staticmethod
    def from_list(paths, device) -> "RaggedPaths":
        lens = [int(p.shape[0]) for p in paths]
        off = [0]
        for L in lens:
            off.append(off[-1] + L)
        pts = torch.cat([torch.as_tensor(p, dtype=torch.float32) for p in paths], 0)
        return RaggedPaths(pts.to(device).contiguous(),
                           torch.tensor(off, dtype=torch.int64, device=device),
                           max(lens) if lens else 1)

    @property
    def n_paths(self) -> int:
        return int(self.offsets.numel()) - 1

    @property
    def dim(self) -> int:
        return int(self.points.shape[1])


PathsLike = Union[torch.Tensor, RaggedPaths]


def _describe(p: PathsLike) -> SkPaths:
    if isinstance(p, RaggedPaths):
        if p.points.dtype != torch.float32 or not p.points.is_cuda:
            raise TypeError("ragged points must be a float32 device tensor")
        if p.offsets.dtype != torch.int64 or not p.offsets.is_cuda:
            raise TypeError("offsets must be an int64 device tensor")
        if not p.points.is_contiguous() or not p.offsets.is_contiguous():
            raise ValueError("ragged tensors must be contiguous")
        return SkPaths(p.points.data_ptr(), p.offsets.data_ptr(), p.n_paths,
                       int(p.max_len), p.dim)
    if not isinstance(p, torch.Tensor) or p.dim() != 3:
        raise TypeError("expected a [n_paths, len, dim] tensor or RaggedPaths")
    if p.dtype != torch.float32 or not p.is_cuda:
        raise TypeError("paths must be a float32 device tensor")
    if not p.is_contiguous():
        raise ValueError("paths must be contiguous")
    return SkPaths(p.data_ptr() if p.numel() else 0, None, int(p.shape[0]),
                   int(p.shape[1]), int(p.shape[2]))


def _device(p: PathsLike) -> torch.device:
    return p.points.device if isinstance(p, RaggedPaths) else p.device


def _n_paths(p: PathsLike) -> int:
    return p.n_paths if isinstance(p, RaggedPaths) else int(p.shape[0])


def _stream_ptr(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def workspace_bytes(op: int, X: PathsLike, Y: PathsLike, dyadic_order: int,
                    flags: int = 0) -> int:
    lib = _lib.load()
    sx, sy = _describe(X), _describe(Y)
    return int(lib.sigkernel_workspace_bytes(op, ctypes.byref(sx), ctypes.byref(sy),
                                             int(dyadic_order), int(flags)))


def _workspace(nbytes: int, device, ws: Optional[torch.Tensor]) -> torch.Tensor:
    if ws is not None:
        if ws.numel() * ws.element_size() < nbytes:
            raise ValueError("workspace too small")
        return ws
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


_GRAM_PRECISION = {"f32": 0, "bf16": _lib.SK_GRAM_BF16, "f16": _lib.SK_GRAM_F16}


def _gram_flag(gram_precision: str) -> int:
    if gram_precision not in _GRAM_PRECISION:
        raise ValueError("gram_precision must be 'f32', 'bf16' or 'f16'")
    return _GRAM_PRECISION[gram_precision]


def _scheme_flag(scheme: str) -> int:
    if scheme not in ("explicit", "implicit"):
        raise ValueError("scheme must be 'explicit' or 'implicit'")
    return _lib.SK_IMPLICIT if scheme == "implicit" else 0


def sigkernel_pair(x: PathsLike, y: PathsLike, dyadic_order: int = 0, *,
                   gram_precision: str = "f32", scheme: str = "explicit",
                   out: Optional[torch.Tensor] = None,
                   workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """out[k] = k_hat(x_k, y_k) of the explicit (or, with scheme='implicit',
    the implicit) scheme on P_lambda.  ``gram_precision`` 'bf16' / 'f16'
    rounds the increments to 16 bits before their inner products (float32
    accumulation)."""
    lib = _lib.load()
    dev = _device(x)
    n = _n_paths(x)
    flags = _gram_flag(gram_precision) | _scheme_flag(scheme)
    sx, sy = _describe(x), _describe(y)
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=dev)
    nbytes = int(lib.sigkernel_workspace_bytes(_lib.SK_OP_PAIR, ctypes.byref(sx),
                                               ctypes.byref(sy), dyadic_order, flags))
    ws = _workspace(nbytes, dev, workspace)
    st = lib.sigkernel_pair(ctypes.byref(sx), ctypes.byref(sy), int(dyadic_order), flags,
                            out.data_ptr() if n else None, ws.data_ptr(),
                            ws.numel() * ws.element_size(), _stream_ptr(dev))
    _lib.check(st, "sigkernel_pair")
    return out


def sigkernel_gram(X: PathsLike, Y: Optional[PathsLike] = None, dyadic_order: int = 0, *,
                   symmetric: bool = False, no_diag: bool = False,
                   gram_precision: str = "f32", scheme: str = "explicit",
                   out: Optional[torch.Tensor] = None,
                   workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """K[a, b] = k_hat(X_a, Y_b).  ``symmetric=True`` (Y omitted or X itself)
    solves a <= b only and mirrors; ``no_diag`` then writes 0 on the diagonal."""
    lib = _lib.load()
    if Y is None:
        Y = X
    if symmetric and Y is not X:
        raise ValueError("symmetric Gram needs Y to be X")
    dev = _device(X)
    nx, ny = _n_paths(X), _n_paths(Y)
    flags = _gram_flag(gram_precision) | _scheme_flag(scheme)
    if symmetric:
        flags |= _lib.SK_SYMMETRIC
        if no_diag:
            flags |= _lib.SK_NO_DIAG
    elif no_diag:
        raise ValueError("no_diag needs symmetric=True")
    sx, sy = _describe(X), _describe(Y)
    if out is None:
        out = torch.empty((nx, ny), dtype=torch.float32, device=dev)
    nbytes = int(lib.sigkernel_workspace_bytes(_lib.SK_OP_GRAM, ctypes.byref(sx),
                                               ctypes.byref(sy), dyadic_order, flags))
    ws = _workspace(nbytes, dev, workspace)
    st = lib.sigkernel_gram(ctypes.byref(sx), ctypes.byref(sy), int(dyadic_order), flags,
                            out.data_ptr() if out.numel() else None, ws.data_ptr(),
                            ws.numel() * ws.element_size(), _stream_ptr(dev))
    _lib.check(st, "sigkernel_gram")
    return out


def _static_kernel(kernel: str, sigma: float):
    if kernel == "rbf":
        if not (sigma > 0):
            raise ValueError("the RBF bandwidth sigma must be positive")
        return _lib.SkStaticKernel(_lib.SK_STATIC_RBF, 0, float(sigma))
    if kernel == "linear":
        return _lib.SkStaticKernel(_lib.SK_STATIC_LINEAR, 0, 0.0)
    raise ValueError("kernel must be 'rbf' or 'linear'")


def sigkernel_pair_lifted(x: PathsLike, y: PathsLike, dyadic_order: int = 0, *,
                          kernel: str = "rbf", sigma: float = 1.0, scheme: str = "explicit",
                          out: Optional[torch.Tensor] = None,
                          workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """out[k] = signature kernel of the lifted pair (x_k, y_k): the scheme on
    P_lambda with the coarse coefficients replaced by second differences of
    the static kernel ('rbf': exp(-|a - b|^2 / (2 sigma^2)); 'linear': the
    plain kernel)."""
    lib = _lib.load()
    dev = _device(x)
    n = _n_paths(x)
    flags = _scheme_flag(scheme)
    sk_ = _static_kernel(kernel, sigma)
    sx, sy = _describe(x), _describe(y)
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=dev)
    nbytes = int(lib.sigkernel_workspace_bytes(_lib.SK_OP_PAIR_LIFTED, ctypes.byref(sx),
                                               ctypes.byref(sy), dyadic_order, flags))
    ws = _workspace(nbytes, dev, workspace)
    st = lib.sigkernel_pair_lifted(ctypes.byref(sx), ctypes.byref(sy), int(dyadic_order), flags,
                                   ctypes.byref(sk_), out.data_ptr() if n else None,
                                   ws.data_ptr(), ws.numel() * ws.element_size(),
                                   _stream_ptr(dev))
    _lib.check(st, "sigkernel_pair_lifted")
    return out


def sigkernel_gram_lifted(X: PathsLike, Y: Optional[PathsLike] = None, dyadic_order: int = 0,
                          *, kernel: str = "rbf", sigma: float = 1.0, symmetric: bool = False,
                          no_diag: bool = False, scheme: str = "explicit",
                          out: Optional[torch.Tensor] = None,
                          workspace: Optional[torch.Tensor] = None) -> torch.Tensor:
    """K[a, b] = lifted signature kernel of (X_a, Y_b) (see
    ``sigkernel_pair_lifted``); ``symmetric`` / ``no_diag`` as in
    ``sigkernel_gram``."""
    lib = _lib.load()
    if Y is None:
        Y = X
    if symmetric and Y is not X:
        raise ValueError("symmetric Gram needs Y to be X")
    if no_diag and not symmetric:
        raise ValueError("no_diag needs symmetric=True")
    dev = _device(X)
    nx, ny = _n_paths(X), _n_paths(Y)
    flags = _scheme_flag(scheme)
    if symmetric:
        flags |= _lib.SK_SYMMETRIC | (_lib.SK_NO_DIAG if no_diag else 0)
    sk_ = _static_kernel(kernel, sigma)
    sx, sy = _describe(X), _describe(Y)
    if out is None:
        out = torch.empty((nx, ny), dtype=torch.float32, device=dev)
    nbytes = int(lib.sigkernel_workspace_bytes(_lib.SK_OP_GRAM_LIFTED, ctypes.byref(sx),
                                               ctypes.byref(sy), dyadic_order, flags))
    ws = _workspace(nbytes, dev, workspace)
    st = lib.sigkernel_gram_lifted(ctypes.byref(sx), ctypes.byref(sy), int(dyadic_order), flags,
                                   ctypes.byref(sk_), out.data_ptr() if out.numel() else None,
                                   ws.data_ptr(), ws.numel() * ws.element_size(),
                                   _stream_ptr(dev))
    _lib.check(st, "sigkernel_gram_lifted")
    return out


def _reduce_inputs(K: torch.Tensor, alpha: Optional[torch.Tensor]):
    if K.dim() != 2 or K.shape[0] != K.shape[1] or not K.is_cuda:
        raise ValueError("K must be a square device tensor")
    K = K.to(torch.float32).contiguous()
    n = K.shape[0]
    if alpha is None:
        alpha = torch.full((n,), 1.0 / n, dtype=torch.float32, device=K.device)
    alpha = alpha.to(device=K.device, dtype=torch.float32).contiguous()
    if alpha.numel() != n:
        raise ValueError("alpha must have one weight per row of K")
    return K, alpha, n


def reduced_measure(K: torch.Tensor, lam: float, iters: int, *,
                    alpha: Optional[torch.Tensor] = None, step: float = 0.0):
    """(beta, loss, step): `iters` proximal-gradient iterations of eq.
    (fixed_point) for eq. (min_lasso) from beta = alpha (default uniform
    weights), on the GPU.  loss[k] is the objective before iteration k and
    after the last; step 0 chooses 1 / (2 * 1.05 * |K|_2)."""
    lib = _lib.load()
    K, alpha, n = _reduce_inputs(K, alpha)
    beta = torch.empty(n, dtype=torch.float64, device=K.device)
    loss = torch.empty(iters + 1, dtype=torch.float64, device=K.device)
    step_out = torch.empty(1, dtype=torch.float64, device=K.device)
    st = lib.sigkernel_reduced_measure(K.data_ptr(), alpha.data_ptr(), n, float(lam),
                                       float(step), int(iters), beta.data_ptr(), loss.data_ptr(),
                                       step_out.data_ptr(), _stream_ptr(K.device))
    _lib.check(st, "sigkernel_reduced_measure")
    return beta, loss, step_out


def reduced_measure_support(K: torch.Tensor, support: int, iters: int = 3000, rounds: int = 40,
                            *, alpha: Optional[torch.Tensor] = None, step: float = 0.0):
    """(beta, lam, step): the penalty found by bisection so that the reduced
    measure has `support` atoms, and its weights (GPU)."""
    lib = _lib.load()
    K, alpha, n = _reduce_inputs(K, alpha)
    beta = torch.empty(n, dtype=torch.float64, device=K.device)
    lam = torch.empty(1, dtype=torch.float64, device=K.device)
    step_out = torch.empty(1, dtype=torch.float64, device=K.device)
    st = lib.sigkernel_reduced_measure_support(K.data_ptr(), alpha.data_ptr(), n, int(support),
                                               int(iters), int(rounds), float(step),
                                               beta.data_ptr(), lam.data_ptr(),
                                               step_out.data_ptr(), _stream_ptr(K.device))
    _lib.check(st, "sigkernel_reduced_measure_support")
    return beta, lam, step_out


def _empty_points(P: PathsLike) -> torch.Tensor:
    """An uninitialised tensor shaped like the points of a batch ([n, len, d],
    or [total, d] for a ragged batch)."""
    return torch.empty_like(P.points if isinstance(P, RaggedPaths) else P)


def sigkernel_gram_backward(X: PathsLike, Y: Optional[PathsLike], dK: torch.Tensor,
                            dyadic_order: int = 0, *, symmetric: bool = False,
                            no_diag: bool = False, need_x: bool = True, need_y: bool = True,
                            workspace: Optional[torch.Tensor] = None):
    """(dX, dY) = gradients of sum(dK * K) with respect to the points of X and
    Y (either None when not wanted), shaped like their points (ragged batches:
    [total, d]).  With ``symmetric=True`` Y must be None or X itself and the
    whole gradient is returned as dX (dY is None)."""
    lib = _lib.load()
    if Y is None:
        Y = X
    if symmetric and Y is not X:
        raise ValueError("symmetric Gram needs Y to be X")
    if no_diag and not symmetric:
        raise ValueError("no_diag needs symmetric=True")
    dev = _device(X)
    flags = 0
    if symmetric:
        flags |= _lib.SK_SYMMETRIC | (_lib.SK_NO_DIAG if no_diag else 0)
        need_y = False
    sx, sy = _describe(X), _describe(Y)
    if dK.dtype != torch.float32 or not dK.is_cuda:
        raise TypeError("dK must be a float32 device tensor")
    dK = dK.contiguous()
    if dK.shape != (_n_paths(X), _n_paths(Y)):
        raise ValueError("dK must be [X.n_paths, Y.n_paths]")
    dX = _empty_points(X) if need_x else None
    dY = _empty_points(Y) if need_y else None
    nbytes = int(lib.sigkernel_workspace_bytes(_lib.SK_OP_GRAM_BACKWARD, ctypes.byref(sx),
                                               ctypes.byref(sy), int(dyadic_order), flags))
    ws = _workspace(nbytes, dev, workspace)
    st = lib.sigkernel_gram_backward(ctypes.byref(sx), ctypes.byref(sy), int(dyadic_order), flags,
                                     dK.data_ptr(), dX.data_ptr() if dX is not None else None,
                                     dY.data_ptr() if dY is not None else None, ws.data_ptr(),
                                     ws.numel() * ws.element_size(), _stream_ptr(dev))
    _lib.check(st, "sigkernel_gram_backward")
    return dX, dY


class SigKernelGram(torch.autograd.Function):
    """K = sigkernel_gram(X, Y); backward through sigkernel_gram_backward."""

    @staticmethod
    def forward(ctx, X, Y, dyadic_order):
        ctx.dyadic_order = dyadic_order
        ctx.save_for_backward(X, Y)
        return sigkernel_gram(X, Y, dyadic_order)

    @staticmethod
    def backward(ctx, dK):
        X, Y = ctx.saved_tensors
        dX, dY = sigkernel_gram_backward(X, Y, dK.to(torch.float32), ctx.dyadic_order,
                                         need_x=ctx.needs_input_grad[0],
                                         need_y=ctx.needs_input_grad[1])
        return dX, dY, None


class SigKernelGramSymmetric(torch.autograd.Function):
    """K = sigkernel_gram(X, X, symmetric=True, no_diag=...) with its gradient."""

    @staticmethod
    def forward(ctx, X, dyadic_order, no_diag):
        ctx.dyadic_order = dyadic_order
        ctx.no_diag = no_diag
        ctx.save_for_backward(X)
        return sigkernel_gram(X, None, dyadic_order, symmetric=True, no_diag=no_diag)

    @staticmethod
    def backward(ctx, dK):
        (X,) = ctx.saved_tensors
        dX, _ = sigkernel_gram_backward(X, None, dK.to(torch.float32), ctx.dyadic_order,
                                        symmetric=True, no_diag=ctx.no_diag)
        return dX, None, None


def gram(X: torch.Tensor, Y: Optional[torch.Tensor] = None, dyadic_order: int = 0, *,
         no_diag: bool = False) -> torch.Tensor:
    """Differentiable Gram matrix; Y None means the symmetric Gram of X."""
    if Y is None:
        return SigKernelGramSymmetric.apply(X, dyadic_order, no_diag)
    return SigKernelGram.apply(X, Y, dyadic_order)


def sigkernel_mmd2(X: PathsLike, Y: PathsLike, dyadic_order: int = 0, *,
                   grad: bool = False, workspace: Optional[torch.Tensor] = None):
    """(mmd2 [1] device tensor, dX or None): unbiased MMD^2 between the batches
    and, with ``grad=True``, its gradient with respect to the points of X."""
    lib = _lib.load()
    dev = _device(X)
    flags = _lib.SK_MMD2_GRAD if grad else 0
    sx, sy = _describe(X), _describe(Y)
    out = torch.empty(1, dtype=torch.float32, device=dev)
    dX = _empty_points(X) if grad else None
    nbytes = int(lib.sigkernel_workspace_bytes(_lib.SK_OP_MMD2, ctypes.byref(sx),
                                               ctypes.byref(sy), int(dyadic_order), flags))
    ws = _workspace(nbytes, dev, workspace)
    st = lib.sigkernel_mmd2(ctypes.byref(sx), ctypes.byref(sy), int(dyadic_order), flags,
                            out.data_ptr(), dX.data_ptr() if dX is not None else None,
                            ws.data_ptr(), ws.numel() * ws.element_size(), _stream_ptr(dev))
    _lib.check(st, "sigkernel_mmd2")
    return out, dX


class SigKernelMMD2(torch.autograd.Function):
    """Unbiased MMD^2 with its gradient computed in the same library call."""

    @staticmethod
    def forward(ctx, X, Y, dyadic_order):
        val, dX = sigkernel_mmd2(X, Y, dyadic_order, grad=ctx.needs_input_grad[0])
        ctx.save_for_backward(dX if dX is not None else torch.empty(0, device=X.device))
        return val[0]

    @staticmethod
    def backward(ctx, g):
        (dX,) = ctx.saved_tensors
        return (dX * g) if dX.numel() else None, None, None


def mmd2(X: torch.Tensor, Y: torch.Tensor, dyadic_order: int = 0) -> torch.Tensor:
    """Differentiable (in X) unbiased signature-kernel MMD^2."""
    return SigKernelMMD2.apply(X, Y, dyadic_order)


def sigkernel_increment_gram(X: torch.Tensor, Y: torch.Tensor, *, gram: bool = True,
                             precision: str = "f32", ld: Optional[int] = None,
                             out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """G0 = <x_{p+1} - x_p, y_{q+1} - y_q> of every pair (float32 VALU, rows in order):
    [nx, ny, Lx-1, Ly-1] (gram) or [n, Lx-1, Ly-1] (pairs).  ``ld`` (>= Ly-1)
    stores each row with that stride: ``out`` then has ld columns, of which
    the first Ly-1 are written and returned as a view."""
    lib = _lib.load()
    sx, sy = _describe(X), _describe(Y)
    m, n = int(X.shape[1]) - 1, int(Y.shape[1]) - 1
    cols = n if ld is None else int(ld)
    lead = (int(X.shape[0]), int(Y.shape[0])) if gram else (int(X.shape[0]),)
    if out is None:
        out = torch.empty(lead + (m, cols), dtype=torch.float32, device=X.device)
    elif tuple(out.shape) != lead + (m, cols) or not out.is_contiguous():
        raise ValueError(f"out must be a contiguous float32 tensor of shape {lead + (m, cols)}")
    st = lib.sigkernel_increment_gram(ctypes.byref(sx), ctypes.byref(sy), 1 if gram else 0,
                                      _gram_flag(precision),
                                      out.data_ptr() if out.numel() else None,
                                      0 if ld is None else cols, _stream_ptr(X.device))
    _lib.check(st, "sigkernel_increment_gram")
    return out if ld is None else out[..., :n]
