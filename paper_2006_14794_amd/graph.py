"""HIP graph replay of library calls (bindings of sigkernel_graph_*).

A :class:`CapturedCalls` records the kernel launches of the library calls a
function issues, once, on a private stream, and replays them with a single
graph launch.  Every pointer is fixed at capture: the function must not
allocate (pass ``out=`` and ``workspace=``), and those tensors, like the
inputs, must outlive the graph.  Replays read the inputs' current contents.
"""
from __future__ import annotations

import ctypes
from typing import Callable, Optional

import torch

from . import _lib


class CapturedCalls:
    def __init__(self, fn: Callable[[], None], device=None):
        lib = _lib.load()
        self._lib = lib
        self._graph = None
        dev = torch.device(device if device is not None else "cuda")
        self.device = dev
        stream = torch.cuda.Stream(dev)
        stream.wait_stream(torch.cuda.current_stream(dev))
        handle = ctypes.c_void_p()
        with torch.cuda.stream(stream):
            _lib.check(lib.sigkernel_graph_begin(stream.cuda_stream), "sigkernel_graph_begin")
            try:
                fn()
            except BaseException:
                if lib.sigkernel_graph_end(stream.cuda_stream, ctypes.byref(handle)) == 0:
                    lib.sigkernel_graph_destroy(handle)
                raise
            _lib.check(lib.sigkernel_graph_end(stream.cuda_stream, ctypes.byref(handle)),
                       "sigkernel_graph_end")
        self._graph = handle

    def replay(self, stream: Optional[torch.cuda.Stream] = None) -> None:
        """One graph launch on ``stream`` (default: the current stream)."""
        if self._graph is None:
            raise RuntimeError("graph destroyed")
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        _lib.check(self._lib.sigkernel_graph_launch(self._graph, s.cuda_stream),
                   "sigkernel_graph_launch")

    def close(self) -> None:
        if self._graph is not None:
            g, self._graph = self._graph, None
            _lib.check(self._lib.sigkernel_graph_destroy(g), "sigkernel_graph_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _buffers(op: int, X, Y, dyadic_order: int, flags: int, n_out):
    from .api import _device, workspace_bytes
    dev = _device(X)
    out = torch.empty(n_out, dtype=torch.float32, device=dev)
    nbytes = workspace_bytes(op, X, Y, dyadic_order, flags)
    ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=dev)
    return out, ws


def capture_gram(X, Y=None, dyadic_order: int = 0, *, symmetric: bool = False,
                 no_diag: bool = False, gram_precision: str = "f32", scheme: str = "explicit"):
    """(graph, K): sigkernel_gram captured once; each ``graph.replay()``
    recomputes K in place from the current contents of X and Y."""
    from .api import _device, _gram_flag, _n_paths, _scheme_flag, sigkernel_gram
    Yv = X if Y is None else Y
    flags = _gram_flag(gram_precision) | _scheme_flag(scheme)
    if symmetric:
        flags |= _lib.SK_SYMMETRIC | (_lib.SK_NO_DIAG if no_diag else 0)
    K, ws = _buffers(_lib.SK_OP_GRAM, X, Yv, dyadic_order, flags, (_n_paths(X), _n_paths(Yv)))
    g = CapturedCalls(lambda: sigkernel_gram(X, Y, dyadic_order, symmetric=symmetric,
                                             no_diag=no_diag, gram_precision=gram_precision,
                                             scheme=scheme, out=K, workspace=ws), _device(X))
    g._keep = (ws,)
    return g, K


def capture_pair(x, y, dyadic_order: int = 0, *, gram_precision: str = "f32",
                 scheme: str = "explicit"):
    """(graph, out): sigkernel_pair captured once (independent pairs)."""
    from .api import _device, _gram_flag, _n_paths, _scheme_flag, sigkernel_pair
    flags = _gram_flag(gram_precision) | _scheme_flag(scheme)
    out, ws = _buffers(_lib.SK_OP_PAIR, x, y, dyadic_order, flags, (_n_paths(x),))
    g = CapturedCalls(lambda: sigkernel_pair(x, y, dyadic_order, gram_precision=gram_precision,
                                             scheme=scheme, out=out, workspace=ws), _device(x))
    g._keep = (ws,)
    return g, out


def capture_mmd2(X, Y, dyadic_order: int = 0, *, grad: bool = False):
    """(graph, mmd2 [1], dX or None): sigkernel_mmd2 captured once."""
    from .api import _describe, _device, _stream_ptr
    lib = _lib.load()
    dev = _device(X)
    flags = _lib.SK_MMD2_GRAD if grad else 0
    from .api import workspace_bytes
    val = torch.empty(1, dtype=torch.float32, device=dev)
    dX = torch.empty_like(X) if grad else None
    ws = torch.empty(max(workspace_bytes(_lib.SK_OP_MMD2, X, Y, dyadic_order, flags), 256),
                     dtype=torch.uint8, device=dev)
    sx, sy = _describe(X), _describe(Y)

    def call():
        _lib.check(lib.sigkernel_mmd2(ctypes.byref(sx), ctypes.byref(sy), int(dyadic_order),
                                      flags, val.data_ptr(),
                                      dX.data_ptr() if dX is not None else None, ws.data_ptr(),
                                      ws.numel(), _stream_ptr(dev)), "sigkernel_mmd2")

    g = CapturedCalls(call, dev)
    g._keep = (ws,)
    return g, val, dX
