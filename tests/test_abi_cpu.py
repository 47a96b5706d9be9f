"""C ABI contract checks that need no GPU.

The library must load without a device, export every function that
include/sigkernel.h declares, and reject bad arguments before it touches HIP
(every error path below returns before any HIP call, so fake device pointers
are safe here).
"""
import ctypes
import os
import re

import pytest

import paper_2006_14794_amd as sk
from paper_2006_14794_amd import _lib
from paper_2006_14794_amd._lib import SkPaths

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = 0x10000  # never dereferenced: every call below fails validation first


def header_functions():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            for m in re.finditer(r"^\s*[\w\s\*]+?\b(sigkernel_\w+)\s*\(", src, re.M):
                names.add(m.group(1))
    return sorted(names)


def test_library_loads_and_exports_every_declared_symbol():
    lib = _lib.load()
    declared = header_functions()
    assert "sigkernel_gram" in declared and "sigkernel_pair" in declared
    for name in declared:
        assert hasattr(lib, name), name
    assert set(declared) == set(_lib.EXPORTED)


def test_status_strings():
    for code in range(-9, 1):
        s = sk.status_string(code)
        assert isinstance(s, str) and s
    assert sk.status_string(123) == "unknown status"
    assert sk.version().count(".") == 2


def paths(n=4, L=16, d=3, pts=FAKE, off=None):
    return SkPaths(pts, off, n, L, d)


def call_gram(X, Y, lam=1, flags=0, K=FAKE, ws=FAKE, nbytes=1 << 30):
    lib = _lib.load()
    return lib.sigkernel_gram(ctypes.byref(X) if X is not None else None,
                              ctypes.byref(Y) if Y is not None else None,
                              lam, flags, K, ws, nbytes, None)


def call_pair(x, y, lam=1, flags=0, out=FAKE, ws=FAKE, nbytes=1 << 30):
    lib = _lib.load()
    return lib.sigkernel_pair(ctypes.byref(x), ctypes.byref(y), lam, flags, out, ws, nbytes,
                              None)


def test_null_arguments():
    assert call_gram(None, paths()) == _lib.SK_ERR_NULL
    assert call_gram(paths(), paths(), K=None) == _lib.SK_ERR_NULL
    assert call_gram(paths(pts=None), paths()) == _lib.SK_ERR_NULL
    assert call_pair(paths(), paths(), out=None) == _lib.SK_ERR_NULL


def test_shape_errors():
    assert call_gram(paths(d=3), paths(d=4)) == _lib.SK_ERR_SHAPE
    assert call_gram(paths(d=0), paths(d=0)) == _lib.SK_ERR_SHAPE
    assert call_gram(paths(L=0), paths()) == _lib.SK_ERR_SHAPE
    assert call_gram(paths(n=-1), paths()) == _lib.SK_ERR_SHAPE
    assert call_pair(paths(n=3), paths(n=4)) == _lib.SK_ERR_SHAPE


def test_order_and_flag_errors():
    assert call_gram(paths(), paths(), lam=-1) == _lib.SK_ERR_ORDER
    # 2^lambda (len - 1) <= 2^20 on both sides: 15 * 2^16 fits, 15 * 2^17 does not
    assert call_gram(paths(L=16), paths(L=16), lam=17) == _lib.SK_ERR_ORDER
    assert call_gram(paths(L=16), paths(L=1025), lam=11) == _lib.SK_ERR_ORDER
    assert call_gram(paths(L=2), paths(L=2), lam=21) == _lib.SK_ERR_ORDER
    assert call_pair(paths(L=16), paths(L=16), lam=17) == _lib.SK_ERR_ORDER
    assert call_gram(paths(), paths(), flags=1 << 20) == _lib.SK_ERR_FLAGS
    assert call_gram(paths(), paths(), flags=_lib.SK_NO_DIAG) == _lib.SK_ERR_FLAGS
    # symmetric needs X and Y to be the same batch
    X, Y = paths(pts=FAKE), paths(pts=FAKE * 2)
    assert call_gram(X, Y, flags=_lib.SK_SYMMETRIC) == _lib.SK_ERR_SHAPE
    assert call_pair(paths(), paths(), flags=_lib.SK_SYMMETRIC) == _lib.SK_ERR_FLAGS


def test_workspace_errors_and_sizing():
    lib = _lib.load()
    X, Y = paths(n=4, L=16, d=3), paths(n=5, L=9, d=3)
    need = lib.sigkernel_workspace_bytes(_lib.SK_OP_GRAM, ctypes.byref(X), ctypes.byref(Y), 1, 0)
    # at least the dense padded increments: 4 floats per segment of each batch
    # plus 128 stream-padding rows on each side, 256-byte aligned
    inc = (256 * ((4 * (4 * 15 + 256) * 4 + 255) // 256)
           + 256 * ((4 * (5 * 8 + 256) * 4 + 255) // 256))
    assert need >= inc and need % 256 == 0
    # ragged batches add a per-path plan (int32 count + int64 start)
    Xr = paths(n=4, L=16, d=3, off=FAKE)
    need_r = lib.sigkernel_workspace_bytes(_lib.SK_OP_GRAM, ctypes.byref(Xr), ctypes.byref(Y), 1, 0)
    assert need_r >= need
    for op in (_lib.SK_OP_PAIR, _lib.SK_OP_GRAM_BACKWARD, _lib.SK_OP_MMD2):
        Xp = paths(n=5, L=16, d=3)
        assert lib.sigkernel_workspace_bytes(op, ctypes.byref(Xp), ctypes.byref(Y), 1, 4) > 0
    assert call_gram(X, Y, ws=None) == _lib.SK_ERR_WORKSPACE
    assert call_gram(X, Y, nbytes=inc - 1) == _lib.SK_ERR_WORKSPACE
    bad = paths(d=0)
    assert lib.sigkernel_workspace_bytes(_lib.SK_OP_GRAM, ctypes.byref(bad), ctypes.byref(Y), 1,
                                         0) == 0


def test_empty_batches_are_no_ops():
    assert call_gram(paths(n=0), paths(n=3), K=None, ws=None) == _lib.SK_OK
    assert call_pair(paths(n=0), paths(n=0), out=None, ws=None) == _lib.SK_OK


def test_gradient_shapes_accepted_and_rejected():
    # the gradient takes tall x paths (row bands) and ragged batches; beyond 16
    # channels it is not compiled.  A workspace that is too small is reported
    # before anything is enqueued (no device memory is touched here).
    lib = _lib.load()
    X = paths(n=2, L=64 * 32 // 8 + 2, d=16)
    Y = paths(n=2, L=8, d=16)
    need = lib.sigkernel_workspace_bytes(_lib.SK_OP_GRAM_BACKWARD, ctypes.byref(X),
                                         ctypes.byref(Y), 3, 0)
    assert need > 0
    st = lib.sigkernel_gram_backward(ctypes.byref(X), ctypes.byref(Y), 3, 0, FAKE, FAKE, FAKE,
                                     FAKE, need - 1, None)
    assert st == _lib.SK_ERR_WORKSPACE
    Xr = paths(n=2, L=16, d=3, off=FAKE)
    Y3 = paths(n=2, L=8, d=3)
    need = lib.sigkernel_workspace_bytes(_lib.SK_OP_GRAM_BACKWARD, ctypes.byref(Xr),
                                         ctypes.byref(Y3), 1, 0)
    st = lib.sigkernel_gram_backward(ctypes.byref(Xr), ctypes.byref(Y3), 1, 0, FAKE, FAKE, FAKE,
                                     FAKE, need - 1, None)
    assert st == _lib.SK_ERR_WORKSPACE
    X17 = paths(n=2, L=16, d=17)
    st = lib.sigkernel_gram_backward(ctypes.byref(X17), ctypes.byref(X17), 1, 0, FAKE, FAKE,
                                     FAKE, FAKE, 1 << 40, None)
    assert st == _lib.SK_ERR_UNSUPPORTED


def test_noalloc_gram_checks_before_any_hip_call():
    # the allocation-free Gram validates like sigkernel_gram and rejects a
    # problem whose workspace exceeds its static array, before touching HIP
    lib = _lib.load()
    cap = lib.sigkernel_gram_noalloc_max_bytes()
    assert cap == 64 << 20
    X = paths(n=4096, L=2049, d=16)
    assert lib.sigkernel_workspace_bytes(_lib.SK_OP_GRAM, ctypes.byref(X), ctypes.byref(X), 1,
                                         0) > cap
    assert lib.sigkernel_gram_noalloc(ctypes.byref(X), ctypes.byref(X), 1, 0, FAKE,
                                      None) == _lib.SK_ERR_WORKSPACE
    assert lib.sigkernel_gram_noalloc(ctypes.byref(paths(d=3)), ctypes.byref(paths(d=4)), 1, 0,
                                      FAKE, None) == _lib.SK_ERR_SHAPE
    assert lib.sigkernel_gram_noalloc(ctypes.byref(paths()), ctypes.byref(paths()), -1, 0, FAKE,
                                      None) == _lib.SK_ERR_ORDER
    assert lib.sigkernel_gram_noalloc(ctypes.byref(paths()), ctypes.byref(paths()), 1, 0, None,
                                      None) == _lib.SK_ERR_NULL


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        _lib.load()


def test_implicit_flag_only_where_defined():
    lib = _lib.load()
    X = paths()
    # the backward, the MMD and the standalone increment Gram have no implicit form
    assert lib.sigkernel_gram_backward(ctypes.byref(X), ctypes.byref(X), 1, _lib.SK_IMPLICIT,
                                       FAKE, FAKE, FAKE, FAKE, 1 << 30, None) == _lib.SK_ERR_FLAGS
    assert lib.sigkernel_increment_gram(ctypes.byref(X), ctypes.byref(X), 1, _lib.SK_IMPLICIT,
                                        FAKE, 0, None) == _lib.SK_ERR_FLAGS
    assert lib.sigkernel_mmd2(ctypes.byref(X), ctypes.byref(X), 1, _lib.SK_IMPLICIT, FAKE, FAKE,
                              FAKE, 1 << 30, None) == _lib.SK_ERR_FLAGS


def test_increment_gram_row_stride_below_the_row_length_is_a_shape_error():
    lib = _lib.load()
    X, Y = paths(L=16), paths(L=40)
    for ldg in (1, 38):  # rows of Y->len - 1 = 39 floats
        assert lib.sigkernel_increment_gram(ctypes.byref(X), ctypes.byref(Y), 1, 0, FAKE, ldg,
                                            None) == _lib.SK_ERR_SHAPE


def test_increment_gram_channel_limit():
    # up to 64 channels (16 on the vector ALUs, 17-64 on the matrix cores);
    # more is refused before anything is enqueued
    lib = _lib.load()
    X, Y = paths(d=65), paths(d=65)
    assert lib.sigkernel_increment_gram(ctypes.byref(X), ctypes.byref(Y), 1, 0, FAKE, 0,
                                        None) == _lib.SK_ERR_UNSUPPORTED


def call_lifted(fn, X, Y, kernel, lam=1, flags=0, out=FAKE, ws=FAKE, nbytes=1 << 30):
    lib = _lib.load()
    return getattr(lib, fn)(ctypes.byref(X), ctypes.byref(Y), lam, flags,
                            ctypes.byref(kernel) if kernel is not None else None, out, ws,
                            nbytes, None)


@pytest.mark.parametrize("fn", ["sigkernel_pair_lifted", "sigkernel_gram_lifted"])
def test_lifted_argument_errors(fn):
    X = paths()
    rbf = _lib.SkStaticKernel(_lib.SK_STATIC_RBF, 0, 1.0)
    assert call_lifted(fn, X, X, None) == _lib.SK_ERR_NULL
    for bad in (_lib.SkStaticKernel(7, 0, 1.0), _lib.SkStaticKernel(_lib.SK_STATIC_RBF, 0, 0.0),
                _lib.SkStaticKernel(_lib.SK_STATIC_RBF, 0, -1.0),
                _lib.SkStaticKernel(_lib.SK_STATIC_RBF, 0, float("nan")),
                _lib.SkStaticKernel(_lib.SK_STATIC_RBF, 0, float("inf")),
                _lib.SkStaticKernel(_lib.SK_STATIC_RBF, 0, 1e-200)):
        assert call_lifted(fn, X, X, bad) == _lib.SK_ERR_VALUE
    # 16-bit increments only mean something for the linear kernel
    assert call_lifted(fn, X, X, rbf, flags=_lib.SK_GRAM_BF16) == _lib.SK_ERR_FLAGS
    assert call_lifted(fn, X, X, rbf, flags=1 << 12) == _lib.SK_ERR_FLAGS
    # the lifted sweep runs the compiled orders only
    assert call_lifted(fn, X, X, rbf, lam=4) == _lib.SK_ERR_ORDER
    assert call_lifted(fn, X, paths(d=2), rbf) == _lib.SK_ERR_SHAPE
    assert call_lifted(fn, X, X, rbf, ws=None) == _lib.SK_ERR_WORKSPACE
    assert call_lifted(fn, X, X, rbf, nbytes=16) == _lib.SK_ERR_WORKSPACE
    # RBF x paths taller than one wave's rows are not compiled
    tall = paths(n=2, L=70000, d=1)
    assert call_lifted(fn, tall, tall, rbf, lam=0) == _lib.SK_ERR_UNSUPPORTED
    if fn == "sigkernel_pair_lifted":
        assert call_lifted(fn, X, X, rbf, flags=_lib.SK_SYMMETRIC) == _lib.SK_ERR_FLAGS
        assert call_lifted(fn, X, paths(n=3), rbf) == _lib.SK_ERR_SHAPE
    else:
        assert call_lifted(fn, X, paths(n=4, L=16, d=3, pts=FAKE + 64), rbf,
                           flags=_lib.SK_SYMMETRIC) == _lib.SK_ERR_SHAPE
        assert call_lifted(fn, X, X, rbf, flags=_lib.SK_NO_DIAG) == _lib.SK_ERR_FLAGS


def test_lifted_workspace_covers_both_static_kernels():
    lib = _lib.load()
    X, Y = paths(n=5, L=40, d=3), paths(n=7, L=30, d=3)
    for op, plain in ((_lib.SK_OP_PAIR_LIFTED, _lib.SK_OP_PAIR),
                      (_lib.SK_OP_GRAM_LIFTED, _lib.SK_OP_GRAM)):
        b = lib.sigkernel_workspace_bytes(op, ctypes.byref(X), ctypes.byref(X if op == 7 else Y),
                                          1, 0)
        p = lib.sigkernel_workspace_bytes(plain, ctypes.byref(X),
                                          ctypes.byref(X if op == 7 else Y), 1, 0)
        # node rows of both batches (padded to 4 channels, 128 rows each side)
        nodes = (5 * 40 + 256) * 4 * 4 + ((5 if op == 7 else 7) * (40 if op == 7 else 30) + 256) * 16
        assert b >= max(p, nodes)


def test_reduced_measure_argument_errors():
    lib = _lib.load()
    f = lib.sigkernel_reduced_measure
    g = lib.sigkernel_reduced_measure_support
    assert f(None, FAKE, 5, 0.1, 0.0, 10, FAKE, None, None, None) == _lib.SK_ERR_NULL
    assert f(FAKE, FAKE, 0, 0.1, 0.0, 10, FAKE, None, None, None) == _lib.SK_ERR_SHAPE
    assert f(FAKE, FAKE, 4097, 0.1, 0.0, 10, FAKE, None, None, None) == _lib.SK_ERR_SHAPE
    assert f(FAKE, FAKE, 5, -0.1, 0.0, 10, FAKE, None, None, None) == _lib.SK_ERR_VALUE
    assert f(FAKE, FAKE, 5, float("nan"), 0.0, 10, FAKE, None, None, None) == _lib.SK_ERR_VALUE
    assert f(FAKE, FAKE, 5, 0.1, -1.0, 10, FAKE, None, None, None) == _lib.SK_ERR_VALUE
    assert f(FAKE, FAKE, 5, 0.1, 0.0, -1, FAKE, None, None, None) == _lib.SK_ERR_SHAPE
    assert g(FAKE, FAKE, 5, 6, 10, 10, 0.0, FAKE, FAKE, None, None) == _lib.SK_ERR_VALUE
    assert g(FAKE, FAKE, 5, 0, 10, 10, 0.0, FAKE, FAKE, None, None) == _lib.SK_ERR_VALUE
    assert g(FAKE, FAKE, 5, 2, 10, 0, 0.0, FAKE, FAKE, None, None) == _lib.SK_ERR_VALUE
    assert g(FAKE, FAKE, 5, 2, 10, 10, 0.0, FAKE, None, None, None) == _lib.SK_ERR_NULL
