"""Launch tuning: bindings of the library's tuning table and autotuner, and a
JSON cache of tuned entries.

A tuning changes how pairs are spread over waves, workgroups and CUs, never a
pair's arithmetic (forward outputs are bit-identical under every tuning).  The
table lives in libsigkernel; this module only marshals keys and values and
reads/writes the cache file.  Setting ``SIGKERNEL_TUNE_CACHE`` to a cache file
loads it when the library is first loaded.
"""
from __future__ import annotations

import ctypes
import json
import os
from typing import Dict, List, Optional, Tuple

from . import _lib
from ._lib import SkTune, SkTuneKey

KEY_FIELDS = ("op", "dyadic_order", "symmetric", "ragged", "nx", "ny", "x_len", "y_len", "dim")
TUNE_FIELDS = ("run", "waves_per_block", "pair_blocks_per_cu", "pair_bands")

OPS = {"pair": _lib.SK_OP_PAIR, "gram": _lib.SK_OP_GRAM,
       "gram_backward": _lib.SK_OP_GRAM_BACKWARD}


def _key_struct(key: Dict[str, int]) -> SkTuneKey:
    k = SkTuneKey()
    for f in KEY_FIELDS:
        setattr(k, f, int(key[f]))
    k.reserved = 0
    return k


def _tune_struct(tune: Dict[str, int]) -> SkTune:
    t = SkTune()
    for f in TUNE_FIELDS:
        setattr(t, f, int(tune.get(f, 0)))
    return t


def _as_dict(s, fields) -> Dict[str, int]:
    return {f: int(getattr(s, f)) for f in fields}


def _op(op) -> int:
    return OPS[op] if isinstance(op, str) else int(op)


def tune_key(op, X, Y, dyadic_order: int, flags: int = 0) -> Dict[str, int]:
    """The table key of a call (op 'pair', 'gram' or 'gram_backward')."""
    from .api import _describe
    lib = _lib.load()
    sx, sy = _describe(X), _describe(Y if Y is not None else X)
    k = SkTuneKey()
    _lib.check(lib.sigkernel_tune_key(_op(op), ctypes.byref(sx), ctypes.byref(sy),
                                      int(dyadic_order), int(flags), ctypes.byref(k)),
               "sigkernel_tune_key")
    return _as_dict(k, KEY_FIELDS)


def tune_set(key: Dict[str, int], tune: Optional[Dict[str, int]]) -> None:
    """Insert or replace the entry of ``key``; ``tune=None`` removes it."""
    lib = _lib.load()
    k = _key_struct(key)
    t = _tune_struct(tune) if tune is not None else None
    _lib.check(lib.sigkernel_tune_set(ctypes.byref(k), ctypes.byref(t) if t is not None else None),
               "sigkernel_tune_set")


def tune_get(key: Dict[str, int]) -> Optional[Dict[str, int]]:
    lib = _lib.load()
    k, t = _key_struct(key), SkTune()
    r = lib.sigkernel_tune_get(ctypes.byref(k), ctypes.byref(t))
    if r < 0:
        _lib.check(r, "sigkernel_tune_get")
    return _as_dict(t, TUNE_FIELDS) if r == 1 else None


def tune_list() -> List[Tuple[Dict[str, int], Dict[str, int]]]:
    lib = _lib.load()
    n = int(lib.sigkernel_tune_list(None, None, 0))
    keys, tunes = (SkTuneKey * max(n, 1))(), (SkTune * max(n, 1))()
    n = min(n, int(lib.sigkernel_tune_list(keys, tunes, n)))
    return [(_as_dict(keys[i], KEY_FIELDS), _as_dict(tunes[i], TUNE_FIELDS)) for i in range(n)]


def tune_clear() -> None:
    _lib.load().sigkernel_tune_clear()


def autotune(op, X, Y=None, dyadic_order: int = 0, *, symmetric: bool = False,
             no_diag: bool = False, gram_precision: str = "f32", scheme: str = "explicit",
             reps: int = 3, cache: Optional[str] = None) -> Tuple[Dict[str, int], float]:
    """Time the candidate tunings of a forward call ('pair' or 'gram') on the
    current stream, keep the fastest in the table and return (tuning, ms).
    With ``cache`` the whole table is then written to that JSON file."""
    import torch

    from .api import (_describe, _device, _gram_flag, _n_paths, _scheme_flag, _stream_ptr,
                      workspace_bytes)
    lib = _lib.load()
    opn = _op(op)
    if opn not in (_lib.SK_OP_PAIR, _lib.SK_OP_GRAM):
        raise ValueError("autotune covers the forward calls 'pair' and 'gram'")
    if Y is None:
        Y = X
    flags = _gram_flag(gram_precision) | _scheme_flag(scheme)
    if symmetric:
        flags |= _lib.SK_SYMMETRIC | (_lib.SK_NO_DIAG if no_diag else 0)
    dev = _device(X)
    n_out = _n_paths(X) if opn == _lib.SK_OP_PAIR else _n_paths(X) * _n_paths(Y)
    out = torch.empty(max(n_out, 1), dtype=torch.float32, device=dev)
    nbytes = workspace_bytes(opn, X, Y, dyadic_order, flags)
    ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=dev)
    sx, sy = _describe(X), _describe(Y)
    best, ms = SkTune(), ctypes.c_float(0.0)
    _lib.check(lib.sigkernel_autotune(opn, ctypes.byref(sx), ctypes.byref(sy), int(dyadic_order),
                                      flags, out.data_ptr(), ws.data_ptr(), ws.numel(),
                                      int(reps), _stream_ptr(dev), ctypes.byref(best),
                                      ctypes.byref(ms)),
               "sigkernel_autotune")
    if cache:
        save_cache(cache)
    return _as_dict(best, TUNE_FIELDS), float(ms.value)


def save_cache(path: str) -> None:
    """Write every table entry to ``path`` (JSON list of {key, tune})."""
    entries = [{"key": k, "tune": t} for k, t in tune_list()]
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump({"version": 1, "entries": entries}, f, indent=1)
    os.replace(tmp, path)


def load_cache(path: str) -> int:
    """Insert the entries of a cache file into the table; returns their count."""
    with open(path) as f:
        data = json.load(f)
    if data.get("version") != 1:
        raise ValueError(f"{path}: unknown tune cache version")
    for e in data["entries"]:
        tune_set(e["key"], e["tune"])
    return len(data["entries"])
