"""Launch-tuning table, its JSON cache and the graph / autotune argument
checks: host-only paths of the C ABI (no GPU; every call that would touch HIP
is rejected first, so fake device pointers are never dereferenced)."""
import ctypes

import pytest

from paper_2006_14794_amd import _lib, tuning
from paper_2006_14794_amd._lib import SkPaths, SkTune, SkTuneKey

FAKE = 0x10000


@pytest.fixture(autouse=True)
def clean_table():
    tuning.tune_clear()
    yield
    tuning.tune_clear()


def key_of(op, X, Y, lam=1, flags=0):
    k = SkTuneKey()
    st = _lib.load().sigkernel_tune_key(op, ctypes.byref(X), ctypes.byref(Y), lam, flags,
                                        ctypes.byref(k))
    assert st == 0
    return tuning._as_dict(k, tuning.KEY_FIELDS)


def test_key_of_a_call():
    X, Y = SkPaths(FAKE, None, 128, 256, 9), SkPaths(FAKE, None, 64, 100, 9)
    k = key_of(_lib.SK_OP_GRAM, X, Y, 2, _lib.SK_SYMMETRIC | _lib.SK_NO_DIAG)
    assert k == dict(op=1, dyadic_order=2, symmetric=1, ragged=0, nx=128, ny=64, x_len=256,
                     y_len=100, dim=9)
    R = SkPaths(FAKE, FAKE, 7, 1024, 16)
    assert key_of(_lib.SK_OP_PAIR, R, R)["ragged"] == 1
    k2 = SkTuneKey()
    assert _lib.load().sigkernel_tune_key(9, ctypes.byref(X), ctypes.byref(Y), 0, 0,
                                          ctypes.byref(k2)) == _lib.SK_ERR_FLAGS
    assert _lib.load().sigkernel_tune_key(1, None, ctypes.byref(Y), 0, 0,
                                          ctypes.byref(k2)) == _lib.SK_ERR_NULL


def test_set_get_replace_remove_list():
    X = SkPaths(FAKE, None, 16, 32, 4)
    ka = key_of(_lib.SK_OP_GRAM, X, X)
    kb = key_of(_lib.SK_OP_PAIR, X, X)
    assert tuning.tune_get(ka) is None
    tuning.tune_set(ka, dict(run=8, waves_per_block=2))
    tuning.tune_set(kb, dict(pair_blocks_per_cu=3, pair_bands=1))
    assert tuning.tune_get(ka) == dict(run=8, waves_per_block=2, pair_blocks_per_cu=0,
                                       pair_bands=0)
    assert tuning.tune_get(kb) == dict(run=0, waves_per_block=0, pair_blocks_per_cu=3,
                                       pair_bands=1)
    tuning.tune_set(ka, dict(run=1, waves_per_block=4))
    assert tuning.tune_get(ka)["run"] == 1
    assert len(tuning.tune_list()) == 2
    tuning.tune_set(ka, None)
    assert tuning.tune_get(ka) is None
    assert [k for k, _ in tuning.tune_list()] == [kb]


@pytest.mark.parametrize("bad", [dict(run=-1), dict(run=1025), dict(waves_per_block=3),
                                 dict(waves_per_block=8), dict(pair_blocks_per_cu=65),
                                 dict(pair_blocks_per_cu=-2), dict(pair_bands=2),
                                 dict(pair_bands=-1)])
def test_out_of_range_tunings_are_rejected(bad):
    X = SkPaths(FAKE, None, 16, 32, 4)
    k = key_of(_lib.SK_OP_GRAM, X, X)
    with pytest.raises(_lib.SigKernelError) as e:
        tuning.tune_set(k, bad)
    assert e.value.status == _lib.SK_ERR_FLAGS
    assert tuning.tune_get(k) is None
    t = SkTune()
    t.pair_bands = 7
    assert _lib.load().sigkernel_tune_set(ctypes.byref(tuning._key_struct(k)),
                                          ctypes.byref(t)) == _lib.SK_ERR_FLAGS


def test_cache_round_trip(tmp_path):
    X = SkPaths(FAKE, None, 128, 256, 9)
    Y = SkPaths(FAKE, FAKE, 4096, 1024, 16)
    entries = [(key_of(_lib.SK_OP_GRAM, X, X, 1), dict(run=4, waves_per_block=4)),
               (key_of(_lib.SK_OP_PAIR, Y, Y, 2), dict(pair_blocks_per_cu=2))]
    for k, t in entries:
        tuning.tune_set(k, t)
    path = str(tmp_path / "tune.json")
    tuning.save_cache(path)
    before = tuning.tune_list()
    tuning.tune_clear()
    assert tuning.tune_list() == []
    assert tuning.load_cache(path) == 2
    assert tuning.tune_list() == before


def test_backward_workspace_follows_the_tuned_run():
    # the per-run x-side partials scale with the number of runs per Gram row
    X = SkPaths(FAKE, None, 32, 64, 4)
    lib = _lib.load()

    def ws():
        return lib.sigkernel_workspace_bytes(_lib.SK_OP_GRAM_BACKWARD, ctypes.byref(X),
                                             ctypes.byref(X), 1, 0)
    k = key_of(_lib.SK_OP_GRAM_BACKWARD, X, X)
    tuning.tune_set(k, dict(run=1))
    w1 = ws()
    tuning.tune_set(k, dict(run=32))
    w32 = ws()
    assert w1 > w32 > 0
    tuning.tune_set(k, None)
    assert ws() > 0


def test_graph_and_autotune_argument_errors():
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.sigkernel_graph_begin(None) == _lib.SK_ERR_NULL
    assert lib.sigkernel_graph_end(None, ctypes.byref(h)) == _lib.SK_ERR_NULL
    assert lib.sigkernel_graph_end(FAKE, None) == _lib.SK_ERR_NULL
    assert lib.sigkernel_graph_launch(None, None) == _lib.SK_ERR_NULL
    assert lib.sigkernel_graph_destroy(None) == _lib.SK_ERR_NULL
    X = SkPaths(FAKE, None, 4, 16, 3)
    best, ms = SkTune(), ctypes.c_float()
    args = (ctypes.byref(X), ctypes.byref(X), 1, 0, FAKE, FAKE, 1 << 20)
    assert lib.sigkernel_autotune(_lib.SK_OP_GRAM_BACKWARD, *args, 3, None, ctypes.byref(best),
                                  ctypes.byref(ms)) == _lib.SK_ERR_FLAGS
    assert lib.sigkernel_autotune(_lib.SK_OP_GRAM, *args, 0, None, ctypes.byref(best),
                                  ctypes.byref(ms)) == _lib.SK_ERR_FLAGS
    assert lib.sigkernel_autotune(_lib.SK_OP_GRAM, *args, 3, None, None,
                                  ctypes.byref(ms)) == _lib.SK_ERR_NULL
    assert _lib.status_string(_lib.SK_ERR_STATE).startswith("not allowed")
