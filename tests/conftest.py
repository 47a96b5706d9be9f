import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: longer CPU test")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


# Gradient parity: |g - g_ref| <= ABS_TOL max|g_ref| for every component, and
# |g - g_ref| <= REL_TOL |g_ref| for every component above REL_FLOOR max|g_ref|.
GRAD_ABS_TOL = 1e-5
GRAD_REL_TOL = 1e-4
GRAD_REL_FLOOR = 1e-3


def grad_close(got, ref, name="grad"):
    """Assert the gradient bar above; print and return (abs, rel) errors."""
    import numpy as np
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    scale = max(float(np.abs(ref).max()), 1e-300)
    err = np.abs(got - ref)
    abs_err = float(err.max()) / scale
    big = np.abs(ref) >= GRAD_REL_FLOOR * scale
    rel_err = float((err[big] / np.abs(ref[big])).max()) if big.any() else 0.0
    print(f"GRADERR {name} abs {abs_err:.3e} rel {rel_err:.3e}")
    assert abs_err <= GRAD_ABS_TOL, (name, abs_err)
    assert rel_err <= GRAD_REL_TOL, (name, rel_err)
    return abs_err, rel_err
