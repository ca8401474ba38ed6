import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def lib():
    """The HIP library through its Python binding (GPU tests only)."""
    from paper_1309_0302_amd import binding
    return binding.load()


def oracle_a1(obj, i=0):
    """A1 of a GPU context (GoDec, GoDecBatch problem i, GoDecLayer member i)
    drawn by the oracle's own generator from the context's seed.  The
    library's copy is only checked against it, bit for bit: no oracle input
    comes from the library."""
    import numpy as np
    from oracle.rng_ref import a1_gaussian
    from paper_1309_0302_amd.binding import GoDecBatch, GoDecLayer
    if isinstance(obj, GoDecBatch):
        X, r, _, seed = obj.specs[i]
        n, lib = X.shape[1], obj.A1(i)
    elif isinstance(obj, GoDecLayer):
        seed, n, r, lib = obj.seed + i, obj.n, obj.r, obj.A1(i)
    else:
        seed, n, r, lib = obj.seed, obj.n, obj.r, obj.A1()
        if obj.a1 is not None:
            A1 = np.ascontiguousarray(obj.a1, dtype=np.float64)
            assert np.array_equal(lib.view(np.uint64), A1.view(np.uint64))
            return A1
    A1 = a1_gaussian(seed, n, r)
    assert np.array_equal(np.ascontiguousarray(lib).view(np.uint64), A1.view(np.uint64))
    return A1

