import functools
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@functools.lru_cache(maxsize=None)
def feeder(name: str, seed: int | None = None):
    from synth import DEFAULT_SEEDS, make_feeder
    return make_feeder(name, DEFAULT_SEEDS[name] if seed is None else seed)


@functools.lru_cache(maxsize=None)
def oracle_lp(name: str):
    from oracle import model
    return model.decompose(feeder(name))


@functools.lru_cache(maxsize=None)
def oracle_prep(name: str):
    from oracle import admm
    return admm.prepare(oracle_lp(name))


def rel_err(a, b) -> float:
    """||a - b||_inf / max(1, ||b||_inf)"""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if a.size == 0:
        return 0.0
    return float(np.abs(a - b).max() / max(1.0, np.abs(b).max()))


@pytest.fixture(scope="session")
def gpu():
    """The HIP binding, only when a GPU and the built library are present."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2310_09410_amd as P
    from paper_2310_09410_amd import _native
    _native.lib()  # raises if the library was not built: no fallback
    return P
