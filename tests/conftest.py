import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    import oracle

    if not os.path.exists(oracle.LIB):
        oracle.build(force=False)
    yield


# ---------------------------------------------------------------------------
# shared helpers
# ---------------------------------------------------------------------------
import functools

import numpy as np

PARITY_TOL = 1e-12


def assert_parity(gpu, ref, abs_scale, tol=PARITY_TOL, what=""):
    """The parity bar: max|gpu - ref| / max|ref| <= tol and, per target,
    |gpu - ref| <= tol * (sum of absolute term values)."""
    gpu = np.asarray(gpu)
    ref = np.asarray(ref)
    assert gpu.shape == ref.shape, (gpu.shape, ref.shape)
    assert np.all(np.isfinite(gpu)), f"{what}: non-finite output"
    d = np.abs(gpu - ref)
    norm = float(np.max(np.abs(ref))) if ref.size else 0.0
    if norm > 0:
        assert d.max() / norm <= tol, f"{what}: rel inf-norm error {d.max() / norm:.3e}"
    bad = d > tol * np.asarray(abs_scale)
    assert not bad.any(), (f"{what}: {int(bad.sum())} targets exceed tol*abs_scale; worst ratio "
                           f"{float(np.max(d / np.maximum(abs_scale, 1e-300))):.3e}")


@functools.lru_cache(maxsize=None)
def cached_workload(name, *args):
    from paper_1811_01110_amd import workloads as W

    return getattr(W, name)(*args)
