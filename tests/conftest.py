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


# observed margins of every parity check: what -> (rel inf-norm error, worst
# per-target ratio |gpu - ref| / abs_scale); written as JSON at the end of the
# session when TSQBX_PARITY_REPORT names a file
MARGINS = {}


def assert_parity(gpu, ref, abs_scale, tol=PARITY_TOL, what=""):
    """The parity bar: max|gpu - ref| / max|ref| <= tol and, per target,
    |gpu - ref| <= tol * (sum of absolute term values).  Returns the two
    observed ratios (to be read against tol)."""
    gpu = np.asarray(gpu)
    ref = np.asarray(ref)
    assert gpu.shape == ref.shape, (gpu.shape, ref.shape)
    assert np.all(np.isfinite(gpu)), f"{what}: non-finite output"
    d = np.abs(gpu - ref)
    norm = float(np.max(np.abs(ref))) if ref.size else 0.0
    rel = float(d.max() / norm) if norm > 0 else 0.0
    worst = float(np.max(d / np.maximum(abs_scale, 1e-300))) if ref.size else 0.0
    if what:
        prev = MARGINS.get(what)
        MARGINS[what] = (max(rel, prev[0]), max(worst, prev[1]), int(ref.size) + prev[2]) \
            if prev else (rel, worst, int(ref.size))
    if norm > 0:
        assert rel <= tol, f"{what}: rel inf-norm error {rel:.3e}"
    bad = d > tol * np.asarray(abs_scale)
    assert not bad.any(), (f"{what}: {int(bad.sum())} targets exceed tol*abs_scale; worst ratio "
                           f"{worst:.3e}")
    return rel, worst


def pytest_sessionfinish(session, exitstatus):
    path = os.environ.get("TSQBX_PARITY_REPORT")
    if path and MARGINS:
        import json

        os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
        with open(path, "w") as f:
            json.dump({k: {"rel_inf": v[0], "worst_per_target": v[1], "targets": v[2]}
                       for k, v in sorted(MARGINS.items())}, f, indent=1)


@functools.lru_cache(maxsize=None)
def cached_workload(name, *args):
    from paper_1811_01110_amd import workloads as W

    return getattr(W, name)(*args)
