"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, CPU only), run on ragged problems with empty rows, duplicate indices,
targets at their centers and orders up to TSQBX_P_MAX: no sanitizer report,
and the same bits as the oracle library the other tests use."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_1811_01110_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path_factory.mktemp("asan") / "oracle_asan")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
           "-std=c11", "-I", oracle.HERE, os.path.join(HERE, "oracle_sanitize_driver.c"),
           oracle.SRC, "-lm", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("sanitizer build unavailable: " + r.stderr[-400:])
    return exe


def _write(path, g, p, layers, threads):
    T = len(g.targets)
    with open(path, "wb") as f:
        np.array([len(g.sources), len(g.centers), T, len(g.list_sources), p, layers, threads],
                 dtype=np.int64).tofile(f)
        for a, dt in ((g.sources, np.float64), (g.weights, np.float64), (g.normals, np.float64),
                      (g.centers, np.float64), (g.list_offsets, np.int64),
                      (g.list_sources, np.int32), (g.targets, np.float64),
                      (g.target_center, np.int32), (g.target_normals, np.float64),
                      (g.sigma, np.float64)):
            np.ascontiguousarray(a, dtype=dt).tofile(f)


@pytest.mark.parametrize("p", [0, 7, 32])
def test_oracle_under_sanitizers(driver, tmp_path, p):
    g = W.fuzz_geometry(7700 + p, n=120, m=25, max_list=40, p=p, layers=7, targets_per_center=2)
    tgt = g.targets.copy()
    tgt[0] = g.centers[g.target_center[0]]  # a target at its center
    g = W.Geometry(g.sources, g.weights, g.normals, g.centers, g.list_offsets, g.list_sources,
                   tgt, g.target_center, g.sigma, p, 7, target_normals=g.target_normals)
    inp, outp = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    _write(inp, g, p, 7, 2)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([driver, inp, outp], capture_output=True, text=True, env=env,
                       timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    got = np.fromfile(outp, dtype=np.float64).reshape(6, -1)
    ref = oracle.evaluate_geometry(g, p=p, layers=7)
    for k, name in enumerate(("slp", "dlp", "sprime")):
        assert np.array_equal(got[k], ref[name]), name
        assert np.array_equal(got[3 + k], ref["abs_" + name]), name
