"""The serving scheduler on the CPU through a fake executor
(tests/server_fake_driver.cc): admission under the memory budget, FIFO order
and no overtaking, slot limits, arena fragmentation, failures of a launch,
of a step and of one job, cancellation, time-outs, shutdown with work in
flight and the bounded ticket history.  The scheduler is the one the library
serves with (paper_1811_01110_amd/csrc/tsqbx_sched.h); the fake executor
delivers outputs computed by the CPU oracle.  Each scenario runs under
AddressSanitizer + UBSan and under ThreadSanitizer."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1811_01110_amd", "csrc")
INCLUDE = os.path.join(ROOT, "include")
ORACLE = os.path.join(ROOT, "oracle")
SCENARIOS = ["mix", "budget", "failures", "cancel_timeout", "fragmentation", "stop_in_flight",
             "history"]
SANITIZERS = {"asan": ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
              "tsan": ["-fsanitize=thread"]}
# ThreadSanitizer needs an interceptor for pthread_cond_clockwait (the timed
# waits of std::condition_variable); GCC 11's runtime lacks it and then
# reports false double locks, so the TSan build uses ROCm's clang.
LLVM = "/opt/rocm/llvm/bin"


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, (" ".join(cmd), r.stdout[-2000:], r.stderr[-4000:])


@pytest.fixture(scope="module", params=sorted(SANITIZERS))
def driver(request, tmp_path_factory):
    if request.param == "tsan":
        cc, cxx = os.path.join(LLVM, "clang"), os.path.join(LLVM, "clang++")
        if not (os.path.exists(cc) and os.path.exists(cxx)):
            pytest.skip("clang for the ThreadSanitizer build not available")
    else:
        cc, cxx = shutil.which("gcc"), shutil.which("g++")
        if cc is None or cxx is None:
            pytest.skip("gcc / g++ not available")
    san = SANITIZERS[request.param]
    tmp = tmp_path_factory.mktemp("server_fake_" + request.param)
    obj = str(tmp / "oracle.o")
    _run([cc, "-O1", "-g", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
          "-fno-omit-frame-pointer", "-c", os.path.join(ORACLE, "tsqbx_oracle.c"), "-o", obj] + san)
    exe = str(tmp / "server_fake")
    _run([cxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-I", INCLUDE, "-I", CSRC,
          "-I", ORACLE, os.path.join(HERE, "server_fake_driver.cc"), obj, "-fopenmp", "-lpthread",
          "-o", exe] + san)
    return request.param, exe


@pytest.mark.parametrize("scenario", SCENARIOS)
def test_scheduler_with_fake_executor(driver, scenario):
    kind, exe = driver
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["TSAN_OPTIONS"] = "halt_on_error=1:second_deadlock_stack=1:ignore_noninstrumented_modules=1"
    env["OMP_NUM_THREADS"] = "1"
    r = subprocess.run([exe, scenario], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (kind, scenario, r.returncode, r.stdout[-2000:], r.stderr[-6000:])
    assert f"{scenario} ok" in r.stdout
    for bad in ("runtime error", "AddressSanitizer", "ThreadSanitizer", "LeakSanitizer"):
        assert bad not in r.stderr, (kind, scenario, r.stderr[-6000:])
