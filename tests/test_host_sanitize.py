"""The library's host runtime under AddressSanitizer and UBSan, on the CPU:
geometry validation, the host layout of a geometry (Morton orders, row remap
and padding), the batch schedule with list lengths whose sums pass 2^31, and
the server's first-fit arena against a byte-map model.  The host-side
translation units (API, plans, server) are compiled with the sanitizers and
linked with the device-code objects of the normal build."""
import os
import shutil
import subprocess

import pytest

from paper_1811_01110_amd import build as B

HERE = os.path.dirname(os.path.abspath(__file__))
HOST_SOURCES = ["tsqbx_api.hip", "tsqbx_plan.hip", "tsqbx_server.hip"]
SAN = ["-Xarch_host", "-fsanitize=address,undefined", "-Xarch_host",
       "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (" ".join(cmd), r.stdout[-2000:], r.stderr[-4000:])
    return r


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    clang = "/opt/rocm/llvm/bin/clang++"
    if not os.path.exists(clang) or shutil.which("hipcc") is None and not os.path.exists(B.hipcc()):
        pytest.skip("ROCm compilers not available")
    tmp = tmp_path_factory.mktemp("host_asan")
    device_objs = [os.path.join(B.BUILD, os.path.splitext(s)[0] + ".o")
                   for s in B.SOURCES if s not in HOST_SOURCES]
    if not all(os.path.exists(o) for o in device_objs):
        B.build()
    objs = []
    for src in HOST_SOURCES:
        o = str(tmp / (os.path.splitext(src)[0] + "_asan.o"))
        _run([B.hipcc(), "-x", "hip", "--cuda-host-only", "-O1", "-g", "-std=c++17", "-fPIC",
              "-ffp-contract=off", "-I", B.INCLUDE, "-I", B.CSRC] + SAN +
             ["-c", os.path.join(B.CSRC, src), "-o", o])
        objs.append(o)
    lib = str(tmp / "libtsqbx_asan.so")
    _run([B.hipcc(), f"--offload-arch={B.ARCH}", "-shared", "-fPIC", "-o", lib] + objs +
         device_objs + ["-lrocprofiler-sdk-roctx", "-lpthread"])
    exe = str(tmp / "host_asan")
    _run([clang, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-I", B.INCLUDE, "-I", B.CSRC,
          os.path.join(HERE, "host_sanitize_driver.cc"), "-L", str(tmp), "-ltsqbx_asan",
          "-Wl,-rpath," + str(tmp), "-o", exe])
    return exe


def test_host_runtime_under_sanitizers(driver):
    env = dict(os.environ)
    env["LD_LIBRARY_PATH"] = "/opt/rocm/lib:" + env.get("LD_LIBRARY_PATH", "")
    # leaks in the uninstrumented runtime libraries at exit are not this code's
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([driver], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    assert "host sanitize ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
