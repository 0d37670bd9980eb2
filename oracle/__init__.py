"""Python access to the plain FP64 CPU oracle (liboracle_tsqbx.so).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg call this; the product library never does.  This module only
marshals arrays; every number comes from tsqbx_oracle.c.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tsqbx_oracle.c")
LIB = os.path.join(HERE, "liboracle_tsqbx.so")

SLP, DLP, SPRIME = 1, 2, 4

_libs = {}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: plain FP64, no fast-math, no FMA contraction."""
    if force or not os.path.exists(LIB):
        compile_source(SRC, LIB)
    return LIB


def compile_source(src: str, out: str) -> str:
    """Compile one C source of the oracle's form into the shared library
    `out`, with the oracle's flags (the tests also build deliberately broken
    copies this way, to show that the pins catch them)."""
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp", "-fPIC",
           "-shared", "-std=c11", "-Wall", "-I", HERE, "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


class _Problem(ctypes.Structure):
    _fields_ = [
        ("n_sources", ctypes.c_int64),
        ("sources", ctypes.c_void_p),
        ("weights", ctypes.c_void_p),
        ("normals", ctypes.c_void_p),
        ("n_centers", ctypes.c_int64),
        ("centers", ctypes.c_void_p),
        ("list_offsets", ctypes.c_void_p),
        ("list_sources", ctypes.c_void_p),
        ("n_targets", ctypes.c_int64),
        ("targets", ctypes.c_void_p),
        ("target_center", ctypes.c_void_p),
        ("target_normals", ctypes.c_void_p),
    ]


def _load(path: str = None):
    """The oracle library at `path` (default: the oracle itself, built on
    first use), with its function signatures declared."""
    path = LIB if path is None else path
    lib = _libs.get(path)
    if lib is None:
        if path == LIB and not os.path.exists(LIB):
            build(force=False)
        lib = ctypes.CDLL(path)
        lib.tsqbx_oracle_pair.argtypes = [ctypes.c_void_p] * 5 + [ctypes.c_int, ctypes.c_void_p]
        lib.tsqbx_oracle_pair.restype = None
        lib.tsqbx_oracle_eval.argtypes = [ctypes.POINTER(_Problem), ctypes.c_int, ctypes.c_uint,
                                          ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        lib.tsqbx_oracle_eval.restype = ctypes.c_int
        lib.tsqbx_oracle_max_threads.restype = ctypes.c_int
        _libs[path] = lib
    return lib


def max_threads() -> int:
    return int(_load().tsqbx_oracle_max_threads())


def _ptr(a):
    return None if a is None else a.ctypes.data


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def pair(t, c, s, nu, p: int, nu_t=None, library: str = None):
    """One pair: [G^(p), nu . grad_s G^(p), |.| yardsticks of both,
    nu_t . grad_t G^(p), its yardstick].  `library` names another build of
    the oracle's source (default: the oracle)."""
    t, c, s = _f64(t, 3), _f64(c, 3), _f64(s, 3)
    nu = None if nu is None else _f64(nu, 3)
    nu_t = None if nu_t is None else _f64(nu_t, 3)
    out = np.zeros(6)
    _load(library).tsqbx_oracle_pair(_ptr(t), _ptr(c), _ptr(s), _ptr(nu), _ptr(nu_t), int(p), _ptr(out))
    return out


def evaluate(sources, weights, normals, centers, list_offsets, list_sources, targets,
             target_center, sigma, p: int, layers: int, select=None, n_threads: int = 0,
             target_normals=None, library: str = None):
    """Potentials at all targets (or the `select`ed ones).

    Returns dict with keys 'slp', 'dlp', 'sprime' and 'abs_' + each (None
    for a layer not requested).  `library` as for pair().
    """
    lib = _load(library)
    src = _f64(sources)
    w = _f64(weights)
    nrm = None if normals is None else _f64(normals)
    ctr = _f64(centers)
    off = np.ascontiguousarray(list_offsets, dtype=np.int64)
    idx = np.ascontiguousarray(list_sources, dtype=np.int32)
    tgt = _f64(targets)
    tc = None if target_center is None else np.ascontiguousarray(target_center, dtype=np.int32)
    tn = None if target_normals is None else _f64(target_normals)
    sig = _f64(sigma)
    prob = _Problem(len(src), _ptr(src), _ptr(w), _ptr(nrm), len(ctr), _ptr(ctr), _ptr(off),
                    _ptr(idx), len(tgt), _ptr(tgt), _ptr(tc), _ptr(tn))
    sel = None if select is None else np.ascontiguousarray(select, dtype=np.int64)
    n_out = len(tgt) if sel is None else len(sel)
    names = ("slp", "dlp", "sprime")
    out = {}
    for bit, k in zip((SLP, DLP, SPRIME), names):
        want = bool(layers & bit)
        out[k] = np.zeros(n_out) if want else None
        out["abs_" + k] = np.zeros(n_out) if want else None
    outs = (ctypes.c_void_p * 3)(*[_ptr(out[k]) for k in names])
    abss = (ctypes.c_void_p * 3)(*[_ptr(out["abs_" + k]) for k in names])
    rc = lib.tsqbx_oracle_eval(ctypes.byref(prob), int(p), int(layers), _ptr(sig),
                               n_out, _ptr(sel), outs, abss, int(n_threads))
    if rc != 0:
        raise ValueError("oracle rejected its arguments")
    return out


def evaluate_geometry(g, p=None, layers=None, sigma=None, select=None, n_threads: int = 0):
    """evaluate() on any object with the workload Geometry attributes."""
    return evaluate(g.sources, g.weights, g.normals, g.centers, g.list_offsets, g.list_sources,
                    g.targets, g.target_center, g.sigma if sigma is None else sigma,
                    g.p if p is None else p, g.layers if layers is None else layers,
                    select=select, n_threads=n_threads,
                    target_normals=getattr(g, "target_normals", None))
