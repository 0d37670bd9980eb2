"""The entry point that allocates nothing (tsqbx_eval_async_noalloc, for
callers that cannot allocate device memory) against tsqbx_eval_async: two
calls in a row through the C ABI, the second on a smaller geometry, each equal
to the existing entry point bit for bit and to the oracle at the parity bar;
the size limit is refused from the counts."""
import ctypes

import numpy as np
import pytest

import oracle
from conftest import assert_parity
from paper_1811_01110_amd import _lib as L
from paper_1811_01110_amd import api
from paper_1811_01110_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _run(lib, entry, ctx, geom, sig, p, layers, outs, stream):
    rc = getattr(lib, entry)(ctx.handle, geom.handle, p, layers, _ptr(sig),
                             *[_ptr(o) for o in outs], 0, ctypes.c_void_p(stream))
    assert rc == 0, (entry, rc, lib.tsqbx_last_error())


def test_noalloc_equals_eval_async_twice():
    lib = L.load()
    ctx = api.Context(0)
    stream = torch.cuda.current_stream().cuda_stream
    try:
        cases = [  # the second smaller than the first
            (W.fuzz_geometry(900, n=3000, m=500, max_list=700, p=16, layers=7), 16, 7),
            (W.fuzz_geometry(901, n=800, m=150, max_list=300, p=9, layers=3), 9, 3),
        ]
        for g, p, layers in cases:
            geom = ctx.geometry(g)
            sig = torch.tensor(g.sigma, device="cuda", dtype=torch.float64)
            a = [torch.full((g.n_targets,), -1.0, device="cuda", dtype=torch.float64)
                 if layers & b else None for b in (1, 2, 4)]
            b = [torch.full((g.n_targets,), -2.0, device="cuda", dtype=torch.float64)
                 if layers & b else None for b in (1, 2, 4)]
            _run(lib, "tsqbx_eval_async_noalloc", ctx, geom, sig, p, layers, a, stream)
            _run(lib, "tsqbx_eval_async", ctx, geom, sig, p, layers, b, stream)
            torch.cuda.synchronize()
            ref = oracle.evaluate_geometry(g, p=p, layers=layers)
            for x, y, bit, name in zip(a, b, (1, 2, 4), ("slp", "dlp", "sprime")):
                if not layers & bit:
                    continue
                xa, ya = x.cpu().numpy(), y.cpu().numpy()
                assert np.array_equal(xa, ya), (g.name, name)
                assert_parity(xa, ref[name], ref["abs_" + name], what=f"noalloc {name}")
            geom.close()
    finally:
        ctx.close()


def test_noalloc_size_limit():
    """Staging beyond the scratch array is refused (TSQBX_E_RANGE) with the
    double layer; the same geometry fits with the single layer alone."""
    lib = L.load()
    ctx = api.Context(0)
    try:
        n = 299592  # N + 1 = 299593 sources' staging exceeds 16 MiB with the double layer
        rng = np.random.default_rng(3)
        src = rng.standard_normal((n, 3))
        src /= np.linalg.norm(src, axis=1)[:, None]
        ctr = np.zeros((1, 3))
        g = W.Geometry(src, np.ones(n), src.copy(), ctr, np.array([0, 4]),
                       np.arange(4, dtype=np.int32), np.array([[0.0, 0.0, 0.1]]), None,
                       np.ones(n), 4, 3)
        geom = ctx.geometry(g)
        sig = torch.ones(n, device="cuda", dtype=torch.float64)
        o1 = torch.zeros(1, device="cuda", dtype=torch.float64)
        o2 = torch.zeros(1, device="cuda", dtype=torch.float64)
        with pytest.raises(api.TsqbxError) as ei:
            ctx.eval_async_noalloc(geom, sig, 4, 3, o1, o2)
        assert ei.value.code == -2
        assert b"scratch" in lib.tsqbx_last_error()
        ctx.eval_async_noalloc(geom, sig, 4, 1, o1)
        ctx.eval_async(geom, sig, 4, 1, o2)
        torch.cuda.synchronize()
        assert torch.equal(o1, o2)
        geom.close()
    finally:
        ctx.close()
