"""Conventional QBX on the GPU (local coefficients formed per center, then
evaluated; Sec. 2.3) against the oracles, through the C ABI.

* Coefficients: element by element against the conventional oracle
  (eqs. sph-harm and local-coeffs), |gpu - oracle| <= 1e-12 times the sum of
  the absolute values of the terms of that coefficient.
* Potentials: against the target-specific oracle (eq. tsqbx says the two
  agree), with the parity bar of the target-specific path.
* The fused launch equals formation followed by evaluation bit for bit.
"""
import numpy as np
import pytest

import oracle
from conftest import assert_parity, cached_workload
from oracle import conventional as conv
from paper_1811_01110_amd import _lib as L
from paper_1811_01110_amd import api
from paper_1811_01110_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device="cuda")


def _run(ctx, geom, g, p, what):
    """Form, evaluate and fused launch; returns (coeffs, u_from_coeffs, u_fused)."""
    nc = (p + 1) ** 2
    sig = _dev(g.sigma)
    coeffs = torch.full((geom.n_centers * nc,), float("nan"), dtype=torch.float64, device="cuda")
    u1 = torch.zeros(geom.n_targets, dtype=torch.float64, device="cuda")
    u2 = torch.zeros(geom.n_targets, dtype=torch.float64, device="cuda")
    print(what, "p", p, "centers", geom.n_centers, "targets", geom.n_targets, flush=True)
    ctx.qbxl_form_async(geom, sig, p, coeffs)
    ctx.qbxl_eval_async(geom, coeffs, p, u1)
    ctx.eval_conventional_async(geom, sig, p, u2)
    torch.cuda.synchronize()
    return (coeffs.cpu().numpy().reshape(geom.n_centers, nc), u1.cpu().numpy(),
            u2.cpu().numpy())


def _check_coeffs(g, C, p, which, what):
    L = conv.form(g.sources, g.weights, g.centers, g.list_offsets, g.list_sources, g.sigma, p,
                  which=which)
    S = conv.coefficient_scale(g.sources, g.weights, g.centers, g.list_offsets, g.list_sources,
                               g.sigma, p, which=which)
    ref = conv.pack(L, p)
    sc = conv.pack(S.astype(np.complex128) * (1 + 1j), p)  # scale of Re and Im parts
    got = C[which]
    assert np.all(np.isfinite(got)), f"{what}: non-finite coefficients"
    err = np.abs(got - ref)
    bad = err > 1e-12 * np.abs(sc) + 1e-300
    assert not bad.any(), f"{what}: worst ratio {np.max(err / np.maximum(np.abs(sc), 1e-300)):.3e}"


@pytest.mark.parametrize("p", [0, 1, 2, 5, 8, 9, 12, 16, 17, 24, 32])
def test_coefficients_and_potentials_every_kernel(ctx, p):
    """Exact-order kernels (5, 8, 16) and the capped ones (<= 16, <= 32), ragged
    lists with empty rows and duplicates, two targets per center."""
    g = W.fuzz_geometry(4000 + p, n=300, m=24, max_list=70, p=p, layers=1, targets_per_center=2)
    geom = ctx.geometry(g)
    C, u1, u2 = _run(ctx, geom, g, p, "fuzz")
    _check_coeffs(g, C, p, np.arange(g.n_centers), f"coeffs p={p}")
    ref = oracle.evaluate_geometry(g, p=p, layers=1)
    assert_parity(u2, ref["slp"], ref["abs_slp"], what=f"fused p={p}")
    assert np.array_equal(u1, u2), "formation + evaluation differs from the fused launch"
    # the same geometry without the Morton reordering: same bits
    geom_n = ctx.geometry(g, flags=api.NO_REORDER)
    Cn, u1n, u2n = _run(ctx, geom_n, g, p, "fuzz no-reorder")
    assert np.array_equal(u2n, u1n)
    assert_parity(u2n, ref["slp"], ref["abs_slp"], what=f"fused p={p} no-reorder")
    geom.close()
    geom_n.close()


def test_oracle_coefficients_evaluate_on_gpu(ctx):
    """QBXL2P alone: the oracle's coefficients evaluated on the GPU."""
    p = 12
    g = W.fuzz_geometry(4100, n=300, m=20, max_list=60, p=p, layers=1, targets_per_center=3)
    geom = ctx.geometry(g)
    L = conv.form(g.sources, g.weights, g.centers, g.list_offsets, g.list_sources, g.sigma, p)
    u = torch.zeros(geom.n_targets, dtype=torch.float64, device="cuda")
    ctx.qbxl_eval_async(geom, _dev(conv.pack(L, p).ravel()), p, u)
    ref = oracle.evaluate_geometry(g, p=p, layers=1)
    assert_parity(u.cpu().numpy(), ref["slp"], ref["abs_slp"], what="eval of oracle coefficients")
    geom.close()


def test_accumulate_and_unused_centers(ctx):
    """ACCUMULATE adds; rows of centers no target uses stay untouched."""
    p = 8
    g0 = W.fuzz_geometry(4200, n=200, m=30, max_list=50, p=p, layers=1)
    used = np.arange(0, 30, 3)
    tc = np.repeat(used, 2).astype(np.int32)
    rng = np.random.default_rng(3)
    tgt = g0.centers[tc] + 0.1 * rng.standard_normal((len(tc), 3))
    g = W.Geometry(g0.sources, g0.weights, g0.normals, g0.centers, g0.list_offsets,
                   g0.list_sources, tgt, tc, g0.sigma, p, 1)
    geom = ctx.geometry(g)
    C, u1, u2 = _run(ctx, geom, g, p, "subset")
    unused = np.setdiff1d(np.arange(30), used)
    assert np.all(np.isnan(C[unused])), "a row of an unused center was written"
    _check_coeffs(g, C, p, used, "subset coeffs")
    ref = oracle.evaluate_geometry(g, p=p, layers=1)
    assert_parity(u2, ref["slp"], ref["abs_slp"], what="subset fused")
    # accumulate: coefficients doubled exactly, potentials added
    nc = (p + 1) ** 2
    sig = _dev(g.sigma)
    co = _dev(np.nan_to_num(C, nan=0.0).ravel())
    ctx.qbxl_form_async(geom, sig, p, co, flags=api.ACCUMULATE)
    u = _dev(u2)
    ctx.eval_conventional_async(geom, sig, p, u, flags=api.ACCUMULATE)
    u3 = _dev(u2)
    ctx.qbxl_eval_async(geom, co, p, u3, flags=api.ACCUMULATE)  # co now holds 2 L
    torch.cuda.synchronize()
    co = co.cpu().numpy().reshape(30, nc)
    assert np.array_equal(co[used], 2 * C[used])
    assert np.array_equal(u.cpu().numpy(), u2 + u2)
    assert np.allclose(u3.cpu().numpy(), 3 * u2, rtol=1e-13, atol=1e-13 * np.abs(u2).max())
    geom.close()


def test_dense_config_a(ctx):
    """Config A (4096 sources, 1024 targets, every list holds every source, p = 8)."""
    g = cached_workload("config_a")
    geom = ctx.geometry(g)
    C, u1, u2 = _run(ctx, geom, g, g.p, "config A")
    ref = oracle.evaluate_geometry(g, p=g.p, layers=1)
    assert_parity(u2, ref["slp"], ref["abs_slp"], what="A conventional")
    assert np.array_equal(u1, u2)
    sel = np.array([0, 17, 511, 1023])
    _check_coeffs(g, C, g.p, sel, "A coeffs")
    geom.close()


def test_config_b_p16(ctx):
    """Geometry B at full size (262144 sources, 65536 targets, p = 16): every
    target's potential against the target-specific oracle, the coefficients of
    sampled centers against the conventional oracle."""
    g = cached_workload("config_b", 1)
    geom = ctx.geometry(g)
    C, u1, u2 = _run(ctx, geom, g, 16, "config B")
    rng = np.random.default_rng(9)
    ref = oracle.evaluate_geometry(g, p=16, layers=1)
    assert_parity(u2, ref["slp"], ref["abs_slp"], what="B conventional p=16 layers=1")
    assert np.array_equal(u1, u2)
    _check_coeffs(g, C, 16, np.sort(rng.choice(g.n_centers, 8, replace=False)), "B coeffs")
    geom.close()


def test_edge_cases(ctx):
    # every list empty: zero coefficients and potentials
    g = W.fuzz_geometry(4300, n=20, m=6, max_list=5, p=4, layers=1)
    off = np.zeros(g.n_centers + 1, dtype=np.int64)
    ge = W.Geometry(g.sources, g.weights, g.normals, g.centers, off, np.zeros(0, dtype=np.int32),
                    g.targets, g.target_center, g.sigma, 4, 1)
    geom = ctx.geometry(ge)
    C, u1, u2 = _run(ctx, geom, ge, 4, "empty lists")
    assert not np.any(C) and not np.any(u1) and not np.any(u2)
    geom.close()
    # target at its center (rho = 0): only n = 0 survives
    one = W.Geometry(np.array([[1.0, 2.0, 0.5], [-0.3, 0.2, 1.1]]), np.array([0.7, 0.4]), None,
                     np.zeros((1, 3)), np.array([0, 2]), np.array([0, 1], dtype=np.int32),
                     np.zeros((1, 3)), None, np.array([1.3, -0.6]), 9, 1)
    geom = ctx.geometry(one)
    C, u1, u2 = _run(ctx, geom, one, 9, "rho=0")
    ref = oracle.evaluate_geometry(one, p=9, layers=1)
    assert_parity(u2, ref["slp"], ref["abs_slp"], what="rho=0")
    geom.close()
    # no targets: nothing to do, nothing written
    g0 = W.Geometry(g.sources, g.weights, g.normals, g.centers, g.list_offsets, g.list_sources,
                    np.zeros((0, 3)), np.zeros(0, dtype=np.int32), g.sigma, 4, 1)
    geom = ctx.geometry(g0)
    C, u1, u2 = _run(ctx, geom, g0, 4, "no targets")
    assert np.all(np.isnan(C)) and u1.size == 0
    geom.close()


def test_errors(ctx):
    g = W.fuzz_geometry(4400, n=30, m=4, max_list=10, p=4, layers=1)
    geom = ctx.geometry(g)
    sig = _dev(g.sigma)
    out = torch.zeros(geom.n_targets, dtype=torch.float64, device="cuda")
    with pytest.raises(api.TsqbxError) as e:
        ctx.eval_conventional_async(geom, sig, 33, out)
    assert e.value.code == L.E_RANGE
    with pytest.raises(api.TsqbxError) as e:
        ctx.eval_conventional_async(geom, sig, -1, out)
    assert e.value.code == L.E_RANGE
    lib = api._lib()
    assert lib.tsqbx_eval_conventional_async(ctx.handle, geom.handle, 4, None, out.data_ptr(), 0,
                                             None) == L.E_INVALID
    assert lib.tsqbx_qbxl_form_async(ctx.handle, geom.handle, 4, sig.data_ptr(), None, 0,
                                     None) == L.E_INVALID
    assert lib.tsqbx_qbxl_eval_async(ctx.handle, geom.handle, 4, None, out.data_ptr(), 0,
                                     None) == L.E_INVALID
    assert lib.tsqbx_qbxl_eval_async(ctx.handle, None, 4, None, None, 0, None) == L.E_INVALID
    geom.close()
