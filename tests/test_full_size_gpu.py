"""The batched (Laplace and Helmholtz) and served workloads at full size, in
the configurations the benchmark times (one plan over all geometries; the
server with pinned submissions), checked against the oracle: every target of
the Laplace workloads, sampled targets of the Helmholtz one."""
import os

import numpy as np
import pytest

import oracle
from conftest import assert_parity, cached_workload
from paper_1811_01110_amd import api
from paper_1811_01110_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


def _check_all(g, p, layers, outs, what, sigma=None):
    ref = oracle.evaluate_geometry(g, p=p, layers=layers, sigma=sigma)
    for bit, name in ((1, "slp"), (2, "dlp")):
        if layers & bit:
            assert_parity(outs[name], ref[name], ref["abs_" + name], what=f"{what} {name}")


def _plan_items(ctx, geoms, p=None, layers=None):
    items = []
    for g in geoms:
        lay = g.layers if layers is None else layers
        items.append(dict(
            geom=ctx.geometry(g), p=g.p if p is None else p, layers=lay, g=g,
            sigma=torch.tensor(g.sigma, device="cuda", dtype=torch.float64),
            out_slp=torch.zeros(g.n_targets, device="cuda", dtype=torch.float64) if lay & 1 else None,
            out_dlp=torch.zeros(g.n_targets, device="cuda", dtype=torch.float64) if lay & 2 else None))
    return items


def test_batched_64_geometries_full_size(ctx):
    """64 geometries, N log-uniform 2048..65536, p in {4, 8, 12, 16}, single layer."""
    geoms = cached_workload("config_c")
    print("64 batched geometries, pairs", sum(int(g.list_offsets[-1]) for g in geoms), flush=True)
    items = _plan_items(ctx, geoms)
    plan = ctx.plan(items)
    plan.execute()
    plan.execute()  # a graph replay after the capturing launch
    torch.cuda.synchronize()
    for it in items:
        outs = {"slp": it["out_slp"].cpu().numpy()}
        _check_all(it["g"], it["p"], 1, outs, f"C batched p={it['p']} layers=1")
    plan.close()
    for it in items:
        it["geom"].close()


def test_high_order_16_geometries_full_size(ctx):
    """16 perturbed spheres of 131072 sources and 32768 targets, k-nearest
    lists of 100..8000 sources, p = 24, double layer."""
    geoms = cached_workload("config_d")
    print("16 high-order geometries, pairs", sum(int(g.list_offsets[-1]) for g in geoms),
          flush=True)
    items = _plan_items(ctx, geoms, p=24, layers=2)
    plan = ctx.plan(items)
    plan.execute()
    torch.cuda.synchronize()
    for it in items:
        outs = {"dlp": it["out_dlp"].cpu().numpy()}
        _check_all(it["g"], 24, 2, outs, "D batched p=24 layers=2")
    plan.close()
    for it in items:
        it["geom"].close()


def test_server_full_size_geometries(ctx):
    """The 32 resident serving geometries (N log-uniform 4096..262144) and a
    burst of requests with p in {8, 16} and one layer each, submitted pinned
    as the benchmark does."""
    geoms = cached_workload("config_e_geometries")
    gs = [ctx.geometry(g) for g in geoms]
    reqs = W.config_e_requests(96, rate_hz=1.0)
    print("serving", len(reqs), "requests over", len(gs), "geometries", flush=True)
    srv = ctx.server(2 << 30, 256)
    sig, outs = [], []
    for r in reqs:
        g = gs[r.geometry]
        s = torch.empty(g.n_sources, dtype=torch.float64, pin_memory=True)
        s.numpy()[:] = W.request_sigma(r, g.n_sources)
        o = torch.zeros(g.n_targets, dtype=torch.float64, pin_memory=True)
        sig.append(s)
        outs.append(o)
        a, b = (o, None) if r.layers == 1 else (None, o)
        srv.submit_pinned(g, s, r.p, r.layers, out_slp=a, out_dlp=b)
    srv.drain(300)
    srv.close()
    for r, s, o in zip(reqs, sig, outs):
        g = geoms[r.geometry]
        name = "slp" if r.layers == 1 else "dlp"
        _check_all(g, r.p, r.layers, {name: o.numpy()}, f"E served p={r.p} layers={r.layers}",
                   sigma=s.numpy())
    for g in gs:
        g.close()


def test_helmholtz_batched_64_geometries_full_size(ctx):
    """The 64 batched geometries with the Helmholtz single and double layer
    (k = 10, each geometry's own order) in one Helmholtz plan, as the
    benchmark times it; sampled targets against the Helmholtz oracle."""
    from oracle import helmholtz as H

    geoms = cached_workload("config_c")
    rng = np.random.default_rng(20181102)
    items = []
    for g in geoms:
        sig = rng.standard_normal(g.n_sources) + 1j * rng.standard_normal(g.n_sources)
        items.append(dict(
            geom=ctx.geometry(g), p=g.p, layers=3, k=10.0, g=g, sig=sig,
            sigma=torch.tensor(sig, device="cuda", dtype=torch.complex128),
            out_slp=torch.zeros(g.n_targets, device="cuda", dtype=torch.complex128),
            out_dlp=torch.zeros(g.n_targets, device="cuda", dtype=torch.complex128)))
    plan = ctx.plan_helmholtz(items)
    plan.execute()
    torch.cuda.synchronize()
    pick = np.random.default_rng(65)
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with H.process_pool(workers) as pool:
        for it in items:
            g = it["g"]
            sel = np.sort(pick.choice(g.n_targets, min(64, g.n_targets), replace=False))
            ref = H.evaluate_parallel(g, 10.0, it["sig"], p=g.p, layers=3, select=sel,
                                      workers=workers, pool=pool)
            for key, name in (("out_slp", "slp"), ("out_dlp", "dlp")):
                got = it[key].cpu().numpy()[sel]
                assert_parity(got, ref[name], ref["abs_" + name],
                              what=f"C Helmholtz batched k=10 layers=3 {name}")
    plan.close()
    for it in items:
        it["geom"].close()
