"""Helmholtz target-specific expansions (single layer, double layer and S') on
the GPU against the Helmholtz oracle, element by element, through the C ABI
(bar: 1e-12 of the per-target sum of term moduli, and 1e-12 of the largest
output)."""
import os

import numpy as np
import pytest

from conftest import assert_parity, cached_workload
from oracle import helmholtz as H
from paper_1811_01110_amd import api
from paper_1811_01110_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


def _sigma(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


ALL = api.SLP | api.DLP | api.SPRIME


WORKERS = max(1, min(16, len(os.sched_getaffinity(0))))


def _check(ctx, g, k, p, layers, sigma, select=None, what="", parallel=False):
    geom = ctx.geometry(g)
    out = ctx.eval_helmholtz(geom, sigma, p, layers, k)
    if parallel:
        ref = H.evaluate_parallel(g, k, sigma, p=p, layers=layers, select=select, workers=WORKERS)
    else:
        ref = H.evaluate_geometry(g, k, sigma, p=p, layers=layers, select=select)
    sel = slice(None) if select is None else select
    for o, bit, key in zip(out, (api.SLP, api.DLP, api.SPRIME), ("slp", "dlp", "sprime")):
        if layers & bit:
            assert_parity(o[sel], ref[key], ref["abs_" + key], what=f"{what} {key}")
        else:
            assert o is None
    geom.close()
    return out


@pytest.mark.parametrize("p", [0, 1, 2, 3, 5, 8, 12, 16, 24, 32])
@pytest.mark.parametrize("k", [0.5, 3.0, 20.0])
def test_orders_and_wavenumbers(ctx, p, k):
    g = W.fuzz_geometry(800 + p, n=250, m=50, max_list=120, p=p, layers=3, targets_per_center=2)
    _check(ctx, g, k, p, ALL, _sigma(g.n_sources, p), what=f"p={p} k={k}")


def test_layer_masks_share_bits(ctx):
    """Every layer is computed the same way whichever others are requested."""
    g = W.fuzz_geometry(850, n=600, m=100, max_list=300, p=16, layers=3)
    sig = _sigma(g.n_sources, 1)
    full = _check(ctx, g, 20.0, 16, ALL, sig, what="all")
    for layers in range(1, 7):
        out = _check(ctx, g, 20.0, 16, layers, sig, what=f"mask {layers}")
        for i, bit in enumerate((api.SLP, api.DLP, api.SPRIME)):
            if layers & bit:
                assert np.array_equal(out[i], full[i]), (layers, bit)


def test_large_and_tiny_k_rho(ctx):
    """k rho > p + 1 takes the upward recurrence for j_n; targets 1e-4 from
    their centers at p = 32 take Miller's recurrence through its rescaling."""
    g = W.fuzz_geometry(851, n=300, m=60, max_list=150, p=4, layers=3)
    _check(ctx, g, 100.0, 4, ALL, _sigma(g.n_sources, 2), what="k=100 p=4")
    h = W.fuzz_geometry(852, n=300, m=60, max_list=150, p=32, layers=3)
    rng = np.random.default_rng(3)
    off = rng.standard_normal((h.n_targets, 3))
    h.targets = h.centers[h.target_center] + 1e-4 * off / np.linalg.norm(off, axis=1)[:, None]
    _check(ctx, h, 1.0, 32, ALL, _sigma(h.n_sources, 4), what="rho=1e-4 p=32")


def test_target_at_center_and_edge_lists(ctx):
    g = W.fuzz_geometry(853, n=200, m=40, max_list=60, p=9, layers=3, targets_per_center=2)
    g.targets[:7] = g.centers[g.target_center[:7]]
    _check(ctx, g, 5.0, 9, ALL, _sigma(g.n_sources, 5), what="t=c")
    off = np.zeros(g.n_centers + 1, dtype=np.int64)
    e = W.Geometry(g.sources, g.weights, g.normals, g.centers, off, np.zeros(0, dtype=np.int32),
                   g.targets, g.target_center, g.sigma, 9, 3, target_normals=g.target_normals)
    geom = ctx.geometry(e)
    out = ctx.eval_helmholtz(geom, _sigma(g.n_sources, 6), 9, ALL, 5.0)
    assert all(np.all(o == 0) for o in out)
    geom.close()


def _morton_keys(points):
    """63-bit Morton keys of points over their bounding box (21 bits per axis)."""
    lo = points.min(axis=0)
    ext = max(float((points.max(axis=0) - lo).max()), 1e-300)
    q = np.minimum(((points - lo) / ext * (1 << 21)).astype(np.int64), (1 << 21) - 1)
    key = np.zeros(len(points), dtype=np.int64)
    for b in range(21):
        for a in range(3):
            key |= ((q[:, a] >> b) & 1) << (3 * b + a)
    return key


def test_config_b_full_size_sampled(ctx):
    """4096 of the 65536 targets, k = 20, p = 16, all three layers: the 512
    targets whose centers come first and the 512 that come last along a Morton
    curve (the first and last blocks of the kernel's target order) and 3072
    drawn at random."""
    g = cached_workload("config_b", 1)
    sig = _sigma(g.n_sources, 7)
    tc = np.arange(g.n_targets) if g.target_center is None else g.target_center
    order = np.argsort(_morton_keys(g.centers[tc]), kind="stable")
    ends = np.concatenate([order[:512], order[-512:]])
    rest = np.setdiff1d(np.arange(g.n_targets), ends)
    rng = np.random.default_rng(8)
    sel = np.sort(np.concatenate([ends, rng.choice(rest, 3072, replace=False)]))
    _check(ctx, g, 20.0, 16, ALL, sig, select=sel, what="B k=20 p=16 layers=7", parallel=True)


def test_async_accumulate_and_tuning_variants(ctx):
    import torch

    g = W.fuzz_geometry(854, n=1500, m=250, max_list=500, p=12, layers=3)
    geom = ctx.geometry(g)
    sig = _sigma(g.n_sources, 9)
    ref = H.evaluate_geometry(g, 8.0, sig, p=12, layers=ALL)
    host = ctx.eval_helmholtz(geom, sig, 12, ALL, 8.0)
    ts = torch.tensor(sig, device="cuda", dtype=torch.complex128)
    dev = [torch.zeros(g.n_targets, device="cuda", dtype=torch.complex128) for _ in range(3)]
    ctx.eval_helmholtz_async(geom, ts, 12, ALL, 8.0, *dev)
    torch.cuda.synchronize()
    for o, h in zip(dev, host):
        assert np.array_equal(o.cpu().numpy(), h)
    ctx.eval_helmholtz_async(geom, ts, 12, ALL, 8.0, *dev, flags=api.ACCUMULATE)
    torch.cuda.synchronize()
    for o, h in zip(dev, host):
        assert np.array_equal(o.cpu().numpy(), h + h)
    acc = [h.copy() for h in host]
    ctx.eval_helmholtz(geom, sig, 12, ALL, 8.0, *acc, flags=api.ACCUMULATE)
    for o, h in zip(acc, host):
        assert np.array_equal(o, h + h)
    mean = max(geom.pairs // geom.n_targets, 1)
    keys = ("slp", "dlp", "sprime")
    base = None
    for G, U in ((64, 1), (64, 2), (32, 2), (16, 2)):
        for w in (1, 4):
            ctx.set_tuning(12, ALL | api.HELMHOLTZ, mean, group_lanes=G, unroll=U, waves_per_block=w)
            out = ctx.eval_helmholtz(geom, sig, 12, ALL, 8.0)
            for o, key in zip(out, keys):
                assert_parity(o, ref[key], ref["abs_" + key], what=f"G{G}U{U}w{w} {key}")
            if G == 64:
                base = out if base is None else base
                assert all(np.array_equal(a, b) for a, b in zip(out, base))
    geom.close()


def test_rejects_bad_requests(ctx):
    g = W.fuzz_geometry(855, n=50, m=10, max_list=20, p=4, layers=1)
    sig = _sigma(g.n_sources, 10)
    geom = ctx.geometry(g)
    for layers, k, code in ((8, 1.0, -1), (1, 0.0, -2), (1, -3.0, -2),
                            (1, float("inf"), -2), (0, 1.0, -1)):
        with pytest.raises(api.TsqbxError) as ei:
            ctx.eval_helmholtz(geom, sig, 4, layers, k)
        assert ei.value.code == code, (layers, k)
    with pytest.raises(api.TsqbxError) as ei:
        ctx.eval_helmholtz(geom, sig, 33, 1, 1.0)
    assert ei.value.code == -2
    geom.close()
    g.normals = None
    geom = ctx.geometry(g)
    with pytest.raises(api.TsqbxError) as ei:
        ctx.eval_helmholtz(geom, sig, 4, api.DLP, 1.0)
    assert ei.value.code == -1
    geom.close()
    g.target_normals = None
    geom = ctx.geometry(g)
    with pytest.raises(api.TsqbxError) as ei:
        ctx.eval_helmholtz(geom, sig, 4, api.SPRIME, 1.0)
    assert ei.value.code == -1
    geom.close()


def _plan_items(ctx, torch, specs, seed):
    """Items (geometry, p, layers, k) on fuzz geometries, complex densities."""
    items = []
    for i, (p, lay, k, share) in enumerate(specs):
        if share:
            g, geom = items[-1]["g"], items[-1]["geom"]
        else:
            g = W.fuzz_geometry(seed + i, n=400 + 60 * i, m=90, max_list=220, p=p, layers=3,
                                targets_per_center=2)
            geom = ctx.geometry(g)
        sig = _sigma(g.n_sources, seed + 100 + i)
        it = dict(g=g, geom=geom, p=p, layers=lay, k=k, sig=sig,
                  sigma=torch.tensor(sig, device="cuda", dtype=torch.complex128))
        for bit, key in ((1, "out_slp"), (2, "out_dlp"), (4, "out_sprime")):
            if lay & bit:
                it[key] = torch.zeros(g.n_targets, device="cuda", dtype=torch.complex128)
        items.append(it)
    return items


def _ceil_mean(pairs, targets):
    return max(-(-pairs // max(targets, 1)), 1)


@pytest.mark.parametrize("G", [16, 64])
def test_plan_matches_plain_bits_and_oracle(ctx, G):
    """A Helmholtz plan (mixed orders, masks and wavenumbers, two items on one
    geometry) equals plain evaluations with the same group width bit for bit,
    and the oracle to the parity bar; replays with new densities and the
    accumulate flag behave as for Laplace plans."""
    import torch

    specs = [(4, 1, 2.0, False), (8, 3, 5.0, False), (12, 4, 10.0, False), (16, 7, 20.0, False),
             (16, 7, 3.0, True), (5, 2, 1.0, False), (0, 5, 3.0, False), (24, 6, 8.0, False)]
    items = _plan_items(ctx, torch, specs, 870)
    # the plan's launch shape comes from (largest p, union of masks, mean list)
    pairs = sum(it["geom"].pairs for it in items)
    targets = sum(it["geom"].n_targets for it in items)
    ctx.set_tuning(24, 7 | api.HELMHOLTZ, _ceil_mean(pairs, targets), group_lanes=G)
    for it in items:
        geom = it["geom"]
        ctx.set_tuning(it["p"], it["layers"] | api.HELMHOLTZ, _ceil_mean(geom.pairs, geom.n_targets),
                       group_lanes=G)
    plan = ctx.plan_helmholtz(items)
    assert plan.info()["n_items"] == len(items)
    keys = ("slp", "dlp", "sprime")

    def check(its, acc=1):
        for it in its:
            g, geom = it["g"], it["geom"]
            plain = ctx.eval_helmholtz(geom, it["sig"], it["p"], it["layers"], it["k"])
            ref = H.evaluate_geometry(g, it["k"], it["sig"], p=it["p"], layers=it["layers"])
            for bit, key, pl in zip((1, 2, 4), keys, plain):
                if not it["layers"] & bit:
                    continue
                got = it["out_" + key].cpu().numpy()
                assert np.array_equal(got, acc * pl), (G, it["p"], it["layers"], key)
                assert_parity(got / acc, ref[key], ref["abs_" + key], what=f"plan p={it['p']} {key}")

    plan.execute()
    torch.cuda.synchronize()
    check(items)
    rng = np.random.default_rng(5)
    for it in items:  # new densities, same plan (graph replay)
        it["sig"] = rng.standard_normal(it["g"].n_sources) + 1j * rng.standard_normal(it["g"].n_sources)
        it["sigma"].copy_(torch.tensor(it["sig"], dtype=torch.complex128))
    torch.cuda.synchronize()
    plan.execute()
    plan.execute()
    torch.cuda.synchronize()
    check(items)
    plan.close()
    acc_plan = ctx.plan_helmholtz(items, flags=api.ACCUMULATE)
    acc_plan.execute()
    torch.cuda.synchronize()
    check(items, acc=2)
    acc_plan.close()


def test_plan_rejects_bad_items(ctx):
    import torch

    items = _plan_items(ctx, torch, [(4, 1, 2.0, False)], 880)
    for bad in (dict(k=0.0), dict(k=float("nan")), dict(p=33), dict(layers=8)):
        it = dict(items[0], **bad)
        with pytest.raises(api.TsqbxError):
            ctx.plan_helmholtz([it])
    it = dict(items[0], layers=3)  # the double layer's output is missing
    with pytest.raises((api.TsqbxError, TypeError, KeyError)):
        ctx.plan_helmholtz([it])


def test_plan_edge_cases(ctx):
    """An empty Helmholtz plan runs and does nothing; an item with every list
    empty gives 0 beside an ordinary item; one with no targets is valid."""
    import torch

    empty = ctx.plan_helmholtz([])
    empty.execute()
    torch.cuda.synchronize()
    empty.close()
    g = W.fuzz_geometry(890, n=300, m=60, max_list=120, p=6, layers=3)
    no_lists = W.Geometry(g.sources, g.weights, g.normals, g.centers,
                          np.zeros(g.n_centers + 1, dtype=np.int64), np.zeros(0, dtype=np.int32),
                          g.targets, g.target_center, g.sigma, 6, 3,
                          target_normals=g.target_normals)
    no_targets = W.Geometry(g.sources, g.weights, g.normals, g.centers, g.list_offsets,
                            g.list_sources, np.zeros((0, 3)), np.zeros(0, dtype=np.int32),
                            g.sigma, 6, 3, target_normals=np.zeros((0, 3)))
    sig = _sigma(g.n_sources, 11)
    items = []
    for geo in (g, no_lists, no_targets):
        geom = ctx.geometry(geo)
        it = dict(g=geo, geom=geom, p=6, layers=ALL, k=4.0,
                  sigma=torch.tensor(sig, device="cuda", dtype=torch.complex128))
        for key in ("out_slp", "out_dlp", "out_sprime"):
            it[key] = torch.full((geo.n_targets,), 7.0 + 0j, device="cuda", dtype=torch.complex128)
        items.append(it)
    plan = ctx.plan_helmholtz(items)
    plan.execute()
    torch.cuda.synchronize()
    ref = H.evaluate_geometry(g, 4.0, sig, p=6, layers=ALL)
    for key in ("slp", "dlp", "sprime"):
        assert_parity(items[0]["out_" + key].cpu().numpy(), ref[key], ref["abs_" + key], what=key)
        assert not items[1]["out_" + key].any()
    plan.close()
    out = ctx.eval_helmholtz(items[2]["geom"], sig, 6, ALL, 4.0)  # no targets, plain path
    assert all(o.size == 0 for o in out)
