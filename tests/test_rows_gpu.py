"""The row kernel of the plain path (one wave per center's list, four, then
two of its targets per walk, then one) against the one-target-per-wave
kernel (TSQBX_PER_TARGET), bit for bit, and against the oracle, for every
layer mask, compiled and run-time orders, target counts per row from 1 to 6
(every mix of the three walks), accumulation, the
device-resident entry points, and plans and servers (which run the
per-target kernels) on the same geometry."""
import numpy as np
import pytest

import oracle
from conftest import assert_parity
from paper_1811_01110_amd import api
from paper_1811_01110_amd import workloads as W

pytestmark = pytest.mark.gpu
KEYS = ("slp", "dlp", "sprime")


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


def _geom(seed, tpc, p, layers, n=5000, m=300, max_list=1400):
    return W.fuzz_geometry(seed, n=n, m=m, max_list=max_list, p=p, layers=layers,
                           targets_per_center=tpc, allow_empty=False)


def _both(ctx, geom, g, p, layers):
    rows = ctx.eval(geom, g.sigma, p, layers)
    per = ctx.eval(geom, g.sigma, p, layers, flags=api.PER_TARGET)
    return rows, per


@pytest.mark.parametrize("tpc,p,layers", [(2, 16, 3), (3, 8, 1), (4, 11, 7), (2, 24, 2),
                                          (4, 16, 4), (3, 12, 5), (2, 4, 6), (5, 0, 3)])
def test_rows_equal_per_target_and_oracle(ctx, tpc, p, layers):
    g = _geom(1300 + 10 * tpc + p, tpc, p, layers)
    geom = ctx.geometry(g)
    assert ctx.get_tuning(p, layers, max(geom.pairs // geom.n_targets, 1))["group_lanes"] == 64
    rows, per = _both(ctx, geom, g, p, layers)
    ref = oracle.evaluate_geometry(g, p=p, layers=layers)
    for bit, key, a, b in zip((1, 2, 4), KEYS, rows, per):
        if layers & bit:
            assert np.array_equal(a, b), key
            assert_parity(a, ref[key], ref["abs_" + key], what=f"rows tpc{tpc} p{p} {key}")
    geom.close()


@pytest.mark.parametrize("lo,hi", [(0, 4), (2, 9)])
def test_mixed_target_counts_and_block_sizes(ctx, lo, hi):
    """Rows with lo..hi-1 targets (odd counts end in the one-target routine;
    the first mix runs the two-target kernel, the second the four-target
    one), some centers without targets, every block size."""
    rng = np.random.default_rng(1390 + lo)
    g = _geom(1390, 1, 12, 3, m=400)
    # give each center lo..hi-1 targets near it
    counts = rng.integers(lo, hi, size=g.n_centers)
    if lo == 0:
        counts[0] = 0
    tc = np.repeat(np.arange(g.n_centers, dtype=np.int32), counts)
    r = np.linalg.norm(g.targets[0] - g.centers[g.target_center[0]])
    dirs = rng.standard_normal((len(tc), 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    tgt = g.centers[tc] + dirs * (r * rng.uniform(0.0, 1.0, size=(len(tc), 1)))
    g2 = W.Geometry(g.sources, g.weights, g.normals, g.centers, g.list_offsets, g.list_sources,
                    tgt, tc, g.sigma, 12, 3, "mixed rows")
    assert (counts % 2 == 1).any() and (counts == 0).any() == (lo == 0)
    rows = np.count_nonzero(counts)
    assert (2 * len(tc) >= 7 * rows) == (lo == 2)
    geom = ctx.geometry(g2)
    mean = max(geom.pairs // geom.n_targets, 1)
    ref = oracle.evaluate_geometry(g2)
    base = None
    for w in (1, 2, 4, 8):
        ctx.set_tuning(12, 3, mean, group_lanes=64, unroll=2, waves_per_block=w, xcd_remap=w % 2)
        rows, per = _both(ctx, geom, g2, 12, 3)
        for k in (0, 1):
            assert np.array_equal(rows[k], per[k])
            assert_parity(rows[k], ref[KEYS[k]], ref["abs_" + KEYS[k]], what=f"mixed w{w}")
        base = rows if base is None else base
        assert all(np.array_equal(a, b) for a, b in zip(rows[:2], base[:2]))
    geom.close()


def test_device_entry_points_accumulate_and_batched_paths(ctx):
    import torch

    g = _geom(1395, 4, 16, 3)
    geom = ctx.geometry(g)
    sig = torch.tensor(g.sigma, device="cuda", dtype=torch.float64)
    T = g.n_targets
    s, d = (torch.zeros(T, device="cuda", dtype=torch.float64) for _ in range(2))
    ctx.eval_async(geom, sig, 16, 3, s, d)
    torch.cuda.synchronize()
    host = ctx.eval(geom, g.sigma, 16, 3, flags=api.PER_TARGET)
    assert np.array_equal(s.cpu().numpy(), host[0]) and np.array_equal(d.cpu().numpy(), host[1])
    ctx.eval_async(geom, sig, 16, 3, s, d, flags=api.ACCUMULATE)
    torch.cuda.synchronize()
    assert np.array_equal(s.cpu().numpy(), host[0] + host[0])
    ctx.stage_async(geom, sig, 3)
    s2, d2 = (torch.zeros(T, device="cuda", dtype=torch.float64) for _ in range(2))
    ctx.eval_staged_async(geom, 16, 3, s2, d2)
    torch.cuda.synchronize()
    assert np.array_equal(s2.cpu().numpy(), host[0]) and np.array_equal(d2.cpu().numpy(), host[1])
    # a plan and a server at the same group width run the per-target kernels
    item = dict(geom=geom, p=16, layers=3, sigma=sig,
                out_slp=torch.zeros(T, device="cuda", dtype=torch.float64),
                out_dlp=torch.zeros(T, device="cuda", dtype=torch.float64))
    plan = ctx.plan([item])
    plan.set_tuning(group_lanes=64, unroll=2)
    plan.execute()
    torch.cuda.synchronize()
    assert np.array_equal(item["out_slp"].cpu().numpy(), host[0])
    assert np.array_equal(item["out_dlp"].cpu().numpy(), host[1])
    plan.close()
    srv = ctx.server(4 * api.Server.request_bytes(geom, 3), 4)
    srv.set_tuning(group_lanes=64, unroll=2)
    t = srv.submit(geom, g.sigma, 16, 3)[0]
    out = srv.wait(t, 60)
    assert np.array_equal(out[0], host[0]) and np.array_equal(out[1], host[1])
    srv.close()
    geom.close()


@pytest.mark.parametrize("p,layers", [(32, 7), (1, 3)])
def test_rows_with_empty_and_short_lists(ctx, p, layers):
    """Empty lists (outputs 0), lists shorter than a wave, the highest and a
    low order, several targets per center."""
    g0 = W.fuzz_geometry(1400 + p, n=3000, m=250, max_list=900, p=p, layers=layers,
                         targets_per_center=4)
    off = g0.list_offsets
    lens = np.diff(off)
    lens[::10] = 0  # every tenth center's list emptied
    new_off = np.zeros_like(off)
    np.cumsum(lens, out=new_off[1:])
    lst = np.concatenate([g0.list_sources[off[i]:off[i] + lens[i]] for i in range(len(lens))])
    g = W.Geometry(g0.sources, g0.weights, g0.normals, g0.centers, new_off, lst.astype(np.int32),
                   g0.targets, g0.target_center, g0.sigma, p, layers, "rows short",
                   target_normals=g0.target_normals)
    assert (lens == 0).any() and ((lens > 0) & (lens < 64)).any()
    geom = ctx.geometry(g)
    mean = max(geom.pairs // geom.n_targets, 1)
    ctx.set_tuning(p, layers, mean, group_lanes=64, unroll=2, waves_per_block=4, xcd_remap=1)
    rows, per = _both(ctx, geom, g, p, layers)
    ref = oracle.evaluate_geometry(g, p=p, layers=layers)
    empty = np.isin(g.target_center, np.flatnonzero(lens == 0))
    for bit, key, a, b in zip((1, 2, 4), KEYS, rows, per):
        if layers & bit:
            assert np.array_equal(a, b), key
            assert np.all(a[empty] == 0.0)
            assert_parity(a, ref[key], ref["abs_" + key], what=f"rows short p{p} {key}")
    geom.close()


def test_crowded_row_runs_one_wave_per_target(ctx):
    """A center with far more targets than the others (here 40 beside rows
    of two): the plain path keeps one wave per target (a row kernel would
    hold that row's whole walk on one wave); same bits and the oracle's
    values either way, for host- and device-built geometries."""
    import torch

    rng = np.random.default_rng(1410)
    g = _geom(1410, 2, 16, 3, m=200)
    tc = g.target_center.copy()
    tc[:40] = 0  # center 0 takes 40 targets
    r = np.linalg.norm(g.targets[0] - g.centers[g.target_center[0]])
    dirs = rng.standard_normal((len(tc), 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    tgt = g.centers[tc] + dirs * (0.5 * r)
    g2 = W.Geometry(g.sources, g.weights, g.normals, g.centers, g.list_offsets, g.list_sources,
                    tgt, tc.astype(np.int32), g.sigma, 16, 3, "crowded row")
    ref = oracle.evaluate_geometry(g2)
    dev = {k: (torch.from_numpy(np.ascontiguousarray(v)).to("cuda:0") if v is not None else None)
           for k, v in dict(sources=g2.sources, weights=g2.weights, normals=g2.normals,
                            centers=g2.centers, list_offsets=g2.list_offsets,
                            list_sources=g2.list_sources, targets=g2.targets,
                            target_center=g2.target_center).items()}
    for geom in (ctx.geometry(g2), ctx.geometry_device(**dev)):
        rows, per = _both(ctx, geom, g2, 16, 3)
        for k in (0, 1):
            assert np.array_equal(rows[k], per[k])
            assert_parity(rows[k], ref[KEYS[k]], ref["abs_" + KEYS[k]], what="crowded row")
        geom.close()
