"""Autotuner, accumulation in plans, server time-outs and shutdown, unusual inputs."""
import numpy as np
import pytest

import oracle
from conftest import assert_parity
from paper_1811_01110_amd import api
from paper_1811_01110_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


def test_autotune_installs_a_supported_tuning(ctx):
    g = W.fuzz_geometry(500, n=3000, m=600, max_list=900, p=16, layers=3)
    geom = ctx.geometry(g)
    tuning, ms = ctx.autotune(geom, 16, 3)
    assert ms > 0
    assert tuning["group_lanes"] in (16, 32, 64) and tuning["waves_per_block"] in (1, 2, 4, 8)
    mean = max(geom.pairs // geom.n_targets, 1)
    assert ctx.get_tuning(16, 3, mean) == tuning
    s, d, _ = ctx.eval(geom, g.sigma, 16, 3)
    ref = oracle.evaluate_geometry(g)
    assert_parity(s, ref["slp"], ref["abs_slp"], what="autotuned slp")
    assert_parity(d, ref["dlp"], ref["abs_dlp"], what="autotuned dlp")
    with pytest.raises(api.TsqbxError):
        ctx.set_tuning(16, 3, mean, group_lanes=48)
    geom.close()


def test_blocks_of_eight_waves_stay_in_the_plain_kernel(ctx):
    """The plain Laplace kernel takes blocks of 8 waves (its default with one
    target per wave); the Helmholtz kernels refuse them, and a plan built
    while the plain tuning has them runs blocks of 4, with the plain path's
    bits."""
    import torch

    g = W.fuzz_geometry(502, n=3000, m=400, max_list=1200, p=16, layers=3, allow_empty=False)
    geom = ctx.geometry(g)
    mean = max(geom.pairs // geom.n_targets, 1)
    assert mean >= 384 and ctx.get_tuning(16, 3, mean)["waves_per_block"] == 8
    assert ctx.get_tuning(16, 3 | api.HELMHOLTZ, mean)["waves_per_block"] == 4
    with pytest.raises(api.TsqbxError):
        ctx.set_tuning(16, 3 | api.HELMHOLTZ, mean, waves_per_block=8)
    for bad in (3, 16):
        with pytest.raises(api.TsqbxError):
            ctx.set_tuning(16, 3, mean, waves_per_block=bad)
    ref = oracle.evaluate_geometry(g)
    outs = []
    for w in (8, 4, 1):
        ctx.set_tuning(16, 3, mean, group_lanes=64, unroll=2, waves_per_block=w, xcd_remap=1)
        s, d, _ = ctx.eval(geom, g.sigma, 16, 3)
        assert_parity(s, ref["slp"], ref["abs_slp"], what=f"w{w} slp")
        assert_parity(d, ref["dlp"], ref["abs_dlp"], what=f"w{w} dlp")
        outs.append((s, d))
    assert all(np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1]) for o in outs)
    ctx.set_tuning(16, 3, mean, group_lanes=64, unroll=2, waves_per_block=8, xcd_remap=1)
    sig = torch.tensor(g.sigma, device="cuda", dtype=torch.float64)
    item = dict(geom=geom, p=16, layers=3, sigma=sig,
                out_slp=torch.zeros(g.n_targets, device="cuda", dtype=torch.float64),
                out_dlp=torch.zeros(g.n_targets, device="cuda", dtype=torch.float64))
    plan = ctx.plan([item])
    t = plan.get_tuning()
    assert t["group_lanes"] == 64 and t["waves_per_block"] == 4
    plan.execute()
    torch.cuda.synchronize()
    assert np.array_equal(item["out_slp"].cpu().numpy(), outs[0][0])
    assert np.array_equal(item["out_dlp"].cpu().numpy(), outs[0][1])
    plan.close()
    geom.close()


def test_plan_accumulates(ctx):
    import torch

    g = W.fuzz_geometry(501, n=800, m=150, max_list=300, p=12, layers=3)
    geom = ctx.geometry(g)
    sig = torch.tensor(g.sigma, device="cuda", dtype=torch.float64)
    base = torch.full((g.n_targets,), 0.5, device="cuda", dtype=torch.float64)
    os_, od_ = base.clone(), base.clone()
    plan = ctx.plan([dict(geom=geom, p=12, layers=3, sigma=sig, out_slp=os_, out_dlp=od_)],
                    flags=api.ACCUMULATE)
    plan.execute()
    plan.execute()
    torch.cuda.synchronize()
    s, d, _ = ctx.eval(geom, g.sigma, 12, 3)
    assert np.array_equal(os_.cpu().numpy(), (0.5 + s) + s)
    assert np.array_equal(od_.cpu().numpy(), (0.5 + d) + d)
    plan.close()
    geom.close()


def test_targets_outside_the_convergence_ball_low_order(ctx):
    """|t - c| > |y - c| is outside the expansion's convergence but the finite
    sum is defined; compare at low order where terms stay moderate."""
    rng = np.random.default_rng(502)
    n, m = 200, 40
    src = rng.standard_normal((n, 3)) * 0.5
    ctr = rng.standard_normal((m, 3)) * 0.5
    tgt = ctr + 2.0 * rng.standard_normal((m, 3))
    off = np.arange(m + 1, dtype=np.int64) * 30
    idx = rng.integers(0, n, size=m * 30).astype(np.int32)
    nrm = rng.standard_normal((n, 3))
    nrm /= np.linalg.norm(nrm, axis=1)[:, None]
    g = W.Geometry(src, rng.uniform(0.1, 1, n), nrm, ctr, off, idx, tgt, None,
                   rng.standard_normal(n), 4, 3)
    geom = ctx.geometry(g)
    for p in (0, 1, 2, 4, 6):
        s, d, _ = ctx.eval(geom, g.sigma, p, 3)
        ref = oracle.evaluate_geometry(g, p=p)
        assert_parity(s, ref["slp"], ref["abs_slp"], what=f"outside p={p} slp")
        assert_parity(d, ref["dlp"], ref["abs_dlp"], what=f"outside p={p} dlp")
    geom.close()


def test_server_wait_times_out_and_destroy_finishes_in_flight_work(ctx):
    g = W.config_b(scale=16)
    geom = ctx.geometry(g)
    srv = ctx.server(16 * api.Server.request_bytes(geom, 3), 8)
    tickets = [srv.submit(geom, g.sigma, 16, 3) for _ in range(8)]
    # a zero wait on a request just queued behind seven others times out
    # (or, if it has somehow finished already, reports it done)
    try:
        srv.wait(tickets[-1][0], 0.0)
        assert srv.poll(tickets[-1][0])
    except api.TsqbxError as e:
        assert e.code == -7
    srv.wait(tickets[-1][0], 120.0)
    more = [srv.submit(geom, g.sigma, 16, 3) for _ in range(4)]
    srv.close()  # returns only after the in-flight requests have completed
    for _, a, b, _t in tickets + more:
        assert np.array_equal(a, tickets[0][1])
        assert np.array_equal(b, tickets[0][2])
    ref = oracle.evaluate_geometry(g)
    assert_parity(tickets[0][1], ref["slp"], ref["abs_slp"], what="served slp")
    assert_parity(tickets[0][2], ref["dlp"], ref["abs_dlp"], what="served dlp")
    geom.close()


def test_server_concurrent_submitters(ctx):
    """Four threads submit at once (submit is thread-safe); every result
    equals the same request served alone."""
    import threading

    geoms = W.config_e_geometries(n_geometries=3, scale=64)
    gs = [ctx.geometry(g) for g in geoms]
    srv = ctx.server(16 * max(api.Server.request_bytes(g, 3) for g in gs), 32)
    rng = np.random.default_rng(77)
    jobs = [(i % 3, (8, 16)[i % 2], (1, 2, 3)[i % 3], rng.standard_normal(geoms[i % 3].n_sources))
            for i in range(80)]
    alone = []
    for k, p, lay, sig in jobs[:12]:
        t, a, b, _ = srv.submit(gs[k], sig, p, lay)
        srv.wait(t, 60)
        alone.append((a, b))
    results = [None] * len(jobs)
    errors = []

    def worker(w):
        try:
            for i in range(w, len(jobs), 4):
                k, p, lay, sig = jobs[i]
                results[i] = srv.submit(gs[k], sig, p, lay)
        except Exception as e:  # reported below
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(w,)) for w in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    assert not errors
    srv.drain(120)
    st = srv.stats()
    assert st["failed"] == 0 and st["completed"] == 12 + len(jobs)
    for i, (a0, b0) in enumerate(alone):
        _, a, b, _ = results[i]
        lay = jobs[i][2]
        if lay & 1:
            assert np.array_equal(a, a0)
        if lay & 2:
            assert np.array_equal(b, b0)
    for (k, p, lay, sig), (t, a, b, _) in list(zip(jobs, results))[12:30]:
        ref = oracle.evaluate_geometry(geoms[k], p=p, layers=lay, sigma=sig)
        if lay & 1:
            assert_parity(a, ref["slp"], ref["abs_slp"], what="threaded slp")
        if lay & 2:
            assert_parity(b, ref["dlp"], ref["abs_dlp"], what="threaded dlp")
    srv.close()


def test_stage_then_eval_staged_equals_eval(ctx):
    """Strengths staged once, then several evaluations from them: the same
    bits as the one-call evaluation; errors when nothing (or not the double
    layer) was staged, and after the autotuner overwrote the staging."""
    import torch

    from paper_1811_01110_amd import _lib as L

    g = W.fuzz_geometry(503, n=2000, m=300, max_list=700, p=16, layers=7)
    geom = ctx.geometry(g)
    sig = torch.tensor(g.sigma, device="cuda", dtype=torch.float64)
    T = g.n_targets
    outs = [torch.zeros(T, device="cuda", dtype=torch.float64) for _ in range(3)]
    ref = [torch.zeros(T, device="cuda", dtype=torch.float64) for _ in range(3)]
    with pytest.raises(api.TsqbxError) as e:
        ctx.eval_staged_async(geom, 16, 1, *outs)
    assert e.value.code == L.E_STATE
    ctx.stage_async(geom, sig, 1)
    with pytest.raises(api.TsqbxError) as e:
        ctx.eval_staged_async(geom, 16, 3, *outs)
    assert e.value.code == L.E_STATE
    ctx.stage_async(geom, sig, 7)
    for p, layers in ((16, 7), (8, 3), (0, 1), (24, 4), (13, 2)):
        ctx.eval_staged_async(geom, p, layers, *outs)
        ctx.eval_async(geom, sig, p, layers, *ref)
        ctx.stage_async(geom, sig, 7)  # eval_async restaged with its own layers
        torch.cuda.synchronize()
        for k in range(3):
            if layers & (1 << k):
                assert torch.equal(outs[k], ref[k]), (p, layers, k)
    ctx.autotune(geom, 16, 3)
    with pytest.raises(api.TsqbxError) as e:
        ctx.eval_staged_async(geom, 16, 1, *outs)
    assert e.value.code == L.E_STATE
    geom.close()
