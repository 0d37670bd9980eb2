"""Batched plans and the request server against plain evaluations and the oracle."""
import time

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


def _items(ctx, geoms, torch):
    out = []
    for g in geoms:
        geom = ctx.geometry(g)
        out.append(dict(
            geom=geom, p=g.p, layers=g.layers, g=g,
            sigma=torch.tensor(g.sigma, device="cuda", dtype=torch.float64),
            out_slp=torch.zeros(g.n_targets, device="cuda", dtype=torch.float64) if g.layers & 1 else None,
            out_dlp=torch.zeros(g.n_targets, device="cuda", dtype=torch.float64) if g.layers & 2 else None))
    return out


def test_plan_matches_plain_and_oracle(ctx):
    import torch

    geoms = W.config_c(n_geometries=10, scale=16)
    geoms += [W.fuzz_geometry(200 + i, n=400, m=80, max_list=200, p=p, layers=lay)
              for i, (p, lay) in enumerate([(0, 3), (5, 2), (24, 3), (32, 1)])]
    items = _items(ctx, geoms, torch)
    plan = ctx.plan(items)
    info = plan.info()
    assert info["n_items"] == len(items) and info["n_units"] > 0
    plan.execute()
    torch.cuda.synchronize()
    mean = max(sum(i["geom"].pairs for i in items) // max(sum(i["geom"].n_targets for i in items), 1), 1)
    G = ctx.get_tuning(max(g.p for g in geoms), 3, mean)["group_lanes"]
    for it in items:
        g = it["g"]
        ref = oracle.evaluate_geometry(g)
        for k, lay in (("out_slp", 1), ("out_dlp", 2)):
            if not g.layers & lay:
                continue
            got = it[k].cpu().numpy()
            name = "slp" if lay == 1 else "dlp"
            assert_parity(got, ref[name], ref["abs_" + name], what=f"plan {g.name} {name}")
        # plain evaluation with the same group width gives the same bits
        mean_i = max(it["geom"].pairs // max(it["geom"].n_targets, 1), 1)
        ctx.set_tuning(g.p, g.layers, mean_i, group_lanes=G, unroll=2)
        s, d, _ = ctx.eval(it["geom"], g.sigma, g.p, g.layers)
        if g.layers & 1:
            assert np.array_equal(s, it["out_slp"].cpu().numpy()), g.name
        if g.layers & 2:
            assert np.array_equal(d, it["out_dlp"].cpu().numpy()), g.name
    plan.close()


def test_plan_graph_replays_follow_inputs(ctx):
    """Each replay of the captured graph reads the current densities."""
    import torch

    geoms = [W.fuzz_geometry(300 + i, n=500, m=120, max_list=250, p=8 + 4 * i, layers=3)
             for i in range(3)]
    items = _items(ctx, geoms, torch)
    plan = ctx.plan(items)
    rng = np.random.default_rng(9)
    for rep in range(4):
        sigmas = [rng.standard_normal(g.n_sources) for g in geoms]
        for it, s in zip(items, sigmas):
            it["sigma"].copy_(torch.tensor(s, dtype=torch.float64))
        torch.cuda.synchronize()
        plan.execute()
        torch.cuda.synchronize()
        for it, s in zip(items, sigmas):
            a, b, _ = ctx.eval(it["geom"], s, it["p"], 3)
            ref = oracle.evaluate_geometry(it["g"], sigma=s)
            assert_parity(it["out_slp"].cpu().numpy(), ref["slp"], ref["abs_slp"], what=f"replay {rep}")
            assert_parity(it["out_dlp"].cpu().numpy(), ref["dlp"], ref["abs_dlp"], what=f"replay {rep}")
            assert_parity(it["out_slp"].cpu().numpy(), a, ref["abs_slp"])
    plan.close()


def test_server_alone_equals_mix(ctx):
    geoms = W.config_e_geometries(n_geometries=4, scale=32)
    gs = [ctx.geometry(g) for g in geoms]
    rng = np.random.default_rng(10)
    reqs = []
    for i in range(24):
        k = int(rng.integers(0, len(geoms)))
        reqs.append((k, int(rng.choice([8, 16])), int(rng.choice([1, 2, 3])),
                     rng.standard_normal(geoms[k].n_sources)))
    budget = 4 * max(api.Server.request_bytes(g, 3) for g in gs)
    srv = ctx.server(budget, 8)
    alone = []
    for k, p, lay, sig in reqs:
        t, a, b, _ = srv.submit(gs[k], sig, p, lay)
        srv.wait(t, 60)
        alone.append((a, b))
    tickets = [srv.submit(gs[k], sig, p, lay) for k, p, lay, sig in reqs]
    srv.drain(120)
    st = srv.stats()
    assert st["completed"] == 2 * len(reqs) and st["failed"] == 0
    assert st["peak_bytes_in_flight"] <= budget
    for (k, p, lay, sig), (t, a, b, _), (a0, b0) in zip(reqs, tickets, alone):
        assert srv.poll(t)
        if lay & 1:
            assert np.array_equal(a, a0)
        if lay & 2:
            assert np.array_equal(b, b0)
    # and against the oracle
    for (k, p, lay, sig), (a0, b0) in list(zip(reqs, alone))[:6]:
        ref = oracle.evaluate_geometry(geoms[k], p=p, layers=lay, sigma=sig)
        if lay & 1:
            assert_parity(a0, ref["slp"], ref["abs_slp"], what="served slp")
        if lay & 2:
            assert_parity(b0, ref["dlp"], ref["abs_dlp"], what="served dlp")
    srv.close()


def test_server_rejects_oversized_and_respects_budget(ctx):
    g = W.fuzz_geometry(400, n=3000, m=500, max_list=100, p=8, layers=3)
    geom = ctx.geometry(g)
    need = api.Server.request_bytes(geom, 3)
    srv = ctx.server(need // 2, 4)
    with pytest.raises(api.TsqbxError) as ei:
        srv.submit(geom, g.sigma, 8, 3)
    assert ei.value.code == -5
    srv.close()
    srv = ctx.server(need + need // 2, 4)  # room for one request at a time
    ts = [srv.submit(geom, g.sigma, 8, 3) for _ in range(6)]
    srv.drain(60)
    st = srv.stats()
    assert st["completed"] == 6 and st["peak_bytes_in_flight"] <= need + need // 2
    for _, a, _b, _t in ts:
        assert np.array_equal(a, ts[0][1])
    srv.close()


def test_server_cancels_a_queued_request(ctx):
    """A request still queued can be withdrawn: it ends with
    TSQBX_E_CANCELED and its outputs stay untouched; one already admitted or
    ended cannot (the scheduler's full failure matrix runs on the CPU in
    test_server_fake.py)."""
    g = W.fuzz_geometry(401, n=3000, m=500, max_list=100, p=8, layers=3)
    geom = ctx.geometry(g)
    need = api.Server.request_bytes(geom, 3)
    srv = ctx.server(need + need // 2, 4)  # one request at a time
    ts = [srv.submit(geom, g.sigma, 8, 3) for _ in range(8)]
    try:
        srv.cancel(ts[-1][0])
        cancelled = True
    except api.TsqbxError as e:  # already admitted: the queue drained first
        assert e.code == -6
        cancelled = False
    with pytest.raises(api.TsqbxError) as ei:
        srv.cancel(10 ** 12)
    assert ei.value.code == -1
    srv.drain(60)
    with pytest.raises(api.TsqbxError) as ei:
        srv.cancel(ts[0][0])  # ended
    assert ei.value.code == -6
    st = srv.stats()
    if cancelled:
        with pytest.raises(api.TsqbxError) as ei:
            srv.wait(ts[-1][0])
        assert ei.value.code == -8
        assert not ts[-1][1].any() and st["completed"] == 7 and st["failed"] == 1
    else:
        assert st["completed"] == 8
    for _, a, _b, _t in ts[:-1]:
        assert np.array_equal(a, ts[0][1])
    srv.close()
    geom.close()


def test_server_autotune_and_tuning_rules():
    """The server autotuner installs a tuning; results then equal plain
    launches at the same group width bit for bit and match the oracle; the
    tuning is fixed once a request has been submitted.  (A context of its
    own: the plain-path tunings it sets stay out of the other tests.)"""
    ctx = api.Context(0)
    g1 = W.fuzz_geometry(402, n=3000, m=400, max_list=120, p=8, layers=3)
    g2 = W.fuzz_geometry(403, n=1500, m=200, max_list=60, p=4, layers=1)
    gg1, gg2 = ctx.geometry(g1), ctx.geometry(g2)
    budget = 16 * max(api.Server.request_bytes(gg1, 3), api.Server.request_bytes(gg2, 1))
    srv = ctx.server(budget, 16)
    assert srv.get_tuning() == {"group_lanes": 16, "unroll": 2, "waves_per_block": 4,
                                "unit_steps": 8, "step_requests": 32, "dma_min_sources": 0}
    import torch

    pinned = [torch.from_numpy(g.sigma).pin_memory() for g in (g1, g2)]
    tuning, ms = srv.autotune([(gg1, 8, 3), (gg2, 4, 1)], n_requests=48, sigmas=pinned)
    assert ms > 0 and tuning == srv.get_tuning()
    assert srv.stats()["submitted"] == 0  # the bursts leave no trace
    t, a, b, _ = srv.submit(gg1, g1.sigma, 8, 3)
    srv.wait(t)
    ref = oracle.evaluate_geometry(g1, p=8, layers=3)
    assert_parity(a, ref["slp"], ref["abs_slp"], what="tuned server slp")
    assert_parity(b, ref["dlp"], ref["abs_dlp"], what="tuned server dlp")
    mean_list = max(1, -(-gg1.pairs // gg1.n_targets))
    ctx.set_tuning(8, 3, mean_list, group_lanes=tuning["group_lanes"],
                   unroll=tuning["unroll"], waves_per_block=4, xcd_remap=1)
    pa, pb, _ = ctx.eval(gg1, g1.sigma, 8, 3)
    assert np.array_equal(a, pa) and np.array_equal(b, pb)
    with pytest.raises(api.TsqbxError) as ei:
        srv.set_tuning(group_lanes=64)
    assert ei.value.code == -6
    with pytest.raises(api.TsqbxError) as ei:
        srv.autotune([(gg1, 8, 3)], n_requests=8)
    assert ei.value.code == -6
    srv.close()
    # a chosen tuning on a fresh server; a bad one is refused
    srv = ctx.server(budget, 16)
    with pytest.raises(api.TsqbxError) as ei:
        srv.set_tuning(group_lanes=8)
    assert ei.value.code == -2
    srv.set_tuning(group_lanes=64, unroll=2, waves_per_block=2, unit_steps=4, step_requests=16,
                   dma_min_sources=1000)  # g2's densities go up by DMA
    ts = [srv.submit(gg2, g2.sigma, 4, 1) for _ in range(5)]
    srv.drain(60)
    ctx.set_tuning(4, 1, max(1, -(-gg2.pairs // gg2.n_targets)), group_lanes=64, unroll=2,
                   waves_per_block=4, xcd_remap=1)
    pa, _, _ = ctx.eval(gg2, g2.sigma, 4, 1)
    for _, o, _b, _t in ts:
        assert np.array_equal(o, pa)
    srv.close()
    gg1.close()
    gg2.close()
    ctx.close()


def test_server_pinned_submissions_match_copying_ones(ctx):
    import torch

    geoms = W.config_e_geometries(n_geometries=3, scale=32)
    gs = [ctx.geometry(g) for g in geoms]
    srv = ctx.server(4 * max(api.Server.request_bytes(g, 3) for g in gs), 6)
    rng = np.random.default_rng(11)
    pending = []
    for i in range(12):
        k = i % 3
        lay = (1, 2, 3)[i % 3]
        s_np = rng.standard_normal(geoms[k].n_sources)
        s_pin = torch.tensor(s_np, dtype=torch.float64).pin_memory()
        t1, a1, b1, _ = srv.submit(gs[k], s_np, 8 + 8 * (i % 2), lay)
        t2, a2, b2, _ = srv.submit_pinned(gs[k], s_pin, 8 + 8 * (i % 2), lay)
        pending.append((lay, a1, b1, a2, b2))
    srv.drain(120)
    for lay, a1, b1, a2, b2 in pending:
        if lay & 1:
            assert np.array_equal(a1, a2.numpy())
        if lay & 2:
            assert np.array_equal(b1, b2.numpy())
    with pytest.raises(api.TsqbxError) as ei:  # pageable memory is refused
        srv.submit_pinned(gs[0], torch.zeros(geoms[0].n_sources, dtype=torch.float64), 8, 1)
    assert ei.value.code == -1
    srv.close()


def test_plan_and_server_with_sprime(ctx):
    """Items and requests asking for S' (alone and beside other layers) run in
    the any-mask persistent kernel and match plain evaluations bit for bit."""
    import torch

    masks = [4, 5, 6, 7, 1, 2, 3]
    geoms = [W.fuzz_geometry(700 + i, n=600, m=150, max_list=250, p=(8, 16, 5)[i % 3], layers=lay)
             for i, lay in enumerate(masks)]
    items = []
    for g in geoms:
        geom = ctx.geometry(g)
        it = dict(geom=geom, p=g.p, layers=g.layers, g=g,
                  sigma=torch.tensor(g.sigma, device="cuda", dtype=torch.float64))
        for bit, key in ((1, "out_slp"), (2, "out_dlp"), (4, "out_sprime")):
            if g.layers & bit:
                it[key] = torch.zeros(g.n_targets, device="cuda", dtype=torch.float64)
        items.append(it)
    plan = ctx.plan(items)
    plan.execute()
    torch.cuda.synchronize()
    mean = max(sum(i["geom"].pairs for i in items) // sum(i["geom"].n_targets for i in items), 1)
    G = ctx.get_tuning(16, 7, mean)["group_lanes"]
    for it in items:
        g = it["g"]
        ref = oracle.evaluate_geometry(g)
        mean_i = max(it["geom"].pairs // max(it["geom"].n_targets, 1), 1)
        ctx.set_tuning(g.p, g.layers, mean_i, group_lanes=G, unroll=2)
        plain = ctx.eval(it["geom"], g.sigma, g.p, g.layers)
        for k, (bit, key, name) in enumerate(((1, "out_slp", "slp"), (2, "out_dlp", "dlp"),
                                              (4, "out_sprime", "sprime"))):
            if not g.layers & bit:
                continue
            got = it[key].cpu().numpy()
            assert_parity(got, ref[name], ref["abs_" + name], what=f"plan mask {g.layers} {name}")
            assert np.array_equal(got, plain[k]), (g.layers, name)
    plan.close()
    # the server: the same requests, all at once
    gs = [it["geom"] for it in items]
    srv = ctx.server(8 * max(api.Server.request_bytes(x, 7) for x in gs), 16)
    tickets = [srv.submit(x, g.sigma, g.p, g.layers) for x, g in zip(gs, geoms)]
    srv.drain(60)
    assert srv.stats()["failed"] == 0
    for (t, *outs), g in zip(tickets, geoms):
        ref = oracle.evaluate_geometry(g)
        for k, (bit, name) in enumerate(((1, "slp"), (2, "dlp"), (4, "sprime"))):
            if g.layers & bit:
                assert_parity(outs[k], ref[name], ref["abs_" + name], what=f"served {name}")
            else:
                assert outs[k] is None
    srv.close()


@pytest.mark.parametrize("p", [8, 16, 11])
def test_plan_single_layer_long_lists_match_plain_bits(ctx, p):
    """One target per wave: the plain kernel unrolls the single layer's
    Clenshaw steps, the persistent kernel reads their constants from a table;
    the results are the same bits."""
    import torch

    geoms = [W.fuzz_geometry(950 + i, n=3000, m=200, max_list=1500, p=p, layers=1,
                             allow_empty=False) for i in range(3)]
    items = _items(ctx, geoms, torch)
    mean = max(sum(i["geom"].pairs for i in items) // sum(i["geom"].n_targets for i in items), 1)
    assert ctx.get_tuning(p, 1, mean)["group_lanes"] == 64
    plan = ctx.plan(items)
    plan.execute()
    torch.cuda.synchronize()
    for it in items:
        g = it["g"]
        mean_i = max(it["geom"].pairs // max(it["geom"].n_targets, 1), 1)
        ctx.set_tuning(p, 1, mean_i, group_lanes=64, unroll=2)
        s, _, _ = ctx.eval(it["geom"], g.sigma, p, 1)
        assert np.array_equal(s, it["out_slp"].cpu().numpy())
        ref = oracle.evaluate_geometry(g)
        assert_parity(s, ref["slp"], ref["abs_slp"], what=f"plan long lists p={p}")
    plan.close()


def test_plan_edge_cases(ctx):
    """An empty plan runs and does nothing; an item with no targets or with
    every list empty is valid (outputs 0) beside an ordinary item."""
    import torch

    empty = ctx.plan([])
    assert empty.info()["n_items"] == 0
    empty.execute()
    torch.cuda.synchronize()
    empty.close()
    g = W.fuzz_geometry(400, n=300, m=60, max_list=120, p=8, layers=3)
    no_lists = W.Geometry(g.sources, g.weights, g.normals, g.centers,
                          np.zeros(g.n_centers + 1, dtype=np.int64), np.zeros(0, dtype=np.int32),
                          g.targets, g.target_center, g.sigma, 8, 3)
    no_targets = W.Geometry(g.sources, g.weights, g.normals, g.centers, g.list_offsets,
                            g.list_sources, np.zeros((0, 3)), np.zeros(0, dtype=np.int32),
                            g.sigma, 8, 3)
    items = _items(ctx, [g, no_lists, no_targets], torch)
    for it in items[1:2]:
        it["out_slp"].fill_(7.0)
        it["out_dlp"].fill_(7.0)
    plan = ctx.plan(items)
    plan.execute()
    torch.cuda.synchronize()
    ref = oracle.evaluate_geometry(g)
    assert_parity(items[0]["out_slp"].cpu().numpy(), ref["slp"], ref["abs_slp"], what="slp")
    assert_parity(items[0]["out_dlp"].cpu().numpy(), ref["dlp"], ref["abs_dlp"], what="dlp")
    assert not items[1]["out_slp"].any() and not items[1]["out_dlp"].any()
    plan.close()


def test_plan_stress_many_tiny_items():
    """Hundreds of tiny items of every order and layer mask in one plan,
    with ACCUMULATE into outputs zeroed before each of 100 graph replays
    (eager fills and synchronisations between them): a target summed twice
    would double, a skipped one stay 0.  Every replay equals the plain
    launches at the same group width bit for bit; a sample matches the
    oracle.  (A context of its own, with the default plain tunings.)"""
    import torch

    ctx = api.Context(0)
    rng = np.random.default_rng(4242)
    geoms = []
    for i in range(360):
        p = int(rng.integers(0, 33))
        layers = int(rng.integers(1, 8))
        geoms.append(W.fuzz_geometry(5000 + i, n=int(rng.integers(8, 200)),
                                     m=int(rng.integers(1, 30)), max_list=int(rng.integers(1, 60)),
                                     p=p, layers=layers,
                                     targets_per_center=int(rng.integers(1, 4))))
    items = []
    for g in geoms:
        geom = ctx.geometry(g)
        it = dict(geom=geom, p=g.p, layers=g.layers, g=g,
                  sigma=torch.tensor(g.sigma, device="cuda", dtype=torch.float64))
        for bit, name in ((1, "out_slp"), (2, "out_dlp"), (4, "out_sprime")):
            if g.layers & bit:
                it[name] = torch.zeros(g.n_targets, device="cuda", dtype=torch.float64)
        items.append(it)
    plan = ctx.plan(items, flags=api.ACCUMULATE)
    plan.set_tuning(group_lanes=16, unroll=2)
    plain = []
    for it in items:  # every mean list is below 384 entries: the plain path runs 16 lanes
        plain.append(ctx.eval(it["geom"], it["g"].sigma, it["p"], it["layers"]))
    outs = [(it.get("out_slp"), it.get("out_dlp"), it.get("out_sprime")) for it in items]
    for rep in range(100):
        for o in outs:
            for t in o:
                if t is not None:
                    t.zero_()
        torch.cuda.synchronize()
        plan.execute()
        torch.cuda.synchronize()
        if rep in (0, 1, 17, 99):
            for k, (o, ref) in enumerate(zip(outs, plain)):
                for t, r in zip(o, ref):
                    if t is not None:
                        assert np.array_equal(t.cpu().numpy(), r), (rep, k)
    for k in range(0, len(items), 37):
        g = items[k]["g"]
        ref = oracle.evaluate_geometry(g)
        for t, name in zip(outs[k], ("slp", "dlp", "sprime")):
            if t is not None:
                assert_parity(t.cpu().numpy(), ref[name], ref["abs_" + name],
                              what=f"stress item {k} {name}")
    plan.close()
    for it in items:
        it["geom"].close()
    ctx.close()


def test_server_mixes_helmholtz_and_laplace_requests(ctx):
    """Helmholtz requests (complex density and outputs) share steps with
    Laplace ones: each result is the same served alone or in the mix, equals
    the plain Helmholtz call with the server's group width bit for bit, and
    the Helmholtz oracle to the parity bar."""
    from oracle import helmholtz as H

    geoms = W.config_e_geometries(n_geometries=4, scale=32)
    gs = [ctx.geometry(g) for g in geoms]
    rng = np.random.default_rng(12)
    reqs = []
    for i in range(30):
        j = int(rng.integers(0, len(geoms)))
        if i % 2:
            sig = rng.standard_normal(geoms[j].n_sources) + 1j * rng.standard_normal(geoms[j].n_sources)
            reqs.append(("h", j, int(rng.choice([4, 8, 12])), int(rng.choice([1, 2, 3, 4, 7])),
                         float(rng.choice([2.0, 10.0])), sig))
        else:
            reqs.append(("l", j, int(rng.choice([8, 16])), int(rng.choice([1, 2, 3])), 0.0,
                         rng.standard_normal(geoms[j].n_sources)))
    budget = 4 * max(max(api.Server.request_bytes(g, 3) for g in gs),
                     max(api.Server.request_bytes_helmholtz(g, 12, 7) for g in gs))
    srv = ctx.server(budget, 8)

    def submit(kind, j, p, lay, k, sig):
        if kind == "h":
            return srv.submit_helmholtz(gs[j], sig, p, lay, k)
        return srv.submit(gs[j], sig, p, lay)

    alone = []
    for rq in reqs:
        t = submit(*rq)
        srv.wait(t[0], 60)
        alone.append(t[1:])
    mixed = [submit(*rq) for rq in reqs]
    srv.drain(120)
    st = srv.stats()
    assert st["completed"] == 2 * len(reqs) and st["failed"] == 0
    assert st["peak_bytes_in_flight"] <= budget
    for rq, a, m in zip(reqs, alone, mixed):
        for x, y in zip(a, m[1:]):
            assert (x is None and y is None) or np.array_equal(x, y), rq[:5]
    # Helmholtz against the plain call (the server runs 16 lanes per target)
    # and the oracle
    checked = 0
    for (kind, j, p, lay, k, sig), a in zip(reqs, alone):
        if kind != "h" or checked >= 5:
            continue
        checked += 1
        geom = gs[j]
        ctx.set_tuning(p, lay | api.HELMHOLTZ, max(-(-geom.pairs // geom.n_targets), 1), group_lanes=16)
        plain = ctx.eval_helmholtz(geom, sig, p, lay, k)
        ref = H.evaluate_geometry(geoms[j], k, sig, p=p, layers=lay)
        for bit, key, got, pl in zip((1, 2, 4), ("slp", "dlp", "sprime"), a, plain):
            if lay & bit:
                assert np.array_equal(got, pl), (p, lay, key)
                assert_parity(got, ref[key], ref["abs_" + key], what=f"served Helmholtz {key}")
    with pytest.raises(api.TsqbxError) as ei:
        srv.submit_helmholtz(gs[0], np.zeros(geoms[0].n_sources, complex), 8, 1, 0.0)
    assert ei.value.code == -2
    srv.close()
    small = ctx.server(api.Server.request_bytes_helmholtz(gs[0], 8, 1) // 2, 2)
    with pytest.raises(api.TsqbxError) as ei:
        small.submit_helmholtz(gs[0], np.zeros(geoms[0].n_sources, complex), 8, 1, 3.0)
    assert ei.value.code == -5
    small.close()


def test_server_pinned_helmholtz_submissions_match_copying_ones(ctx):
    import torch

    geoms = W.config_e_geometries(n_geometries=3, scale=32)
    gs = [ctx.geometry(g) for g in geoms]
    srv = ctx.server(4 * max(api.Server.request_bytes_helmholtz(g, 16, 7) for g in gs), 6)
    rng = np.random.default_rng(13)
    runs = []
    for i in range(9):
        j, p, lay = i % 3, (8, 16)[i % 2], (1, 3, 7)[i % 3]
        sig = rng.standard_normal(geoms[j].n_sources) + 1j * rng.standard_normal(geoms[j].n_sources)
        pin = torch.empty(geoms[j].n_sources, dtype=torch.complex128, pin_memory=True)
        pin.numpy()[:] = sig
        runs.append((srv.submit_helmholtz(gs[j], sig, p, lay, 6.0),
                     srv.submit_helmholtz_pinned(gs[j], pin, p, lay, 6.0), pin))
    srv.drain(120)
    assert srv.stats()["failed"] == 0
    for copied, pinned, _ in runs:
        for a, b in zip(copied[1:], pinned[1:]):
            assert (a is None and b is None) or np.array_equal(a, b.numpy())
    srv.close()


def test_schedule_preview_matches_plan(ctx):
    """The host-only preview yields the schedule a plan builds (units counted by
    the plan), for geometries kept in the caller's order."""
    import torch

    geoms = [W.fuzz_geometry(300 + i, n=500, m=120, max_list=250, p=p, layers=lay)
             for i, (p, lay) in enumerate([(8, 1), (16, 3), (4, 2), (12, 1)])]
    items = []
    for g in geoms:
        geom = ctx.geometry(g, flags=api.NO_REORDER)
        items.append(dict(
            geom=geom, p=g.p, layers=g.layers,
            sigma=torch.tensor(g.sigma, device="cuda", dtype=torch.float64),
            out_slp=torch.zeros(g.n_targets, device="cuda", dtype=torch.float64),
            out_dlp=torch.zeros(g.n_targets, device="cuda", dtype=torch.float64)))
    plan = ctx.plan(items)
    info = plan.info()
    mean = max(sum(it["geom"].pairs for it in items) // sum(it["geom"].n_targets for it in items), 1)
    G = ctx.get_tuning(max(g.p for g in geoms), 3, mean)["group_lanes"]
    rows = []
    for g in geoms:
        tc = g.target_center if g.target_center is not None else np.arange(g.n_targets)
        lens = (g.list_offsets[1:] - g.list_offsets[:-1])[tc]
        rows.append((lens, g.p, g.layers))
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    units, wb = api.schedule_preview(rows, group_lanes=G, max_waves=cus * 4 * 6 * 8)
    print("plan units", info["n_units"], "preview units", len(units), "G", G, flush=True)
    assert info["n_units"] == len(units)
    plan.close()
    for it in items:
        it["geom"].close()


def test_server_keeps_a_bounded_history(ctx):
    """A long-running server forgets the tickets of old completed requests
    (the last 4096 stay queryable), so its host memory stays bounded; the
    counters still count every request and the results stay right."""
    g = W.fuzz_geometry(700, n=120, m=12, max_list=24, p=4, layers=1, allow_empty=False)
    geom = ctx.geometry(g)
    srv = ctx.server(64 * api.Server.request_bytes(geom, 1), 64)
    n = 4300
    rng = np.random.default_rng(70)
    tickets, outs, sigmas = [], [], []
    for i in range(n):
        s = rng.standard_normal(g.n_sources)
        t, o, _, _ = srv.submit(geom, s, 4, api.SLP)
        tickets.append(t)
        if i >= n - 3:
            outs.append(o)
            sigmas.append(s)
    srv.drain(300)
    st = srv.stats()
    assert st["completed"] == n and st["failed"] == 0
    with pytest.raises(api.TsqbxError) as ei:
        srv.poll(tickets[0])
    assert ei.value.code == -1
    assert srv.poll(tickets[-1]) and srv.poll(tickets[n - 4096])
    for o, s in zip(outs, sigmas):
        ref = oracle.evaluate_geometry(g, p=4, layers=1, sigma=s)
        assert_parity(o, ref["slp"], ref["abs_slp"], what="bounded history")
    srv.close()
    geom.close()
