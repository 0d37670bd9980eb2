"""Plan tuning: the autotuner over the persistent kernel's launch shape and
schedule, per-kernel profiling, and the saved tuning table."""
import os

import numpy as np
import pytest

import oracle
from conftest import assert_parity
from paper_1811_01110_amd import api
from paper_1811_01110_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


def _geoms():
    geoms = W.config_c(n_geometries=8, scale=16)
    geoms += [W.fuzz_geometry(500 + i, n=400, m=80, max_list=300, p=p, layers=lay)
              for i, (p, lay) in enumerate([(0, 3), (7, 2), (24, 3), (16, 1)])]
    return geoms


def _items(ctx, geoms):
    out = []
    for g in geoms:
        out.append(dict(
            geom=ctx.geometry(g), p=g.p, layers=g.layers, g=g,
            sigma=torch.tensor(g.sigma, device="cuda", dtype=torch.float64),
            out_slp=torch.zeros(g.n_targets, device="cuda", dtype=torch.float64) if g.layers & 1 else None,
            out_dlp=torch.zeros(g.n_targets, device="cuda", dtype=torch.float64) if g.layers & 2 else None))
    return out


def _check_against_plain_and_oracle(ctx, items, G, what):
    for it in items:
        g = it["g"]
        ref = oracle.evaluate_geometry(g)
        mean_i = max(it["geom"].pairs // max(it["geom"].n_targets, 1), 1)
        ctx.set_tuning(g.p, g.layers, mean_i, group_lanes=G, unroll=2)
        s, d, _ = ctx.eval(it["geom"], g.sigma, g.p, g.layers)
        for key, lay, plain in (("out_slp", 1, s), ("out_dlp", 2, d)):
            if not g.layers & lay:
                continue
            got = it[key].cpu().numpy()
            name = "slp" if lay == 1 else "dlp"
            assert_parity(got, ref[name], ref["abs_" + name], what=f"{what} {name}")
            # a plan equals the plain path at the same group width, bit for bit
            assert np.array_equal(got, plain), (what, g.name, name)


def test_autotuned_plan_matches_plain_and_oracle(ctx, tmp_path):
    geoms = _geoms()
    items = _items(ctx, geoms)
    plan = ctx.plan(items)
    t0 = plan.get_tuning()
    prof = plan.profile(reps=3)
    assert prof["reps"] == 3 and prof["eval_ms"] > 0 and prof["stage_ms"] > 0
    best, ms = plan.autotune()
    print("tuned", best, f"{ms:.4f} ms (default {t0}, {prof['eval_ms']:.4f} ms)", flush=True)
    assert best == plan.get_tuning() and ms > 0
    assert ms <= prof["eval_ms"] * 1.5
    for it in items:  # outputs from the last timing run; zero them and run the tuned plan
        for key in ("out_slp", "out_dlp"):
            if it[key] is not None:
                it[key].zero_()
    plan.execute()
    plan.execute()
    torch.cuda.synchronize()
    _check_against_plain_and_oracle(ctx, items, best["group_lanes"], "tuned plan")

    # every supported group width, with a non-default schedule, against plain
    for G, U in ((64, 1), (32, 2), (16, 2)):
        plan.set_tuning(group_lanes=G, unroll=U, waves_per_block=2, oversubscription=3,
                        step_cost=0)
        assert plan.get_tuning()["group_lanes"] == G
        plan.execute()
        torch.cuda.synchronize()
        _check_against_plain_and_oracle(ctx, items, G, f"plan G{G}")

    # out-of-range tunings are refused and leave the plan as it was
    before = plan.get_tuning()
    for bad in (dict(group_lanes=8), dict(group_lanes=32, unroll=1), dict(waves_per_block=3),
                dict(oversubscription=0), dict(oversubscription=33), dict(step_cost=-1)):
        with pytest.raises(api.TsqbxError) as ei:
            plan.set_tuning(**bad)
        assert ei.value.code == -1, bad
        assert plan.get_tuning() == before

    # the tuned entry is saved, loaded into another context and picked up by
    # a new plan of the same bucket
    path = str(tmp_path / "tuning.jsonl")
    ctx.tuning_save(path)
    text = open(path).read()
    assert '"kind": "plan"' in text
    c2 = api.Context(0)
    try:
        assert c2.tuning_load(path) >= 1
        items2 = _items(c2, geoms)
        p2 = c2.plan(items2)
        assert p2.get_tuning() == best
        p2.execute()
        torch.cuda.synchronize()
        for a, b in zip(items, items2):
            a_out = a["out_slp"] if a["out_slp"] is not None else a["out_dlp"]
            b_out = b["out_slp"] if b["out_slp"] is not None else b["out_dlp"]
            assert a_out is not None and b_out is not None
        p2.close()
        for it in items2:
            it["geom"].close()
        # a file of another form is refused
        bad = str(tmp_path / "bad.jsonl")
        with open(bad, "w") as f:
            f.write('{"kind": "plan", "arch": "x"}\n')
        with pytest.raises(api.TsqbxError):
            c2.tuning_load(bad)
        # entries of another architecture are skipped
        other = str(tmp_path / "other.jsonl")
        with open(other, "w") as f:
            f.write(text.replace('"arch": "', '"arch": "other-'))
        assert c2.tuning_load(other) == 0
        with pytest.raises(api.TsqbxError):
            c2.tuning_load(str(tmp_path / "missing.jsonl"))
    finally:
        c2.close()
    plan.close()
    for it in items:
        it["geom"].close()


def test_helmholtz_plan_tuning(ctx):
    """The Helmholtz plan takes the same tuning calls; its results equal the
    plain Helmholtz path at 64 lanes (the plan's default) bit for bit."""
    geoms = [W.fuzz_geometry(520 + i, n=300, m=60, max_list=150, p=p, layers=3)
             for i, p in enumerate((4, 9, 16))]
    rng = np.random.default_rng(5)
    items = []
    for g in geoms:
        sig = rng.standard_normal(g.n_sources) + 1j * rng.standard_normal(g.n_sources)
        items.append(dict(geom=ctx.geometry(g), p=g.p, layers=3, k=4.0, g=g, sig=sig,
                          sigma=torch.tensor(sig, device="cuda", dtype=torch.complex128),
                          out_slp=torch.zeros(g.n_targets, device="cuda", dtype=torch.complex128),
                          out_dlp=torch.zeros(g.n_targets, device="cuda", dtype=torch.complex128)))
    plan = ctx.plan_helmholtz(items)
    best, ms = plan.autotune()
    assert ms > 0 and best == plan.get_tuning()
    plan.set_tuning(group_lanes=64, unroll=2, waves_per_block=4, oversubscription=2, step_cost=15)
    plan.execute()
    torch.cuda.synchronize()
    for it in items:
        g = it["g"]
        mean_i = max(it["geom"].pairs // max(it["geom"].n_targets, 1), 1)
        ctx.set_tuning(g.p, 3 | api.HELMHOLTZ, mean_i, group_lanes=64, unroll=2)
        s, d, _ = ctx.eval_helmholtz(it["geom"], it["sig"], g.p, 3, 4.0)
        assert np.array_equal(s, it["out_slp"].cpu().numpy())
        assert np.array_equal(d, it["out_dlp"].cpu().numpy())
    plan.close()
    for it in items:
        it["geom"].close()
