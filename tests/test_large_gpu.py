"""A geometry with more than 2^31 list entries, so that row offsets beyond
the 32-bit range are exercised in the plain, batched and Helmholtz paths.

33000 targets, each with its own center, list all 4096 sources 16 times
over (2.16e9 entries, 8.6 GB of indices; duplicates are summed as listed).
Every output is therefore 16 times the output for a single copy of each
list, which the oracles compute directly: for every target in the Laplace
paths, for a sample of targets in the Helmholtz path."""
import numpy as np
import pytest

import oracle
from conftest import assert_parity
from oracle import helmholtz as H
from paper_1811_01110_amd import api
from paper_1811_01110_amd import workloads as W

pytestmark = pytest.mark.gpu

N, T, REP = 4096, 33000, 16


def _geometry(rep):
    rng = np.random.default_rng(20181101)
    src = W.random_sphere_points(N, rng)
    ctr = 0.3 * W.random_sphere_points(T, rng)
    tgt = ctr + 0.05 * W.random_sphere_points(T, rng)
    tnrm = W.random_sphere_points(T, rng)
    sigma = rng.standard_normal(N)
    offsets = np.arange(T + 1, dtype=np.int64) * (N * rep)
    idx = np.tile(np.arange(N, dtype=np.int32), T * rep)
    return W.Geometry(src, np.full(N, 4 * np.pi / N), src.copy(), ctr, offsets, idx, tgt, None,
                      sigma, 4, 3, target_normals=tnrm)


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def big(ctx):
    g = _geometry(REP)
    assert g.list_offsets[-1] > 2 ** 31
    geom = ctx.geometry(g)
    del g.list_sources  # the library holds its own copy on the device
    yield g, geom
    geom.close()


@pytest.fixture(scope="module")
def single():
    return _geometry(1)


@pytest.mark.timeout(600)
def test_plain_and_plan_beyond_2_31_entries(ctx, big, single):
    import torch

    g, geom = big
    assert geom.pairs == T * N * REP
    ref = oracle.evaluate_geometry(single, p=4, layers=7)
    s, d, t = ctx.eval(geom, g.sigma, 4, 7)
    for got, key in ((s, "slp"), (d, "dlp"), (t, "sprime")):
        assert_parity(got, REP * ref[key], REP * ref["abs_" + key], what=f"plain {key}")
    sig = torch.tensor(g.sigma, device="cuda", dtype=torch.float64)
    outs = [torch.zeros(T, device="cuda", dtype=torch.float64) for _ in range(2)]
    plan = ctx.plan([dict(geom=geom, p=4, layers=3, sigma=sig, out_slp=outs[0], out_dlp=outs[1])])
    plan.execute()
    torch.cuda.synchronize()
    for got, key in zip(outs, ("slp", "dlp")):
        assert_parity(got.cpu().numpy(), REP * ref[key], REP * ref["abs_" + key], what=f"plan {key}")
    plan.close()


@pytest.mark.timeout(600)
def test_helmholtz_beyond_2_31_entries(ctx, big, single):
    g, geom = big
    rng = np.random.default_rng(7)
    sig = g.sigma + 1j * rng.standard_normal(N)
    got = ctx.eval_helmholtz(geom, sig, 2, 7, 3.0)
    sel = np.sort(np.concatenate([rng.choice(T, 200, replace=False), np.arange(T - 40, T)]))
    ref = H.evaluate_geometry(single, 3.0, sig, p=2, layers=7, select=sel)
    for o, key in zip(got, ("slp", "dlp", "sprime")):
        assert_parity(o[sel], REP * ref[key], REP * ref["abs_" + key], what=f"Helmholtz {key}")
