"""GPU path vs the CPU oracle, element by element, through the C ABI.

Bar: max|gpu - oracle| / max|oracle| <= 1e-12 and, per target,
|gpu - oracle| <= 1e-12 * (the oracle's sum of absolute term values).
"""
import numpy as np
import pytest

import oracle
from conftest import assert_parity, cached_workload
from paper_1811_01110_amd import api
from paper_1811_01110_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


def _check(ctx, g, p=None, layers=None, select=None, flags=0, what=""):
    p = g.p if p is None else p
    layers = g.layers if layers is None else layers
    geom = ctx.geometry(g, flags=flags)
    s, d, t = ctx.eval(geom, g.sigma, p, layers)
    ref = oracle.evaluate_geometry(g, p=p, layers=layers, select=select)
    sel = slice(None) if select is None else select
    if layers & api.SLP:
        assert_parity(s[sel], ref["slp"], ref["abs_slp"], what=f"{what} slp")
    if layers & api.DLP:
        assert_parity(d[sel], ref["dlp"], ref["abs_dlp"], what=f"{what} dlp")
    if layers & api.SPRIME:
        assert_parity(t[sel], ref["sprime"], ref["abs_sprime"], what=f"{what} sprime")
    geom.close()
    return s, d, t


def test_config_a_dense_lists(ctx):
    g = cached_workload("config_a")
    print("config A", g.n_sources, g.n_targets, flush=True)
    _check(ctx, g, what="A")


def test_config_b_scaled(ctx):
    g = cached_workload("config_b", 64)
    print("config B/64", g.n_sources, g.n_targets, g.nnz, flush=True)
    _check(ctx, g, what="B/64")


def test_config_b_full_size(ctx):
    """Every one of the 65536 targets of the 262144-source perturbed sphere,
    p = 16, single + double layer (the benchmark's workload)."""
    g = cached_workload("config_b", 1)
    print("config B full", g.n_sources, g.n_targets, g.nnz, flush=True)
    _check(ctx, g, what="B p=16 layers=3")


@pytest.mark.parametrize("p", list(range(0, 33)))
def test_every_order_ragged_lists(ctx, p):
    g = W.fuzz_geometry(p, n=300, m=70, max_list=140, p=p, layers=3, targets_per_center=2)
    _check(ctx, g, what=f"fuzz p={p}")


@pytest.mark.parametrize("p", list(range(24, 33)))
def test_near_convergence_edge_high_order(ctx, p):
    """|t - c| / |y - c| up to 0.99 at p = 24..32, with targets aimed at and
    away from their nearest source (cos gamma = +-1): the closed forms of the
    sums of b_n and (n+1) b_n cancel most there.  All three layers, every
    mask class, and the single layer alone (Clenshaw)."""
    g = W.fuzz_near_boundary(p, n=400, m=80, max_list=300, p=p, layers=7)
    for lay in (7, 3, 1):
        _check(ctx, g, layers=lay, what=f"boundary 0.99 p={p} layers={lay}")


@pytest.mark.parametrize("p", list(range(0, 5)))
def test_outside_convergence_low_order(ctx, p):
    """|t - c| = 1.3 |y - c|_min: pairs outside the expansion's convergence
    (a finite sum all the same) at p <= 4."""
    g = W.fuzz_near_boundary(100 + p, n=300, m=60, max_list=200, p=p, layers=7, ratio=1.3)
    for lay in (7, 1):
        _check(ctx, g, layers=lay, what=f"boundary 1.3 p={p} layers={lay}")


@pytest.mark.parametrize("p", list(range(0, 33)))
def test_single_layer_alone_every_order(ctx, p):
    """The single layer alone runs Clenshaw's backward recurrence: every
    compiled and run-time order, with short and long lists (one and four
    targets per wave)."""
    g = W.fuzz_geometry(900 + p, n=400, m=80, max_list=700, p=p, layers=1, targets_per_center=2)
    geom = ctx.geometry(g)
    ref = oracle.evaluate_geometry(g, p=p, layers=1)
    mean = max(geom.pairs // max(geom.n_targets, 1), 1)
    for G, U in ((64, 2), (64, 1), (16, 2)):
        ctx.set_tuning(p, 1, mean, group_lanes=G, unroll=U)
        s, _, _ = ctx.eval(geom, g.sigma, p, 1)
        assert_parity(s, ref["slp"], ref["abs_slp"], what=f"slp alone p={p} G{G}U{U}")
    geom.close()


@pytest.mark.parametrize("layers", [1, 2, 3])
def test_layers_separately(ctx, layers):
    g = W.fuzz_geometry(100 + layers, n=500, m=90, max_list=300, p=16, layers=layers)
    _check(ctx, g, layers=layers, what=f"layers={layers}")


def test_edge_cases(ctx):
    # no targets at all
    g = W.fuzz_geometry(7, n=20, m=5, max_list=5, p=4, layers=3)
    g0 = W.Geometry(g.sources, g.weights, g.normals, g.centers, g.list_offsets, g.list_sources,
                    np.zeros((0, 3)), np.zeros(0, dtype=np.int32), g.sigma, 4, 3)
    geom = ctx.geometry(g0)
    s, d, _ = ctx.eval(geom, g.sigma, 4, 3)
    assert s.size == 0 and d.size == 0
    # every list empty
    off = np.zeros(g.n_centers + 1, dtype=np.int64)
    ge = W.Geometry(g.sources, g.weights, g.normals, g.centers, off, np.zeros(0, dtype=np.int32),
                    g.targets, g.target_center, g.sigma, 4, 3)
    geom = ctx.geometry(ge)
    s, d, _ = ctx.eval(geom, g.sigma, 4, 3)
    assert np.all(s == 0) and np.all(d == 0)
    # one source, list of length one, target at its center (rho = 0)
    one = W.Geometry(np.array([[1.0, 2.0, 0.5]]), np.array([0.7]), np.array([[0.0, 0.6, 0.8]]),
                     np.zeros((1, 3)), np.array([0, 1]), np.array([0], dtype=np.int32),
                     np.zeros((1, 3)), None, np.array([1.3]), 9, 3)
    _check(ctx, one, what="rho=0")


def test_tuning_variants(ctx):
    g = W.fuzz_geometry(11, n=2000, m=300, max_list=700, p=16, layers=3)
    geom = ctx.geometry(g)
    ref = oracle.evaluate_geometry(g)
    mean = max(geom.pairs // max(geom.n_targets, 1), 1)
    base = None
    for G, U in ((64, 1), (64, 2), (64, 4), (32, 2), (16, 2)):
        for w in (1, 2, 4, 8):
            for remap in (0, 1):
                ctx.set_tuning(16, 3, mean, waves_per_block=w, group_lanes=G, unroll=U,
                               xcd_remap=remap)
                s, d, _ = ctx.eval(geom, g.sigma, 16, 3)
                assert_parity(s, ref["slp"], ref["abs_slp"], what=f"G{G}U{U}w{w}")
                assert_parity(d, ref["dlp"], ref["abs_dlp"], what=f"G{G}U{U}w{w}")
                if G == 64:
                    if base is None:
                        base = (s.copy(), d.copy())
                    # the summation order depends only on the group width
                    assert np.array_equal(s, base[0]) and np.array_equal(d, base[1])
    geom.close()


def test_async_device_path_and_accumulate(ctx):
    import torch

    g = W.fuzz_geometry(12, n=800, m=200, max_list=400, p=12, layers=3)
    geom = ctx.geometry(g)
    s_host, d_host, _ = ctx.eval(geom, g.sigma, 12, 3)
    sig = torch.tensor(g.sigma, device="cuda", dtype=torch.float64)
    os_ = torch.zeros(g.n_targets, device="cuda", dtype=torch.float64)
    od_ = torch.zeros(g.n_targets, device="cuda", dtype=torch.float64)
    ctx.eval_async(geom, sig, 12, 3, os_, od_)
    torch.cuda.synchronize()
    assert np.array_equal(os_.cpu().numpy(), s_host)
    assert np.array_equal(od_.cpu().numpy(), d_host)
    ctx.eval_async(geom, sig, 12, 3, os_, od_, flags=api.ACCUMULATE)
    torch.cuda.synchronize()
    assert np.array_equal(os_.cpu().numpy(), s_host + s_host)
    assert np.array_equal(od_.cpu().numpy(), d_host + d_host)
    # the single layer alone runs its own recurrence (equal to 1e-12, not bitwise)
    s_only, _, _ = ctx.eval(geom, g.sigma, 12, api.SLP)
    ref = oracle.evaluate_geometry(g, p=12, layers=1)
    assert_parity(s_only, ref["slp"], ref["abs_slp"], what="slp alone")
    base_s = np.full(g.n_targets, 0.25)
    out_s = base_s.copy()
    ctx.eval(geom, g.sigma, 12, api.SLP, out_slp=out_s, flags=api.ACCUMULATE)
    assert np.array_equal(out_s, base_s + s_only)
    geom.close()


def test_no_reorder_same_result(ctx):
    g = W.fuzz_geometry(13, n=600, m=100, max_list=300, p=8, layers=3, targets_per_center=3)
    a = _check(ctx, g, what="reorder")
    b = _check(ctx, g, flags=api.NO_REORDER, what="no reorder")
    ref = oracle.evaluate_geometry(g)
    assert_parity(a[0], b[0], ref["abs_slp"])
    assert_parity(a[1], b[1], ref["abs_dlp"])


def test_rejects_bad_requests(ctx):
    g = W.fuzz_geometry(14, n=50, m=10, max_list=20, p=4, layers=1)
    g.normals = None
    geom = ctx.geometry(g)
    with pytest.raises(api.TsqbxError) as ei:
        ctx.eval(geom, g.sigma, 4, api.DLP)
    assert ei.value.code == -1
    with pytest.raises(api.TsqbxError) as ei:
        ctx.eval(geom, g.sigma, 33, api.SLP)
    assert ei.value.code == -2
    geom.close()


def test_config_d_geometry_full(ctx):
    """Every target of one high-order geometry (131072 sources, k-nearest
    lists of 100..8000), p = 24, double layer, in a plain launch."""
    g = cached_workload("config_d", 1)[0]
    print("config D[0]", g.n_sources, g.n_targets, g.nnz, flush=True)
    _check(ctx, g, what="D[0] plain p=24 layers=2")


# ---------------------------------------------------------------------------
# S': the normal derivative of the single layer at the target (App. A)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("p", list(range(0, 33)))
def test_sprime_every_order_ragged_lists(ctx, p):
    g = W.fuzz_geometry(600 + p, n=300, m=70, max_list=140, p=p, layers=7, targets_per_center=2)
    _check(ctx, g, layers=7, what=f"fuzz p={p} all layers")


def test_sprime_layer_masks_share_the_derivative_recurrence(ctx):
    """Masks 4..7 against the oracle; every mask with the double layer or S'
    runs the same recurrence, so S' (and the double layer, and the single
    layer beside either) has the same bits in every such mask."""
    g = W.fuzz_geometry(640, n=700, m=120, max_list=400, p=16, layers=7)
    res = {lay: _check(ctx, g, layers=lay, what=f"mask {lay}") for lay in (2, 3, 4, 5, 6, 7)}
    for lay in (5, 6, 7):
        assert np.array_equal(res[lay][2], res[4][2]), lay
    for lay in (3, 6, 7):
        assert np.array_equal(res[lay][1], res[2][1]), lay
    for lay in (5, 7):
        assert np.array_equal(res[lay][0], res[3][0]), lay


def test_sprime_config_b_full_size(ctx):
    """Every target of the perturbed sphere with all three layers, and S'
    alone, p = 16."""
    g = cached_workload("config_b", 1)
    assert g.target_normals is not None
    _check(ctx, g, layers=7, what="B p=16 layers=7")
    _check(ctx, g, layers=4, what="B p=16 layers=4")


def test_sprime_at_center_and_tuning_variants(ctx):
    g = W.fuzz_geometry(641, n=1500, m=250, max_list=600, p=12, layers=7)
    g.targets[:5] = g.centers[g.target_center[:5]]  # t = c: only the n = 1 term
    geom = ctx.geometry(g)
    ref = oracle.evaluate_geometry(g, layers=4)
    mean = max(geom.pairs // max(geom.n_targets, 1), 1)
    base = None
    for G, U in ((64, 1), (64, 2), (64, 4), (32, 2), (16, 2)):
        ctx.set_tuning(12, 4, mean, group_lanes=G, unroll=U)
        _, _, t = ctx.eval(geom, g.sigma, 12, 4)
        assert_parity(t, ref["sprime"], ref["abs_sprime"], what=f"G{G}U{U}")
        if G == 64:
            base = t.copy() if base is None else base
            assert np.array_equal(t, base)
    geom.close()


def test_sprime_needs_target_normals(ctx):
    g = W.fuzz_geometry(642, n=50, m=10, max_list=20, p=4, layers=1)
    g.target_normals = None
    geom = ctx.geometry(g)
    assert not geom.has_target_normals
    with pytest.raises(api.TsqbxError) as ei:
        ctx.eval(geom, g.sigma, 4, api.SPRIME)
    assert ei.value.code == -1
    with pytest.raises(api.TsqbxError) as ei:
        ctx.eval(geom, g.sigma, 4, 8)
    assert ei.value.code == -1
    geom.close()


@pytest.mark.parametrize("G", [64, 32, 16])
def test_several_targets_per_center(ctx, G):
    """Several targets share one center (and so one row of the layout): every
    target against the oracle, all three layers, at each group width and
    block size the plain kernel takes."""
    g = W.fuzz_geometry(1200 + G, n=4000, m=300, max_list=900, p=12, layers=7,
                        targets_per_center=4)
    geom = ctx.geometry(g)
    mean = max(geom.pairs // geom.n_targets, 1)
    ref = oracle.evaluate_geometry(g, p=12, layers=7)
    for w in (2, 8):
        ctx.set_tuning(12, 7, mean, group_lanes=G, unroll=2, waves_per_block=w, xcd_remap=1)
        s, d, t = ctx.eval(geom, g.sigma, 12, 7)
        for out, key in ((s, "slp"), (d, "dlp"), (t, "sprime")):
            assert_parity(out, ref[key], ref["abs_" + key], what=f"tpc4 G{G} w{w} {key}")
    geom.close()
