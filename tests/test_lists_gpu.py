"""Near-field lists built on the device against the brute-force oracle,
bit for bit (integer output: identical CSR)."""
import ctypes

import numpy as np
import pytest

from conftest import cached_workload
from oracle import lists as LO
from paper_1811_01110_amd import _lib as L
from paper_1811_01110_amd import api

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = api.Context(0)
    yield c
    c.close()


def _gpu(ctx, src, ctr, r):
    off, idx = ctx.ball_lists(src, ctr, r)
    return off.cpu().numpy(), idx.cpu().numpy()


@pytest.mark.parametrize("r", [0.01, 0.07, 0.2, 0.6])
def test_random_cloud_equals_brute_force(ctx, r):
    rng = np.random.default_rng(int(r * 1000))
    src = rng.uniform(-1, 1, (6000, 3))
    ctr = rng.uniform(-1.3, 1.3, (700, 3))
    off, idx = _gpu(ctx, src, ctr, r)
    ref_off, ref_idx = LO.ball_lists(src, ctr, r)
    assert np.array_equal(off, ref_off)
    assert np.array_equal(idx, ref_idx)


def test_exact_boundary_distances(ctx):
    """Grid points at exactly representable distances: members on the sphere
    r = 0.25 are kept (closed ball) exactly as the oracle decides."""
    g = np.arange(-8, 9) / 16.0
    src = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    ctr = src[::37].copy()
    for r in (0.25, 0.125, 0.3125):
        off, idx = _gpu(ctx, src, ctr, r)
        ref_off, ref_idx = LO.ball_lists(src, ctr, r)
        assert np.array_equal(off, ref_off) and np.array_equal(idx, ref_idx)


def test_degenerate_and_empty_inputs(ctx):
    src = np.tile([[0.3, -0.2, 0.1]], (5000, 1))  # every source in one point
    ctr = np.array([[0.3, -0.2, 0.1], [0.3, -0.2, 0.2], [5.0, 5.0, 5.0]])
    off, idx = _gpu(ctx, src, ctr, 0.1)
    ref_off, ref_idx = LO.ball_lists(src, ctr, 0.1)
    assert np.array_equal(off, ref_off) and np.array_equal(idx, ref_idx)
    off, idx = _gpu(ctx, np.zeros((0, 3)), ctr, 0.5)
    assert list(off) == [0, 0, 0, 0] and idx.size == 0
    off, idx = _gpu(ctx, src, np.zeros((0, 3)), 0.5)
    assert list(off) == [0] and idx.size == 0


def test_config_b_scaled_equals_brute_force(ctx):
    g = cached_workload("config_b", 16)
    r = 0.15 * 4.0
    off, idx = _gpu(ctx, g.sources, g.centers, r)
    assert np.array_equal(off, g.list_offsets) and np.array_equal(idx, g.list_sources)
    rows = LO.ball_rows(g.sources, g.centers, r, rows=range(0, g.n_centers, 97))
    for i, row in zip(range(0, g.n_centers, 97), rows):
        assert np.array_equal(idx[off[i]:off[i + 1]], row)


def test_config_b_full_size(ctx):
    """The 262144-source lists of the headline workload: identical to the
    host generator (itself pinned equal to the brute force) and, on sampled
    rows, to the brute force directly."""
    g = cached_workload("config_b", 1)
    off, idx = _gpu(ctx, g.sources, g.centers, 0.15)
    assert np.array_equal(off, g.list_offsets)
    assert np.array_equal(idx, g.list_sources)
    sel = np.random.default_rng(11).choice(g.n_centers, 64, replace=False)
    for i, row in zip(sel, LO.ball_rows(g.sources, g.centers, 0.15, rows=sel)):
        assert np.array_equal(idx[off[i]:off[i + 1]], row)


def test_capacity_and_row_limit_errors(ctx):
    import torch

    rng = np.random.default_rng(12)
    src = torch.tensor(rng.uniform(-1, 1, (3000, 3)), device="cuda", dtype=torch.float64)
    ctr = torch.tensor(rng.uniform(-1, 1, (50, 3)), device="cuda", dtype=torch.float64)
    off = torch.empty(51, device="cuda", dtype=torch.int64)
    nnz = ctypes.c_int64(-1)
    lib = L.load()
    stream = torch.cuda.current_stream().cuda_stream
    rc = lib.tsqbx_ball_lists(ctx.handle, 3000, src.data_ptr(), 50, ctr.data_ptr(), 0.4,
                              off.data_ptr(), None, 0, ctypes.byref(nnz), stream)
    ref_off, _ = LO.ball_lists(src.cpu().numpy(), ctr.cpu().numpy(), 0.4)
    assert rc == L.E_RANGE and nnz.value == ref_off[-1] > 0
    assert np.array_equal(off.cpu().numpy(), ref_off)
    big = torch.zeros((9000, 3), device="cuda", dtype=torch.float64)  # one ball of 9000
    off1 = torch.empty(2, device="cuda", dtype=torch.int64)
    idx = torch.empty(9000, device="cuda", dtype=torch.int32)
    rc = lib.tsqbx_ball_lists(ctx.handle, 9000, big.data_ptr(), 1, big.data_ptr(), 0.5,
                              off1.data_ptr(), idx.data_ptr(), 9000, ctypes.byref(nnz), stream)
    assert rc == L.E_RANGE and nnz.value == 9000
    for r in (0.0, -1.0, float("nan")):
        rc = lib.tsqbx_ball_lists(ctx.handle, 3000, src.data_ptr(), 50, ctr.data_ptr(), r,
                                  off.data_ptr(), None, 0, ctypes.byref(nnz), stream)
        assert rc == L.E_RANGE


def test_lists_feed_a_geometry(ctx):
    """Device-built lists used as the geometry's lists give the same
    potentials as the host-built ones."""
    from paper_1811_01110_amd import workloads as W

    g = cached_workload("config_b", 16)
    off, idx = ctx.ball_lists(g.sources, g.centers, 0.6)
    h = W.Geometry(g.sources, g.weights, g.normals, g.centers, off.cpu().numpy(),
                   idx.cpu().numpy(), g.targets, g.target_center, g.sigma, 16, 3)
    a = ctx.eval(ctx.geometry(g), g.sigma, 16, 3)
    b = ctx.eval(ctx.geometry(h), g.sigma, 16, 3)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


# ---- k nearest -------------------------------------------------------------

def _knn(ctx, src, ctr, counts):
    off, idx = ctx.knn_lists(src, ctr, counts)
    return off.cpu().numpy(), idx.cpu().numpy()


@pytest.mark.parametrize("kmax", [1, 40, 600, 8192])
def test_knn_random_cloud_equals_brute_force(ctx, kmax):
    rng = np.random.default_rng(kmax)
    src = rng.uniform(-1, 1, (9000, 3))
    ctr = rng.uniform(-1.3, 1.3, (500, 3))
    counts = rng.integers(0, kmax + 1, 500)
    counts[:2] = [0, kmax]
    off, idx = _knn(ctx, src, ctr, counts)
    ref_off, ref_idx = LO.knn_lists(src, ctr, counts)
    assert np.array_equal(off, ref_off)
    assert np.array_equal(idx, ref_idx)


def test_knn_surface_points_and_every_source(ctx):
    """Sources on a sphere (the workloads' shape), counts up to all sources."""
    from paper_1811_01110_amd import workloads as W

    rng = np.random.default_rng(21)
    src = W.random_sphere_points(6000, rng)
    ctr = 0.97 * W.random_sphere_points(300, rng)
    counts = np.exp(rng.uniform(0, np.log(6000), 300)).astype(np.int64)
    counts[:3] = [6000, 5999, 1]
    off, idx = _knn(ctx, src, ctr, counts)
    ref_off, ref_idx = LO.knn_lists(src, ctr, counts)
    assert np.array_equal(off, ref_off) and np.array_equal(idx, ref_idx)


def test_knn_exact_ties_go_to_the_smaller_index(ctx):
    g = np.arange(-6, 7) / 8.0
    src = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    src = src[np.random.default_rng(22).permutation(len(src))]  # ties across index order
    ctr = src[::29].copy()
    counts = np.resize([1, 7, 19, 27, 33, 81, 125, 1000, 2197], len(ctr))
    off, idx = _knn(ctx, src, ctr, counts)
    ref_off, ref_idx = LO.knn_lists(src, ctr, counts)
    assert np.array_equal(off, ref_off) and np.array_equal(idx, ref_idx)


def test_knn_degenerate_inputs(ctx):
    src = np.tile([[0.3, -0.2, 0.1]], (5000, 1))  # every source in one point
    ctr = np.array([[0.3, -0.2, 0.1], [9.0, 9.0, 9.0], [0.0, 0.0, 0.0]])
    counts = [5000, 300, 0]
    off, idx = _knn(ctx, src, ctr, counts)
    ref_off, ref_idx = LO.knn_lists(src, ctr, counts)
    assert np.array_equal(off, ref_off) and np.array_equal(idx, ref_idx)
    off, idx = _knn(ctx, src, np.zeros((0, 3)), np.zeros(0, dtype=np.int32))
    assert list(off) == [0] and idx.size == 0
    off, idx = _knn(ctx, np.zeros((0, 3)), ctr, [0, 0, 0])
    assert list(off) == [0, 0, 0, 0] and idx.size == 0


def test_knn_config_d_scaled_equals_the_workload_lists(ctx):
    """Config D's lists (k-d tree on the host; continuous points, so no ties)
    rebuilt on the device: identical CSR."""
    from paper_1811_01110_amd import workloads as W

    g = W.config_d(n_geometries=1, scale=8)[0]
    counts = np.diff(g.list_offsets)
    off, idx = _knn(ctx, g.sources, g.centers, counts)
    assert np.array_equal(off, g.list_offsets)
    assert np.array_equal(idx, g.list_sources)


def test_knn_rejects_bad_counts(ctx):
    import torch

    rng = np.random.default_rng(23)
    src = torch.tensor(rng.uniform(-1, 1, (3000, 3)), device="cuda", dtype=torch.float64)
    ctr = torch.tensor(rng.uniform(-1, 1, (4, 3)), device="cuda", dtype=torch.float64)
    off = torch.empty(5, device="cuda", dtype=torch.int64)
    idx = torch.empty(20000, device="cuda", dtype=torch.int32)
    nnz = ctypes.c_int64(-1)
    lib = L.load()
    stream = torch.cuda.current_stream().cuda_stream
    for bad in ([5, 5, -1, 5], [5, 3001, 5, 5]):
        cnt = torch.tensor(bad, device="cuda", dtype=torch.int32)
        rc = lib.tsqbx_knn_lists(ctx.handle, 3000, src.data_ptr(), 4, ctr.data_ptr(),
                                 cnt.data_ptr(), off.data_ptr(), idx.data_ptr(), 20000,
                                 ctypes.byref(nnz), stream)
        assert rc == L.E_RANGE, bad
    big = torch.zeros((9000, 3), device="cuda", dtype=torch.float64)
    cnt = torch.tensor([8193, 1, 1, 1], device="cuda", dtype=torch.int32)
    rc = lib.tsqbx_knn_lists(ctx.handle, 9000, big.data_ptr(), 4, ctr.data_ptr(), cnt.data_ptr(),
                             off.data_ptr(), idx.data_ptr(), 20000, ctypes.byref(nnz), stream)
    assert rc == L.E_RANGE
    cnt = torch.tensor([100, 200, 300, 400], device="cuda", dtype=torch.int32)
    rc = lib.tsqbx_knn_lists(ctx.handle, 3000, src.data_ptr(), 4, ctr.data_ptr(), cnt.data_ptr(),
                             off.data_ptr(), idx.data_ptr(), 999, ctypes.byref(nnz), stream)
    assert rc == L.E_RANGE and nnz.value == 1000
    assert list(off.cpu().numpy()) == [0, 100, 300, 600, 1000]
