"""Seeded input generators: determinism, list correctness, geometric invariants."""
import math

import numpy as np

from paper_1811_01110_amd import workloads as W


def _brute_ball(centers, points, r):
    rows = []
    for c in centers:
        d = np.linalg.norm(points - c, axis=1)
        rows.append(np.nonzero(d <= r)[0])
    return rows


def test_csr_ball_matches_brute_force():
    rng = np.random.default_rng(1)
    pts = rng.uniform(-1, 1, (3000, 3))
    ctr = rng.uniform(-1.1, 1.1, (200, 3))
    off, idx = W.csr_ball(ctr, pts, 0.23, chunk=37)
    ref = _brute_ball(ctr, pts, 0.23)
    assert off[0] == 0 and off[-1] == len(idx)
    for i, row in enumerate(ref):
        got = idx[off[i]:off[i + 1]]
        assert np.array_equal(got, row)


def test_csr_knn_matches_brute_force():
    rng = np.random.default_rng(2)
    pts = rng.uniform(-1, 1, (2000, 3))
    ctr = rng.uniform(-1, 1, (50, 3))
    counts = rng.integers(1, 300, size=50)
    off, idx = W.csr_knn(ctr, pts, counts, chunk=7)
    for i, c in enumerate(ctr):
        d = np.linalg.norm(pts - c, axis=1)
        ref = np.sort(np.argsort(d, kind="stable")[:counts[i]])
        assert np.array_equal(idx[off[i]:off[i + 1]], ref)


def test_generators_are_deterministic():
    a = W.config_b(scale=256)
    b = W.config_b(scale=256)
    for f in ("sources", "weights", "normals", "centers", "list_offsets", "list_sources",
              "targets", "sigma"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    c = W.config_c(n_geometries=3, scale=8)
    d = W.config_c(n_geometries=3, scale=8)
    for x, y in zip(c, d):
        assert np.array_equal(x.list_sources, y.list_sources)
        assert x.p == y.p


def test_config_a_shape():
    g = W.config_a()
    assert g.n_sources == 4096 and g.n_targets == 1024 and g.p == 8 and g.layers == 1
    assert g.nnz == 4096 * 1024
    assert np.allclose(np.linalg.norm(g.sources, axis=1), 1.0)
    assert np.allclose(g.centers, 0.95 * g.targets)
    assert math.isclose(g.weights.sum(), 4 * math.pi)


def _check_surface_geometry(g, offset_max):
    assert np.allclose(np.linalg.norm(g.normals, axis=1), 1.0)
    assert np.all(g.weights > 0)
    rho = np.linalg.norm(g.targets - g.centers, axis=1)
    assert np.all(rho <= offset_max * (1 + 1e-12))
    rows = np.repeat(np.arange(g.n_centers), g.row_lengths())
    R = np.linalg.norm(g.sources[g.list_sources] - g.centers[rows], axis=1)
    # every listed source lies outside the ball |t - c| <= rho of its center
    assert np.all(R >= rho[rows] * (1 - 1e-9))
    assert np.all(np.diff(g.list_offsets) >= 0)
    # indices ascending within each row
    d = np.diff(g.list_sources.astype(np.int64))
    starts = g.list_offsets[1:-1] - 1
    mask = np.ones(len(d), dtype=bool)
    mask[starts[(starts >= 0) & (starts < len(d))]] = False
    assert np.all(d[mask] > 0)


def test_config_b_scaled_structure():
    g = W.config_b(scale=64)
    assert g.p == 16 and g.layers == 3
    _check_surface_geometry(g, 0.02)
    # the surface area of r = 1 + 0.1 f is close to that of the unit sphere
    assert 0.8 * 4 * math.pi < g.weights.sum() < 1.3 * 4 * math.pi
    assert 500 < g.row_lengths().mean() < 3000


def test_config_c_and_e_structure():
    gs = W.config_c(n_geometries=4, scale=4)
    for g in gs:
        assert g.p in (4, 8, 12, 16) and g.layers == 1
        assert g.n_targets == max(g.n_sources // 4, 1)
        _check_surface_geometry(g, 1.0)
    reqs = W.config_e_requests(200, rate_hz=1000.0)
    t = np.array([r.arrival_s for r in reqs])
    assert np.all(np.diff(t) >= 0)
    assert {r.p for r in reqs} <= {8, 16} and {r.layers for r in reqs} <= {1, 2}


def test_config_d_skewed_knn_lists():
    gs = W.config_d(n_geometries=1, scale=32)
    g = gs[0]
    assert g.p == 24 and g.layers == 2
    lens = g.row_lengths()
    assert lens.min() >= 100 and lens.max() <= 131072 // 32
    _check_surface_geometry(g, 1.0)


def test_fuzz_geometry_ragged():
    g = W.fuzz_geometry(3, n=50, m=20, max_list=9, p=4, layers=3, targets_per_center=2)
    assert g.n_targets == 40
    assert np.all(np.bincount(g.target_center, minlength=20) == 2)
    assert (g.row_lengths() == 0).any()


def test_near_boundary_generator_reaches_the_edge():
    """Every listed pair of the near-boundary generator has |t - c| / |y - c|
    between 0.85 * ratio and ratio, and the aimed targets sit on the line of
    their nearest source (cos gamma = +1 and -1)."""
    for ratio in (0.99, 1.3):
        g = W.fuzz_near_boundary(3, n=300, m=60, max_list=150, p=30, layers=7, ratio=ratio)
        assert np.array_equal(g.list_offsets, np.sort(g.list_offsets))
        seen = {0: 0, 1: 0}
        for i, c in enumerate(g.target_center):
            lo, hi = int(g.list_offsets[c]), int(g.list_offsets[c + 1])
            if hi == lo:
                continue
            d = g.sources[g.list_sources[lo:hi]] - g.centers[c]
            R = np.linalg.norm(d, axis=1)
            delta = g.targets[i] - g.centers[c]
            rho = np.linalg.norm(delta)
            q = rho / R
            assert q.max() <= ratio * (1 + 1e-12) and q.max() >= ratio * (1 - 1e-12)
            assert q.min() >= 0.85 * ratio
            j = int(np.argmin(R))
            cosg = float(delta @ d[j]) / (rho * R[j])
            if i % 3 in (0, 1):
                assert abs(cosg - (1.0 if i % 3 == 0 else -1.0)) < 1e-12
                seen[i % 3] += 1
        assert seen[0] > 5 and seen[1] > 5
