"""Pins of the list oracle: geometric facts and a second, independent
construction (scipy's k-d tree ball query), away from the boundary sphere
where the two may round differently."""
import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import lists as LO


def test_matches_kdtree_ball_query_off_the_boundary():
    rng = np.random.default_rng(1)
    src = rng.uniform(-1, 1, (4000, 3))
    ctr = rng.uniform(-1.2, 1.2, (300, 3))
    r = 0.21
    off, idx = LO.ball_lists(src, ctr, r)
    tree = cKDTree(src)
    for i, c in enumerate(ctr):
        row = idx[off[i]:off[i + 1]]
        assert np.all(np.diff(row) > 0)
        d = np.linalg.norm(src - c, axis=1)
        far_from_edge = np.abs(d - r) > 1e-12
        ref = np.array(sorted(tree.query_ball_point(c, r)), dtype=np.int32)
        assert set(row[far_from_edge[row]]) == set(ref[far_from_edge[ref]])


def test_closed_ball_boundary_and_edge_cases():
    # a source exactly at distance r along an axis is a member (closed ball)
    src = np.array([[0.0, 0.0, 0.0], [0.5, 0.0, 0.0], [0.0, 0.75, 0.0], [0.0, 0.0, 2.0]])
    ctr = np.array([[0.0, 0.0, 0.0], [10.0, 10.0, 10.0]])
    off, idx = LO.ball_lists(src, ctr, 0.75)
    assert list(off) == [0, 3, 3]
    assert list(idx) == [0, 1, 2]
    off, idx = LO.ball_lists(np.zeros((0, 3)), ctr, 1.0)
    assert list(off) == [0, 0, 0] and idx.size == 0
    off, idx = LO.ball_lists(src, np.zeros((0, 3)), 1.0)
    assert list(off) == [0] and idx.size == 0


def test_translation_moves_nothing_and_growth_is_monotone():
    rng = np.random.default_rng(2)
    src = rng.integers(-64, 64, (3000, 3)) / 64.0   # exactly representable after a shift
    ctr = rng.integers(-64, 64, (100, 3)) / 64.0
    a = LO.ball_lists(src, ctr, 0.3)
    b = LO.ball_lists(src + 8.0, ctr + 8.0, 0.3)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    small = LO.ball_rows(src, ctr, 0.2)
    big = LO.ball_rows(src, ctr, 0.3)
    for s, g in zip(small, big):
        assert set(s) <= set(g)


def test_agrees_with_the_workload_generator():
    """The grid-based generator of the workloads and the brute force take
    the same membership decision on every pair."""
    from paper_1811_01110_amd import workloads as W

    g = W.config_b(scale=64)
    r = 0.15 * 8.0
    off, idx = LO.ball_lists(g.sources, g.centers, r)
    assert np.array_equal(off, g.list_offsets)
    assert np.array_equal(idx, g.list_sources)


# ---- k nearest ---------------------------------------------------------------

def test_knn_matches_kdtree_when_distances_are_distinct():
    rng = np.random.default_rng(5)
    src = rng.uniform(-1, 1, (3000, 3))
    ctr = rng.uniform(-1.2, 1.2, (200, 3))
    counts = rng.integers(0, 400, 200)
    counts[:3] = [0, 1, 3000]
    off, idx = LO.knn_lists(src, ctr, counts)
    assert np.array_equal(np.diff(off), counts)
    tree = cKDTree(src)
    for i, c in enumerate(ctr):
        row = idx[off[i]:off[i + 1]]
        assert np.all(np.diff(row) > 0)
        if counts[i] == 0:
            continue
        _, nb = tree.query(c, k=int(counts[i]))
        assert set(row) == set(np.atleast_1d(nb))


def test_knn_breaks_equal_distances_by_index():
    # six sources at distance 1 along the axes, one at the center, one far away
    src = np.array([[1.0, 0, 0], [0, 1.0, 0], [0, 0, 1.0], [-1.0, 0, 0], [0, -1.0, 0],
                    [0, 0, -1.0], [0, 0, 0], [5.0, 5.0, 5.0]])
    ctr = np.zeros((4, 3))
    off, idx = LO.knn_lists(src, ctr, [1, 3, 7, 8])
    rows = [list(idx[off[i]:off[i + 1]]) for i in range(4)]
    assert rows == [[6], [0, 1, 6], [0, 1, 2, 3, 4, 5, 6], list(range(8))]
    # every source in one point: the smallest indices
    off, idx = LO.knn_lists(np.ones((50, 3)), np.zeros((1, 3)), [7])
    assert list(idx) == list(range(7))


def test_knn_selected_precede_the_rest():
    """In (d2, index) order every listed source comes before every unlisted
    one, with d2 formed as the definition states."""
    rng = np.random.default_rng(6)
    src = rng.integers(-8, 8, (2000, 3)) / 8.0   # many exact ties
    ctr = rng.integers(-8, 8, (50, 3)) / 8.0
    counts = rng.integers(1, 2000, 50)
    rows = LO.knn_rows(src, ctr, counts)
    for c, k, row in zip(ctr, counts, rows):
        d = src - c
        d2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
        inside = np.zeros(len(src), dtype=bool)
        inside[row] = True
        assert inside.sum() == k
        worst = max((d2[j], j) for j in row)
        best_out = min(((d2[j], j) for j in np.nonzero(~inside)[0]), default=(np.inf, 0))
        assert worst < best_out


def test_knn_agrees_with_the_workload_generator():
    """Config D's k-d tree lists (continuous random points, no ties) equal the
    brute force on sampled rows."""
    from paper_1811_01110_amd import workloads as W

    g = W.config_d(n_geometries=1, scale=64)[0]
    counts = np.diff(g.list_offsets)
    sel = range(0, g.n_centers, 7)
    for i, row in zip(sel, LO.knn_rows(g.sources, g.centers, counts, rows=sel)):
        assert np.array_equal(g.list_sources[g.list_offsets[i]:g.list_offsets[i + 1]], row)
