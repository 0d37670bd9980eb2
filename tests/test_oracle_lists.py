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
