"""The device layout of a geometry, previewed on the host
(tsqbx_geometry_layout, no device): orders, rows, padding and the Morton
ordering, checked against their definitions."""
import numpy as np
import pytest

from paper_1811_01110_amd import api
from paper_1811_01110_amd import workloads as W


def _arrays(g):
    return dict(sources=g.sources, weights=g.weights, normals=g.normals, centers=g.centers,
                list_offsets=g.list_offsets, list_sources=g.list_sources, targets=g.targets,
                target_center=g.target_center)


def _morton(points):
    """63-bit Morton keys over the points' bounding box, 21 bits per axis with
    x in the highest position of each triple (the library's stated order is a
    Morton curve; the test only needs keys that are monotone along it)."""
    lo = points.min(axis=0)
    span = max(float((points.max(axis=0) - lo).max()), 1e-300)
    q = np.clip(((points - lo) * (((1 << 21) - 1) / span)), 0, (1 << 21) - 1).astype(np.int64)
    key = np.zeros(len(points), dtype=np.int64)
    for b in range(21):
        for a in range(3):
            key |= ((q[:, a] >> b) & 1) << (3 * b + (2 - a))
    return key


@pytest.mark.parametrize("tpc", [1, 3])
def test_layout_rows_orders_and_padding(tpc):
    g = W.fuzz_geometry(40 + tpc, n=700, m=90, max_list=200, p=4, layers=1,
                        targets_per_center=tpc)
    lay = api.geometry_layout(**_arrays(g))
    N, T = g.n_sources, g.n_targets
    so, to, tr = lay["source_order"], lay["target_order"], lay["target_row"]
    assert np.array_equal(np.sort(so), np.arange(N)) and np.array_equal(np.sort(to), np.arange(T))
    rank = np.empty(N, dtype=np.int64)
    rank[so] = np.arange(N)
    # sources along a Morton curve; targets by the Morton key of their center
    assert np.all(np.diff(_morton(g.sources)[so]) >= 0)
    tc = g.target_center
    ck = _morton(g.centers)[tc[to]]
    assert np.all(np.diff(ck) >= 0)
    # one row per distinct center in order of first use; rows sorted and padded
    centers_in_order = []
    for c in tc[to]:
        if c not in centers_in_order:
            centers_in_order.append(c)
    assert lay["n_rows"] == len(centers_in_order)
    off, rows = lay["row_offsets"], lay["rows"]
    assert off[0] == 0 and lay["nnz"] == off[-1] == len(rows)
    for r, c in enumerate(centers_in_order):
        lst = g.list_sources[g.list_offsets[c]:g.list_offsets[c + 1]]
        row = rows[off[r]:off[r + 1]]
        assert len(row) % 16 == 0 and len(row) - len(lst) < 16
        assert np.array_equal(row[:len(lst)], np.sort(rank[lst]))
        assert np.all(row[len(lst):] == N)
    for k in range(T):
        assert centers_in_order[tr[k]] == tc[to[k]]
    lens = np.diff(g.list_offsets)[tc]
    assert lay["pairs"] == lens.sum() and lay["max_list"] == lens.max()


def test_layout_without_reorder_and_errors():
    g = W.fuzz_geometry(43, n=300, m=40, max_list=50, p=4, layers=1)
    lay = api.geometry_layout(flags=api.NO_REORDER, **_arrays(g))
    assert np.array_equal(lay["source_order"], np.arange(g.n_sources))
    assert np.array_equal(lay["target_order"], np.arange(g.n_targets))
    bad = _arrays(g)
    bad["list_sources"] = bad["list_sources"].copy()
    bad["list_sources"][3] = g.n_sources
    with pytest.raises(api.TsqbxError) as ei:
        api.geometry_layout(**bad)
    assert ei.value.code == -2
