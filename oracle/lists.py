"""Brute-force CPU oracle for near-field list construction.

TEST INFRASTRUCTURE ONLY: the test suite and the benchmark's CPU-baseline leg
call this; the product library never does.  It shares no code with the GPU
path.

What it computes: the near-field source set of a QBX center (Sec. 3.3: the
sources a center's expansion interacts with directly) taken, as in the
workloads of this repository, either as every source inside the closed ball
of radius r about the center, or as the k_c sources nearest to center c,
listed in ascending source index (CSR).  Every (center, source) distance is
computed, in FP64 exactly as written here, each operation rounded on its own:
dx = y_x - c_x (likewise y, z), d2 = (dx*dx + dy*dy) + dz*dz.  Ball: member
iff d2 <= r*r.  Nearest: the k_c smallest sources in the order of
(d2, source index), so equal distances are broken by the smaller index.
"""
from __future__ import annotations

import numpy as np


def ball_rows(sources, centers, radius: float, rows=None):
    """Rows of the ball lists: a list of int32 arrays (ascending source
    indices), for every center or for the centers in `rows`."""
    src = np.ascontiguousarray(sources, dtype=np.float64)
    ctr = np.ascontiguousarray(centers, dtype=np.float64)
    r2 = np.float64(radius) * np.float64(radius)
    sel = range(len(ctr)) if rows is None else rows
    out = []
    for i in sel:
        c = ctr[i]
        dx = src[:, 0] - c[0]
        dy = src[:, 1] - c[1]
        dz = src[:, 2] - c[2]
        d2 = (dx * dx + dy * dy) + dz * dz
        out.append(np.nonzero(d2 <= r2)[0].astype(np.int32))
    return out


def ball_lists(sources, centers, radius: float):
    """The ball lists of every center as CSR (offsets int64 [M+1], indices
    int32 [nnz], ascending within each row)."""
    rows = ball_rows(sources, centers, radius)
    offsets = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum([len(r) for r in rows], out=offsets[1:])
    idx = np.concatenate(rows) if rows else np.zeros(0, dtype=np.int32)
    return offsets, idx.astype(np.int32)


def knn_rows(sources, centers, counts, rows=None):
    """Rows of the k-nearest lists: a list of int32 arrays (ascending source
    indices), for every center or for the centers in `rows`; counts[c] is the
    number of sources listed for center c."""
    src = np.ascontiguousarray(sources, dtype=np.float64)
    ctr = np.ascontiguousarray(centers, dtype=np.float64)
    counts = np.asarray(counts)
    idx = np.arange(len(src))
    sel = range(len(ctr)) if rows is None else rows
    out = []
    for i in sel:
        c = ctr[i]
        dx = src[:, 0] - c[0]
        dy = src[:, 1] - c[1]
        dz = src[:, 2] - c[2]
        d2 = (dx * dx + dy * dy) + dz * dz
        order = np.lexsort((idx, d2))  # by d2, then by index
        out.append(np.sort(order[:int(counts[i])]).astype(np.int32))
    return out


def knn_lists(sources, centers, counts):
    """The k-nearest lists of every center as CSR (offsets int64 [M+1],
    indices int32, ascending within each row)."""
    rows = knn_rows(sources, centers, counts)
    offsets = np.zeros(len(rows) + 1, dtype=np.int64)
    np.cumsum([len(r) for r in rows], out=offsets[1:])
    idx = np.concatenate(rows) if rows else np.zeros(0, dtype=np.int32)
    return offsets, idx.astype(np.int32)
