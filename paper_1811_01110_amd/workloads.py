"""Seeded synthetic inputs for the target-specific QBX near-field evaluation.

This module produces geometry only: source points with quadrature-times-area
weights and outward unit normals, densities, on-surface targets with one QBX
center each placed along the inward normal, and per-center near-field source
lists in compressed-sparse-row (CSR) form.  It performs none of the method's
arithmetic (no expansion, no Legendre recurrence), so both the GPU path and the
CPU oracle may take their inputs from here.

Why these shapes: the paper's experiments evaluate layer potentials on the
surface with one target per QBX center, the center displaced from the target
along the normal (Sec. 2.4 and the stage-1 discretization of Sec. 2.5), and
every center sees a near field of sources gathered from nearby boxes
(Sec. 3.3, the QBX near field of Algorithm 1).  The meshes used there (urchin,
torus grid, plane) are not reproduced; star-shaped and ellipsoidal point
clouds with the same structure stand in for them.

Every generator draws from ``numpy.random.default_rng(SeedSequence([20181101,
config_id, item_id]))`` so that both sides see bit-identical inputs.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np
import scipy.special as sps

SEED_BASE = 20181101
GOLDEN_ANGLE = math.pi * (3.0 - math.sqrt(5.0))

CONFIG_IDS = {"A": 0, "B": 1, "C": 2, "D": 3, "E": 4, "fuzz": 90, "sphere": 91,
              "boundary": 92}


def rng_for(config: str, item: int = 0) -> np.random.Generator:
    """The seeded generator for (config, item)."""
    cid = CONFIG_IDS[config] if isinstance(config, str) else int(config)
    return np.random.default_rng(np.random.SeedSequence([SEED_BASE, cid, int(item)]))


@dataclasses.dataclass
class Geometry:
    """One evaluation problem in the layout the C ABI takes.

    sources      (N, 3) float64   source points y
    weights      (N,)   float64   quadrature x area weights w_y
    normals      (N, 3) float64   outward unit normals at y (double layer)
    centers      (M, 3) float64   QBX expansion centers c
    list_offsets (M+1,) int64     CSR row pointers, offsets[0] = 0
    list_sources (nnz,) int32     CSR column indices into sources
    targets      (T, 3) float64   targets t
    target_center (T,)  int32     center of each target (None: target i uses center i)
    sigma        (N,)   float64   density samples at the sources
    p            int              expansion order
    layers       int              bitmask, 1 = single layer, 2 = double layer,
                                  4 = normal derivative of the single layer at the target (S')
    target_normals (T, 3) float64 unit normals at the targets (S'), or None
    """

    sources: np.ndarray
    weights: np.ndarray
    normals: Optional[np.ndarray]
    centers: np.ndarray
    list_offsets: np.ndarray
    list_sources: np.ndarray
    targets: np.ndarray
    target_center: Optional[np.ndarray]
    sigma: np.ndarray
    p: int
    layers: int
    name: str = ""
    target_normals: Optional[np.ndarray] = None

    @property
    def n_sources(self) -> int:
        return int(self.sources.shape[0])

    @property
    def n_targets(self) -> int:
        return int(self.targets.shape[0])

    @property
    def n_centers(self) -> int:
        return int(self.centers.shape[0])

    @property
    def nnz(self) -> int:
        return int(self.list_offsets[-1])

    def row_lengths(self) -> np.ndarray:
        return np.diff(self.list_offsets)

    def pairs(self) -> int:
        """Number of (target, listed source) pairs."""
        lens = self.row_lengths()
        if self.target_center is None:
            return int(lens.sum())
        return int(lens[self.target_center].sum())

    def pair_terms(self, p: Optional[int] = None, layers: Optional[int] = None) -> int:
        """Pairs x (p+1), counted once per layer evaluated."""
        p = self.p if p is None else p
        layers = self.layers if layers is None else layers
        return self.pairs() * (p + 1) * bin(layers).count("1")


# ----------------------------------------------------------------------------
# point sets on the unit sphere
# ----------------------------------------------------------------------------

def random_sphere_points(n: int, rng: np.random.Generator) -> np.ndarray:
    """n directions uniform on the unit sphere (normalized Gaussians)."""
    g = rng.standard_normal((n, 3))
    return g / np.linalg.norm(g, axis=1)[:, None]


def fibonacci_angles(n: int, phase: float = 0.0):
    """Polar and azimuthal angles of an n-point Fibonacci lattice (near equal-area)."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    theta = np.arccos(z)
    phi = np.mod(i * GOLDEN_ANGLE + phase, 2.0 * math.pi)
    return theta, phi


def _angles_to_xyz(theta, phi):
    st = np.sin(theta)
    return np.stack([st * np.cos(phi), st * np.sin(phi), np.cos(theta)], axis=1)


def _random_rotation(rng: np.random.Generator) -> np.ndarray:
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


# ----------------------------------------------------------------------------
# surfaces
# ----------------------------------------------------------------------------

class PerturbedSphere:
    """r(theta, phi) = 1 + amp * f(theta, phi), f a sum of real spherical harmonics.

    f = sum_k a_k Yreal_{l_k m_k} with l_k uniform in 1..lmax, m_k uniform in
    -l_k..l_k and a_k ~ N(0, 1), scaled so that max |f| = 1 on a
    128 x 256 angular grid, which keeps r within [1 - amp, 1 + amp].
    """

    def __init__(self, rng: np.random.Generator, n_terms: int = 20, lmax: int = 6,
                 amp: float = 0.1):
        self.l = rng.integers(1, lmax + 1, size=n_terms)
        self.m = np.array([rng.integers(-l, l + 1) for l in self.l])
        self.a = rng.standard_normal(n_terms)
        self.amp = amp
        self.scale = 1.0
        th = (np.arange(128) + 0.5) * math.pi / 128
        ph = np.arange(256) * 2.0 * math.pi / 256
        TH, PH = np.meshgrid(th, ph, indexing="ij")
        f, _, _ = self._f(TH.ravel(), PH.ravel())
        self.scale = 1.0 / np.max(np.abs(f))

    def _f(self, theta, phi):
        f = np.zeros_like(theta)
        ft = np.zeros_like(theta)
        fp = np.zeros_like(theta)
        for a, l, m in zip(self.a, self.l, self.m):
            y, dy = sps.sph_harm_y(int(l), abs(int(m)), theta, phi, diff_n=1)
            if m > 0:
                v, vt, vp = (math.sqrt(2) * y.real, math.sqrt(2) * dy[..., 0].real,
                             math.sqrt(2) * dy[..., 1].real)
            elif m < 0:
                v, vt, vp = (math.sqrt(2) * y.imag, math.sqrt(2) * dy[..., 0].imag,
                             math.sqrt(2) * dy[..., 1].imag)
            else:
                v, vt, vp = y.real, dy[..., 0].real, dy[..., 1].real
            f += a * v
            ft += a * vt
            fp += a * vp
        s = self.scale
        return f * s, ft * s, fp * s

    def sample(self, theta, phi, n_total: int):
        """Points, outward unit normals and area weights at the given angles.

        The weight is the area element of the radial graph times the
        equal-area share 4 pi / n_total of the unit-sphere lattice.
        """
        f, ft, fp = self._f(theta, phi)
        r = 1.0 + self.amp * f
        r_t = self.amp * ft
        r_p_over_sin = self.amp * fp / np.sin(theta)
        omega = _angles_to_xyz(theta, phi)
        th_hat = np.stack([np.cos(theta) * np.cos(phi), np.cos(theta) * np.sin(phi),
                           -np.sin(theta)], axis=1)
        ph_hat = np.stack([-np.sin(phi), np.cos(phi), np.zeros_like(phi)], axis=1)
        x = r[:, None] * omega
        nrm = omega - (r_t / r)[:, None] * th_hat - (r_p_over_sin / r)[:, None] * ph_hat
        nrm /= np.linalg.norm(nrm, axis=1)[:, None]
        w = (4.0 * math.pi / n_total) * r * np.sqrt(r * r + r_t * r_t + r_p_over_sin ** 2)
        return x, nrm, w


class Ellipsoid:
    """x = D y_hat with D = diag(a, b, c), y_hat on the unit sphere."""

    def __init__(self, axes):
        self.axes = np.asarray(axes, dtype=np.float64)

    def sample(self, theta, phi, n_total: int):
        yh = _angles_to_xyz(theta, phi)
        x = yh * self.axes[None, :]
        g = yh / self.axes[None, :]
        gn = np.linalg.norm(g, axis=1)
        nrm = g / gn[:, None]
        w = (4.0 * math.pi / n_total) * np.prod(self.axes) * gn
        return x, nrm, w

    def min_curvature_radius(self) -> float:
        return float(self.axes.min() ** 2 / self.axes.max())


# ----------------------------------------------------------------------------
# near-field lists
# ----------------------------------------------------------------------------

def csr_ball(centers: np.ndarray, points: np.ndarray, radius: float, chunk: int = 1024):
    """All points within `radius` of each center, as CSR with ascending indices.

    A uniform grid of cell size `radius` is used; the 27 neighbouring cells of
    each center hold every candidate.  Chunks of centers run on a thread pool.
    """
    import concurrent.futures as cf
    import os

    centers = np.ascontiguousarray(centers, dtype=np.float64)
    points = np.ascontiguousarray(points, dtype=np.float64)
    n = len(points)
    lo = np.minimum(points.min(0), centers.min(0)) - radius
    cell = float(radius)
    pijk = np.floor((points - lo) / cell).astype(np.int64)
    dims = np.maximum(pijk.max(0), np.floor((centers - lo) / cell).astype(np.int64).max(0)) + 2
    key = (pijk[:, 0] * dims[1] + pijk[:, 1]) * dims[2] + pijk[:, 2]
    order = np.argsort(key, kind="stable")
    skey = key[order]
    spts = points[order]
    offs = np.array([(i, j, k) for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)],
                    dtype=np.int64)
    r2 = radius * radius

    def one(s):
        c = centers[s:s + chunk]
        cijk = np.floor((c - lo) / cell).astype(np.int64)
        nijk = cijk[:, None, :] + offs[None, :, :]
        nkey = (nijk[..., 0] * dims[1] + nijk[..., 1]) * dims[2] + nijk[..., 2]
        st = np.searchsorted(skey, nkey, side="left").ravel()
        en = np.searchsorted(skey, nkey, side="right").ravel()
        cnt = en - st
        tot = int(cnt.sum())
        rep_cell = np.repeat(np.arange(cnt.size), cnt)
        first = np.cumsum(cnt) - cnt
        pos = st[rep_cell] + (np.arange(tot) - first[rep_cell])
        crow = rep_cell // 27
        d = spts[pos] - c[crow]
        keep = (d * d).sum(axis=1) <= r2
        comb = crow[keep] * n + order[pos[keep]]
        comb.sort()
        counts = np.bincount(comb // n, minlength=len(c))
        return counts, (comb % n).astype(np.int32)

    starts = list(range(0, len(centers), chunk))
    workers = max(1, min(16, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        res = list(ex.map(one, starts))
    counts = np.concatenate([r[0] for r in res]) if res else np.zeros(0, dtype=np.int64)
    offsets = np.zeros(len(centers) + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    idx = np.concatenate([r[1] for r in res]) if res else np.zeros(0, dtype=np.int32)
    return offsets, idx


def csr_knn(centers: np.ndarray, points: np.ndarray, counts: np.ndarray, chunk: int = 256):
    """The counts[i] nearest points to center i, as CSR with ascending indices."""
    from scipy.spatial import cKDTree

    tree = cKDTree(points)
    counts = np.asarray(counts, dtype=np.int64)
    order = np.argsort(counts, kind="stable")
    offsets = np.zeros(len(centers) + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    idx = np.empty(int(offsets[-1]), dtype=np.int32)
    for s in range(0, len(order), chunk):
        ids = order[s:s + chunk]
        k = int(counts[ids].max())
        _, nb = tree.query(centers[ids], k=k, workers=-1)
        nb = nb.reshape(len(ids), k)
        for row, ci in enumerate(ids):
            L = int(counts[ci])
            idx[offsets[ci]:offsets[ci + 1]] = np.sort(nb[row, :L])
    return offsets, idx


# ----------------------------------------------------------------------------
# the five workload configurations
# ----------------------------------------------------------------------------

def _ys32_real(theta, phi):
    """Real part of the orthonormal spherical harmonic of degree 3, order 2."""
    return sps.sph_harm_y(3, 2, theta, phi).real


def config_a(scale: int = 1) -> Geometry:
    """Dense near field on the unit sphere, single layer, p = 8.

    4096 uniform random sources, weights 4 pi / N, sigma ~ N(0, 1); 1024
    further random targets t, each with center 0.95 t; every center lists all
    sources.  `scale` divides both counts (for quick runs).
    """
    rng = rng_for("A")
    n, k = 4096 // scale, 1024 // scale
    src = random_sphere_points(n, rng)
    w = np.full(n, 4.0 * math.pi / n)
    sigma = rng.standard_normal(n)
    tgt = random_sphere_points(k, rng)
    ctr = 0.95 * tgt
    offsets = np.arange(k + 1, dtype=np.int64) * n
    idx = np.tile(np.arange(n, dtype=np.int32), k)
    return Geometry(src, w, src.copy(), ctr, offsets, idx, tgt, None, sigma, 8, 1, "A",
                    target_normals=tgt.copy())


def _on_surface_targets(surface, n_src, n_tgt, rng, offset, phase_tgt):
    th, ph = fibonacci_angles(n_src)
    src, nrm, w = surface.sample(th, ph, n_src)
    tth, tph = fibonacci_angles(n_tgt, phase=phase_tgt)
    tgt, tnrm, _ = surface.sample(tth, tph, n_tgt)
    ctr = tgt - offset * tnrm
    return src, nrm, w, (th, ph), tgt, ctr, tnrm


def config_b(scale: int = 1, radius: float = 0.15) -> Geometry:
    """Perturbed sphere, single + double layer, p = 16.

    262144 Fibonacci-lattice sources on r = 1 + 0.1 f, sigma = Re Y_3^2 +
    0.1 N(0, 1); 65536 targets on a second lattice, centers 0.02 inside along
    the normal; lists hold every source within `radius` of the center.
    `scale` divides the counts and grows the radius by sqrt(scale) so that the
    list lengths stay about the same.
    """
    rng = rng_for("B")
    surf = PerturbedSphere(rng)
    n, k = 262144 // scale, 65536 // scale
    src, nrm, w, (th, ph), tgt, ctr, tnrm = _on_surface_targets(
        surf, n, k, rng, 0.02, phase_tgt=0.5 * GOLDEN_ANGLE)
    sigma = _ys32_real(th, ph) + 0.1 * rng.standard_normal(n)
    r = radius * math.sqrt(scale)
    offsets, idx = csr_ball(ctr, src, r)
    return Geometry(src, w, nrm, ctr, offsets, idx, tgt, None, sigma, 16, 3, "B",
                    target_normals=tnrm)


def config_b_shared(targets_per_center: int = 4, scale: int = 1,
                    radius: float = 0.15) -> Geometry:
    """Geometry B's sources and density with several targets per center.

    A quarter as many centers as B has targets (16384), each 0.02 inside the
    perturbed sphere along the normal, with `targets_per_center` targets on
    the segment from the center to the surface, at 1, 3/4, 1/2, ... of the
    way (the first on the surface): near-surface targets sharing one QBX
    expansion.  Lists hold every source within `radius` of the center, so
    the pairs per target are those of B.
    """
    rng = rng_for("B")
    surf = PerturbedSphere(rng)
    n, k = 262144 // scale, 65536 // scale // targets_per_center
    src, nrm, w, (th, ph), tgt0, ctr, tnrm0 = _on_surface_targets(
        surf, n, k, rng, 0.02, phase_tgt=0.5 * GOLDEN_ANGLE)
    sigma = _ys32_real(th, ph) + 0.1 * rng.standard_normal(n)
    r = radius * math.sqrt(scale)
    offsets, idx = csr_ball(ctr, src, r)
    frac = 1.0 - np.arange(targets_per_center) / (targets_per_center)
    tgt = (ctr[:, None, :] + 0.02 * frac[None, :, None] * tnrm0[:, None, :]).reshape(-1, 3)
    tc = np.repeat(np.arange(k, dtype=np.int32), targets_per_center)
    tnrm = np.repeat(tnrm0, targets_per_center, axis=0)
    return Geometry(src, w, nrm, ctr, offsets, idx, tgt, tc, sigma, 16, 3,
                    f"B shared x{targets_per_center}", target_normals=tnrm)


def _random_surface(rng):
    if rng.random() < 0.5:
        axes = rng.uniform(0.5, 2.0, size=3)
        surf = Ellipsoid(axes)
        curv = surf.min_curvature_radius()
        area_est = 4.0 * math.pi * ((axes[0] * axes[1]) ** 1.6 + (axes[0] * axes[2]) ** 1.6
                                    + (axes[1] * axes[2]) ** 1.6) ** (1 / 1.6) / 3 ** (1 / 1.6)
        kind = "ellipsoid"
    else:
        surf = PerturbedSphere(rng)
        curv = 0.5
        area_est = 4.0 * math.pi
        kind = "perturbed_sphere"
    return surf, curv, area_est, kind


def _batched_geometry(config: str, item: int, n: int, p: int, layers: int,
                      list_radius_h: float = 8.0, knn_counts=None, surface=None) -> Geometry:
    rng = rng_for(config, item)
    if surface is None:
        surf, curv, area, kind = _random_surface(rng)
    else:
        surf, curv, area, kind = surface(rng)
    k = max(n // 4, 1)
    h = math.sqrt(area / n)
    offset = min(2.0 * h, 0.5 * curv)
    src, nrm, w, _, tgt, ctr, tnrm = _on_surface_targets(surf, n, k, rng, offset,
                                                         phase_tgt=rng.uniform(0, 2 * math.pi))
    sigma = rng.standard_normal(n)
    if knn_counts is None:
        offsets, idx = csr_ball(ctr, src, list_radius_h * h)
    else:
        counts = knn_counts(rng, k)
        offsets, idx = csr_knn(ctr, src, counts)
    return Geometry(src, w, nrm, ctr, offsets, idx, tgt, None, sigma, p, layers,
                    f"{config}{item}:{kind}", target_normals=tnrm)


def config_c(n_geometries: int = 64, scale: int = 1) -> List[Geometry]:
    """64 geometries (ellipsoids with semi-axes U(0.5, 2) or perturbed spheres).

    N log-uniform in [2048, 65536], N/4 targets, p uniform in {4, 8, 12, 16},
    single layer, lists of radius 8 h with h = sqrt(area / N).
    """
    meta = rng_for("C", 10_000)
    ns = np.exp(meta.uniform(math.log(2048), math.log(65536), size=n_geometries)).astype(int)
    ps = meta.choice([4, 8, 12, 16], size=n_geometries)
    return [_batched_geometry("C", i, max(int(ns[i]) // scale, 64), int(ps[i]), 1)
            for i in range(n_geometries)]


def config_d(n_geometries: int = 16, scale: int = 1) -> List[Geometry]:
    """16 perturbed spheres, N = 131072, T = 32768, p = 24, double layer only.

    Each center lists its L nearest sources with L log-uniform in [100, 8000].
    """
    def counts(rng, k):
        lo, hi = 100, min(8000, 131072 // scale)
        return np.exp(rng.uniform(math.log(lo), math.log(hi), size=k)).astype(np.int64)

    def sphere(rng):
        return PerturbedSphere(rng), 0.5, 4.0 * math.pi, "perturbed_sphere"

    return [_batched_geometry("D", i, 131072 // scale, 24, 2, knn_counts=counts, surface=sphere)
            for i in range(n_geometries)]


def config_e_geometries(n_geometries: int = 32, scale: int = 1) -> List[Geometry]:
    """32 resident geometries drawn as in the batched configuration, N in [4096, 262144]."""
    meta = rng_for("E", 10_000)
    ns = np.exp(meta.uniform(math.log(4096), math.log(262144), size=n_geometries)).astype(int)
    return [_batched_geometry("E", i, max(int(ns[i]) // scale, 64), 16, 3)
            for i in range(n_geometries)]


@dataclasses.dataclass
class Request:
    arrival_s: float
    geometry: int
    p: int
    layers: int
    sigma_seed: int


def config_e_requests(n_requests: int, rate_hz: float, n_geometries: int = 32) -> List[Request]:
    """Poisson arrivals at `rate_hz`; geometry uniform, p in {8, 16}, one layer each."""
    rng = rng_for("E", 20_000)
    gaps = rng.exponential(1.0 / rate_hz, size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    geo = rng.integers(0, n_geometries, size=n_requests)
    ps = rng.choice([8, 16], size=n_requests)
    lay = rng.choice([1, 2], size=n_requests)
    return [Request(float(t[i]), int(geo[i]), int(ps[i]), int(lay[i]), i)
            for i in range(n_requests)]


def request_sigma(req: Request, n: int) -> np.ndarray:
    return rng_for("E", 100_000 + req.sigma_seed).standard_normal(n)


def fuzz_geometry(seed: int, n: int, m: int, max_list: int, p: int, layers: int,
                  targets_per_center: int = 1, allow_empty: bool = True,
                  allow_duplicates: bool = True) -> Geometry:
    """A small random problem with ragged lists, optional empty rows and duplicates.

    Sources lie in the shell 1 <= |y| <= 1.5 and centers within 0.4 of the
    origin, with targets within 0.3 of their center, so |t - c| < |y - c|.
    """
    rng = rng_for("fuzz", seed)
    d = random_sphere_points(n, rng)
    src = d * rng.uniform(1.0, 1.5, size=(n, 1))
    nrm = random_sphere_points(n, rng)
    w = rng.uniform(0.1, 1.0, size=n)
    sigma = rng.standard_normal(n)
    ctr = random_sphere_points(m, rng) * rng.uniform(0.0, 0.4, size=(m, 1))
    lens = rng.integers(0 if allow_empty else 1, max_list + 1, size=m)
    offsets = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    idx = rng.integers(0, n, size=int(offsets[-1])).astype(np.int32)
    if not allow_duplicates:
        for i in range(m):
            L = int(lens[i])
            idx[offsets[i]:offsets[i + 1]] = rng.choice(n, size=min(L, n), replace=False)
    tc = np.repeat(np.arange(m, dtype=np.int32), targets_per_center)
    rng.shuffle(tc)
    tgt = ctr[tc] + random_sphere_points(len(tc), rng) * rng.uniform(0.0, 0.3, size=(len(tc), 1))
    tnrm = random_sphere_points(len(tc), rng)  # drawn last: earlier draws stay as they were
    return Geometry(src, w, nrm, ctr, offsets, idx, tgt, tc, sigma, p, layers, f"fuzz{seed}",
                    target_normals=tnrm)


def fuzz_near_boundary(seed: int, n: int, m: int, max_list: int, p: int, layers: int,
                       ratio: float = 0.99, targets_per_center: int = 2) -> Geometry:
    """Pairs close to the edge of the expansion's convergence (App. A needs
    |t - c| < |y - c|), where the terms decay slowest.

    Sources lie on the unit sphere and centers within 0.05 of the origin, so
    every |y - c| is within 0.95..1.05; each target sits at
    |t - c| = ratio * (the smallest |y - c| of its center's list), which puts
    every listed pair's |t - c| / |y - c| between about 0.9 * ratio and ratio.
    One target in three points from its center at its nearest listed source
    (cos gamma = 1), one in three away from it (cos gamma = -1), the rest in
    random directions.  ratio > 1 gives pairs outside convergence, for small p
    only.  Lists are ragged with empty rows and duplicates; a target of an
    empty list lies 0.5 from its center.
    """
    rng = rng_for("boundary", seed)
    src = random_sphere_points(n, rng)
    nrm = random_sphere_points(n, rng)
    w = rng.uniform(0.1, 1.0, size=n)
    sigma = rng.standard_normal(n)
    ctr = random_sphere_points(m, rng) * rng.uniform(0.0, 0.05, size=(m, 1))
    lens = rng.integers(0, max_list + 1, size=m)
    offsets = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    idx = rng.integers(0, n, size=int(offsets[-1])).astype(np.int32)
    tc = np.repeat(np.arange(m, dtype=np.int32), targets_per_center)
    rng.shuffle(tc)
    dirs = random_sphere_points(len(tc), rng)
    tgt = np.empty((len(tc), 3))
    for i, c in enumerate(tc):
        lo, hi = int(offsets[c]), int(offsets[c + 1])
        if hi == lo:
            tgt[i] = ctr[c] + 0.5 * dirs[i]
            continue
        d = src[idx[lo:hi]] - ctr[c]
        R = np.sqrt(np.einsum("ij,ij->i", d, d))
        j = int(np.argmin(R))
        u = d[j] / R[j]
        v = u if i % 3 == 0 else (-u if i % 3 == 1 else dirs[i])
        tgt[i] = ctr[c] + (ratio * R[j]) * v
    tnrm = random_sphere_points(len(tc), rng)
    return Geometry(src, w, nrm, ctr, offsets, idx, tgt, tc, sigma, p, layers,
                    f"boundary{seed}", target_normals=tnrm)
