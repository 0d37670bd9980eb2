"""Plain FP64 CPU oracle for target-specific QBX with the Helmholtz kernel.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg call this; the product library never does.  It
shares no code with the GPU path.

What it computes (Wala & Kloeckner, App. A, the Helmholtz case): for a real
wavenumber k > 0, with gamma the angle between t - c and s - c,

    G_k^(p)(t, s) = (i k / 4 pi) sum_{n=0..p} (2n+1) j_n(k|t-c|) h_n(k|s-c|) P_n(cos gamma),

the p-th order target-specific expansion of exp(ik|t-s|) / (4 pi |t-s|)
(the addition theorem App. A cites from DLMF 10.60), and its source gradient
dotted with the normal nu at s,

    nu . grad_s G_k^(p)(t, s) = (i k / 4 pi) sum_{n=0..p} (2n+1) j_n(k|t-c|) / |s-c|
        [ k (nu . (s-c)) h_n'(k|s-c|) P_n(x) + (nu . t_hat - (nu . s_hat) x) h_n(k|s-c|) P_n'(x) ],

x = cos gamma, and its target gradient dotted with a normal nu_t at t (S'),

    nu_t . grad_t G_k^(p)(t, s) = (i k / 4 pi) sum_{n=0..p} (2n+1) h_n(k|s-c|) / |t-c|
        [ k (nu_t . (t-c)) j_n'(k|t-c|) P_n(x) + (nu_t . s_hat - (nu_t . t_hat) x) j_n(k|t-c|) P_n'(x) ],

j_n is the spherical Bessel function of the first kind and
h_n = j_n + i y_n the spherical Hankel function of the first kind; scipy's
spherical_jn / spherical_yn (and their derivatives) are used as library
primitives.  P_n and P_n' come from Bonnet's recurrence and
P_{n+1}' = x P_n' + (n+1) P_n.  Potentials sum q_y = w_y sigma_y over each
center's list, sigma complex (eq. pt-pot), in list order.

Readings where the paper is silent: k is real and positive; at t = c the angle
is undefined and t_hat = 0 (then j_n(0) = 0 for n >= 1 leaves the n = 0 term
of the potentials, and S' keeps its limit: j_n(k rho) / rho -> k / 3 for n = 1
and 0 otherwise, so only (i k / 4 pi) k h_1(k|s-c|) (nu_t . s_hat) is left);
|s - c| = 0 is invalid.  The yardsticks abs_* are the sums of the moduli of
the terms (the double layer with |nu| times the length of each gradient term),
against which rounding is measured.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.special as sps

SLP, DLP, SPRIME = 1, 2, 4


def _legendre_and_derivative(x, p):
    """P_n(x) and P_n'(x), n = 0..p, by Bonnet's recurrence and
    P_{n+1}' = x P_n' + (n+1) P_n; arrays of shape (p+1,) + x.shape."""
    P = np.zeros((p + 1,) + x.shape)
    dP = np.zeros((p + 1,) + x.shape)
    P[0] = 1.0
    if p >= 1:
        P[1] = x
        dP[1] = 1.0
    for n in range(1, p):
        P[n + 1] = ((2 * n + 1) * x * P[n] - n * P[n - 1]) / (n + 1)
        dP[n + 1] = x * dP[n] + (n + 1) * P[n]
    return P, dP


def pair_terms(t, c, s, nu, k: float, p: int):
    """Kernel values for one target t (center c) against sources s[m] (m, 3).

    Returns (G, D, G_abs, D_abs): the single-layer kernel G_k^(p), the
    double-layer kernel nu . grad_s G_k^(p) (None if nu is None) and their
    yardsticks, each of shape (m,), 1/(4 pi) included."""
    t = np.asarray(t, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    s = np.atleast_2d(np.asarray(s, dtype=np.float64))
    dt = t - c
    rho = math.sqrt(float(dt @ dt))
    that = dt / rho if rho > 0 else np.zeros(3)
    d = s - c
    R = np.sqrt(np.einsum("ij,ij->i", d, d))
    shat = d / R[:, None]
    x = shat @ that
    P, dP = _legendre_and_derivative(x, p)
    n = np.arange(p + 1)
    jt = sps.spherical_jn(n, k * rho)                      # (p+1,)
    jr = sps.spherical_jn(n[:, None], k * R[None, :])      # (p+1, m)
    yr = sps.spherical_yn(n[:, None], k * R[None, :])
    h = jr + 1j * yr
    coef = (1j * k / (4 * math.pi)) * (2 * n + 1) * jt    # (p+1,)
    terms = coef[:, None] * h * P
    G = terms.sum(axis=0)
    G_abs = np.abs(terms).sum(axis=0)
    if nu is None:
        return G, None, G_abs, None
    nu = np.atleast_2d(np.asarray(nu, dtype=np.float64))
    djr = sps.spherical_jn(n[:, None], k * R[None, :], derivative=True)
    dyr = sps.spherical_yn(n[:, None], k * R[None, :], derivative=True)
    dh = djr + 1j * dyr
    nu_d = np.einsum("ij,ij->i", nu, d)
    nu_t = nu @ that
    nu_s = np.einsum("ij,ij->i", nu, shat)
    nu_len = np.linalg.norm(nu, axis=1)
    perp = np.linalg.norm(that[None, :] - shat * x[:, None], axis=1)
    a = k * nu_d[None, :] * dh * P
    b = (nu_t - nu_s * x)[None, :] * h * dP
    dterms = coef[:, None] / R[None, :] * (a + b)
    D = dterms.sum(axis=0)
    D_abs = (np.abs(coef)[:, None] / R[None, :] * nu_len[None, :]
             * (k * R[None, :] * np.abs(dh) * np.abs(P) + perp[None, :] * np.abs(h) * np.abs(dP))
             ).sum(axis=0)
    return G, D, G_abs, D_abs


def target_normal_terms(t, c, s, nu_t, k: float, p: int):
    """S' kernel nu_t . grad_t G_k^(p)(t, s) for one target t (center c, unit
    or any normal nu_t) against sources s[m] (m, 3), and its yardstick: the
    sum over n of |i k (2n+1) / (4 pi)| |h_n| (k |nu_t| |j_n'| |P_n| +
    |nu_t| |s_hat - t_hat x| |j_n / rho| |P_n'|).  Both of shape (m,)."""
    t = np.asarray(t, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    nu_t = np.asarray(nu_t, dtype=np.float64)
    s = np.atleast_2d(np.asarray(s, dtype=np.float64))
    dt = t - c
    rho = math.sqrt(float(dt @ dt))
    d = s - c
    R = np.sqrt(np.einsum("ij,ij->i", d, d))
    shat = d / R[:, None]
    n = np.arange(p + 1)
    if rho > 0:
        that = dt / rho
        djt = sps.spherical_jn(n, k * rho, derivative=True)
        jt_rho = sps.spherical_jn(n, k * rho) / rho
    else:  # limits at t = c: j_n'(0) = 1/3 and j_n(k rho) / rho -> k/3 for n = 1 only
        that = np.zeros(3)
        djt = np.where(n == 1, 1.0 / 3.0, 0.0)
        jt_rho = np.where(n == 1, k / 3.0, 0.0)
    x = shat @ that
    P, dP = _legendre_and_derivative(x, p)
    h = (sps.spherical_jn(n[:, None], k * R[None, :])
         + 1j * sps.spherical_yn(n[:, None], k * R[None, :]))
    coef = (1j * k / (4 * math.pi)) * (2 * n + 1)
    nt_t = float(nu_t @ that)
    nt_s = shat @ nu_t
    a = (k * nt_t) * djt[:, None] * P
    b = (nt_s - nt_t * x)[None, :] * jt_rho[:, None] * dP
    terms = coef[:, None] * h * (a + b)
    nu_len = float(np.linalg.norm(nu_t))
    perp = np.linalg.norm(shat - that[None, :] * x[:, None], axis=1)
    ab = (np.abs(coef)[:, None] * np.abs(h) * nu_len
          * (k * np.abs(djt)[:, None] * np.abs(P) + perp[None, :] * np.abs(jt_rho)[:, None] * np.abs(dP)))
    return terms.sum(axis=0), ab.sum(axis=0)


def evaluate(sources, weights, normals, centers, list_offsets, list_sources, targets,
             target_center, sigma, k: float, p: int, layers: int, select=None,
             target_normals=None):
    """Helmholtz potentials at all targets (or the `select`ed ones).

    sigma is complex (N,).  Returns a dict with complex 'slp', 'dlp', 'sprime'
    and real 'abs_' + each (None for a layer not requested)."""
    if not k > 0:
        raise ValueError("the wavenumber must be positive")
    if layers & DLP and normals is None:
        raise ValueError("the double layer needs normals")
    if layers & SPRIME and target_normals is None:
        raise ValueError("S' needs target normals")
    sources = np.asarray(sources, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.complex128)
    q = np.asarray(weights, dtype=np.float64) * sigma
    tsel = np.arange(len(targets)) if select is None else np.asarray(select)
    out = {key: None for key in ("slp", "dlp", "sprime", "abs_slp", "abs_dlp", "abs_sprime")}
    if layers & SLP:
        out["slp"] = np.zeros(len(tsel), dtype=np.complex128)
        out["abs_slp"] = np.zeros(len(tsel))
    if layers & DLP:
        out["dlp"] = np.zeros(len(tsel), dtype=np.complex128)
        out["abs_dlp"] = np.zeros(len(tsel))
    if layers & SPRIME:
        out["sprime"] = np.zeros(len(tsel), dtype=np.complex128)
        out["abs_sprime"] = np.zeros(len(tsel))
    for i, ti in enumerate(tsel):
        ci = ti if target_center is None else int(target_center[ti])
        lo, hi = int(list_offsets[ci]), int(list_offsets[ci + 1])
        if hi == lo:
            continue
        idx = np.asarray(list_sources[lo:hi])
        nu = normals[idx] if layers & DLP else None
        G, D, Ga, Da = pair_terms(targets[ti], centers[ci], sources[idx], nu, k, p)
        qi = q[idx]
        # sequential sums in list order
        if layers & SLP:
            acc = 0j
            for v in qi * G:
                acc += v
            out["slp"][i] = acc
            out["abs_slp"][i] = float(np.sum(np.abs(qi) * Ga))
        if layers & DLP:
            acc = 0j
            for v in qi * D:
                acc += v
            out["dlp"][i] = acc
            out["abs_dlp"][i] = float(np.sum(np.abs(qi) * Da))
        if layers & SPRIME:
            Sp, Spa = target_normal_terms(targets[ti], centers[ci], sources[idx],
                                          target_normals[ti], k, p)
            acc = 0j
            for v in qi * Sp:
                acc += v
            out["sprime"][i] = acc
            out["abs_sprime"][i] = float(np.sum(np.abs(qi) * Spa))
    return out


def evaluate_geometry(g, k: float, sigma, p=None, layers=None, select=None):
    """evaluate() on any object with the workload Geometry attributes."""
    return evaluate(g.sources, g.weights, g.normals, g.centers, g.list_offsets, g.list_sources,
                    g.targets, g.target_center, sigma, k, g.p if p is None else p,
                    g.layers if layers is None else layers, select=select,
                    target_normals=getattr(g, "target_normals", None))


def _evaluate_rows(args):
    (sources, weights, normals, centers, offsets, rows, targets, sigma, k, p, layers,
     target_normals) = args
    return evaluate(sources, weights, normals, centers, offsets, rows, targets, None, sigma, k, p,
                    layers, target_normals=target_normals)


def process_pool(workers: int):
    """A pool of fresh interpreter processes (spawned, so that nothing of the
    caller's process state, a GPU runtime included, is inherited)."""
    import concurrent.futures as cf
    import multiprocessing as mp

    return cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn"))


def evaluate_parallel(g, k: float, sigma, p=None, layers=None, select=None, workers: int = 8,
                      pool=None):
    """evaluate_geometry() split over `workers` processes by target: each
    process evaluates a slice of the selected targets (with their centers' rows
    cut out of the CSR), one target at a time as evaluate() does, so the
    results are those of evaluate_geometry() bit for bit.  `pool` (from
    process_pool) is used if given, else one is made for the call."""
    p = g.p if p is None else p
    layers = g.layers if layers is None else layers
    tsel = np.arange(g.n_targets) if select is None else np.asarray(select)
    tc = np.arange(g.n_targets) if g.target_center is None else np.asarray(g.target_center)
    tn = getattr(g, "target_normals", None)
    jobs = []
    for part in np.array_split(tsel, max(1, min(workers, len(tsel)))):
        cs = tc[part]
        lo = np.asarray(g.list_offsets)[cs]
        hi = np.asarray(g.list_offsets)[cs + 1]
        offs = np.zeros(len(part) + 1, dtype=np.int64)
        np.cumsum(hi - lo, out=offs[1:])
        rows = (np.concatenate([np.asarray(g.list_sources[a:b]) for a, b in zip(lo, hi)])
                if len(part) else np.zeros(0, dtype=np.int32))
        jobs.append((g.sources, g.weights, g.normals, np.asarray(g.centers)[cs], offs, rows,
                     np.asarray(g.targets)[part], sigma, k, p, layers,
                     None if tn is None else np.asarray(tn)[part]))
    if pool is None:
        with process_pool(len(jobs)) as ex:
            parts = list(ex.map(_evaluate_rows, jobs))
    else:
        parts = list(pool.map(_evaluate_rows, jobs))
    out = {}
    for key in ("slp", "dlp", "sprime", "abs_slp", "abs_dlp", "abs_sprime"):
        out[key] = None if parts[0][key] is None else np.concatenate([q[key] for q in parts])
    return out
