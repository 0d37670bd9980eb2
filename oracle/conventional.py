"""Plain FP64 CPU oracle for conventional QBX: local expansions formed from
the sources of each center's list, then evaluated at the targets.

TEST INFRASTRUCTURE ONLY: the test suite calls this; the product library
never does.  It shares no code with the GPU path.

What it computes (Wala & Kloeckner, Sec. 2.3, the first approach of
Sec. 2.4):

* eq. (sph-harm): Y_n^m(theta, phi) = sqrt((2n+1)/(4 pi) (n-|m|)!/(n+|m|)!)
  P_n^{|m|}(cos theta) e^{i m phi}, with P_n^m the associated Legendre
  function written without the Condon-Shortley factor (so that
  Y_n^{-m} = conj(Y_n^m)); scipy's lpmv, a library primitive, carries that
  factor, which is divided out here;
* eq. (local-coeffs), summed over the list L(c) of a center c with the
  strengths q_y = w_y sigma_y of eq. (pt-pot):
      L_n^m(c) = sum_{y in L(c)} q_y Y_n^{-m}(y - c) / ((2n+1) |y - c|^{n+1}),
  n = 0..p, |m| <= n (the angles of y - c in the polar/azimuthal convention
  theta = acos(z/r), phi = atan2(y, x));
* eq. (local-expansion) truncated after n = p, at each target t of center c:
      u(t) = sum_{n=0..p} sum_{|m|<=n} L_n^m(c) |t - c|^n Y_n^m(t - c).

By eq. (tsqbx) u(t) equals the target-specific single layer of the same list
up to rounding.  At t = c only n = 0 survives (|t - c|^0 = 1, Y_0^0 is
constant), and the angles of t - c are then immaterial.

Compact real layout of one center's coefficients (real densities give
L_n^{-m} = conj(L_n^m)): (p+1)^2 doubles, degree n at offset n^2, holding
Re L_n^0, then Re L_n^m, Im L_n^m for m = 1..n.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.special as sps


def n_coeffs(p: int) -> int:
    return (p + 1) * (p + 1)


def _norm(n: int, m: int) -> float:
    am = abs(m)
    return math.sqrt((2 * n + 1) / (4 * math.pi)
                     * math.exp(math.lgamma(n - am + 1) - math.lgamma(n + am + 1)))


def ylm(n: int, m: int, theta, phi):
    """Y_n^m of eq. (sph-harm), P_n^{|m|} without the Condon-Shortley factor."""
    am = abs(m)
    plm = sps.lpmv(am, n, np.cos(theta)) * (-1.0) ** am
    return _norm(n, m) * plm * np.exp(1j * m * phi)


def _angles(v):
    r = np.sqrt(np.einsum("ij,ij->i", v, v))
    cos_t = np.clip(v[:, 2] / np.where(r > 0, r, 1.0), -1.0, 1.0)
    return r, np.arccos(cos_t), np.arctan2(v[:, 1], v[:, 0])


def form(sources, weights, centers, offsets, lists, sigma, p: int, which=None):
    """L_n^m of the centers `which` (default all) as a complex array
    [center, n, m + p] (entries with |m| > n are zero), summed in list order."""
    sources = np.asarray(sources, dtype=np.float64)
    q_all = np.asarray(weights, dtype=np.float64) * np.asarray(sigma, dtype=np.float64)
    centers = np.asarray(centers, dtype=np.float64)
    which = np.arange(len(centers)) if which is None else np.asarray(which)
    out = np.zeros((len(which), p + 1, 2 * p + 1), dtype=np.complex128)
    for k, c in enumerate(which):
        sel = np.asarray(lists[offsets[c]:offsets[c + 1]], dtype=np.int64)
        if sel.size == 0:
            continue
        R, th, ph = _angles(sources[sel] - centers[c])
        q = q_all[sel]
        for n in range(p + 1):
            scale = q / ((2 * n + 1) * R ** (n + 1))
            for m in range(-n, n + 1):
                terms = scale * ylm(n, -m, th, ph)
                acc = 0.0 + 0.0j
                for v in terms:  # list order
                    acc += v
                out[k, n, m + p] = acc
    return out


def evaluate(L, centers, targets, target_center, p: int, which=None):
    """u(t) of eq. (local-expansion) for each target, with L the array of
    `form` for the centers `which` (default: all centers, in order)."""
    centers = np.asarray(centers, dtype=np.float64)
    targets = np.asarray(targets, dtype=np.float64)
    which = np.arange(len(centers)) if which is None else np.asarray(which)
    slot = {int(c): k for k, c in enumerate(which)}
    out = np.zeros(len(targets))
    for i, t in enumerate(targets):
        c = int(target_center[i])
        d = (t - centers[c])[None, :]
        rho, th, ph = _angles(d)
        acc = 0.0 + 0.0j
        for n in range(p + 1):
            rn = rho[0] ** n
            for m in range(-n, n + 1):
                acc += L[slot[c], n, m + p] * rn * ylm(n, m, th[0], ph[0])
        out[i] = acc.real
    return out


def coefficient_scale(sources, weights, centers, offsets, lists, sigma, p: int, which=None):
    """Sum over the list of |q_y Y_n^{-m}(y - c)| / ((2n+1)|y-c|^{n+1}) for each
    coefficient, the yardstick rounding in L_n^m is measured against; same
    array shape as `form` (real)."""
    sources = np.asarray(sources, dtype=np.float64)
    q_all = np.abs(np.asarray(weights, dtype=np.float64) * np.asarray(sigma, dtype=np.float64))
    centers = np.asarray(centers, dtype=np.float64)
    which = np.arange(len(centers)) if which is None else np.asarray(which)
    out = np.zeros((len(which), p + 1, 2 * p + 1))
    for k, c in enumerate(which):
        sel = np.asarray(lists[offsets[c]:offsets[c + 1]], dtype=np.int64)
        if sel.size == 0:
            continue
        R, th, ph = _angles(sources[sel] - centers[c])
        for n in range(p + 1):
            scale = q_all[sel] / ((2 * n + 1) * R ** (n + 1))
            for m in range(-n, n + 1):
                out[k, n, m + p] = np.sum(scale * np.abs(ylm(n, -m, th, ph)))
    return out


def pack(L, p: int):
    """Complex [center, n, m + p] -> compact real layout [center, (p+1)^2]."""
    out = np.zeros((L.shape[0], n_coeffs(p)))
    for n in range(p + 1):
        base = n * n
        out[:, base] = L[:, n, p].real
        for m in range(1, n + 1):
            out[:, base + 2 * m - 1] = L[:, n, m + p].real
            out[:, base + 2 * m] = L[:, n, m + p].imag
    return out


def unpack(C, p: int):
    """Compact real layout -> complex [center, n, m + p], with
    L_n^{-m} = conj(L_n^m) (real densities)."""
    C = np.atleast_2d(np.asarray(C, dtype=np.float64))
    L = np.zeros((C.shape[0], p + 1, 2 * p + 1), dtype=np.complex128)
    for n in range(p + 1):
        base = n * n
        L[:, n, p] = C[:, base]
        for m in range(1, n + 1):
            v = C[:, base + 2 * m - 1] + 1j * C[:, base + 2 * m]
            L[:, n, m + p] = v
            L[:, n, p - m] = np.conj(v)
    return L
