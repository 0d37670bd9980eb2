"""Pins of the oracles' rounding yardsticks from above and from below.

The per-target half of the parity bar, |gpu_t - oracle_t| <= 1e-12 abs_t,
trusts the yardsticks abs_slp, abs_dlp, abs_sprime (the C oracle) and the
Helmholtz abs_* (oracle/helmholtz.py): sums over a target's list of |q| times
the size of each term of App. A.  A yardstick that came out too small fails
the oracle's own rounding pins; one that came out too large would loosen the
bar and pass them.  So each yardstick is pinned here by facts that do not
come from the oracle:

* equalities where no term cancels: collinear points (P_n(+-1) = (+-1)^n and
  no perpendicular part), the target at its center, orders 0, 1 and 2 at a
  known angle; against geometric series and closed forms of j_0, h_0, h_1;
* upper bounds with the Legendre factors at their maxima, |P_n| <= 1 and
  |P_n'| <= n(n+1)/2 (Helmholtz: spherical Bessel values from mpmath, not
  from scipy, which the Helmholtz oracle uses);
* two-sided bounds against the length of each term's gradient: the yardstick
  adds the lengths of two orthogonal parts of the gradient, so it lies
  between the gradient's length and sqrt(2) times it.  The gradients come from
  complex-step differentiation of an independent evaluation of each term
  (numpy's Legendre basis);
* the per-target sums depend on |q| only: sign flips of the density leave
  them unchanged, and with every term of one sign they equal the modulus of
  the potential.

Every check also runs against copies of the oracle with one mistake planted
in a yardstick (built on the CPU from a modified copy of the source), and
each copy must fail at least one check.
"""
import math
import os
import types

import mpmath as mp
import numpy as np
import numpy.polynomial.legendre as npleg
import pytest

import oracle
from oracle import helmholtz as H

FOUR_PI = 4.0 * math.pi
SQRT2 = math.sqrt(2.0)


def _unit(rng, n=None):
    v = rng.standard_normal(3 if n is None else (n, 3))
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _frame(rng):
    """Two orthonormal vectors."""
    e1 = _unit(rng)
    e2 = np.cross(e1, _unit(rng))
    return e1, e2 / np.linalg.norm(e2)


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


# ---------------------------------------------------------------------------
# Laplace: yardsticks k[2] (single layer), k[3] (double layer), k[5] (S') of
# one pair, and abs_* of the per-target sums
# ---------------------------------------------------------------------------

def _random_pairs(rng, n, p_max=24):
    """Pairs with |t-c| < |y-c|, normals of random length, about a third of
    them nearly collinear (x near +-1), where the P_n' part is smallest."""
    out = []
    for i in range(n):
        c = rng.uniform(-1, 1, 3)
        R = rng.uniform(0.3, 2.0)
        u = rng.uniform(0.02, 0.95)
        e = _unit(rng)
        y = c + R * e
        if i % 3 == 0:
            tdir = np.sign(rng.standard_normal()) * e + 1e-3 * _unit(rng)
            tdir /= np.linalg.norm(tdir)
        else:
            tdir = _unit(rng)
        t = c + u * R * tdir
        nu = _unit(rng) * rng.uniform(0.2, 3.0)
        nu_t = _unit(rng) * rng.uniform(0.2, 3.0)
        p = int(rng.integers(0, p_max + 1))
        out.append((t, c, y, nu, nu_t, p))
    return out


def check_laplace_triangle(lib):
    """|potential| <= yardstick for every layer, and yardsticks >= 0."""
    rng = np.random.default_rng(31)
    for t, c, y, nu, nu_t, p in _random_pairs(rng, 150):
        k = oracle.pair(t, c, y, nu, p, nu_t, library=lib)
        assert k[2] >= 0 and k[3] >= 0 and k[5] >= 0, k
        assert abs(k[0]) <= k[2] * (1 + 1e-13), ("slp", k)
        assert abs(k[1]) <= k[3] * (1 + 1e-13), ("dlp", k)
        assert abs(k[4]) <= k[5] * (1 + 1e-13) + 1e-300, ("sprime", k)


def _series(f, p, lo=0):
    return math.fsum(f(n) for n in range(lo, p + 1))


def check_laplace_collinear(lib):
    """Source and target on one line through the center (x = +1 or -1):
    P_n(x) = x^n and the P_n' direction has length 0, so every yardstick is
    a series in u = |t-c|/|y-c| with no cancellation:
      4 pi abs_slp    = sum_n u^n / R                       (both signs),
      4 pi abs_dlp    = |nu| sum_n (n+1) u^n / R^2          (nu along the line),
      4 pi abs_sprime = |nu_t| sum_{n>=1} n u^(n-1) / R^2   (nu_t along the line).
    With x = +1 every single-layer term is positive, so abs_slp equals the
    potential bit for bit."""
    rng = np.random.default_rng(32)
    for sign in (1.0, -1.0):
        for u in (0.1, 0.5, 0.9, 0.99):
            for p in (0, 1, 2, 5, 16, 24, 32):
                c = rng.uniform(-1, 1, 3)
                e = _unit(rng)
                R = rng.uniform(0.5, 2.0)
                y = c + R * e
                t = c + sign * u * R * e
                a, b = 2.5, 1.7
                k = oracle.pair(t, c, y, a * e, p, b * sign * e, library=lib)
                s_ref = _series(lambda n: u ** n, p) / R / FOUR_PI
                d_ref = a * _series(lambda n: (n + 1) * u ** n, p) / R ** 2 / FOUR_PI
                t_ref = b * _series(lambda n: n * u ** (n - 1), p, 1) / R ** 2 / FOUR_PI
                assert _rel(k[2], s_ref) <= 1e-13, ("slp", sign, u, p, k[2], s_ref)
                assert _rel(k[3], d_ref) <= 1e-13, ("dlp", sign, u, p, k[3], d_ref)
                if p == 0:
                    assert k[5] == 0.0
                else:
                    assert _rel(k[5], t_ref) <= 1e-13, ("sprime", sign, u, p, k[5], t_ref)
                if sign > 0:
                    assert k[2] == k[0], (u, p)
    # the closed forms of the same series at u = 1/2, p = 16
    u, p, R = 0.5, 16, 1.0
    assert _rel(_series(lambda n: u ** n, p), (1 - u ** (p + 1)) / (1 - u)) <= 1e-15
    assert _rel(_series(lambda n: (n + 1) * u ** n, p),
                (1 - (p + 2) * u ** (p + 1) + (p + 1) * u ** (p + 2)) / (1 - u) ** 2) <= 1e-15


def check_laplace_center_and_low_orders(lib):
    """The target at its center (only the n = 0 term, and S''s n = 1 term,
    survive), order 0 anywhere, and orders 1 and 2 at a known angle theta
    between t - c and y - c (x = cos theta, s = sin theta, u = rho/R):
      p = 0:  4 pi abs_slp = 1/R,  4 pi abs_dlp = |nu|/R^2,  abs_sprime = 0;
      t = c:  the same, and 4 pi abs_sprime = |nu_t|/R^2;
      p = 1:  4 pi abs_slp = (1 + u|x|)/R,
              4 pi abs_dlp = |nu| (1 + u(2|x| + s))/R^2,
              4 pi abs_sprime = |nu_t| (|x| + s)/R^2;
      p = 2:  adds u^2 |P_2|/R, |nu| u^2 (3|P_2| + 3|x| s)/R^2 and
              |nu_t| u (2|P_2| + 3|x| s)/R^2, with P_2 = (3x^2 - 1)/2, P_2' = 3x."""
    rng = np.random.default_rng(33)
    for _ in range(20):
        c = rng.uniform(-1, 1, 3)
        R = rng.uniform(0.3, 2.0)
        y = c + R * _unit(rng)
        nu = _unit(rng) * rng.uniform(0.2, 3.0)
        nu_t = _unit(rng) * rng.uniform(0.2, 3.0)
        ln, lt = np.linalg.norm(nu), np.linalg.norm(nu_t)
        for p in (0, 3, 16):
            k = oracle.pair(c, c, y, nu, p, nu_t, library=lib)
            assert _rel(k[2], 1 / (FOUR_PI * R)) <= 1e-14, ("t=c slp", k)
            assert _rel(k[3], ln / (FOUR_PI * R * R)) <= 1e-14, ("t=c dlp", k)
            if p == 0:
                assert k[5] == 0.0
            else:
                assert _rel(k[5], lt / (FOUR_PI * R * R)) <= 1e-14, ("t=c sprime", k)
        t = c + rng.uniform(0.1, 0.9) * R * _unit(rng)
        k = oracle.pair(t, c, y, nu, 0, nu_t, library=lib)
        assert _rel(k[2], 1 / (FOUR_PI * R)) <= 1e-14 and k[5] == 0.0
        assert _rel(k[3], ln / (FOUR_PI * R * R)) <= 1e-14
    for theta in (0.3, 1.0, math.pi / 2, 2.0, 2.9):
        for u in (0.2, 0.7):
            c = rng.uniform(-1, 1, 3)
            R = rng.uniform(0.5, 2.0)
            e1, e2 = _frame(rng)
            y = c + R * e1
            t = c + u * R * (math.cos(theta) * e1 + math.sin(theta) * e2)
            nu = _unit(rng) * 1.3
            nu_t = _unit(rng) * 0.8
            x, s = abs(math.cos(theta)), math.sin(theta)
            P2, dP2 = abs(1.5 * math.cos(theta) ** 2 - 0.5), 3 * x
            k1 = oracle.pair(t, c, y, nu, 1, nu_t, library=lib)
            k2 = oracle.pair(t, c, y, nu, 2, nu_t, library=lib)
            refs = [
                (k1[2], (1 + u * x) / R),
                (k1[3], 1.3 * (1 + u * (2 * x + s)) / R ** 2),
                (k1[5], 0.8 * (x + s) / R ** 2),
                (k2[2], (1 + u * x + u * u * P2) / R),
                (k2[3], 1.3 * (1 + u * (2 * x + s) + u * u * (3 * P2 + dP2 * s)) / R ** 2),
                (k2[5], 0.8 * (x + s + u * (2 * P2 + dP2 * s)) / R ** 2),
            ]
            for i, (got, ref) in enumerate(refs):
                assert _rel(got, ref / FOUR_PI) <= 1e-13, (theta, u, i, got, ref / FOUR_PI)


def check_laplace_upper_bounds(lib):
    """|P_n| <= 1, |P_n'| <= n(n+1)/2 and perpendicular lengths <= 1 bound
    each yardstick by a series in rho and R alone."""
    rng = np.random.default_rng(34)
    for t, c, y, nu, nu_t, p in _random_pairs(rng, 150, p_max=32):
        rho, R = np.linalg.norm(t - c), np.linalg.norm(y - c)
        ln, lt = np.linalg.norm(nu), np.linalg.norm(nu_t)
        k = oracle.pair(t, c, y, nu, p, nu_t, library=lib)
        bs = _series(lambda n: rho ** n / R ** (n + 1), p)
        bd = ln * _series(lambda n: rho ** n / R ** (n + 2) * ((n + 1) + n * (n + 1) / 2), p)
        bt = lt * _series(lambda n: rho ** (n - 1) / R ** (n + 1) * (n + n * (n + 1) / 2), p, 1)
        assert FOUR_PI * k[2] <= bs * (1 + 1e-13), ("slp", p, FOUR_PI * k[2], bs)
        assert FOUR_PI * k[3] <= bd * (1 + 1e-13), ("dlp", p, FOUR_PI * k[3], bd)
        assert FOUR_PI * k[5] <= bt * (1 + 1e-13) + 1e-300, ("sprime", p, FOUR_PI * k[5], bt)


def _term(n, t, c, y):
    """rho^n P_n(x) / R^(n+1) through numpy's Legendre basis, analytic in
    every coordinate (no abs, no conj), for complex-step derivatives."""
    d = y - c
    dl = t - c
    R = np.sqrt(np.sum(d * d))
    rho = np.sqrt(np.sum(dl * dl))
    x = np.sum(dl * d) / (rho * R)
    coef = np.zeros(n + 1)
    coef[n] = 1.0
    return rho ** n * npleg.legval(x, coef) / R ** (n + 1)


def _grad(n, t, c, y, wrt):
    h = 1e-30
    g = np.zeros(3)
    for i in range(3):
        e = np.zeros(3, dtype=complex)
        e[i] = 1j * h
        if wrt == "y":
            g[i] = _term(n, t.astype(complex), c.astype(complex), y + e).imag / h
        else:
            g[i] = _term(n, t + e, c.astype(complex), y.astype(complex)).imag / h
    return g


def check_laplace_gradient_sandwich(lib):
    """Per term, the double-layer yardstick adds the lengths of the two
    orthogonal parts of the term's source gradient (along y - c, and along
    t_hat - s_hat x), so  sum_n |nu| |grad_y T_n| <= 4 pi abs_dlp <= sqrt(2)
    times that; likewise S' with the target gradient (parts along t - c and
    s_hat - t_hat x); the single-layer yardstick is sum_n |T_n|."""
    rng = np.random.default_rng(35)
    for t, c, y, nu, nu_t, p in _random_pairs(rng, 40, p_max=16):
        if np.linalg.norm(t - c) < 1e-3:
            continue
        k = oracle.pair(t, c, y, nu, p, nu_t, library=lib)
        ln, lt = np.linalg.norm(nu), np.linalg.norm(nu_t)
        ts = [_term(n, t, c, y) for n in range(p + 1)]
        gy = [np.linalg.norm(_grad(n, t, c, y, "y")) for n in range(p + 1)]
        gt = [np.linalg.norm(_grad(n, t, c, y, "t")) for n in range(1, p + 1)]
        s_abs = math.fsum(abs(v) for v in ts)
        assert _rel(FOUR_PI * k[2], s_abs) <= 1e-13, ("slp", p, FOUR_PI * k[2], s_abs)
        lo = ln * math.fsum(gy)
        assert lo * (1 - 1e-12) <= FOUR_PI * k[3] <= SQRT2 * lo * (1 + 1e-12), (
            "dlp", p, FOUR_PI * k[3], lo)
        if p >= 1:
            lo = lt * math.fsum(gt)
            assert lo * (1 - 1e-12) <= FOUR_PI * k[5] <= SQRT2 * lo * (1 + 1e-12), (
                "sprime", p, FOUR_PI * k[5], lo)


def _collinear_problem(rng, n=40):
    """Sources on a ray from the center, targets on the same ray closer in:
    every term of the single layer is positive, every term of the double
    layer (normals along the ray) negative, every S' term (target normals
    along the ray) positive, for positive strengths."""
    c = np.array([0.1, -0.2, 0.3])
    e = _unit(rng)
    src = c + np.outer(rng.uniform(0.5, 1.5, n), e)
    w = rng.uniform(0.1, 1.0, n)
    nrm = np.tile(e, (n, 1))
    tgt = c + np.outer(rng.uniform(0.0, 0.45, 5), e)
    off = np.array([0, n], dtype=np.int64)
    idx = np.arange(n, dtype=np.int32)
    return src, w, nrm, c[None, :], off, idx, tgt, np.zeros(5, dtype=np.int32), np.tile(e, (5, 1))


def check_laplace_per_target_sums(lib):
    """abs_* depend on |w sigma| only, and without cancellation equal the
    modulus of the potential."""
    rng = np.random.default_rng(36)
    src, w, nrm, ctr, off, idx, tgt, tc, tn = _collinear_problem(rng)
    sigma = rng.uniform(0.5, 2.0, len(src))
    r = oracle.evaluate(src, w, nrm, ctr, off, idx, tgt, tc, sigma, 12, 7, target_normals=tn,
                        library=lib)
    assert np.array_equal(r["abs_slp"], r["slp"])
    assert np.all(np.abs(r["abs_dlp"] + r["dlp"]) <= 1e-14 * r["abs_dlp"])
    sp = r["sprime"][1:]  # the first target sits where t - c may be 0
    assert np.all(np.abs(r["abs_sprime"][1:] - sp) <= 1e-14 * r["abs_sprime"][1:])
    # random problem: sign flips of sigma leave every yardstick's bits alone
    n, m = 300, 40
    src = _unit(rng, n) * rng.uniform(1.0, 1.5, (n, 1))
    nrm = _unit(rng, n) * rng.uniform(0.5, 2.0, (n, 1))
    w = rng.uniform(0.1, 1.0, n)
    ctr = _unit(rng, m) * rng.uniform(0, 0.3, (m, 1))
    lens = rng.integers(0, 60, m)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    idx = rng.integers(0, n, int(off[-1])).astype(np.int32)
    tgt = ctr + _unit(rng, m) * rng.uniform(0, 0.3, (m, 1))
    tn = _unit(rng, m)
    sigma = rng.standard_normal(n)
    flip = np.where(rng.uniform(size=n) < 0.5, -1.0, 1.0)
    a = oracle.evaluate(src, w, nrm, ctr, off, idx, tgt, None, sigma, 9, 7, target_normals=tn,
                        library=lib)
    b = oracle.evaluate(src, w, nrm, ctr, off, idx, tgt, None, sigma * flip, 9, 7,
                        target_normals=tn, library=lib)
    for key in ("abs_slp", "abs_dlp", "abs_sprime"):
        assert np.array_equal(a[key], b[key]), key


LAPLACE_CHECKS = [check_laplace_triangle, check_laplace_collinear,
                  check_laplace_center_and_low_orders, check_laplace_upper_bounds,
                  check_laplace_gradient_sandwich, check_laplace_per_target_sums]


@pytest.mark.parametrize("check", LAPLACE_CHECKS, ids=lambda f: f.__name__)
def test_laplace_yardsticks(check):
    check(None)


# Mistakes planted in a copy of the C oracle: (what, original text, replacement).
LAPLACE_MUTATIONS = [
    ("1/(4 pi) dropped from the single-layer yardstick",
     "k[2] = ks_abs * inv4pi;", "k[2] = ks_abs;"),
    ("no modulus in the single-layer yardstick",
     "ks_abs += fabs(term_s);", "ks_abs += term_s;"),
    ("1/|y-c| dropped from the double-layer yardstick",
     "kd_abs += radial_d * nu_len", "kd_abs += radial * nu_len"),
    ("|nu| dropped from the double-layer yardstick",
     "kd_abs += radial_d * nu_len *", "kd_abs += radial_d *"),
    ("the projection nu . s_hat instead of |nu| in the double-layer yardstick",
     "kd_abs += radial_d * nu_len *", "kd_abs += radial_d * fabs(nu_sh) *"),
    ("(n+1) dropped from the double-layer yardstick",
     "nu_len * ((double)(n + 1) * fabs(P)", "nu_len * (fabs(P)"),
    ("perpendicular length dropped from the double-layer yardstick",
     "fabs(dP) * perp)", "fabs(dP))"),
    ("1/(4 pi) dropped from the double-layer yardstick",
     "k[3] = kd_abs * inv4pi;", "k[3] = kd_abs;"),
    ("|nu_t| dropped from the S' yardstick",
     "kt_abs += radial_t * m_len *", "kt_abs += radial_t *"),
    ("n dropped from the S' yardstick",
     "m_len * ((double)n * fabs(P)", "m_len * (fabs(P)"),
    ("perpendicular length dropped from the S' yardstick",
     "fabs(dP) * m_perp)", "fabs(dP))"),
    ("1/(4 pi) dropped from the S' yardstick",
     "k[5] = kt_abs * inv4pi;", "k[5] = kt_abs;"),
    ("signed strength in the single-layer sum of yardsticks",
     "sum_abs[0] += fabs(q) * k[2];", "sum_abs[0] += q * k[2];"),
    ("single-layer yardstick summed for the double layer",
     "sum_abs[1] += fabs(q) * k[3];", "sum_abs[1] += fabs(q) * k[2];"),
]


@pytest.mark.parametrize("what,old,new", LAPLACE_MUTATIONS, ids=[m[0] for m in LAPLACE_MUTATIONS])
def test_planted_laplace_yardstick_mistakes_are_caught(what, old, new, tmp_path):
    text = open(oracle.SRC).read()
    assert text.count(old) == 1, f"mutation site not unique: {old!r}"
    src = tmp_path / "mutant.c"
    src.write_text(text.replace(old, new))
    lib = oracle.compile_source(str(src), str(tmp_path / "libmutant.so"))
    failed = []
    for check in LAPLACE_CHECKS:
        try:
            check(lib)
        except AssertionError:
            failed.append(check.__name__)
    assert failed, f"no check caught: {what}"


# ---------------------------------------------------------------------------
# Helmholtz: yardsticks G_abs, D_abs (pair_terms) and the S' yardstick
# (target_normal_terms); spherical Bessel values from mpmath
# ---------------------------------------------------------------------------

mp.mp.dps = 30


def _jn(n, z):
    z = mp.mpf(z)
    return mp.sqrt(mp.pi / (2 * z)) * mp.besselj(n + mp.mpf(1) / 2, z)


def _yn(n, z):
    z = mp.mpf(z)
    return mp.sqrt(mp.pi / (2 * z)) * mp.bessely(n + mp.mpf(1) / 2, z)


def _hn(n, z):
    return mp.mpc(_jn(n, z), _yn(n, z))


def _dfn(f, n, z):
    """f_n'(z) = f_{n-1}(z) - (n+1)/z f_n(z), f_0' = -f_1 (DLMF 10.51.2)."""
    if n == 0:
        return -f(1, z)
    return f(n - 1, z) - (n + 1) / mp.mpf(z) * f(n, z)


def check_helm_triangle(HM):
    rng = np.random.default_rng(41)
    for t, c, y, nu, nu_t, p in _random_pairs(rng, 40, p_max=16):
        for k in (0.5, 5.0, 20.0):
            G, D, Ga, Da = HM.pair_terms(t, c, y[None, :], nu[None, :], k, p)
            Sp, Spa = HM.target_normal_terms(t, c, y[None, :], nu_t, k, p)
            assert abs(G[0]) <= Ga[0] * (1 + 1e-13), ("slp", k, p)
            assert abs(D[0]) <= Da[0] * (1 + 1e-13), ("dlp", k, p)
            assert abs(Sp[0]) <= Spa[0] * (1 + 1e-13) + 1e-300, ("sprime", k, p)


def check_helm_center_and_order_zero(HM):
    """With j_0(w) = sin w / w, j_0'(w) = (w cos w - sin w)/w^2, |h_0(z)| = 1/z
    and |h_0'(z)| = |h_1(z)| = sqrt(1 + z^2)/z^2 (z = k|y-c|, w = k|t-c|):
      t = c:  abs_slp = 1/(4 pi R), abs_dlp = k^2 |nu| |h_1(z)| / (4 pi),
              abs_sprime = k^2 |nu_t| |h_1(z)| / (4 pi);
      p = 0:  abs_slp = k |j_0(w)| / (4 pi z), abs_dlp = k^2 |j_0(w)| |nu| |h_1(z)| / (4 pi),
              abs_sprime = k^2 |j_0'(w)| |nu_t| / (4 pi z)."""
    rng = np.random.default_rng(42)
    for _ in range(12):
        c = rng.uniform(-1, 1, 3)
        R = rng.uniform(0.3, 2.0)
        y = c + R * _unit(rng)
        nu = _unit(rng) * rng.uniform(0.3, 2.0)
        nu_t = _unit(rng) * rng.uniform(0.3, 2.0)
        ln, lt = np.linalg.norm(nu), np.linalg.norm(nu_t)
        for k in (0.5, 3.0, 20.0):
            z = k * R
            h1 = math.sqrt(1 + z * z) / (z * z)
            for p in (0, 4, 12):
                _, _, Ga, Da = HM.pair_terms(c, c, y[None, :], nu[None, :], k, p)
                _, Spa = HM.target_normal_terms(c, c, y[None, :], nu_t, k, p)
                assert _rel(Ga[0], 1 / (FOUR_PI * R)) <= 1e-13, ("t=c slp", k, p)
                assert _rel(Da[0], k * k * ln * h1 / FOUR_PI) <= 1e-13, ("t=c dlp", k, p)
                if p >= 1:
                    assert _rel(Spa[0], k * k * lt * h1 / FOUR_PI) <= 1e-13, ("t=c sp", k, p)
            t = c + rng.uniform(0.05, 0.9) * R * _unit(rng)
            w = k * np.linalg.norm(t - c)
            j0 = abs(math.sin(w) / w)
            dj0 = abs((w * math.cos(w) - math.sin(w)) / (w * w))
            _, _, Ga, Da = HM.pair_terms(t, c, y[None, :], nu[None, :], k, 0)
            _, Spa = HM.target_normal_terms(t, c, y[None, :], nu_t, k, 0)
            assert _rel(Ga[0], k * j0 / (FOUR_PI * z)) <= 1e-13, ("p=0 slp", k)
            assert _rel(Da[0], k * k * j0 * ln * h1 / FOUR_PI) <= 1e-13, ("p=0 dlp", k)
            assert _rel(Spa[0], k * k * dj0 * lt / (FOUR_PI * z)) <= 1e-12, ("p=0 sp", k)


def check_helm_collinear_and_upper_bounds(HM):
    """Collinear points (x = +-1, no perpendicular part, normals along the
    line):  abs_slp = (k/4pi) sum (2n+1) |j_n(w)| |h_n(z)|,
    abs_dlp = (k/4pi) |nu| k sum (2n+1) |j_n(w)| |h_n'(z)|,
    abs_sprime = (k/4pi) |nu_t| k sum (2n+1) |j_n'(w)| |h_n(z)|.
    At any angle the same sums (with n(n+1)/2 |j_n(w)/w| |h_n(z)| k added for
    the P_n' parts) bound the yardsticks from above."""
    rng = np.random.default_rng(43)
    for k in (0.7, 6.0, 20.0):
        for u in (0.2, 0.8):
            for p in (1, 6, 14):
                c = rng.uniform(-1, 1, 3)
                e = _unit(rng)
                R = rng.uniform(0.4, 1.5)
                z, w = k * R, k * u * R
                J = [_jn(n, w) for n in range(p + 1)]
                Hh = [_hn(n, z) for n in range(p + 1)]
                dJ = [_dfn(_jn, n, w) for n in range(p + 1)]
                dH = [_dfn(_hn, n, z) for n in range(p + 1)]
                s_ref = float(k / (4 * mp.pi) * mp.fsum((2 * n + 1) * abs(J[n]) * abs(Hh[n])
                                                        for n in range(p + 1)))
                d_ref = float(k * k / (4 * mp.pi) * mp.fsum((2 * n + 1) * abs(J[n]) * abs(dH[n])
                                                            for n in range(p + 1)))
                t_ref = float(k * k / (4 * mp.pi) * mp.fsum((2 * n + 1) * abs(dJ[n]) * abs(Hh[n])
                                                            for n in range(p + 1)))
                for sign in (1.0, -1.0):
                    y = c + R * e
                    t = c + sign * u * R * e
                    _, _, Ga, Da = HM.pair_terms(t, c, y[None, :], 1.6 * e[None, :], k, p)
                    _, Spa = HM.target_normal_terms(t, c, y[None, :], 0.7 * sign * e, k, p)
                    assert _rel(Ga[0], s_ref) <= 1e-12, ("slp", k, u, p, sign)
                    assert _rel(Da[0], 1.6 * d_ref) <= 1e-12, ("dlp", k, u, p, sign)
                    assert _rel(Spa[0], 0.7 * t_ref) <= 1e-12, ("sprime", k, u, p, sign)
                # any angle: |P_n| <= 1, |P_n'| <= n(n+1)/2, perpendicular parts <= 1
                y = c + R * e
                t = c + u * R * _unit(rng)
                nu = _unit(rng) * 1.1
                nu_t = _unit(rng) * 0.9
                _, _, Ga, Da = HM.pair_terms(t, c, y[None, :], nu[None, :], k, p)
                _, Spa = HM.target_normal_terms(t, c, y[None, :], nu_t, k, p)
                dbound = 1.1 * float(k / (4 * mp.pi) * mp.fsum(
                    (2 * n + 1) * abs(J[n]) * (k * abs(dH[n]) + n * (n + 1) / 2 * abs(Hh[n]) / R)
                    for n in range(p + 1)))
                tbound = 0.9 * float(k / (4 * mp.pi) * mp.fsum(
                    (2 * n + 1) * abs(Hh[n]) * (k * abs(dJ[n]) + n * (n + 1) / 2 * abs(J[n]) / (u * R))
                    for n in range(p + 1)))
                assert Ga[0] <= s_ref * (1 + 1e-12), ("slp bound", k, u, p)
                assert Da[0] <= dbound * (1 + 1e-12), ("dlp bound", k, u, p)
                assert Spa[0] <= tbound * (1 + 1e-12), ("sprime bound", k, u, p)


def check_helm_per_target_sums(HM):
    """abs_* depend on |q| only: sign flips of the complex density leave them
    unchanged bit for bit."""
    rng = np.random.default_rng(44)
    n, m = 120, 15
    src = _unit(rng, n) * rng.uniform(1.0, 1.5, (n, 1))
    nrm = _unit(rng, n) * rng.uniform(0.5, 2.0, (n, 1))
    w = rng.uniform(0.1, 1.0, n)
    ctr = _unit(rng, m) * rng.uniform(0, 0.3, (m, 1))
    lens = rng.integers(0, 30, m)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    idx = rng.integers(0, n, int(off[-1])).astype(np.int32)
    tgt = ctr + _unit(rng, m) * rng.uniform(0, 0.3, (m, 1))
    tn = _unit(rng, m)
    sigma = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    flip = np.where(rng.uniform(size=n) < 0.5, -1.0, 1.0)
    a = HM.evaluate(src, w, nrm, ctr, off, idx, tgt, None, sigma, 5.0, 8, 7, target_normals=tn)
    b = HM.evaluate(src, w, nrm, ctr, off, idx, tgt, None, sigma * flip, 5.0, 8, 7,
                    target_normals=tn)
    for key in ("abs_slp", "abs_dlp", "abs_sprime"):
        assert np.array_equal(a[key], b[key]), key
        assert np.all(np.abs(a[key[4:]]) <= a[key] * (1 + 1e-13)), key


HELM_CHECKS = [check_helm_triangle, check_helm_center_and_order_zero,
               check_helm_collinear_and_upper_bounds, check_helm_per_target_sums]


@pytest.mark.parametrize("check", HELM_CHECKS, ids=lambda f: f.__name__)
def test_helmholtz_yardsticks(check):
    check(H)


HELM_MUTATIONS = [
    ("1/(4 pi) dropped from the single-layer yardstick",
     "G_abs = np.abs(terms).sum(axis=0)", "G_abs = 4 * math.pi * np.abs(terms).sum(axis=0)"),
    ("1/|y-c| dropped from the double-layer yardstick",
     "D_abs = (np.abs(coef)[:, None] / R[None, :] * nu_len[None, :]",
     "D_abs = (np.abs(coef)[:, None] * nu_len[None, :]"),
    ("|nu| dropped from the double-layer yardstick",
     "D_abs = (np.abs(coef)[:, None] / R[None, :] * nu_len[None, :]",
     "D_abs = (np.abs(coef)[:, None] / R[None, :]"),
    ("k|y-c| dropped from the double-layer yardstick",
     "* (k * R[None, :] * np.abs(dh) * np.abs(P)", "* (np.abs(dh) * np.abs(P)"),
    ("perpendicular length dropped from the double-layer yardstick",
     "+ perp[None, :] * np.abs(h) * np.abs(dP))", "+ np.abs(h) * np.abs(dP))"),
    ("k dropped from the S' yardstick",
     "* (k * np.abs(djt)[:, None] * np.abs(P)", "* (np.abs(djt)[:, None] * np.abs(P)"),
    ("|nu_t| dropped from the S' yardstick",
     "ab = (np.abs(coef)[:, None] * np.abs(h) * nu_len", "ab = (np.abs(coef)[:, None] * np.abs(h)"),
    ("perpendicular length dropped from the S' yardstick",
     "+ perp[None, :] * np.abs(jt_rho)[:, None] * np.abs(dP)))",
     "+ np.abs(jt_rho)[:, None] * np.abs(dP)))"),
    ("real part of the strength in the single-layer sum of yardsticks",
     'out["abs_slp"][i] = float(np.sum(np.abs(qi) * Ga))',
     'out["abs_slp"][i] = float(np.sum(qi.real * Ga))'),
]


@pytest.mark.parametrize("what,old,new", HELM_MUTATIONS, ids=[m[0] for m in HELM_MUTATIONS])
def test_planted_helmholtz_yardstick_mistakes_are_caught(what, old, new):
    path = os.path.join(os.path.dirname(oracle.__file__), "helmholtz.py")
    text = open(path).read()
    assert text.count(old) == 1, f"mutation site not unique: {old!r}"
    mod = types.ModuleType("helmholtz_mutant")
    exec(compile(text.replace(old, new), "helmholtz_mutant", "exec"), mod.__dict__)
    failed = []
    for check in HELM_CHECKS:
        try:
            check(mod)
        except AssertionError:
            failed.append(check.__name__)
    assert failed, f"no check caught: {what}"
