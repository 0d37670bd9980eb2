"""Pins of the conventional-QBX oracle (local coefficients formed from the
sources, then evaluated; Sec. 2.3 eqs. (sph-harm), (local-coeffs),
(local-expansion)) to facts that do not come from its own formulas: the
independently written target-specific oracle (eq. (tsqbx) says the two
agree), Cartesian closed forms of the low-order solid harmonics, the axis
and equator values of P_n^m, and the symmetries of Y_n^m under rotation
about the z-axis and conjugation.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import conventional as conv


def _rand_unit(rng, n):
    v = rng.standard_normal((n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _problem(seed, n_centers=4, ns=7, nt_per=2):
    rng = np.random.default_rng(seed)
    centers = rng.uniform(-0.5, 0.5, (n_centers, 3))
    src, lists, offs = [], [], [0]
    tgt, tc = [], []
    for c in range(n_centers):
        y = centers[c] + _rand_unit(rng, ns) * rng.uniform(1.0, 1.4, (ns, 1))
        lists.extend(range(c * ns, c * ns + ns))
        src.extend(y)
        offs.append(offs[-1] + ns)
        for _ in range(nt_per):
            tgt.append(centers[c] + _rand_unit(rng, 1)[0] * rng.uniform(0.0, 0.8))
            tc.append(c)
    src = np.array(src)
    w = rng.uniform(0.5, 1.5, len(src))
    sigma = rng.standard_normal(len(src))
    return dict(src=src, w=w, sigma=sigma, centers=centers, offs=np.array(offs, dtype=np.int64),
                lists=np.array(lists, dtype=np.int32), tgt=np.array(tgt),
                tc=np.array(tc, dtype=np.int32))


@pytest.mark.parametrize("p", [0, 1, 2, 5, 9, 16, 24])
def test_form_then_evaluate_equals_target_specific_oracle(p):
    """eq. (tsqbx): the p-th order local expansion evaluated at t equals the
    target-specific sum; checked against the C oracle, written separately."""
    pr = _problem(500 + p)
    L = conv.form(pr["src"], pr["w"], pr["centers"], pr["offs"], pr["lists"], pr["sigma"], p)
    u = conv.evaluate(L, pr["centers"], pr["tgt"], pr["tc"], p)
    ts = oracle.evaluate(pr["src"], pr["w"], None, pr["centers"], pr["offs"], pr["lists"],
                         pr["tgt"], pr["tc"], pr["sigma"], p, oracle.SLP)
    err = np.abs(u - ts["slp"])
    assert np.all(err <= 1e-13 * ts["abs_slp"]), (err / ts["abs_slp"]).max()


def _single(y, c, q, p):
    return conv.form(np.array([y]), np.array([1.0]), np.array([c]), np.array([0, 1]),
                     np.array([0]), np.array([q]), p)[0]


@pytest.mark.parametrize("sign", [1.0, -1.0])
def test_source_on_axis_leaves_only_m_zero(sign):
    """theta = 0 or pi: P_n^m(+-1) = 0 for m > 0 and P_n(+-1) = (+-1)^n, so
    L_n^0 = q (+-1)^n sqrt((2n+1)/(4 pi)) / ((2n+1) R^{n+1}) and the rest is 0."""
    p, R, q = 12, 1.3, 0.7
    c = np.array([0.1, -0.2, 0.3])
    L = _single(c + np.array([0.0, 0.0, sign * R]), c, q, p)
    for n in range(p + 1):
        ref = q * sign ** n * math.sqrt((2 * n + 1) / (4 * math.pi)) / ((2 * n + 1) * R ** (n + 1))
        assert abs(L[n, p] - ref) <= 1e-15 * abs(ref)
        for m in range(1, n + 1):
            assert abs(L[n, p + m]) <= 1e-15 * abs(ref) and abs(L[n, p - m]) <= 1e-15 * abs(ref)


def test_source_on_equator_has_no_odd_n_plus_m():
    """theta = pi/2: P_n^m(0) = 0 when n + m is odd."""
    p = 10
    c = np.zeros(3)
    L = _single(np.array([0.6, -0.9, 0.0]), c, 1.0, p)
    big = np.abs(L).max()
    for n in range(p + 1):
        for m in range(-n, n + 1):
            if (n + m) % 2:
                assert abs(L[n, m + p]) <= 1e-15 * big


def test_low_orders_match_cartesian_solid_harmonics():
    """Textbook Cartesian forms of Y_n^{-m} r^n for n <= 2 (no Condon-Shortley
    factor): Y_0^0 = 1/sqrt(4 pi); r Y_1^0 = sqrt(3/(4 pi)) z;
    r Y_1^{-1} = sqrt(3/(8 pi)) (x - i y); r^2 Y_2^{-1} = sqrt(15/(8 pi)) z (x - i y);
    r^2 Y_2^{-2} = sqrt(15/(32 pi)) (x - i y)^2; r^2 Y_2^0 = sqrt(5/(16 pi)) (2z^2 - x^2 - y^2)."""
    rng = np.random.default_rng(7)
    c = rng.uniform(-1, 1, 3)
    d = np.array([0.4, -0.7, 0.5])
    q = -1.7
    R = np.linalg.norm(d)
    L = _single(c + d, c, q, 3)
    x, y, z = d
    w = x - 1j * y
    ref = {
        (0, 0): q / (math.sqrt(4 * math.pi) * R),
        (1, 0): q * math.sqrt(3 / (4 * math.pi)) * z / (3 * R ** 3),
        (1, 1): q * math.sqrt(3 / (8 * math.pi)) * w / (3 * R ** 3),
        (2, 0): q * math.sqrt(5 / (16 * math.pi)) * (2 * z * z - x * x - y * y) / (5 * R ** 5),
        (2, 1): q * math.sqrt(15 / (8 * math.pi)) * z * w / (5 * R ** 5),
        (2, 2): q * math.sqrt(15 / (32 * math.pi)) * w * w / (5 * R ** 5),
    }
    for (n, m), v in ref.items():
        assert abs(L[n, m + 3] - v) <= 2e-15 * abs(v), (n, m, L[n, m + 3], v)
        # L_n^{-m} = conj(L_n^m) for a real strength (no Condon-Shortley factor)
        assert abs(L[n, 3 - m] - np.conj(v)) <= 2e-15 * abs(v), (n, -m)


def test_rotation_about_z_multiplies_by_phase():
    """Rotating every source by alpha about the z-axis through c adds alpha to
    phi, so Y_n^{-m} and L_n^m pick up exp(-i m alpha)."""
    p, alpha = 8, 0.83
    rng = np.random.default_rng(11)
    c = np.array([0.2, 0.1, -0.3])
    d = _rand_unit(rng, 5) * 1.2
    q = rng.standard_normal(5)
    rot = np.array([[math.cos(alpha), -math.sin(alpha), 0], [math.sin(alpha), math.cos(alpha), 0],
                    [0, 0, 1.0]])
    args = (np.array([c]), np.array([0, 5]), np.arange(5), q, p)
    L0 = conv.form(c + d, np.ones(5), *args)[0]
    L1 = conv.form(c + d @ rot.T, np.ones(5), *args)[0]
    for n in range(p + 1):
        for m in range(-n, n + 1):
            ref = L0[n, m + p] * np.exp(-1j * m * alpha)
            assert abs(L1[n, m + p] - ref) <= 1e-14 * (abs(L0).max())


def test_unit_coefficient_evaluates_to_solid_harmonic():
    """Only L_1^{+-1} = 1: u = |d| (Y_1^1 + Y_1^{-1})(d) = 2 sqrt(3/(8 pi)) d_x."""
    p = 2
    L = np.zeros((1, p + 1, 2 * p + 1), dtype=np.complex128)
    L[0, 1, p + 1] = 1.0
    L[0, 1, p - 1] = 1.0
    c = np.array([0.3, 0.2, 0.1])
    t = c + np.array([0.25, -0.1, 0.05])
    u = conv.evaluate(L, np.array([c]), np.array([t]), np.array([0]), p)
    assert abs(u[0] - 2 * math.sqrt(3 / (8 * math.pi)) * 0.25) <= 1e-15


def test_target_at_center_is_monopole():
    """t = c: only n = 0 survives, u = sum q / (4 pi R)."""
    pr = _problem(3, n_centers=2)
    pr["tgt"] = pr["centers"][pr["tc"]].copy()
    L = conv.form(pr["src"], pr["w"], pr["centers"], pr["offs"], pr["lists"], pr["sigma"], 6)
    u = conv.evaluate(L, pr["centers"], pr["tgt"], pr["tc"], 6)
    for i, c in enumerate(pr["tc"]):
        sel = pr["lists"][pr["offs"][c]:pr["offs"][c + 1]]
        R = np.linalg.norm(pr["src"][sel] - pr["centers"][c], axis=1)
        ref = np.sum(pr["w"][sel] * pr["sigma"][sel] / R) / (4 * math.pi)
        assert abs(u[i] - ref) <= 1e-15 * np.sum(np.abs(pr["w"][sel] * pr["sigma"][sel] / R))


def test_pack_roundtrip_and_scale_bounds():
    pr = _problem(21, n_centers=3)
    p = 7
    L = conv.form(pr["src"], pr["w"], pr["centers"], pr["offs"], pr["lists"], pr["sigma"], p)
    C = conv.pack(L, p)
    assert C.shape == (3, 64)
    assert np.array_equal(conv.unpack(C, p), L)
    S = conv.coefficient_scale(pr["src"], pr["w"], pr["centers"], pr["offs"], pr["lists"],
                               pr["sigma"], p)
    assert np.all(np.abs(L) <= S * (1 + 1e-14))
    # empty list: all zeros
    offs = pr["offs"].copy()
    offs[2] = offs[1]
    L2 = conv.form(pr["src"], pr["w"], pr["centers"], offs, pr["lists"], pr["sigma"], p,
                   which=[1])
    assert not np.any(L2)
