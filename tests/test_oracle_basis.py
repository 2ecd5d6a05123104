"""Pins of the oracle's basis functions (Def. 1.2, Def. 2.1, Thm. 2.2, Lemma 3.5)."""

import math
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest
from scipy import special

from oracle import basis as BS, quadrature as Q

rng = np.random.default_rng(7)


def test_low_degree_spherical_harmonics_closed_forms():
    th = rng.uniform(0, math.pi, 50)
    ph = rng.uniform(0, 2 * math.pi, 50)
    P = BS.legendre_table(3, th)
    Y00 = BS.legendre_signed(P, 0, 0)
    Y10 = BS.legendre_signed(P, 1, 0)
    Y11 = BS.legendre_signed(P, 1, 1) * np.exp(1j * ph)
    Y1m1 = BS.legendre_signed(P, 1, -1) * np.exp(-1j * ph)
    np.testing.assert_allclose(Y00, 1 / (2 * math.sqrt(math.pi)), rtol=1e-15)
    np.testing.assert_allclose(Y10, math.sqrt(3 / (4 * math.pi)) * np.cos(th), rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(Y11, -math.sqrt(3 / (8 * math.pi)) * np.sin(th) * np.exp(1j * ph), rtol=1e-14)
    np.testing.assert_allclose(Y1m1, math.sqrt(3 / (8 * math.pi)) * np.sin(th) * np.exp(-1j * ph), rtol=1e-14)


def _rodrigues(l, m, t):
    """P_lm(t) from the Rodrigues form of Def. 2.1, with exact rational polynomial
    arithmetic for the derivative: (-1)^m / (2^l l!) (1-t^2)^{m/2} d^{l+m}/dt^{l+m} (t^2-1)^l."""
    # (t^2 - 1)^l as coefficient list (index = power)
    poly = [Fraction(0)] * (2 * l + 1)
    for k in range(l + 1):
        poly[2 * k] = Fraction(math.comb(l, k) * (-1) ** (l - k))
    for _ in range(l + m):
        poly = [poly[i] * i for i in range(1, len(poly))] or [Fraction(0)]
    vals = []
    for tv in np.atleast_1d(t):
        tq = Fraction(float(tv))          # exact rational value of the FP64 abscissa
        vals.append(float(sum(c * tq ** i for i, c in enumerate(poly))))
    val = np.array(vals)
    return (-1) ** m / (2 ** l * math.factorial(l)) * (1 - t * t) ** (m / 2) * val


@pytest.mark.parametrize("l", range(0, 9))
def test_legendre_matches_rodrigues_exact_derivative(l):
    th = np.linspace(0.05, math.pi - 0.05, 17)
    P = BS.legendre_table(l + 1, th)
    t = np.cos(th)
    for m in range(-l, l + 1):
        M = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - m) / math.factorial(l + m))
        ref = M * _rodrigues(l, m, t)
        got = BS.legendre_signed(P, l, m)
        assert np.abs(got - ref).max() <= 1e-14 * np.abs(ref).max(), (l, m)


@pytest.mark.parametrize("B", [20, 64])
def test_legendre_matches_scipy(B):
    """Against scipy's spherical harmonics (independent library routine)."""
    th = rng.uniform(0.01, math.pi - 0.01, 40)
    P = BS.legendre_table(B, th)
    for l in range(0, B, 3):
        for m in range(-l, l + 1, max(1, l // 5)):
            ref = special.sph_harm_y(l, m, th, 0.0).real
            got = BS.legendre_signed(P, l, m)
            scale = max(np.abs(ref).max(), 1e-300)
            assert np.abs(got - ref).max() <= 1e-12 * scale + 1e-300, (l, m)


def test_legendre_parity():
    """Pbar_lm(-t) = (-1)^{l+m} Pbar_lm(t): theta_j and theta_{2B-1-j} are mirror images."""
    B = 16
    th = Q.polar_angles(B)
    P = BS.legendre_table(B, th)
    for m in range(B):
        for l in range(m, B):
            scale = np.abs(P[m, l]).max()
            assert np.abs(P[m, l, ::-1] - (-1) ** (l + m) * P[m, l]).max() <= 1e-13 * scale, (l, m)


def test_laguerre_low_degree_closed_forms():
    """L_0 = 1, L_1 = 1 + alpha - t, L_2 = (a+1)(a+2)/2 - (a+2) t + t^2/2 (Eq. associated_laguerre_explicit),
    through the radial table with the normalization and r^l removed."""
    r = np.linspace(0.1, 4.0, 23)
    t = r * r
    R = BS.radial_table(4, r)
    for l in range(2):
        a = l + 0.5
        for k, L in enumerate([np.ones_like(t), 1 + a - t, (a + 1) * (a + 2) / 2 - (a + 2) * t + t * t / 2]):
            n = k + l + 1
            if n > 4:
                continue
            Nnl = math.sqrt(2 * math.factorial(k) / math.gamma(n + 0.5))
            np.testing.assert_allclose(R[n, l], Nnl * L * r ** l, rtol=1e-13, atol=1e-14)


def _laguerre_explicit(k, alpha, t):
    """Eq. associated_laguerre_explicit with exact rationals (alpha half-integer, t rational)."""
    tot = Fraction(0)
    for j in range(k + 1):
        # binom(k+alpha, k-j) for rational alpha
        num = Fraction(1)
        for q in range(k - j):
            num *= (Fraction(k) + alpha - q)
        binom = num / math.factorial(k - j)
        tot += Fraction((-1) ** j, math.factorial(j)) * binom * t ** j
    return tot


@pytest.mark.parametrize("l", [0, 1, 4, 9])
def test_radial_matches_explicit_sum(l):
    ts = [Fraction(1, 7), Fraction(3, 2), Fraction(9, 1), Fraction(29, 3)]
    r = np.array([math.sqrt(float(t)) for t in ts])
    B = l + 12
    R = BS.radial_table(B, r)
    for k in range(0, 12):
        n = k + l + 1
        Nnl = math.sqrt(2 * math.factorial(k) / math.gamma(n + 0.5))
        ref = np.array([Nnl * float(_laguerre_explicit(k, Fraction(2 * l + 1, 2), t)) * float(t) ** (l / 2) for t in ts])
        scale = np.abs(ref).max()
        assert np.abs(R[n, l] - ref).max() <= 1e-12 * scale, (l, k)


def test_radial_matches_scipy_genlaguerre():
    r = rng.uniform(0.05, 6, 30)
    B = 30
    R = BS.radial_table(B, r)
    for l in range(0, B, 4):
        for n in range(l + 1, B + 1, 3):
            k = n - l - 1
            Nnl = math.exp(0.5 * (math.log(2) + math.lgamma(k + 1) - math.lgamma(n + 0.5)))
            ref = Nnl * special.eval_genlaguerre(k, l + 0.5, r * r) * r ** l
            assert np.abs(R[n, l] - ref).max() <= 1e-11 * np.abs(ref).max(), (n, l)


def test_radial_start_and_lemma_recurrence():
    """Lemma 3.5: R_{l+1,l} = sqrt(2/Gamma(l+3/2)) r^l and the normalized three-term
    recurrence in n hold for the oracle's radial functions (built from Eq.
    laguerre_recursion, a different route)."""
    r = np.linspace(0.2, 5.0, 31)
    B = 24
    R = BS.radial_table(B, r)
    t = r * r
    for l in range(B):
        np.testing.assert_allclose(R[l + 1, l], math.sqrt(2 / math.gamma(l + 1.5)) * r ** l, rtol=1e-13)
        for n in range(l + 1, B):
            c1 = (2 * n - l - 0.5 - t) / math.sqrt((n + 0.5) * (n - l))
            c2 = math.sqrt((n - 0.5) / (n + 0.5) * (n - l - 1) / (n - l))
            prev = R[n - 1, l] if n - 1 > l else 0.0
            pred = c1 * R[n, l] - c2 * prev
            scale = np.abs(R[l + 1:B + 1, l]).max(axis=0)
            assert np.all(np.abs(R[n + 1, l] - pred) <= 1e-12 * scale), (n, l)


def test_H100_constant():
    r = rng.uniform(0, 3, 10)
    th = rng.uniform(0, math.pi, 10)
    ph = rng.uniform(0, 2 * math.pi, 10)
    np.testing.assert_allclose(BS.sgl_function(1, 0, 0, r, th, ph), math.pi ** -0.75, rtol=1e-15)


@pytest.mark.parametrize("B", [4, 16, 32])
def test_radial_gram_identity(B):
    """Sect. 3.3 (iDRT): sum_i a_i r_i^2 Rhat_nl(r_i) Rhat_n'l(r_i) = delta_nn',
    i.e. the rows of rho_l = [sigma_i Rhat_nl(r_i)] are orthonormal."""
    g = Q.sgl_grid(B)
    rho = BS.radial_table(B, g["r"], g["log_sigma"])
    for l in range(B):
        M = rho[l + 1:B + 1, l, :]
        assert np.abs(M @ M.T - np.eye(B - l)).max() < 2e-13, l
    assert np.abs(rho).max() <= 1.0


def test_scaled_radial_matches_mpmath():
    """rho_nl(r_i) against 30-digit mpmath Laguerre values at B = 8."""
    B = 8
    g = Q.sgl_grid(B)
    rr = Q.radial_rule(2 * B)
    rho = BS.radial_table(B, g["r"], g["log_sigma"])
    with mp.workdps(30):
        for l in range(B):
            for n in range(l + 1, B + 1):
                for i in range(2 * B):
                    x = rr.r_mp[i]
                    sig = mp.exp(rr.log_a_mp[i] / 2) * x
                    v = sig * mp.sqrt(2 * mp.factorial(n - l - 1) / mp.gamma(n + mp.mpf(1) / 2)) \
                        * mp.laguerre(n - l - 1, l + mp.mpf(1) / 2, x * x) * x ** l
                    assert abs(float(v) - rho[n, l, i]) <= 1e-14, (n, l, i)
