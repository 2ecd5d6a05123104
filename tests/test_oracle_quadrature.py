"""Pins of the oracle's quadrature rules (Thm. 3.1, Lemma 3.2, Thm. 3.3)."""

import math

import mpmath as mp
import numpy as np
import pytest
from scipy import special

from oracle import mp_direct, quadrature as Q


@pytest.mark.parametrize("B", [1, 2, 3, 8, 17, 64])
def test_polar_weights_positive_symmetric_and_total(B):
    """Lemma 3.2: b_j > 0; the rule is symmetric under theta -> pi - theta;
    the printed weights integrate sin(theta) (sum 2), the corrected ones the
    whole sphere (sum over j, k of b~_j = 4 pi)."""
    b = Q.polar_weights_printed(B)
    bt = Q.polar_weights(B)
    assert np.all(b > 0) and np.all(bt > 0)
    np.testing.assert_allclose(bt, bt[::-1], rtol=1e-14, atol=0)
    assert abs(b.sum() - 2.0) < 1e-13
    assert abs(bt.sum() * 2 * B - 4 * math.pi) < 1e-12


def _sph_gram(B, weights):
    th = Q.polar_angles(B)
    ph = Q.azimuth_angles(B)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    Y = []
    for l in range(B):
        for m in range(-l, l + 1):
            # scipy's sph_harm_y(l, m, polar, azimuth) includes the Condon-Shortley phase
            Y.append(special.sph_harm_y(l, m, TH, PH).reshape(-1))
    Y = np.array(Y)
    w = np.repeat(weights, 2 * B)
    return (Y * w) @ Y.conj().T


@pytest.mark.parametrize("B", [2, 5, 8, 16])
def test_spherical_rule_exact_with_corrected_weight(B):
    """Thm. 3.1 with b~_j: sum_{jk} b~_j Y_lm conj(Y_l'm') = delta for l, l' < B.
    Y_lm taken from scipy (independent of the oracle's Legendre code)."""
    G = _sph_gram(B, Q.polar_weights(B))
    assert np.abs(G - np.eye(B * B)).max() < 1e-13


def test_printed_weight_misses_azimuthal_step():
    """Reading of Thm. 3.1: the printed b_j in the double sum gives B/pi times
    the identity, i.e. the missing factor is exactly pi/B."""
    B = 6
    G = _sph_gram(B, Q.polar_weights_printed(B))
    assert np.abs(G - (B / math.pi) * np.eye(B * B)).max() < 1e-13
    assert np.abs(G - np.eye(B * B)).max() > 0.5


def test_polar_angles():
    B = 4
    np.testing.assert_allclose(Q.polar_angles(B), [(2 * j + 1) * math.pi / 16 for j in range(8)], rtol=0, atol=1e-15)
    np.testing.assert_allclose(Q.azimuth_angles(B), [k * math.pi / 4 for k in range(8)], rtol=0, atol=1e-15)


def test_radial_rule_one_point_closed_form():
    """N = 1: the node is mu_1/mu_0 = 1/sqrt(pi) and the weight mu_0 = sqrt(pi)/2."""
    rr = Q.radial_rule(1)
    assert abs(rr.r[0] - 1 / math.sqrt(math.pi)) < 1e-16
    assert abs(rr.a[0] - math.sqrt(math.pi) / 2) < 4e-16


@pytest.mark.parametrize("N", [2, 4, 6, 8])
def test_radial_rule_matches_hankel_route(N):
    """Nodes and weights agree with an independent route: roots of the Hankel
    determinant polynomial and the Lagrange-integral weight formula of Thm. 3.3."""
    r, a = mp_direct.radial_rule(N)
    rr = Q.radial_rule(N)
    with mp.workdps(40):
        for i in range(N):
            assert abs(rr.r_mp[i] - r[i]) <= mp.mpf(10) ** -30 * r[i]
            assert abs(rr.log_a_mp[i] - mp.log(a[i])) <= mp.mpf(10) ** -30


@pytest.mark.parametrize("N", [16, 64, 128])
def test_radial_rule_moment_exactness(N):
    """Thm. 3.3: sum_i a_i r_i^k = int_0^inf r^k exp(-r^2) dr for all k <= 2N-1
    (checked at 40 digits with the moments from mpmath's quadrature at low k)."""
    rr = Q.radial_rule(N)
    with mp.workdps(40):
        for k in range(0, 2 * N):
            s = mp.fsum(mp.exp(rr.log_a_mp[i]) * rr.r_mp[i] ** k for i in range(N))
            ex = mp.gamma(mp.mpf(k + 1) / 2) / 2
            assert abs(s / ex - 1) < mp.mpf(10) ** -28, (N, k)
        # the closed-form moments themselves
        for k in (0, 1, 2, 5):
            q = mp.quad(lambda x: x ** k * mp.exp(-x * x), [0, mp.inf])
            assert abs(q - mp.gamma(mp.mpf(k + 1) / 2) / 2) < mp.mpf(10) ** -30
        # one degree beyond is not integrated exactly (the defect shrinks like
        # 2^-N relative to mu_2N, so it is visible at 40 digits only for small N)
        if N <= 16:
            k = 2 * N
            s = mp.fsum(mp.exp(rr.log_a_mp[i]) * rr.r_mp[i] ** k for i in range(N))
            assert abs(s / (mp.gamma(mp.mpf(k + 1) / 2) / 2) - 1) > mp.mpf(10) ** -20


@pytest.mark.parametrize("N", [32, 256])
def test_radial_rule_fp64_fields(N):
    """FP64 fields are consistent with each other and lie in the expected ranges."""
    rr = Q.radial_rule(N)
    assert np.all(np.diff(rr.r) > 0) and rr.r[0] > 0
    np.testing.assert_allclose(rr.log_atilde, rr.log_a + rr.r ** 2 + 2 * np.log(rr.r), rtol=1e-14, atol=1e-12)
    np.testing.assert_allclose(rr.log_sigma, 0.5 * rr.log_a + np.log(rr.r), rtol=1e-14, atol=1e-12)
    assert np.all(np.isfinite(rr.log_a))
    # sum of weights = sqrt(pi)/2, in log-sum-exp form (a_i underflows at N=256)
    m = rr.log_a.max()
    tot = math.exp(m) * np.sum(np.exp(rr.log_a - m))
    assert abs(tot - math.sqrt(math.pi) / 2) < 1e-14
