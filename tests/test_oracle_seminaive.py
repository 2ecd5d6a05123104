"""Pins of the seminaive (cosine-domain) Legendre oracle, oracle/seminaive.py.

Each pin compares with something other than the seminaive code itself: the
defining properties of the DCT of Eq. DCT (orthogonality; vanishing beyond the
degree of a trigonometric polynomial, checked on monomials cos^d), the direct
weighted Legendre sums of Eq. DLT formed from the basis tables by a plain matrix
product, and the quadrature sums of the direct transforms (Alg. 1, Alg. 2).
"""

import numpy as np
import pytest

from oracle import direct as D
from oracle import seminaive as S
from oracle import quadrature as Q

RNG = np.random.default_rng(20260412)


@pytest.mark.parametrize("N", [2, 8, 16, 24])
def test_dct_matrix_is_orthogonal(N):
    C = S.dct_matrix(N)
    assert np.abs(C @ C.T - np.eye(N)).max() < 1e-14


@pytest.mark.parametrize("N", [8, 16])
def test_dct_of_cosine_powers_vanishes_beyond_degree(N):
    # cos^d th is a trigonometric polynomial of degree d
    th = (2 * np.arange(N) + 1) * np.pi / (2 * N)
    C = S.dct_matrix(N)
    for d in range(N):
        v = C @ np.cos(th) ** d
        assert np.abs(v[d + 1:]).max(initial=0.0) < 1e-13, d
        # the top index is the leading term 2^(1-d) cos(d th): sum_j cos^2(d th_j) = N/2
        lead = np.sqrt(N) if d == 0 else 2.0 ** -d * np.sqrt(2.0 * N)
        assert abs(v[d] - lead) < 1e-13, d


@pytest.mark.parametrize("B", [5, 12])
def test_cosine_legendre_vectors_are_sparse(B):
    """[C q_lm]_k = 0 for k > l - par(m) (the sparsity the seminaive method stores)."""
    T = S.get_tables(B)
    for m in range(B):
        for l in range(m, B):
            v = T.Cq[m, l]
            d = l - S.parity(m)
            assert np.abs(v[d + 1:]).max(initial=0.0) < 1e-12 * max(1.0, np.abs(v).max()), (m, l)


@pytest.mark.parametrize("B", [6, 11])
def test_dlt_matches_direct_weighted_sum(B):
    """Eq. dct_trick: the cosine-domain sum equals sum_j b~_j Pbar_lm t_j, every order."""
    g = Q.sgl_grid(B)
    T = S.get_tables(B)
    for m in range(1 - B, B):
        t = RNG.standard_normal(2 * B) + 1j * RNG.standard_normal(2 * B)
        P = np.array([T.Pbar[abs(m), l] * (-1.0) ** (abs(m) * (m < 0)) for l in range(abs(m), B)])
        ref = P @ (g["btilde"] * t)
        got = S.dlt_forward(t, B, m)
        assert np.abs(got - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max()), m
        # inverse step: F_j = sum_l Pbar_lm(cos th_j) g_l
        c = RNG.standard_normal(B - abs(m)) + 1j * RNG.standard_normal(B - abs(m))
        ref_i = P.T @ c
        got_i = S.dlt_inverse(c, B, m)
        assert np.abs(got_i - ref_i).max() <= 1e-13 * max(1.0, np.abs(ref_i).max()), m


@pytest.mark.parametrize("B", [4, 7])
def test_seminaive_transforms_match_quadrature_sums(B):
    """Whole transforms: seminaive forward = quadrature sum (Alg. 1) for arbitrary
    samples; seminaive inverse = synthesis sum (Alg. 2) for arbitrary coefficients."""
    s = RNG.standard_normal(D.num_samples(B)) + 1j * RNG.standard_normal(D.num_samples(B))
    c = RNG.standard_normal(D.num_coeffs(B)) + 1j * RNG.standard_normal(D.num_coeffs(B))
    f_ref = D.forward(s, B)
    f_got = S.forward(s, B)
    assert np.abs(f_got - f_ref).max() <= 1e-12 * np.abs(f_ref).max()
    s_ref = D.inverse(c, B)
    s_got = S.inverse(c, B)
    assert np.abs(s_got - s_ref).max() <= 1e-12 * np.abs(s_ref).max()


def test_seminaive_round_trip():
    B = 9
    c = RNG.standard_normal(D.num_coeffs(B)) + 1j * RNG.standard_normal(D.num_coeffs(B))
    assert np.abs(S.forward(S.inverse(c, B), B) - c).max() < 1e-12
