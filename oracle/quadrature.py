"""Quadrature rules of the SGL sampling theorem (oracle; test infrastructure only).

* Equiangular rule on the sphere, Thm. 3.1 (after Driscoll and Healy), order
  L = B: theta_j = (2j+1) pi / (4B), phi_k = k pi / B, j, k < 2B.
* Half-range Gauss-Hermite rule, Thm. 3.3, order N = 2B: Gauss rule for the
  weight exp(-r^2) on [0, inf).

Reading of Thm. 3.1 (weight constant): the printed b_j sum to 2, the integral of
sin(theta) over [0, pi]; the theorem's double sum over (j, k) also needs the
azimuthal step 2 pi / (2B).  The oracle therefore uses b~_j = (pi/B) b_j.  The
spherical Gram test and the closed-form transform pins fail without it.

Reading of Sect. 3.1 (how r_i and a_i are computed): the paper cites special
recurrences and a standard eigenvalue route without giving them.  The oracle
builds the unique N-point Gauss rule from its definition: the three-term
recurrence coefficients of the monic orthogonal polynomials of exp(-r^2) on
[0, inf) follow from the moments mu_k = Gamma((k+1)/2)/2 by the Chebyshev
algorithm in multiple precision; the nodes are the zeros of p_N (Newton on the
recurrence); the weights are the Christoffel numbers 1 / sum_k phat_k(r_i)^2,
which equal the weight formula of Thm. 3.3.
"""

from __future__ import annotations

import functools
import math

import mpmath as mp
import numpy as np


# --------------------------------------------------------------------------
# Sphere (Thm. 3.1)
# --------------------------------------------------------------------------

def polar_angles(B: int) -> np.ndarray:
    """theta_j = (2j+1) pi / (4B), j = 0..2B-1 (Thm. 3.1 with L = B)."""
    j = np.arange(2 * B, dtype=np.float64)
    return (2.0 * j + 1.0) * math.pi / (4.0 * B)


def azimuth_angles(B: int) -> np.ndarray:
    """phi_k = k pi / B, k = 0..2B-1 (Thm. 3.1 with L = B)."""
    return np.arange(2 * B, dtype=np.float64) * math.pi / B


@functools.lru_cache(maxsize=None)
def _polar_weights_mp(B: int):
    with mp.workdps(40):
        out = []
        for j in range(2 * B):
            s = mp.fsum(mp.sin((2 * j + 1) * (2 * l + 1) * mp.pi / (4 * B)) / (2 * l + 1)
                        for l in range(B))
            bj = mp.sin((2 * j + 1) * mp.pi / (4 * B)) * 2 / B * s
            out.append(bj)
        return tuple(out)


def polar_weights_printed(B: int) -> np.ndarray:
    """b_j exactly as printed in Thm. 3.1 (sums to 2 over j)."""
    return np.array([float(v) for v in _polar_weights_mp(B)], dtype=np.float64)


def polar_weights(B: int) -> np.ndarray:
    """b~_j = (pi/B) b_j: the S^2 weight that makes the double sum over (j, k)
    of Thm. 3.1 exact (reading of Thm. 3.1; pinned by the spherical Gram test)."""
    with mp.workdps(40):
        return np.array([float(mp.pi / B * v) for v in _polar_weights_mp(B)], dtype=np.float64)


# --------------------------------------------------------------------------
# Half line (Thm. 3.3)
# --------------------------------------------------------------------------

def _moment(k: int):
    """mu_k = int_0^inf r^k exp(-r^2) dr = Gamma((k+1)/2) / 2."""
    return mp.gamma(mp.mpf(k + 1) / 2) / 2


@functools.lru_cache(maxsize=None)
def recurrence_coefficients(N: int):
    """Monic recurrence p_{k+1} = (r - alpha_k) p_k - beta_k p_{k-1}, k < N, for
    the weight exp(-r^2) on [0, inf); beta_0 = mu_0.

    Chebyshev algorithm on the ordinary moments.  The moment map loses about
    1.15 N decimal digits, so the working precision is 1.25 N + 60 digits.
    Returns two tuples of mpf at that precision.
    """
    dps = int(1.25 * N) + 60
    with mp.workdps(dps):
        mu = [_moment(k) for k in range(2 * N)]
        alpha = [mp.mpf(0)] * N
        beta = [mp.mpf(0)] * N
        # sigma_{k,l} = int p_k(r) r^l w(r) dr, kept for rows k-1 and k.
        sig_prev = [mp.mpf(0)] * (2 * N)
        sig = list(mu)
        alpha[0] = mu[1] / mu[0]
        beta[0] = mu[0]
        for k in range(1, N):
            new = [mp.mpf(0)] * (2 * N)
            for l in range(k, 2 * N - k):
                new[l] = sig[l + 1] - alpha[k - 1] * sig[l] - beta[k - 1] * sig_prev[l]
            alpha[k] = new[k + 1] / new[k] - sig[k] / sig[k - 1]
            beta[k] = new[k] / sig[k - 1]
            sig_prev, sig = sig, new
        return tuple(alpha), tuple(beta)


class RadialRule:
    """N-point half-range Gauss-Hermite rule (Thm. 3.3) in FP64 plus logs.

    Attributes (numpy float64 arrays of length N, ascending nodes):
      r          nodes r_i
      log_a      ln a_i (a_i underflows FP64 for N >~ 280)
      a          a_i (0 where it underflows)
      log_atilde ln(a_i exp(r_i^2) r_i^2)    (modified weight of Sect. 3.2)
      atilde     a_i exp(r_i^2) r_i^2
      log_sigma  ln sigma_i, sigma_i = sqrt(a_i) r_i  (sample scaling)
      sigma      sigma_i
    and the same nodes/log-weights as mpf tuples (r_mp, log_a_mp) at 40 digits.
    """

    def __init__(self, N, r_mp, log_a_mp):
        self.N = N
        self.r_mp = r_mp
        self.log_a_mp = log_a_mp
        with mp.workdps(40):
            self.r = np.array([float(x) for x in r_mp])
            self.log_a = np.array([float(x) for x in log_a_mp])
            la = [x for x in log_a_mp]
            self.log_atilde = np.array([float(la[i] + r_mp[i] ** 2 + 2 * mp.log(r_mp[i]))
                                        for i in range(N)])
            self.log_sigma = np.array([float(la[i] / 2 + mp.log(r_mp[i])) for i in range(N)])
        self.a = np.exp(self.log_a)
        self.atilde = np.exp(self.log_atilde)
        self.sigma = np.exp(self.log_sigma)


@functools.lru_cache(maxsize=None)
def radial_rule(N: int) -> RadialRule:
    """Half-range Gauss-Hermite rule of order N (Thm. 3.3).

    Nodes: zeros of p_N.  FP64 eigenvalues of the Jacobi matrix serve only as
    starting points; each zero is then refined by Newton's method on p_N and
    p_N' evaluated with the three-term recurrence at 40 digits.  Weights:
    a_i = 1 / sum_{k<N} phat_k(r_i)^2 with phat_k the orthonormal polynomials
    (Christoffel numbers; equal to the weight formula of Thm. 3.3).
    """
    alpha_hp, beta_hp = recurrence_coefficients(N)
    with mp.workdps(40):
        alpha = [+a for a in alpha_hp]
        beta = [+b for b in beta_hp]
        # starting points from the FP64 Jacobi matrix
        d = np.array([float(a) for a in alpha])
        e = np.array([float(mp.sqrt(b)) for b in beta[1:]])
        J = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
        guess = np.sort(np.linalg.eigvalsh(J))

        def p_and_dp(x):
            p0, p1 = mp.mpf(0), mp.mpf(1)
            d0, d1 = mp.mpf(0), mp.mpf(0)
            for k in range(N):
                p2 = (x - alpha[k]) * p1 - (beta[k] * p0 if k > 0 else 0)
                d2 = p1 + (x - alpha[k]) * d1 - (beta[k] * d0 if k > 0 else 0)
                p0, p1 = p1, p2
                d0, d1 = d1, d2
            return p1, d1

        nodes = []
        for g in guess:
            x = mp.mpf(float(g))
            for _ in range(20):
                p, dp = p_and_dp(x)
                dx = p / dp
                x -= dx
                if abs(dx) <= mp.mpf(10) ** -34 * abs(x):
                    break
            nodes.append(x)
        for a_, b_ in zip(nodes, nodes[1:]):
            if not b_ > a_:
                raise ArithmeticError("half-range Gauss-Hermite: Newton merged two zeros")

        sqb = [mp.sqrt(b) for b in beta]
        log_a = []
        for x in nodes:
            ph0 = mp.mpf(0)
            ph1 = 1 / sqb[0]
            s = ph1 ** 2
            for k in range(N - 1):
                ph2 = ((x - alpha[k]) * ph1 - (sqb[k] * ph0 if k > 0 else 0)) / sqb[k + 1]
                ph0, ph1 = ph1, ph2
                s += ph1 ** 2
            log_a.append(-mp.log(s))
        return RadialRule(N, tuple(nodes), tuple(log_a))


@functools.lru_cache(maxsize=None)
def sgl_grid(B: int):
    """All FP64 grid data of the SGL sampling theorem (Thm. 3.4) for bandlimit B:
    radial rule of order 2B, polar angles/weights and azimuths of order B."""
    rr = radial_rule(2 * B)
    return {
        "B": B,
        "r": rr.r,
        "log_a": rr.log_a,
        "a": rr.a,
        "atilde": rr.atilde,
        "log_sigma": rr.log_sigma,
        "sigma": rr.sigma,
        "theta": polar_angles(B),
        "btilde": polar_weights(B),
        "phi": azimuth_angles(B),
    }
