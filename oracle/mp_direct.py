"""50-digit brute-force SGL transforms for tiny bandlimits (oracle; test infrastructure only).

Independent of the FP64 oracle's routes, used to pin it:
  * radial Gauss rule from its definition (Thm. 3.3): p_N is the monic
    orthogonal polynomial, written as the Hankel determinant
        p_N(x) = det[[mu_0 .. mu_N], ..., [mu_{N-1} .. mu_{2N-1}], [1, x, .., x^N]] / D_{N-1},
    its zeros are found by a polynomial root finder, and each weight is the
    integral of the Lagrange polynomial p_N(r) / ((r - r_i) p_N'(r_i)) against
    exp(-r^2), evaluated term by term with the moments (the formula of Thm. 3.3);
  * basis values from mpmath's own Laguerre and associated Legendre routines
    (the Legendre routine carries the Condon-Shortley factor (-1)^m, as the
    Rodrigues form of Def. 2.1 does);
  * the printed S^2 weight of Thm. 3.1 multiplied by pi/B (reading of Thm. 3.1);
  * Alg. 1 and Alg. 2 summed literally, with a~_i = a_i exp(r_i^2) r_i^2 and
    the basis weighted by exp(-r_i^2) as in Alg. 1.
Cost grows like B^7: meant for B <= 3.
"""

from __future__ import annotations

import mpmath as mp

DPS = 50


def _moments(n):
    return [mp.gamma(mp.mpf(k + 1) / 2) / 2 for k in range(n)]


def radial_rule(N: int):
    """(nodes, weights) of the N-point half-range Gauss-Hermite rule at DPS digits."""
    with mp.workdps(3 * DPS):
        mu = _moments(2 * N + 1)
        # coefficients of p_N(x) = sum_k c_k x^k by cofactor expansion along the last row
        H = mp.matrix(N, N)
        for a in range(N):
            for b in range(N):
                H[a, b] = mu[a + b]
        D = mp.det(H)
        coeffs = []
        for k in range(N + 1):
            M = mp.matrix(N, N)
            cols = [c for c in range(N + 1) if c != k]
            for a in range(N):
                for b, c in enumerate(cols):
                    M[a, b] = mu[a + c]
            coeffs.append((-1) ** (N + k) * mp.det(M) / D)
        # coeffs[k] multiplies x^k; coeffs[N] == 1
        roots = mp.polyroots(list(reversed(coeffs)), maxsteps=200, extraprec=4 * DPS)
        roots = sorted([mp.re(x) for x in roots])
        dcoef = [k * coeffs[k] for k in range(1, N + 1)]
        weights = []
        for x in roots:
            dp = sum(dcoef[k] * x ** k for k in range(N))
            # synthetic division p_N(r) / (r - x) = sum_k q_k r^k
            q = [mp.mpf(0)] * N
            carry = mp.mpf(0)
            for k in range(N, 0, -1):
                carry = coeffs[k] + carry * x
                q[k - 1] = carry
            weights.append(sum(q[k] * mu[k] for k in range(N)) / dp)
        return roots, weights


def _grid(B):
    r, a = radial_rule(2 * B)
    th = [(2 * j + 1) * mp.pi / (4 * B) for j in range(2 * B)]
    ph = [k * mp.pi / B for k in range(2 * B)]
    b = []
    for j in range(2 * B):
        s = mp.fsum(mp.sin((2 * j + 1) * (2 * l + 1) * mp.pi / (4 * B)) / (2 * l + 1) for l in range(B))
        b.append(mp.pi / B * mp.sin(th[j]) * 2 / B * s)
    return r, a, th, ph, b


def H(n, l, m, r, th, ph):
    """H_nlm (Def. 1.2) with mpmath's Laguerre and Legendre routines."""
    Nnl = mp.sqrt(2 * mp.factorial(n - l - 1) / mp.gamma(n + mp.mpf(1) / 2))
    R = mp.laguerre(n - l - 1, l + mp.mpf(1) / 2, r ** 2) * r ** l
    Mlm = mp.sqrt((2 * l + 1) / (4 * mp.pi) * mp.factorial(l - m) / mp.factorial(l + m))
    P = mp.legenp(l, m, mp.cos(th), type=2)
    return Nnl * R * Mlm * P * mp.expj(m * ph)


def nlm_list(B):
    return [(n, l, m) for n in range(1, B + 1) for l in range(n) for m in range(-l, l + 1)]


def forward_raw(f, B):
    """Alg. 1 on raw samples f[i][j][k] (nested lists of mpc/float)."""
    with mp.workdps(DPS):
        r, a, th, ph, b = _grid(B)
        at = [a[i] * mp.exp(r[i] ** 2) * r[i] ** 2 for i in range(2 * B)]
        out = []
        for (n, l, m) in nlm_list(B):
            acc = mp.mpc(0)
            for i in range(2 * B):
                for j in range(2 * B):
                    for k in range(2 * B):
                        acc += (at[i] * b[j] * f[i][j][k]) * (
                            mp.conj(H(n, l, m, r[i], th[j], ph[k])) * mp.exp(-r[i] ** 2))
            out.append(acc)
        return out


def inverse_raw(c, B):
    """Alg. 2: raw samples f[i][j][k] from coefficients c (omega order)."""
    with mp.workdps(DPS):
        r, a, th, ph, b = _grid(B)
        lst = nlm_list(B)
        f = [[[mp.mpc(0)] * (2 * B) for _ in range(2 * B)] for _ in range(2 * B)]
        for i in range(2 * B):
            for j in range(2 * B):
                for k in range(2 * B):
                    f[i][j][k] = mp.fsum(c[q] * H(n, l, m, r[i], th[j], ph[k])
                                         for q, (n, l, m) in enumerate(lst))
        return f


def sigma(B):
    """sigma_i = sqrt(a_i) r_i at DPS digits."""
    with mp.workdps(DPS):
        r, a = radial_rule(2 * B)
        return [mp.sqrt(a[i]) * r[i] for i in range(2 * B)]
