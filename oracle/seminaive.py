"""The seminaive Legendre step in the cosine domain (oracle; test infrastructure only).

Sect. 3.3.1 (the seminaive algorithm): for one order m the discrete Legendre
transform of Eq. DLT,  g_l = sum_j b~_j Pbar_lm(cos th_j) t_j  for |m| <= l < B,
is evaluated after a DCT.  C_N is the orthonormal DCT matrix of Eq. DCT; with
N = 2B its angles (2j+1) pi / 2N are the polar nodes th_j.  Two facts carry the
method: C_N is orthogonal, so <u, v> = <C u, C v> (Eq. dct_trick); and C_N
applied to a trigonometric polynomial of degree d on these nodes vanishes
beyond index d.

Pbar_lm(cos th) is a trigonometric polynomial of degree l when m is even.  When
m is odd it is sin th times a cosine polynomial of degree l - 1; the sin th
factor then moves to the data side (this is how the odd orders are "treated
similarly" here).  With par = |m| mod 2,
    q_lm(th) = Pbar_lm(cos th) / sin^par th,      u_j = b~_j t_j sin^par th_j,
    g_l = sum_{k <= l - par} [C q_lm]_k [C u]_k .
The inverse step is the transpose (end of Sect. 3.3.1, C^T = C^-1):
    F_j = sin^par th_j sum_k C[k, j] V_k,   V_k = sum_{l >= k + par} [C q_lm]_k g_l .

forward / inverse below are whole transforms with this step in place of the
direct Legendre sum, in the paper's separation-of-variables order (Eq.
SFFT_rearranged with the radial sums of Sect. 3.3.2): an FFT over phi (numpy),
the seminaive step over theta, then the radial products with the table
rho_nl(r_i) = sigma_i N_nl R_nl(r_i).  They are pinned against the quadrature
sums of direct.py, which share no step with them beyond the basis tables.
"""

from __future__ import annotations

import numpy as np

from . import basis, quadrature
from .direct import nlm_list, num_coeffs, omega


def dct_matrix(N: int) -> np.ndarray:
    """C_N of Eq. DCT: C[k, j] = s_k cos(k (2j+1) pi / 2N), s_0 = sqrt(1/N), s_k = sqrt(2/N)."""
    k = np.arange(N)[:, None]
    j = np.arange(N)[None, :]
    s = np.full((N, 1), np.sqrt(2.0 / N))
    s[0, 0] = np.sqrt(1.0 / N)
    return s * np.cos(k * (2 * j + 1) * np.pi / (2 * N))


def parity(m: int) -> int:
    return abs(m) % 2


class Tables:
    """Grid, Pbar, the cosine-domain Legendre vectors and rho for bandlimit B (FP64)."""

    def __init__(self, B: int):
        g = quadrature.sgl_grid(B)
        self.B = B
        self.grid = g
        th = g["theta"]
        self.sin = np.sin(th)
        self.C = dct_matrix(2 * B)
        self.Pbar = basis.legendre_table(B, th)                      # [m][l][j]
        self.rho = basis.radial_table(B, g["r"], g["log_sigma"])     # [n][l][i]
        # Cq[m][l] = C_{2B} (Pbar_lm / sin^par) for m >= 0 (rows l < m are zero)
        self.Cq = np.zeros((B, B, 2 * B))
        for m in range(B):
            q = self.Pbar[m] / self.sin[None, :] ** parity(m)
            self.Cq[m] = q @ self.C.T

    def cq(self, l: int, m: int) -> np.ndarray:
        """[C q_lm]_k for any |m| <= l (q_{l,-m} = (-1)^m q_lm, like Pbar)."""
        v = self.Cq[abs(m), l]
        return v if m >= 0 or abs(m) % 2 == 0 else -v


_CACHE: dict = {}


def get_tables(B: int) -> Tables:
    if B not in _CACHE:
        _CACHE[B] = Tables(B)
    return _CACHE[B]


def dlt_forward(t, B: int, m: int) -> np.ndarray:
    """g_l = sum_j b~_j Pbar_lm(cos th_j) t_j for l = |m|..B-1, by the cosine-domain sum."""
    T = get_tables(B)
    par = parity(m)
    u = T.grid["btilde"] * np.asarray(t) * T.sin ** par
    U = T.C @ u
    out = np.zeros(B - abs(m), dtype=np.result_type(U, np.float64))
    for l in range(abs(m), B):
        d = l - par  # highest nonzero cosine index of q_lm
        out[l - abs(m)] = np.dot(T.cq(l, m)[:d + 1], U[:d + 1])
    return out


def dlt_inverse(g, B: int, m: int) -> np.ndarray:
    """F_j = sum_l Pbar_lm(cos th_j) g_l (l = |m|..B-1) through the cosine domain."""
    T = get_tables(B)
    par = parity(m)
    g = np.asarray(g)
    V = np.zeros(2 * B, dtype=np.result_type(g, np.float64))
    for l in range(abs(m), B):
        d = l - par
        V[:d + 1] += T.cq(l, m)[:d + 1] * g[l - abs(m)]
    return T.sin ** par * (T.C.T @ V)


def forward(samples, B: int) -> np.ndarray:
    """Scaled samples s (psi order) -> coefficients (omega order), seminaive Legendre step."""
    T = get_tables(B)
    L = 2 * B
    s = np.asarray(samples, dtype=np.complex128).reshape(L, L, L)
    # azimuthal sums F[i, j, m] = sum_k s_ijk exp(-i m ph_k)  (ph_k = k pi / B)
    F = np.fft.fft(s, axis=2)
    out = np.zeros(num_coeffs(B), dtype=np.complex128)
    for m in range(1 - B, B):
        g = np.array([dlt_forward(F[i, :, m % L], B, m) for i in range(L)])  # [i][l - |m|]
        for l in range(abs(m), B):
            for n in range(l + 1, B + 1):
                out[omega(n, l, m)] = np.dot(T.rho[n, l], g[:, l - abs(m)])
    return out


def inverse(coeffs, B: int) -> np.ndarray:
    """Coefficients (omega order) -> scaled samples s (psi order), seminaive Legendre step."""
    T = get_tables(B)
    L = 2 * B
    c = np.asarray(coeffs, dtype=np.complex128).reshape(-1)
    F = np.zeros((L, L, L), dtype=np.complex128)  # [i][j][m mod L]
    for m in range(1 - B, B):
        g = np.zeros((L, B - abs(m)), dtype=np.complex128)
        for l in range(abs(m), B):
            for n in range(l + 1, B + 1):
                g[:, l - abs(m)] += T.rho[n, l] * c[omega(n, l, m)]
        for i in range(L):
            F[i, :, m % L] = dlt_inverse(g[i], B, m)
    # s_ijk = sum_m F[i, j, m] exp(+i m ph_k)
    return (np.fft.ifft(F, axis=2) * L).reshape(-1)


__all__ = ["dct_matrix", "parity", "Tables", "get_tables", "dlt_forward", "dlt_inverse", "forward", "inverse",
           "nlm_list"]
