"""SGL basis functions evaluated point by point (oracle; test infrastructure only).

H_nlm(r, theta, phi) = N_nl R_nl(r) Y_lm(theta, phi)                  (Def. 1.2)
  N_nl = sqrt(2 (n-l-1)! / Gamma(n + 1/2)),
  R_nl(r) = L^{(l+1/2)}_{n-l-1}(r^2) r^l,
  Y_lm(theta, phi) = M_lm P_lm(cos theta) exp(i m phi),                 (Def. 2.1)
  M_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!),
  P_lm the associated Legendre function of the Rodrigues form (Def. 2.1), which
  carries the factor (-1)^m.

Legendre part: the three-term recurrence of Eq. legendre_recurrence,
  (l+1-m) P_{l+1,m} = (2l+1) t P_lm - (l+m) P_{l-1,m},
started from P_mm = (-1)^m (2m-1)!! (1-t^2)^{m/2} (from the Rodrigues form) and
P_{m-1,m} = 0.  To stay inside the FP64 range the recurrence is run on
Pbar_lm = M_lm P_lm, with its two coefficients multiplied by ratios of M_lm
taken from log-gamma values.  Negative orders follow from the Rodrigues form:
P_{l,-m} = (-1)^m (l-m)!/(l+m)! P_lm, hence Pbar_{l,-m} = (-1)^m Pbar_lm.

Radial part: generalized Laguerre recurrence of Eq. laguerre_recursion,
  (k+1) L_{k+1} = (2k + alpha + 1 - t) L_k - (k + alpha) L_{k-1},
  L_0 = 1, L_1 = 1 + alpha - t (explicit sum, Eq. associated_laguerre_explicit),
with alpha = l + 1/2, t = r^2, k = n - l - 1.  Values are carried with a
per-point power-of-ten exponent so that neither L_k nor r^l overflows; the
products with N_nl, r^l and the sample scale sigma_i are formed in log space.
"""

from __future__ import annotations

import math

import numpy as np

_LOG_4PI = math.log(4.0 * math.pi)


def _log_M(l: int, m: int) -> float:
    """ln M_lm, M_lm = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!), 0 <= m <= l."""
    return 0.5 * (math.log(2 * l + 1) - _LOG_4PI + math.lgamma(l - m + 1) - math.lgamma(l + m + 1))


def legendre_table(B: int, theta: np.ndarray) -> np.ndarray:
    """Pbar[m, l, j] = M_lm P_lm(cos theta_j) for 0 <= m <= l < B (0 for l < m).

    Shape (B, B, len(theta)), float64.
    """
    theta = np.asarray(theta, dtype=np.float64)
    t = np.cos(theta)
    log_st = np.log(np.sin(theta))
    out = np.zeros((B, B, theta.size), dtype=np.float64)
    with np.errstate(under="ignore"):
        for m in range(B):
            # ln|P_mm| = ln (2m-1)!! + m ln sin(theta);  (2m-1)!! = (2m)! / (2^m m!)
            log_dfact = math.lgamma(2 * m + 1) - m * math.log(2.0) - math.lgamma(m + 1)
            cur = (-1.0) ** m * np.exp(_log_M(m, m) + log_dfact + m * log_st)
            prev = np.zeros_like(cur)
            out[m, m] = cur
            for l in range(m, B - 1):
                # Eq. legendre_recurrence with P replaced by Pbar / M.
                c1 = (2 * l + 1) / (l + 1 - m) * math.exp(_log_M(l + 1, m) - _log_M(l, m))
                if l > m:
                    c2 = (l + m) / (l + 1 - m) * math.exp(_log_M(l + 1, m) - _log_M(l - 1, m))
                    nxt = c1 * t * cur - c2 * prev
                else:
                    nxt = c1 * t * cur
                prev, cur = cur, nxt
                out[m, l + 1] = cur
    return out


def legendre_signed(Pbar: np.ndarray, l: int, m: int) -> np.ndarray:
    """Pbar_{l,m} for any |m| <= l from the m >= 0 table: Pbar_{l,-m} = (-1)^m Pbar_{l,m}."""
    if m >= 0:
        return Pbar[m, l]
    return (-1.0) ** (-m) * Pbar[-m, l]


def radial_table(B: int, r: np.ndarray, log_scale=None) -> np.ndarray:
    """rho[n, l, i] = s_i * N_nl * R_nl(r_i) for 1 <= n <= B, 0 <= l < n.

    s_i = exp(log_scale[i]) (1 if log_scale is None).  With log_scale = ln sigma
    this is the radial factor that multiplies scaled samples; with None it is
    the plain normalized radial function.  Shape (B+1, B, len(r)); row n = 0
    and entries with l >= n are 0.
    """
    r = np.asarray(r, dtype=np.float64)
    t = r * r
    log_r = np.log(r)
    ls = np.zeros_like(r) if log_scale is None else np.asarray(log_scale, dtype=np.float64)
    out = np.zeros((B + 1, B, r.size), dtype=np.float64)
    big = 1e100
    with np.errstate(under="ignore", divide="ignore"):
        for l in range(B):
            alpha = l + 0.5
            Lm1 = np.zeros_like(t)          # L_{-1}
            L0 = np.ones_like(t)            # L_0
            expo = np.zeros_like(t)         # L_k = Lk * 10^expo
            for k in range(B - l):
                n = k + l + 1
                log_N = 0.5 * (math.log(2.0) + math.lgamma(k + 1) - math.lgamma(n + 0.5))
                mag = np.log(np.abs(L0)) + expo * math.log(10.0)
                val = np.sign(L0) * np.exp(ls + log_N + l * log_r + mag)
                out[n, l] = val
                if k + 1 < B - l:
                    # Eq. laguerre_recursion; k = 0 uses L_1 = 1 + alpha - t.
                    if k == 0:
                        L1 = (1.0 + alpha - t) * L0
                    else:
                        L1 = ((2 * k + alpha + 1 - t) * L0 - (k + alpha) * Lm1) / (k + 1)
                    Lm1, L0 = L0, L1
                    over = np.abs(L0) > big
                    if np.any(over):
                        Lm1 = np.where(over, Lm1 / big, Lm1)
                        L0 = np.where(over, L0 / big, L0)
                        expo = np.where(over, expo + 100.0, expo)
    return out


def sh(l: int, m: int, theta, phi, Pbar=None, B=None):
    """Y_lm(theta, phi) (Def. 2.1) at the given points (helper for tests).

    theta/phi broadcast together; Pbar is recomputed unless a table for the
    same theta is passed.
    """
    theta = np.asarray(theta, dtype=np.float64)
    if Pbar is None:
        Pbar = legendre_table(l + 1 if B is None else B, theta.ravel())
    p = legendre_signed(Pbar, l, m).reshape(theta.shape)
    return p * np.exp(1j * m * np.asarray(phi, dtype=np.float64))


def sgl_function(n: int, l: int, m: int, r, theta, phi) -> np.ndarray:
    """H_nlm(r, theta, phi) (Def. 1.2) at arbitrary points (no scaling)."""
    r = np.atleast_1d(np.asarray(r, dtype=np.float64))
    theta = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    phi = np.atleast_1d(np.asarray(phi, dtype=np.float64))
    rad = radial_table(n, r.ravel())[n, l].reshape(r.shape)
    ang = sh(l, m, theta, phi)
    return rad * ang
