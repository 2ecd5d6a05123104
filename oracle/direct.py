"""Direct SGL transforms by quadrature (oracle; test infrastructure only).

Forward (naive DSGLFT, Alg. 1, from the SGL sampling theorem, Thm. 3.4):
    fhat_nlm = sum_{i,j,k < 2B} a_i r_i^2 b~_j f(r_i, th_j, ph_k) conj(H_nlm(r_i, th_j, ph_k))
Inverse (naive iDSGLFT, Alg. 2):
    f(r_i, th_j, ph_k) = sum_{n<=B, l<n, |m|<=l} fhat_nlm H_nlm(r_i, th_j, ph_k)

Coefficients are stored in the order omega(n,l,m) = n(n-1)(2n-1)/6 + l(l+1) + m
and samples in the order psi(i,j,k) = 4B^2 i + 2B j + k (Sect. 3.4).

Scaled samples (reading of Sect. 3.2 / Sect. 5 on the exp(r^2) compensation):
s_ijk = sigma_i f(r_i, th_j, ph_k) with sigma_i = sqrt(a_i) r_i.  Because
a_i r_i^2 = sigma_i^2, the forward sum becomes
    fhat_nlm = sum_{ijk} b~_j s_ijk conj(sigma_i H_nlm(r_i, th_j, ph_k)),
and the inverse produces s directly by synthesizing with sigma_i H_nlm.  In
exact arithmetic this is the same linear map; it keeps every value inside the
FP64 range for all bandlimits (raw samples grow like 10^B at the outer radii).

The sums below are written per coefficient (forward) or per sample point
(inverse) over the full grid or the full coefficient set: there is no
separation of variables, no FFT and no reuse between coefficients.
"""

from __future__ import annotations

import math

import numpy as np

from . import basis, quadrature


def num_coeffs(B: int) -> int:
    """Omega = B(B+1)(2B+1)/6 (Sect. 3.4)."""
    return B * (B + 1) * (2 * B + 1) // 6


def num_samples(B: int) -> int:
    """Psi = 8 B^3 (Sect. 3.4)."""
    return 8 * B ** 3


def omega(n: int, l: int, m: int) -> int:
    """omega(n,l,m) = n(n-1)(2n-1)/6 + l(l+1) + m (Sect. 3.4)."""
    return n * (n - 1) * (2 * n - 1) // 6 + l * (l + 1) + m


def nlm_list(B: int):
    """All (n, l, m) with |m| <= l < n <= B, in omega order."""
    out = []
    for n in range(1, B + 1):
        for l in range(n):
            for m in range(-l, l + 1):
                out.append((n, l, m))
    return out


class Basis:
    """Everything the direct sums need for bandlimit B, in FP64."""

    def __init__(self, B: int):
        g = quadrature.sgl_grid(B)
        self.B = B
        self.grid = g
        self.Pbar = basis.legendre_table(B, g["theta"])                    # [m][l][j]
        self.rho = basis.radial_table(B, g["r"], g["log_sigma"])           # [n][l][i]
        self.nlm = nlm_list(B)

    def scaled_function(self, n: int, l: int, m: int, i_slice=slice(None)) -> np.ndarray:
        """sigma_i H_nlm(r_i, th_j, ph_k) on the grid (rows i of i_slice), shape (ni, 2B, 2B)."""
        g = self.grid
        rad = self.rho[n, l, i_slice]
        pol = basis.legendre_signed(self.Pbar, l, m)
        az = np.exp(1j * m * g["phi"])
        return rad[:, None, None] * pol[None, :, None] * az[None, None, :]


_CACHE: dict = {}


def get_basis(B: int) -> Basis:
    if B not in _CACHE:
        _CACHE[B] = Basis(B)
    return _CACHE[B]


def _as_grid(samples: np.ndarray, B: int) -> np.ndarray:
    s = np.asarray(samples, dtype=np.complex128)
    if s.size != num_samples(B):
        raise ValueError("expected 8B^3 samples")
    return s.reshape(2 * B, 2 * B, 2 * B)


def forward(samples, B: int, omegas=None, raw: bool = False, i_chunk: int = 64,
            radial_scale: float = 1.0) -> np.ndarray:
    """Forward SGL transform by the quadrature sum of Thm. 3.4.

    samples: 8B^3 complex values in psi order; scaled (s = sigma f) unless raw.
    omegas:  optional list of coefficient indices; default all Omega.
    radial_scale: the radially scaled basis H^s_nlm(x) = s^(-3/2) H_nlm(x/s)
             (orthonormal on R^3 for every s > 0; the radially scaled SGL
             functions named in Sect. 5).  Its samples are taken at radii
             s r_i, and the change of variables x = s y turns the integral of
             f conj(H^s) into s^(3/2) times the unit-basis quadrature sum of the
             same sample values.
    Returns complex128 coefficients for the requested omegas.
    """
    bs = get_basis(B)
    s = _as_grid(samples, B)
    if raw:
        # a_i r_i^2 f = sigma_i^2 f = sigma_i (sigma_i f)
        s = s * bs.grid["sigma"][:, None, None]
    w = bs.grid["btilde"][None, :, None]
    idx = range(num_coeffs(B)) if omegas is None else omegas
    out = np.empty(len(idx), dtype=np.complex128)
    for q, om in enumerate(idx):
        n, l, m = bs.nlm[om]
        acc = 0.0 + 0.0j
        for i0 in range(0, 2 * B, i_chunk):
            sl = slice(i0, min(2 * B, i0 + i_chunk))
            h = bs.scaled_function(n, l, m, sl)
            acc += np.sum(w * s[sl] * np.conj(h))
        out[q] = acc
    if radial_scale != 1.0:
        out = out * radial_scale ** 1.5
    return out


def inverse(coeffs, B: int, points=None, raw: bool = False, radial_scale: float = 1.0) -> np.ndarray:
    """Inverse SGL transform by direct synthesis (Alg. 2).

    coeffs: Omega complex values in omega order.
    points: optional array of (i, j, k) triples; default the full grid.
    radial_scale: synthesis in the radially scaled basis H^s_nlm(x) =
             s^(-3/2) H_nlm(x/s) at the points (s r_i, th_j, ph_k): the unit
             synthesis times s^(-3/2).
    Returns scaled samples s = sigma f (raw f if raw) for the requested points,
    as a flat psi-ordered array for the full grid.
    """
    bs = get_basis(B)
    c = np.asarray(coeffs, dtype=np.complex128)
    if c.size != num_coeffs(B):
        raise ValueError("expected Omega coefficients")
    if radial_scale != 1.0:
        c = c * radial_scale ** -1.5
    g = bs.grid
    if points is None:
        out = np.zeros((2 * B, 2 * B, 2 * B), dtype=np.complex128)
        for om, (n, l, m) in enumerate(bs.nlm):
            if c[om] != 0:
                out += c[om] * bs.scaled_function(n, l, m)
        if raw:
            out = out / g["sigma"][:, None, None]
        return out.reshape(-1)
    pts = np.asarray(points, dtype=np.int64).reshape(-1, 3)
    n_arr = np.array([t[0] for t in bs.nlm])
    l_arr = np.array([t[1] for t in bs.nlm])
    m_arr = np.array([t[2] for t in bs.nlm])
    sign = np.where((m_arr < 0) & (np.abs(m_arr) % 2 == 1), -1.0, 1.0)
    out = np.empty(len(pts), dtype=np.complex128)
    for q, (i, j, k) in enumerate(pts):
        rad = bs.rho[n_arr, l_arr, i]
        pol = sign * bs.Pbar[np.abs(m_arr), l_arr, j]
        az = np.exp(1j * m_arr * g["phi"][k])
        v = np.sum(c * rad * pol * az)
        if raw:
            v = v / g["sigma"][i]
        out[q] = v
    return out


def error_metrics(ref: np.ndarray, got: np.ndarray) -> dict:
    """Error of got against ref (reading of Sect. 4's error measures).

    e_inf  = max |d| / max |ref|     (gate metric)
    e_2    = ||d||_2 / ||ref||_2
    paper  = max |d| / |ref|          (the paper's relative error, entries with ref != 0)
    abs    = max |d|                  (the paper's absolute error)
    """
    ref = np.asarray(ref).reshape(-1)
    got = np.asarray(got).reshape(-1)
    d = np.abs(got - ref)
    a = np.abs(ref)
    nz = a > 0
    return {
        "e_inf": float(d.max() / a.max()) if a.max() > 0 else float(d.max()),
        "e_2": float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300)),
        "paper": float((d[nz] / a[nz]).max()) if nz.any() else 0.0,
        "abs": float(d.max()),
    }


def sample_grid_points(B: int, radial_scale: float = 1.0):
    """Cartesian coordinates (x, y, z) of every grid point, psi order, shape (8B^3, 3)
    (radii s r_i for the radially scaled basis)."""
    g = quadrature.sgl_grid(B)
    r = radial_scale * g["r"][:, None, None]
    th = g["theta"][None, :, None]
    ph = g["phi"][None, None, :]
    x = r * np.sin(th) * np.cos(ph)
    y = r * np.sin(th) * np.sin(ph)
    z = r * np.cos(th) * np.ones_like(ph)
    return np.stack([x, y, z], axis=-1).reshape(-1, 3)


def scale_raw(values_raw: np.ndarray, B: int) -> np.ndarray:
    """Raw samples f (psi order) -> scaled samples sigma_i f."""
    sig = quadrature.sgl_grid(B)["sigma"]
    v = np.asarray(values_raw, dtype=np.complex128).reshape(2 * B, 4 * B * B)
    return (v * sig[:, None]).reshape(-1)


LOG_PI = math.log(math.pi)
