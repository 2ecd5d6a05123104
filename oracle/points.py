"""SGL expansions off the sampling grid (oracle; test infrastructure only).

synthesize(coeffs, B, xyz):     f(x_p) = sum_{n,l,m} fhat_nlm H_nlm(x_p) at arbitrary points.
midpoint_forward(values, ...):  the Cartesian midpoint-rule projection that Sect. 5 describes as
                                the field's practice: fhat_nlm ~ dV sum_c f(x_c) conj(H_nlm(x_c))
                                exp(-|x_c|^2) over the cells of a regular grid (the weight exp(-|x|^2)
                                is that of the SGL inner product, Def. 1.2 and
                                Eq. laguerre_ortho_transformed; the displayed sum in Sect. 5 writes
                                basis functions that carry the Gaussian themselves).

Grid convention: nx cells per axis on [-h, h]^3, cell side d = 2h/nx, midpoints
-h + (i + 1/2) d; values in the order (ix nx + iy) nx + iz.
radial_scale s: the radially scaled basis H^s_nlm(x) = s^(-3/2) H_nlm(x/s), weight
exp(-|x|^2/s^2) (see direct.forward).
"""

from __future__ import annotations

import numpy as np

from . import basis
from .direct import nlm_list, num_coeffs


def cartesian_midpoints(nx: int, h: float) -> np.ndarray:
    """(nx^3, 3) cell midpoints of the regular grid on [-h, h]^3, order (ix, iy, iz)."""
    d = 2.0 * h / nx
    c = -h + (np.arange(nx) + 0.5) * d
    x, y, z = np.meshgrid(c, c, c, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def _spherical(xyz: np.ndarray):
    x, y, z = xyz[:, 0], xyz[:, 1], xyz[:, 2]
    r = np.sqrt(x * x + y * y + z * z)
    theta = np.arccos(np.clip(np.where(r > 0, z / np.where(r > 0, r, 1.0), 1.0), -1.0, 1.0))
    phi = np.arctan2(y, x)
    return r, theta, phi


def _basis_columns(B: int, xyz: np.ndarray):
    """H_nlm at the points for every omega, as (Omega, npts) (Def. 1.2: N_nl R_nl(r) Y_lm)."""
    r, theta, phi = _spherical(xyz)
    P = basis.legendre_table(B, theta)    # [m, l, p]
    R = basis.radial_table(B, r)          # [n, l, p], N_nl R_nl(r)
    out = np.empty((num_coeffs(B), len(r)), dtype=np.complex128)
    for om, (n, l, m) in enumerate(nlm_list(B)):
        out[om] = R[n, l] * basis.legendre_signed(P, l, m) * np.exp(1j * m * phi)
    return out


def synthesize(coeffs, B: int, xyz, radial_scale: float = 1.0) -> np.ndarray:
    """f(x_p) = sum fhat_nlm H^s_nlm(x_p) at arbitrary points xyz (npts, 3)."""
    c = np.asarray(coeffs, dtype=np.complex128).reshape(-1)
    y = np.asarray(xyz, dtype=np.float64).reshape(-1, 3) / radial_scale
    return (radial_scale ** -1.5) * (c @ _basis_columns(B, y))


def midpoint_forward(values, B: int, nx: int, h: float, radial_scale: float = 1.0) -> np.ndarray:
    """Midpoint-rule coefficients dV sum_c f(x_c) conj(H^s_nlm(x_c)) exp(-|x_c|^2/s^2)."""
    f = np.asarray(values, dtype=np.complex128).reshape(-1)
    xyz = cartesian_midpoints(nx, h)
    if f.size != len(xyz):
        raise ValueError("expected nx^3 values")
    y = xyz / radial_scale
    w = np.exp(-np.sum(y * y, axis=1)) * (2.0 * h / nx) ** 3
    return (radial_scale ** -1.5) * (np.conj(_basis_columns(B, y)) @ (f * w))
