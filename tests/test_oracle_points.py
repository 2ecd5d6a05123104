"""Pins of the oracle's off-grid routines (Sect. 5's Cartesian midpoint projection,
synthesis at arbitrary points): golden closed forms, the sampling-theorem
transform at grid points, and the midpoint rule's convergence."""

import numpy as np
import pytest

from closed_forms import DEGREE, load_closed_forms, poly
from oracle import direct as D, points as PT
from paper_1604_05140_amd import synth


def _closed(B, name, s=1.0):
    ref = np.zeros(D.num_coeffs(B), dtype=np.complex128)
    for (nm, n, l, m, v) in load_closed_forms():
        if nm == name:
            ref[D.omega(n, l, m)] = v * s ** (1.5 + DEGREE[name])
    return ref


@pytest.mark.parametrize("s", [1.0, 1.7])
def test_synthesis_of_closed_forms_is_the_polynomial(s):
    """sum fhat H^s at random points reproduces the polynomial whose exact
    coefficients are the golden closed forms."""
    B = 3
    xyz = np.random.default_rng(5).uniform(-3, 3, (200, 3))
    for name in DEGREE:
        got = PT.synthesize(_closed(B, name, s), B, xyz, radial_scale=s)
        ref = poly(name, xyz[:, 0], xyz[:, 1], xyz[:, 2])
        assert np.abs(got - ref).max() < 1e-12 * max(1.0, np.abs(ref).max()), name


def test_synthesis_matches_grid_synthesis():
    """At the sampling-theorem grid points, synthesis equals the direct inverse (raw)."""
    B = 4
    c = synth.complex_normal_coeffs(B, 1, seed=17)[0]
    xyz = D.sample_grid_points(B)
    assert np.allclose(PT.synthesize(c, B, xyz), D.inverse(c, B, raw=True), rtol=0, atol=1e-12)


@pytest.mark.parametrize("s", [1.0, 0.8])
def test_midpoint_converges_to_closed_forms(s):
    """For these Gaussian-weighted polynomials the midpoint rule converges fast as
    the cells shrink (and the cube grows past the Gaussian); fine grids reach the
    exact coefficients, coarse ones do not."""
    B = 3
    h = 7.0 * s
    errs = []
    for nx in (8, 16, 48):
        xyz = PT.cartesian_midpoints(nx, h)
        f = poly("r2", xyz[:, 0], xyz[:, 1], xyz[:, 2]) + 0.5 * poly("z", xyz[:, 0], xyz[:, 1], xyz[:, 2])
        ref = _closed(B, "r2", s) + 0.5 * _closed(B, "z", s)
        errs.append(np.abs(PT.midpoint_forward(f, B, nx, h, radial_scale=s) - ref).max())
    assert errs[2] < 1e-11
    assert errs[0] > 1e3 * errs[2]
