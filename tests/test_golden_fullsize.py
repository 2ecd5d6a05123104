"""CPU checks of the full-size oracle fixtures (tests/golden/fullsize_b<B>.npz):
they cover the edge coefficients and grid points they promise, and a few stored
values are reproduced by the oracle from the regenerated seeded inputs (so a
change of the generators or of the oracle shows here, not as a GPU failure)."""

import importlib.util
import os

import numpy as np
import pytest

from oracle import direct as D

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _maker():
    spec = importlib.util.spec_from_file_location("mkfix", os.path.join(GOLD, "make_fullsize_fixtures.py"))
    mk = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mk)
    return mk


@pytest.mark.parametrize("B", [128, 129, 150, 251, 256])
def test_fixture_covers_edges(B):
    mk = _maker()
    z = np.load(os.path.join(GOLD, f"fullsize_b{B}.npz"))
    assert int(z["B"]) == B
    oms, pts = z["omegas"], z["points"]
    n_rand = mk.CASES[B][2]
    assert len(oms) >= n_rand and len(pts) >= mk.CASES[B][3]
    assert set(mk.edge_omegas(B)) <= set(oms.tolist())
    for nlm in [(B, B - 1, -(B - 1)), (B, B - 1, B - 1), (B, B - 1, 0), (1, 0, 0)]:
        assert D.omega(*nlm) in set(oms.tolist())
    corners = {(i, j, k) for i in (0, 2 * B - 1) for j in (0, 2 * B - 1) for k in (0, 2 * B - 1)}
    assert corners <= {tuple(p) for p in pts.tolist()}
    assert np.all((oms >= 0) & (oms < D.num_coeffs(B)))
    assert np.all((pts >= 0) & (pts < 2 * B))
    assert np.isfinite(z["forward"]).all() and np.isfinite(z["inverse"]).all()
    assert len(z["forward"]) == len(oms) and len(z["inverse"]) == len(pts)


def test_fixture_values_reproduce_at_b128():
    """Three stored forward sums (the extreme order included) and three stored
    synthesis sums at B = 128 recomputed from the regenerated inputs."""
    B = 128
    mk = _maker()
    z = np.load(os.path.join(GOLD, f"fullsize_b{B}.npz"))
    s, c = mk.inputs(B)
    oms = z["omegas"]
    pick = [0, int(np.where(oms == D.omega(B, B - 1, B - 1))[0][0]), len(oms) // 2]
    f = D.forward(s.astype(np.complex128), B, omegas=oms[pick])
    assert np.abs(f - z["forward"][pick]).max() <= 1e-13 * np.abs(z["forward"]).max()
    pk = [0, len(z["points"]) - 1, len(z["points"]) // 3]
    v = D.inverse(c.astype(np.complex128), B, points=z["points"][pk])
    assert np.abs(v - z["inverse"][pk]).max() <= 1e-13 * np.abs(z["inverse"]).max()
