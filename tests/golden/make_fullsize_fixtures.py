"""Write the full-size oracle fixtures tests/golden/fullsize_b<B>.npz.

Calls only oracle/ (the direct quadrature and synthesis sums, Thm. 3.4 with
Alg. 1 / Alg. 2) and the seeded input generators of paper_1604_05140_amd/synth.py;
no GPU code is imported.  At these bandlimits the full direct transforms are out
of reach on a CPU, so each fixture holds, for one function of bandlimit B:

  forward:  seeded complex-normal samples on the whole grid (not bandlimited:
            the forward map is the quadrature sum for any samples), rounded to
            complex64 so that the reduced-precision forms read the same values;
            the oracle's quadrature sums at a seeded subset of coefficients plus
            edge coefficients (n = B, l = B - 1, |m| = B - 1; m = 0; n = l + 1;
            the lowest degrees);
  inverse:  seeded complex-normal coefficients times n^-decay, rounded to
            complex64; the oracle's synthesis sums at a seeded subset of grid
            points plus edge points (i, j, k in {0, 2B - 1} and mid-grid ones).

The samples and coefficients themselves are not stored (up to 2 GB): the tests
regenerate them from the stored seeds with the same generators.

Usage: python tests/golden/make_fullsize_fixtures.py [B ...]   (default: all)
"""

from __future__ import annotations

import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import direct as D  # noqa: E402
from paper_1604_05140_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
BASE = synth.BASE_SEED

# B: (seed base, coefficient decay, random coefficients, random points)
CASES = {
    128: (BASE + 3100, 1.0, 200, 200),
    256: (BASE + 5100, 1.5, 200, 200),
    # ring lengths 258..510 with odd factors (generic mixed-radix FFT path)
    129: (BASE + 6100, 1.0, 40, 40),   # 258 = 2 * 3 * 43
    150: (BASE + 6200, 1.0, 40, 40),   # 300 = 4 * 3 * 5 * 5
    251: (BASE + 6300, 1.0, 40, 40),   # 502 = 2 * 251
}


def edge_omegas(B: int) -> list[int]:
    h = B // 2
    nlm = [(1, 0, 0), (2, 1, -1), (2, 1, 0), (2, 1, 1), (B, 0, 0), (B, 1, -1), (B, 1, 1),
           (B, B - 1, -(B - 1)), (B, B - 1, 0), (B, B - 1, B - 1), (B, B - 1, 1), (B - 1, B - 2, B - 2),
           (h + 1, h, -h), (h + 1, h, 0), (h + 1, h, h), (B, h, -h), (B, h, 0)]
    return sorted({D.omega(n, l, m) for n, l, m in nlm})


def edge_points(B: int) -> np.ndarray:
    e = [0, 2 * B - 1]
    pts = [(i, j, k) for i in e for j in e for k in e]
    pts += [(0, 0, B), (2 * B - 1, 2 * B - 1, B - 1), (B, B, B), (0, B - 1, 0), (2 * B - 1, B, 2 * B - 1),
            (B - 1, 0, 1), (1, 2 * B - 1, B + 1)]
    return np.array(pts, dtype=np.int64)


def inputs(B: int):
    """The seeded inputs the fixture describes (also used by the tests)."""
    seed, decay, _, _ = CASES[B]
    s = synth.complex_normal_samples(B, 1, seed=seed)[0].astype(np.complex64)
    c = synth.complex_normal_coeffs(B, 1, seed=seed + 1, decay=decay)[0].astype(np.complex64)
    return s, c


_S = None
_C = None
_B = None


def _fwd(oms):
    return D.forward(_S, _B, omegas=oms)


def _inv(pts):
    return D.inverse(_C, _B, points=pts)


def make(B: int, workers: int = 4) -> str:
    global _S, _C, _B
    seed, decay, ncoef, npts = CASES[B]
    t0 = time.time()
    D.get_basis(B)  # grid and tables, inherited by the workers
    s, c = inputs(B)
    _S, _C, _B = s.astype(np.complex128), c.astype(np.complex128), B
    oms = np.union1d(synth.subset(ncoef, D.num_coeffs(B), seed=seed + 2), edge_omegas(B)).astype(np.int64)
    rnd = synth.grid_points(npts, B, seed=seed + 3)
    pts = np.unique(np.concatenate([rnd, edge_points(B)]), axis=0).astype(np.int64)
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        f_parts = pool.map(_fwd, np.array_split(oms, workers * 4))
        s_parts = pool.map(_inv, np.array_split(pts, workers * 4))
    fwd = np.concatenate(f_parts)
    inv = np.concatenate(s_parts)
    out = os.path.join(HERE, f"fullsize_b{B}.npz")
    np.savez(out, B=B, seed=seed, decay=decay, omegas=oms, forward=fwd, points=pts, inverse=inv,
             numpy_version=np.__version__)
    print(f"B={B}: {len(oms)} coefficients, {len(pts)} points, {time.time() - t0:.0f} s -> {out}", flush=True)
    return out


if __name__ == "__main__":
    Bs = [int(a) for a in sys.argv[1:]] or sorted(CASES)
    for B in Bs:
        make(B)
