"""Exact SGL coefficients of low-degree polynomials (tests/golden/closed_form_transforms.txt)."""

import os

import mpmath as mp
import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

# polynomial degree of each closed-form function (all are homogeneous)
DEGREE = {"1": 0, "z": 1, "x+iy": 1, "x-iy": 1, "r2": 2}


def load_closed_forms():
    """Rows (function, n, l, m, value) of the golden file, values in 30-digit arithmetic."""
    rows = []
    with open(os.path.join(GOLDEN, "closed_form_transforms.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            name, n, l, m, expr = line.split(None, 4)
            with mp.workdps(30):
                val = float(eval(expr, {"__builtins__": {}}, {"pi": mp.pi, "sqrt": mp.sqrt}))
            rows.append((name, int(n), int(l), int(m), val))
    return rows


def poly(name, x, y, z):
    return {"1": np.ones_like(x), "z": z, "x+iy": x + 1j * y, "x-iy": x - 1j * y,
            "r2": x * x + y * y + z * z}[name]
