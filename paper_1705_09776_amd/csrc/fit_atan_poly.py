"""Fits the arctangent polynomial of describe.hip's angle_2pi().

atan(t) on [0, 1] is approximated by the odd polynomial t P(t^2), P of
degree 5 (6 coefficients, degree 11 in t), with the smallest largest
absolute error: Lawson's iteratively reweighted least squares (C. L. Lawson,
"Contributions to the theory of linear least maximum approximation", 1961)
on 4001 Chebyshev nodes of [0, 1], in float64, then rounded to float32.
Prints the coefficients from the highest power of t^2 down, the order in
which the kernel's Horner chain uses them.

    python paper_1705_09776_amd/csrc/fit_atan_poly.py
"""
from __future__ import annotations

import numpy as np

DEGREE = 5          # of P in s = t^2
NODES = 4001
ITERATIONS = 400


def fit() -> np.ndarray:
    """float32 coefficients c[0] (of s^DEGREE) .. c[DEGREE] (of s^0)."""
    k = np.arange(NODES)
    t = 0.5 - 0.5 * np.cos(np.pi * (k + 0.5) / NODES)      # Chebyshev nodes of [0, 1]
    A = t[:, None] * (t * t)[:, None] ** np.arange(DEGREE, -1, -1)[None, :]
    y = np.arctan(t)
    w = np.full(NODES, 1.0 / NODES)
    for _ in range(ITERATIONS):
        sw = np.sqrt(w)
        c, *_ = np.linalg.lstsq(A * sw[:, None], y * sw, rcond=None)
        e = np.abs(A @ c - y)
        w = w * e
        w /= w.sum()
    return c.astype(np.float32)


def max_error(c: np.ndarray, n: int = 200001) -> float:
    """Largest |t P(t^2) - atan t| on [0, 1] with the coefficients as given
    (evaluated in float64)."""
    t = np.linspace(0.0, 1.0, n)
    return float(np.abs(np.polyval(c.astype(np.float64), t * t) * t - np.arctan(t)).max())


if __name__ == "__main__":
    c = fit()
    print(f"max |error| {max_error(c):.3e}")
    print(f"float p = {float(c[0])!r}f;")
    for v in c[1:]:
        print(f"p = fmaf(p, s, {float(v)!r}f);")
