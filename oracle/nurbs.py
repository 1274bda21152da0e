"""NURBS curves for the tests (test infrastructure only): plain definitions.

``basis`` is the Cox-de Boor recursion for the B-spline basis functions of a
clamped knot vector; ``nurbs_point`` is the rational curve
C(t) = sum_i N_{i,p}(t) w_i P_i / sum_i N_{i,p}(t) w_i; ``bezier_point`` is the
rational Bernstein form of one segment.  Nothing here is shared with the HIP
library.
"""
from math import comb

import numpy as np


def basis(knots, p: int, t: float) -> np.ndarray:
    """N_{i,p}(t) for i = 0 .. len(knots) - p - 2 (half-open spans; at the
    clamped right end the last function is 1)."""
    U = np.asarray(knots, dtype=np.float64)
    n = len(U) - p - 1
    if t >= U[-1]:
        N = np.zeros(n)
        N[-1] = 1.0
        return N
    N = np.array([1.0 if U[i] <= t < U[i + 1] else 0.0 for i in range(len(U) - 1)])
    for d in range(1, p + 1):
        M = np.zeros(len(U) - 1 - d)
        for i in range(len(M)):
            a = 0.0 if U[i + d] == U[i] else (t - U[i]) / (U[i + d] - U[i]) * N[i]
            b = 0.0 if U[i + d + 1] == U[i + 1] else (U[i + d + 1] - t) / (U[i + d + 1] - U[i + 1]) * N[i + 1]
            M[i] = a + b
        N = M
    return N[:n]


def nurbs_point(knots, p: int, cp, w, t: float) -> np.ndarray:
    N = basis(knots, p, t)
    cp = np.asarray(cp, dtype=np.float64)
    ww = np.ones(len(cp)) if w is None else np.asarray(w, dtype=np.float64)
    den = np.sum(N * ww)
    return (N * ww) @ cp / den


def bezier_point(cp, w, t: float) -> np.ndarray:
    cp = np.asarray(cp, dtype=np.float64)
    n = len(cp) - 1
    ww = np.ones(n + 1) if w is None else np.asarray(w, dtype=np.float64)
    b = np.array([comb(n, k) * t ** k * (1.0 - t) ** (n - k) for k in range(n + 1)]) * ww
    return b @ cp / np.sum(b)
