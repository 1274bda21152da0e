"""NURBS curves for the tests (test infrastructure only): plain definitions.

``basis`` is the Cox-de Boor recursion for the B-spline basis functions of a
clamped knot vector; ``nurbs_point`` is the rational curve
C(t) = sum_i N_{i,p}(t) w_i P_i / sum_i N_{i,p}(t) w_i; ``bezier_point`` is the
rational Bernstein form of one segment; ``spans_to_bezier`` gives each knot
span's Bezier form by interpolating the homogeneous curve (not by knot
insertion, which is the library's method).  Nothing here is shared with the
HIP library.
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


def homogeneous_point(knots, p: int, cp, w, t: float) -> np.ndarray:
    """(sum N_i w_i x_i, sum N_i w_i y_i, sum N_i w_i) at t."""
    N = basis(knots, p, t)
    cp = np.asarray(cp, dtype=np.float64)
    ww = np.ones(len(cp)) if w is None else np.asarray(w, dtype=np.float64)
    return np.array([np.sum(N * ww * cp[:, 0]), np.sum(N * ww * cp[:, 1]), np.sum(N * ww)])


def spans_to_bezier(knots, p: int, cp, w):
    """Each knot span of nonzero length as one rational Bezier segment, by
    interpolation: on a span the homogeneous curve is a polynomial of degree
    p, so its p + 1 Bernstein coefficients are fixed by its values at p + 1
    distinct parameters (Chebyshev nodes of the span, values by Cox-de Boor).
    Returns [(control points [(p+1), 2], weights [p+1] or None)]."""
    U = np.asarray(knots, dtype=np.float64)
    spans = [(U[k], U[k + 1]) for k in range(p, len(U) - p - 1) if U[k + 1] > U[k]]
    s = 0.5 - 0.5 * np.cos(np.pi * (np.arange(p + 1) + 0.5) / (p + 1))  # nodes in (0, 1)
    B = np.array([[comb(p, k) * x ** k * (1.0 - x) ** (p - k) for k in range(p + 1)] for x in s])
    out = []
    for a, b in spans:
        # the right end of the last span is closed: evaluate inside the span
        H = np.array([homogeneous_point(U, p, cp, w, a + (b - a) * x) for x in s])
        C = np.linalg.solve(B, H)  # Bernstein coefficients of (wx, wy, w)
        wts = C[:, 2]
        pts = C[:, :2] / wts[:, None]
        out.append((pts, None if w is None else wts))
    return out
