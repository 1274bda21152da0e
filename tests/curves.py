"""Test-local curve helpers (independent of both the oracle and the HIP
library): exact constructions used to pin the oracle."""
from math import comb

import numpy as np

SQ2 = np.sqrt(0.5)


def circle_arcs(radius=1.0, center=(0.0, 0.0), cw=False):
    """Unit circle as 4 rational quadratic quarter arcs (weights 1, cos 45deg, 1)."""
    cx, cy = center
    pts = [(1, 0), (1, 1), (0, 1), (-1, 1), (-1, 0), (-1, -1), (0, -1), (1, -1), (1, 0)]
    segs = []
    for k in range(4):
        cp = np.array([pts[2 * k], pts[2 * k + 1], pts[2 * k + 2]], dtype=np.float64) * radius
        cp[:, 0] += cx
        cp[:, 1] += cy
        segs.append((cp, np.array([1.0, SQ2, 1.0])))
    if cw:
        segs = [(cp[::-1].copy(), w[::-1].copy()) for cp, w in reversed(segs)]
    return segs


def polygon(points):
    P = np.asarray(points, dtype=np.float64)
    return [(np.stack([P[i], P[(i + 1) % len(P)]]), None) for i in range(len(P))]


def eval_curve(cp, w, t):
    cp = np.asarray(cp, dtype=np.float64)
    n = len(cp) - 1
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))[:, None]
    j = np.arange(n + 1)
    b = np.array([comb(n, int(i)) for i in j]) * t ** j * (1 - t) ** (n - j)
    ww = np.ones(n + 1) if w is None else np.asarray(w)
    b = b * ww
    return (b @ cp) / b.sum(axis=1, keepdims=True)


def eval_deriv(cp, w, t):
    """Derivative of a rational Bezier curve via the quotient rule."""
    cp = np.asarray(cp, dtype=np.float64)
    n = len(cp) - 1
    ww = np.ones(n + 1) if w is None else np.asarray(w, dtype=np.float64)
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))[:, None]
    j = np.arange(n + 1)
    B = np.array([comb(n, int(i)) for i in j]) * t ** j * (1 - t) ** (n - j)
    # derivative of Bernstein basis
    jm = np.arange(n)
    Bm = np.array([comb(n - 1, int(i)) for i in jm]) * t ** jm * (1 - t) ** (n - 1 - jm)
    dB = np.zeros_like(B)
    dB[:, 1:] += n * Bm
    dB[:, :-1] -= n * Bm
    Wt = B @ ww
    dWt = dB @ ww
    Nt = (B * ww) @ cp
    dNt = (dB * ww) @ cp
    return (dNt * Wt[:, None] - Nt * dWt[:, None]) / (Wt[:, None] ** 2)


def split(cp, w, t):
    """de Casteljau split of a rational curve at parameter t (homogeneous)."""
    cp = np.asarray(cp, dtype=np.float64)
    ww = np.ones(len(cp)) if w is None else np.asarray(w, dtype=np.float64)
    H = np.column_stack([cp * ww[:, None], ww])
    n = len(cp) - 1
    left, right = [H[0]], [H[n]]
    cur = H.copy()
    for k in range(1, n + 1):
        cur = (1 - t) * cur[:-1] + t * cur[1:]
        left.append(cur[0])
        right.append(cur[-1])
    L = np.array(left)
    R = np.array(right[::-1])
    wl, wr = L[:, 2], R[:, 2]
    out_w = None if w is None else (wl, wr)
    return (L[:, :2] / wl[:, None], None if w is None else wl), (R[:, :2] / wr[:, None], None if w is None else wr)


def elevate(cp, w):
    """Degree elevation by one (same curve, one more control point)."""
    cp = np.asarray(cp, dtype=np.float64)
    n = len(cp) - 1
    ww = np.ones(n + 1) if w is None else np.asarray(w, dtype=np.float64)
    H = np.column_stack([cp * ww[:, None], ww])
    E = np.zeros((n + 2, 3))
    E[0], E[n + 1] = H[0], H[n]
    for i in range(1, n + 1):
        a = i / (n + 1)
        E[i] = a * H[i - 1] + (1 - a) * H[i]
    return E[:, :2] / E[:, 2:3], (None if w is None else E[:, 2])


def winding_quadrature(cp, w, x, y):
    """(1/2pi) * integral of (dx*y' - dy*x')/(dx^2+dy^2) dt by adaptive Gauss-Kronrod."""
    from scipy.integrate import quad

    def f(t):
        p = eval_curve(cp, w, t)[0]
        d = eval_deriv(cp, w, t)[0]
        dx, dy = p[0] - x, p[1] - y
        return (dx * d[1] - dy * d[0]) / (dx * dx + dy * dy)

    val, err = quad(f, 0.0, 1.0, epsabs=1e-15, epsrel=1e-14, limit=500)
    return val / (2 * np.pi), err / (2 * np.pi)


def dense_polyline(segs, m=4000):
    pts = [eval_curve(cp, w, np.linspace(0, 1, m, endpoint=False)) for cp, w in segs]
    return np.vstack(pts)


def crossing_winding(poly, pts):
    """Signed crossing number of a closed polygon (independent integer method)."""
    P = poly
    Q = np.roll(P, -1, axis=0)
    out = np.zeros(len(pts), dtype=np.int64)
    for k, (x, y) in enumerate(pts):
        up = (P[:, 1] <= y) & (Q[:, 1] > y)
        dn = (P[:, 1] > y) & (Q[:, 1] <= y)
        cr = (Q[:, 0] - P[:, 0]) * (y - P[:, 1]) - (x - P[:, 0]) * (Q[:, 1] - P[:, 1])
        out[k] = np.sum(up & (cr > 0)) - np.sum(dn & (cr < 0))
    return out


def polyline_distance(poly, pts):
    P = poly
    Q = np.roll(P, -1, axis=0)
    d = P - Q
    L2 = np.maximum((d * d).sum(1), 1e-300)
    out = np.empty(len(pts))
    for k, p in enumerate(pts):
        t = np.clip(((p - Q) * d).sum(1) / L2, 0, 1)
        c = Q + t[:, None] * d
        out[k] = np.sqrt(((c - p) ** 2).sum(1)).min()
    return out
