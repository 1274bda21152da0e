"""Alg. 1's depth in exact rational arithmetic (test-only brute force).

For a Bezier segment with rational control points and weights and a
rational query, every quantity Alg. 1 (Sec. 4.1, sub-segment bound of
Sec. 4.2) compares can be decided exactly:

  * curve points at dyadic parameters are rational (Bernstein sums);
  * the bound B (Lemma 1, App. A.1) is a square root of a rational: only B^2
    is formed, from the squared lengths, and the smaller of the two rational
    bounds is taken by comparing their squares;
  * the ellipse test sqrt(A) + sqrt(C) <= sqrt(G), with A, C the squared
    distances to the node's end points and G = B^2 4^-k, holds iff
    G - A - C >= 0 and 4 A C <= (G - A - C)^2 (squaring twice);
  * the eps test d < eps is A < eps^2;
  * with cp_bound, a node's own control points are exact halvings of its
    parent's (rational), so its control-point bound squared is rational too.

The nodes are enumerated level by level (breadth first), the reverse of the
recursion's order: a node of level k + 1 is tested iff its parent failed
its test.  The depth is the deepest tested level.
"""
from __future__ import annotations

from decimal import Decimal, getcontext
from fractions import Fraction
from math import comb


def _point(cps, ws, t):
    n = len(cps) - 1
    sx = sy = sw = Fraction(0)
    for i in range(n + 1):
        b = comb(n, i) * t ** i * (1 - t) ** (n - i) * ws[i]
        sx += b * cps[i][0]
        sy += b * cps[i][1]
        sw += b
    return (sx / sw, sy / sw)


def _d2(p, q):
    return (p[0] - q[0]) ** 2 + (p[1] - q[1]) ** 2


def bound_squared(cps, ws=None) -> Fraction:
    """B^2 of Lemma 1 (polynomial) or App. A.1 (rational: min of the two)."""
    n = len(cps) - 1
    maxd2 = max(_d2(cps[i], cps[i - 1]) for i in range(1, n + 1))
    if ws is None:
        return n * n * maxd2
    r = Fraction(max(ws)) / Fraction(min(ws))
    diam2 = max(_d2(cps[i], cps[j]) for i in range(n + 1) for j in range(i + 1, n + 1))
    b1 = n * n * r * r * diam2
    b2 = n * n * r ** 4 * maxd2
    return min(b1, b2)


def _sqrt(q: Fraction) -> Decimal:
    return (Decimal(q.numerator) / Decimal(q.denominator)).sqrt()


def _halves(hom):
    """De Casteljau at 1/2 of homogeneous control points [(wx, wy, w)]."""
    n = len(hom) - 1
    t = list(hom)
    left, right = [t[0]], [t[n]]
    for r in range(1, n + 1):
        t = [tuple((p + q) / 2 for p, q in zip(t[i], t[i + 1])) for i in range(n - r + 1)] + t[n - r + 1:]
        left.append(t[0])
        right.append(t[n - r])
    return left, right[::-1]


def _piece_bound_squared(hom, rational):
    cps = [(X / W, Y / W) for X, Y, W in hom]
    return bound_squared(cps, [W for _, _, W in hom] if rational else None)


def depth(cps, ws, x, eps, max_level=40, cp_bound=False):
    """Exact Alg. 1 on one pair.  cps: [(Fraction, Fraction)], ws: weights or
    None, x: query (Fraction, Fraction), eps: Fraction.  cp_bound: the axis
    of a node is the smaller of B (b - a) and the bound of the node's own
    control points (exact de Casteljau halving of its parent's).

    Returns (depth, on_boundary, splits, leaves, min_abs_margin,
    min_rel_margin): the smallest |d1 + d2 - axis| over the tested nodes,
    absolute and relative to the axis, evaluated to 50 digits."""
    getcontext().prec = 50
    cps = [(Fraction(a), Fraction(b)) for a, b in cps]
    ws_ = [Fraction(1)] * len(cps) if ws is None else [Fraction(w) for w in ws]
    x = (Fraction(x[0]), Fraction(x[1]))
    B2 = bound_squared(cps, None if ws is None else ws_)
    eps2 = Fraction(eps) ** 2
    root = [(w * px, w * py, w) for (px, py), w in zip(cps, ws_)]
    level_nodes = [(Fraction(0), Fraction(1), cps[0], cps[-1], root)]
    deepest, splits, leaves = 0, 0, 0
    min_rel = min_abs = Decimal("Infinity")
    for k in range(max_level + 1):
        if not level_nodes:
            break
        deepest = k
        G = B2 / Fraction(4) ** k
        nxt = []
        for a, b, pa, pb, hom in level_nodes:
            A, C = _d2(pa, x), _d2(pb, x)
            if A < eps2 or C < eps2:
                return deepest, True, splits, leaves, min_abs, min_rel
            Gn = min(G, _piece_bound_squared(hom, ws is not None)) if cp_bound else G
            axis = _sqrt(Gn)
            gap = abs(_sqrt(A) + _sqrt(C) - axis)
            min_abs = min(min_abs, gap)
            min_rel = min(min_rel, gap / axis)
            R = Gn - A - C
            inside = R >= 0 and 4 * A * C <= R * R
            if not inside:
                leaves += 1
                continue
            splits += 1
            m = (a + b) / 2
            pm = _point(cps, ws_, m)
            lh, rh = _halves(hom) if cp_bound else (None, None)
            nxt.append((a, m, pa, pm, lh))
            nxt.append((m, b, pm, pb, rh))
        level_nodes = nxt
    if level_nodes:
        raise RuntimeError("exact recursion passed max_level")
    return deepest, False, splits, leaves, min_abs, min_rel
