"""Pins of the oracle's Alg. 1 depth mirror (CPU only).

The mirror (oracle/wn_oracle_alg1.inc) runs Alg. 1 (Sec. 4.1) with the
sub-segment bound of Sec. 4.2 in FP64 and reports the depth, split and leaf
counts of each (query, segment) pair.  It is pinned here by

  * exact rational arithmetic (tests/alg1_exact.py) on random small curves of
    degree 1-5, polynomial and rational: every output must agree wherever the
    exact margin of every tested node is clear of rounding;
  * closed forms: a circular arc seen from its centre (all sub-arcs have
    d1 + d2 = 2r, so the depth is fixed by B alone, App. A.1), and straight
    segments (B = chord length: no point off the segment ever recurses);
  * the distance bounds behind the termination argument of Sec. 4.2: a node
    whose end point is farther than B (b - a) from the query is a leaf, and a
    node that contains the parameter of a curve point within delta of the
    query is split whenever 2 delta <= (B - V)(b - a), V = max |gamma'|;
  * reversal of the segment, which maps dyadic nodes to dyadic nodes.
"""
from fractions import Fraction

import numpy as np
import pytest

from tests import alg1_exact

EPS = 1e-12
# a node whose exact |d1 + d2 - B (b - a)| is below this is "borderline":
# FP64 rounding of the same formula may decide it either way
BORDER_ABS = 1e-12
BORDER_REL = 1e-10


def _random_curve(rng, rational):
    n = int(rng.integers(1, 6))
    cps = [(Fraction(int(rng.integers(-64, 65)), 64), Fraction(int(rng.integers(-64, 65)), 64)) for _ in range(n + 1)]
    # distinct consecutive points (a zero-length control leg is allowed by the
    # method, but keeps B meaningful for these pins)
    for i in range(1, n + 1):
        if cps[i] == cps[i - 1]:
            cps[i] = (cps[i][0] + Fraction(1, 64), cps[i][1])
    ws = None
    if rational:
        ws = [Fraction(int(rng.choice([2, 3, 4, 5, 6, 8])), 4) for _ in range(n + 1)]
    return cps, ws


def _exact_point(cps, ws, t):
    w = [Fraction(1)] * len(cps) if ws is None else ws
    return alg1_exact._point(cps, w, Fraction(t))


def test_mirror_matches_exact_arithmetic(oracle_lib):
    rng = np.random.default_rng(20251025)
    compared = border = 0
    depths = []
    for case in range(240):
        cps, ws = _random_curve(rng, rational=bool(case % 2))
        t0 = Fraction(int(rng.integers(1, 1 << 12)), 1 << 12)
        px, py = _exact_point(cps, ws, t0)
        e = int(rng.integers(4, 26))
        off = (float(rng.uniform(-1, 1)) * 2.0 ** -e, float(rng.uniform(-1, 1)) * 2.0 ** -e)
        qx, qy = float(px) + off[0], float(py) + off[1]
        ex = alg1_exact.depth(cps, ws, (Fraction(qx), Fraction(qy)), Fraction(EPS))
        cp = np.array([[float(a), float(b)] for a, b in cps])
        w = None if ws is None else np.array([float(x) for x in ws])
        m = oracle_lib.alg1_segment(cp, w, qx, qy, eps=EPS)
        d, onb, sp, lf, mabs, mrel = ex
        if (mabs < BORDER_ABS or mrel < BORDER_REL) and not onb:
            border += 1
            continue
        compared += 1
        depths.append(d)
        assert bool(m["onb"][0]) == onb, (case, ex, m)
        if not onb:
            assert int(m["depth"][0]) == d, (case, ex, m)
            assert int(m["splits"][0]) == sp and int(m["leaves"][0]) == lf, (case, ex, m)
    assert compared >= 220 and border <= 20
    # the cases reach a range of depths, not only the root
    assert max(depths) >= 15 and np.mean(np.array(depths) == 0) < 0.5


def test_bound_matches_exact_formula(oracle_lib):
    rng = np.random.default_rng(5)
    for case in range(60):
        cps, ws = _random_curve(rng, rational=bool(case % 2))
        B2 = alg1_exact.bound_squared(cps, ws)
        cp = np.array([[float(a), float(b)] for a, b in cps])
        w = None if ws is None else np.array([float(x) for x in ws])
        B = oracle_lib.alg1_bound(cp, w)
        assert abs(B - float(B2) ** 0.5) <= 1e-14 * B


def _arc(phi):
    """Unit circular arc of angle 2 phi from (1, 0), rational quadratic."""
    cp = np.array([[1.0, 0.0], [1.0, np.tan(phi)], [np.cos(2 * phi), np.sin(2 * phi)]])
    return cp, np.array([1.0, np.cos(phi), 1.0])


@pytest.mark.parametrize("deg", [10, 30, 50, 60, 70, 80, 85])
def test_arc_centre_closed_form(oracle_lib, deg):
    phi = np.radians(deg)
    cp, w = _arc(phi)
    # App. A.1 on this arc: W/w = 1/cos(phi), control legs tan(phi), chord 2 sin(phi)
    b1 = 2.0 * max(np.tan(phi), 2 * np.sin(phi)) / np.cos(phi)
    b2 = 2.0 * np.tan(phi) / np.cos(phi) ** 2
    B = min(b1, b2)
    assert abs(oracle_lib.alg1_bound(cp, w) - B) <= 1e-13 * B
    # every sub-arc's end points lie on the circle: d1 + d2 = 2 at every node,
    # so the nodes of level k are leaves iff 2 > B 2^-k
    want = 0
    while not (2.0 > B * 2.0 ** -want):
        want += 1
    assert abs(np.log2(B / 2.0) - round(np.log2(B / 2.0))) > 1e-6  # not a tie
    r = oracle_lib.alg1_segment(cp, w, 0.0, 0.0, eps=EPS)
    assert int(r["depth"][0]) == want
    # a full binary tree down to level `want`
    assert int(r["splits"][0]) == 2 ** want - 1 and int(r["leaves"][0]) == 2 ** want


def test_straight_segments_never_recurse(oracle_lib):
    rng = np.random.default_rng(3)
    for _ in range(50):
        a, b = rng.uniform(-1, 1, 2), rng.uniform(-1, 1, 2)
        n = int(rng.integers(1, 6))
        # evenly spaced collinear control points: gamma is the uniform line, B = |b - a|
        cp = np.array([a + (b - a) * i / n for i in range(n + 1)])
        x = rng.uniform(-1.5, 1.5, 200)
        y = rng.uniform(-1.5, 1.5, 200)
        # off the segment by at least 1e-3 of its length
        t = np.clip(((x - a[0]) * (b - a)[0] + (y - a[1]) * (b - a)[1]) / np.dot(b - a, b - a), 0, 1)
        d = np.hypot(x - (a[0] + t * (b - a)[0]), y - (a[1] + t * (b - a)[1]))
        keep = d > 1e-3 * np.linalg.norm(b - a)
        r = oracle_lib.alg1_segment(cp, None, x[keep], y[keep], eps=EPS)
        assert np.all(r["depth"] == 0) and np.all(r["splits"] == 0)


def _cubic_speed_max(cp):
    """max |gamma'| over [0, 1] of a polynomial cubic: |gamma'|^2 is a quartic,
    its maximum sits at an end or at a real root of its derivative."""
    d = 3.0 * np.diff(cp, axis=0)  # gamma' = sum d_i B_i^2(t)
    # power basis of gamma'(t): d0 (1-t)^2 + 2 d1 t (1-t) + d2 t^2
    c0 = d[0]
    c1 = 2 * (d[1] - d[0])
    c2 = d[0] - 2 * d[1] + d[2]
    px = np.polynomial.Polynomial([c0[0], c1[0], c2[0]])
    py = np.polynomial.Polynomial([c0[1], c1[1], c2[1]])
    s2 = px * px + py * py
    ts = [0.0, 1.0] + [r.real for r in s2.deriv().roots() if abs(r.imag) < 1e-12 and 0 <= r.real <= 1]
    return max(np.sqrt(s2(t)) for t in ts)


def test_termination_distance_bounds(oracle_lib):
    """Hermite cubics of a star curve, queries offset from a curve point by
    delta along random directions: the depth obeys both bounds."""
    rng = np.random.default_rng(11)
    checked = 0
    for _ in range(40):
        th0 = rng.uniform(0, 2 * np.pi)
        dth = rng.uniform(0.05, 0.4)
        k = rng.integers(2, 6)
        amp = rng.uniform(0.05, 0.3)

        def c(t):
            r = 1 + amp * np.cos(k * t)
            return np.array([r * np.cos(t), r * np.sin(t)])

        def dc(t):
            r = 1 + amp * np.cos(k * t)
            dr = -amp * k * np.sin(k * t)
            return np.array([dr * np.cos(t) - r * np.sin(t), dr * np.sin(t) + r * np.cos(t)])

        p0, p3 = c(th0), c(th0 + dth)
        cp = np.array([p0, p0 + dth / 3 * dc(th0), p3 - dth / 3 * dc(th0 + dth), p3])
        B = oracle_lib.alg1_bound(cp, None)
        V = _cubic_speed_max(cp)
        assert V <= B * (1 + 1e-12)  # Lemma 1

        def g(t):
            tt = np.array([(1 - t) ** 3, 3 * t * (1 - t) ** 2, 3 * t ** 2 * (1 - t), t ** 3])
            return tt @ cp

        for _ in range(10):
            ts = rng.uniform(0.05, 0.95)
            delta = 10.0 ** rng.uniform(-9, -2)
            phi = rng.uniform(0, 2 * np.pi)
            q = g(ts) + delta * np.array([np.cos(phi), np.sin(phi)])
            # a lower bound of the query's distance to the segment: the least
            # distance over a grid zoomed in six times around its minimum, less
            # V times the final spacing (and the evaluation's rounding)
            lo_t, hi_t = 0.0, 1.0
            for _ in range(6):
                grid = np.linspace(lo_t, hi_t, 2001)
                pts = np.array([g(t) for t in grid])
                dd = np.hypot(pts[:, 0] - q[0], pts[:, 1] - q[1])
                i = int(np.argmin(dd))
                h = grid[1] - grid[0]
                lo_t, hi_t = max(grid[i] - h, 0.0), min(grid[i] + h, 1.0)
            dist = float(dd[i]) - V * h - 1e-15
            r = oracle_lib.alg1_segment(cp, None, q[0], q[1], eps=1e-15)
            d = int(r["depth"][0])
            # upper: at the first level k with B 2^-k < dist every node is a leaf
            kup = 0
            while not (B * 2.0 ** -kup < dist * (1 - 1e-6)):
                kup += 1
            assert d <= kup, (d, kup, B, dist)
            # lower: the nodes containing ts are split while 2 delta <= (B - V) 2^-k
            if B > V:
                klo = 0
                while 2 * delta * (1 + 1e-6) <= (B - V) * 2.0 ** -(klo + 1):
                    klo += 1
                if 2 * delta * (1 + 1e-6) <= (B - V):
                    assert d >= klo + 1, (d, klo, B, V, delta)
            checked += 1
    assert checked == 400


def test_reversal_invariance(oracle_lib):
    rng = np.random.default_rng(17)
    same = total = 0
    for case in range(200):
        n = int(rng.integers(1, 6))
        cp = rng.uniform(-1, 1, (n + 1, 2))
        w = rng.uniform(0.5, 2.0, n + 1) if case % 2 else None
        t = rng.uniform(0, 1)
        tt = np.array([[(1 - t) ** (n - i) * t ** i for i in range(n + 1)]])
        from math import comb

        bern = tt * np.array([comb(n, i) for i in range(n + 1)])
        ww = np.ones(n + 1) if w is None else w
        p = ((bern * ww) @ cp / float((bern * ww).sum())).ravel()
        q = p + 10.0 ** rng.uniform(-8, -2) * rng.standard_normal(2)
        a = oracle_lib.alg1_segment(cp, w, q[0], q[1], eps=EPS)
        b = oracle_lib.alg1_segment(cp[::-1].copy(), None if w is None else w[::-1].copy(), q[0], q[1], eps=EPS)
        if a["margin_rel"][0] < 1e-9 or b["margin_rel"][0] < 1e-9:
            continue
        total += 1
        same += int(a["depth"][0] == b["depth"][0] and a["splits"][0] == b["splits"][0] and
                    a["leaves"][0] == b["leaves"][0])
    assert total >= 180 and same == total


# Planted mistakes: each variant of the mirror below carries one plausible
# error (a dropped factor, a wrong index or operand, a shifted midpoint, an
# off-by-one level) and must fail the exact-arithmetic pin or a closed form.
MUTATIONS = {
    "bound without the degree factor": ("if (!cw) return n * maxd;", "if (!cw) return maxd;"),
    "rational bound with W/w not squared": ("b2 = n * r * r * maxd", "b2 = n * r * maxd"),
    "second distance to the wrong end": ("d2 = hypot(bx - c->x, by - c->y)", "d2 = hypot(ax - c->x, ay - c->y)"),
    "midpoint at a quarter": ("double t = 0.5 * (a + b)", "double t = a + 0.25 * (b - a)"),
    "children one level too deep": ("alg1_node(c, a, t, level + 1,", "alg1_node(c, a, t, level + 2,"),
    "axis of the whole segment at every level": ("double axis = c->B * (b - a);", "double axis = c->B;"),
}
# ... and in the control-point bound variant (checked against its own exact pin)
CP_MUTATIONS = {
    "control-point bound ignored": ("fmin(c->B * (b - a), bcp)", "c->B * (b - a)"),
    "halves swapped": ("alg1_node_cp(c, a, tm, level + 1, lx, ly, lw,", "alg1_node_cp(c, a, tm, level + 1, rx, ry, rw,"),
    "weights dropped from the piece bound": ("c->rational ? W : NULL", "NULL"),
    "apex not divided by its weight": ("mx = tx[0] / tw[0]", "mx = tx[0]"),
}


def _mutant_segment(lib, cp, w, x, y, eps, cp_bound=0):
    import ctypes

    cp = np.asarray(cp, dtype=np.float64)
    n = len(cp) - 1
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    y = np.atleast_1d(np.asarray(y, dtype=np.float64))
    sco = np.array([0, n + 1], dtype=np.int64)
    cu, cv = np.ascontiguousarray(cp[:, 0]), np.ascontiguousarray(cp[:, 1])
    cw = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    seg = np.zeros(len(x), dtype=np.int32)
    out = np.empty((len(x), 6))
    P = ctypes.c_void_p
    ptr = lambda a: None if a is None else a.ctypes.data_as(P)
    lib.wno_alg1_pairs(1, ptr(sco), ptr(cu), ptr(cv), ptr(cw), len(x), ptr(seg), ptr(x), ptr(y), ctypes.c_double(eps),
                       cp_bound, 1, ptr(out))
    return out


def _build_mutant(tmp_path, old, new):
    import ctypes
    import os
    import shutil
    import subprocess

    import oracle

    src = os.path.dirname(oracle.__file__)
    for f in ("wn_oracle.c", "wn_oracle_core.inc", "wn_oracle_periodic.inc", "wn_oracle_alg1.inc"):
        shutil.copy(os.path.join(src, f), tmp_path / f)
    text = (tmp_path / "wn_oracle_alg1.inc").read_text()
    assert text.count(old) == 1, old
    (tmp_path / "wn_oracle_alg1.inc").write_text(text.replace(old, new))
    so = tmp_path / "mutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", str(so), str(tmp_path / "wn_oracle.c"),
                    "-lpthread", "-lm"], check=True)
    lib = ctypes.CDLL(str(so))
    lib.wno_alg1_pairs.restype = ctypes.c_int
    return lib


@pytest.mark.parametrize("name", sorted(CP_MUTATIONS))
def test_planted_mistakes_fail_the_cp_pin(tmp_path, name):
    lib = _build_mutant(tmp_path, *CP_MUTATIONS[name])
    rng = np.random.default_rng(123)
    failed = False
    for case in range(60):
        if failed:
            break
        cps, ws = _random_curve(rng, rational=bool(case % 2))
        t0 = Fraction(int(rng.integers(1, 1 << 12)), 1 << 12)
        px, py = _exact_point(cps, ws, t0)
        e = int(rng.integers(4, 18))
        qx = float(px) + float(rng.uniform(-1, 1)) * 2.0 ** -e
        qy = float(py) + float(rng.uniform(-1, 1)) * 2.0 ** -e
        d, onb, sp, lf, mabs, mrel = alg1_exact.depth(cps, ws, (Fraction(qx), Fraction(qy)), Fraction(EPS),
                                                      cp_bound=True)
        if onb or mabs < BORDER_ABS or mrel < BORDER_REL:
            continue
        cp = np.array([[float(a), float(b)] for a, b in cps])
        w = None if ws is None else np.array([float(x) for x in ws])
        r = _mutant_segment(lib, cp, w, qx, qy, EPS, cp_bound=1)
        failed |= int(r[0, 0]) != d or int(r[0, 2]) != sp or int(r[0, 3]) != lf
    assert failed, f"planted mistake '{name}' passed the control-point pin"


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistakes_fail_the_pins(tmp_path, name):
    lib = _build_mutant(tmp_path, *MUTATIONS[name])
    failed = False
    # the arc closed forms
    for deg in (30, 60, 80):
        phi = np.radians(deg)
        cp, w = _arc(phi)
        b1 = 2.0 * max(np.tan(phi), 2 * np.sin(phi)) / np.cos(phi)
        b2 = 2.0 * np.tan(phi) / np.cos(phi) ** 2
        B = min(b1, b2)
        want = 0
        while not (2.0 > B * 2.0 ** -want):
            want += 1
        r = _mutant_segment(lib, cp, w, 0.0, 0.0, EPS)
        failed |= int(r[0, 0]) != want or int(r[0, 2]) != 2 ** want - 1
    # the exact-arithmetic pin on a few random curves
    rng = np.random.default_rng(99)
    for case in range(40):
        if failed:
            break
        cps, ws = _random_curve(rng, rational=bool(case % 2))
        t0 = Fraction(int(rng.integers(1, 1 << 12)), 1 << 12)
        px, py = _exact_point(cps, ws, t0)
        e = int(rng.integers(4, 20))
        qx = float(px) + float(rng.uniform(-1, 1)) * 2.0 ** -e
        qy = float(py) + float(rng.uniform(-1, 1)) * 2.0 ** -e
        d, onb, sp, lf, mabs, mrel = alg1_exact.depth(cps, ws, (Fraction(qx), Fraction(qy)), Fraction(EPS))
        if onb or mabs < BORDER_ABS or mrel < BORDER_REL:
            continue
        cp = np.array([[float(a), float(b)] for a, b in cps])
        w = None if ws is None else np.array([float(x) for x in ws])
        r = _mutant_segment(lib, cp, w, qx, qy, EPS)
        failed |= int(r[0, 0]) != d or int(r[0, 2]) != sp or int(r[0, 3]) != lf
    assert failed, f"planted mistake '{name}' passed the pins"


# --- the subdivided control-point bound variant (Sec. 4.2 / Table 1 contrast)

def test_cp_mirror_matches_exact_arithmetic(oracle_lib):
    """The FP64 mirror's control-point bound mode against exact rational
    arithmetic (exact halvings, exact squared bounds): every output agrees
    wherever every tested node's exact margin is clear of rounding."""
    rng = np.random.default_rng(20251103)
    compared = border = 0
    depths = []
    for case in range(160):
        cps, ws = _random_curve(rng, rational=bool(case % 2))
        t0 = Fraction(int(rng.integers(1, 1 << 12)), 1 << 12)
        px, py = _exact_point(cps, ws, t0)
        e = int(rng.integers(4, 22))
        off = (float(rng.uniform(-1, 1)) * 2.0 ** -e, float(rng.uniform(-1, 1)) * 2.0 ** -e)
        qx, qy = float(px) + off[0], float(py) + off[1]
        ex = alg1_exact.depth(cps, ws, (Fraction(qx), Fraction(qy)), Fraction(EPS), cp_bound=True)
        cp = np.array([[float(a), float(b)] for a, b in cps])
        w = None if ws is None else np.array([float(x) for x in ws])
        m = oracle_lib.alg1_segment(cp, w, qx, qy, eps=EPS, cp_bound=True)
        d, onb, sp, lf, mabs, mrel = ex
        if (mabs < BORDER_ABS or mrel < BORDER_REL) and not onb:
            border += 1
            continue
        compared += 1
        depths.append(d)
        assert bool(m["onb"][0]) == onb, (case, ex, m)
        if not onb:
            assert int(m["depth"][0]) == d, (case, ex, m)
            assert int(m["splits"][0]) == sp and int(m["leaves"][0]) == lf, (case, ex, m)
    assert compared >= 140 and border <= 20
    assert max(depths) >= 12


def test_cp_bound_prunes_a_subtree_of_the_global_tree():
    """Exact arithmetic: a node's control-point bound never exceeds B (b - a)
    for polynomial curves (the restricted hodograph's control points are
    convex combinations of the whole one's), and the variant takes the
    smaller of the two, so every node it tests is tested by the global-bound
    recursion too: depth, splits and leaves can only shrink, and they do on
    curved segments."""
    rng = np.random.default_rng(77)
    shrunk = 0
    for case in range(60):
        cps, ws = _random_curve(rng, rational=bool(case % 3 == 0))
        t0 = Fraction(int(rng.integers(1, 1 << 10)), 1 << 10)
        px, py = _exact_point(cps, ws, t0)
        q = (px + Fraction(int(rng.integers(-64, 65)), 1 << 14), py + Fraction(int(rng.integers(-64, 65)), 1 << 14))
        g = alg1_exact.depth(cps, ws, q, Fraction(1, 1 << 40))
        c = alg1_exact.depth(cps, ws, q, Fraction(1, 1 << 40), cp_bound=True)
        if g[1] or c[1]:
            continue
        assert c[0] <= g[0] and c[2] <= g[2] and c[3] <= g[3], (case, g, c)
        shrunk += c[2] < g[2]
        if ws is None:
            hom = [(x, y, Fraction(1)) for x, y in cps]
            B2 = alg1_exact.bound_squared(cps)
            for lvl in range(1, 5):
                hom = alg1_exact._halves(hom)[int(rng.integers(0, 2))]
                assert alg1_exact._piece_bound_squared(hom, False) <= B2 / Fraction(4) ** lvl
    assert shrunk >= 10


def test_cp_bound_on_straight_segments_changes_nothing(oracle_lib):
    """A straight segment's sub-pieces have control-point bound = their length
    = B (b - a): both modes give the same counts (closed form)."""
    rng = np.random.default_rng(5)
    for _ in range(20):
        a, b = rng.uniform(-1, 1, 2), rng.uniform(-1, 1, 2)
        n = int(rng.integers(1, 6))
        t = np.linspace(0, 1, n + 1)[:, None]
        cp = a + t * (b - a)  # evenly spaced: a degree-n parametrisation of the segment at constant speed
        q = a + rng.uniform(0.2, 0.8) * (b - a) + rng.normal(0, 1e-3, 2)
        g = oracle_lib.alg1_segment(cp, None, q[0], q[1], eps=EPS)
        c = oracle_lib.alg1_segment(cp, None, q[0], q[1], eps=EPS, cp_bound=True)
        for k in ("depth", "splits", "leaves"):
            assert int(g[k][0]) == int(c[k][0]), (k, g, c)
