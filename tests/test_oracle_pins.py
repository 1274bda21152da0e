"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms (Sec. 3.2 definition and its homotopy consequences), invariants
(additivity, orientation, translation, subdivision and degree elevation),
an independent integer method (crossing number of a dense polygon), adaptive
Gauss-Kronrod quadrature of the defining integral, and the oracle's own long
double twin on tiny inputs.  No GPU is involved.
"""
import json
import os

import numpy as np
import pytest

from paper_2510_25159_amd import workloads as W
from tests import curves as C

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _face(segs):
    """One face with one loop made of ``segs``."""
    return W.faces_from_loops([[segs]])


def _omega(oracle_lib, segs, pts, **kw):
    F = _face(segs)
    Q = W.queries_for_faces([np.asarray(pts, dtype=np.float64).reshape(-1, 2)])
    return oracle_lib.query_faces(F, Q, **kw)


# -- closed forms -------------------------------------------------------------
def test_line_segment_known_angle(oracle_lib):
    """A straight segment whose end points lie on a circle around x subtends
    exactly the difference of their polar angles (definition, Sec. 3.2)."""
    rng = np.random.default_rng(11)
    for _ in range(200):
        x = rng.uniform(-2, 2, 2)
        r1, r2 = rng.uniform(0.1, 3, 2)
        a = rng.uniform(-np.pi, np.pi)
        d = rng.uniform(-0.999 * np.pi, 0.999 * np.pi)
        A = x + r1 * np.array([np.cos(a), np.sin(a)])
        B = x + r2 * np.array([np.cos(a + d), np.sin(a + d)])
        for deg in (1, 3, 5):  # degree-elevated straight segments: same curve
            cp = A + np.linspace(0, 1, deg + 1)[:, None] * (B - A)
            w, near = oracle_lib.segment_winding(cp, None, x[0], x[1])
            assert near == 0
            assert abs(w - d / (2 * np.pi)) < 2e-15


def test_golden_cases(oracle_lib):
    """Hand-derived values (tests/golden/closed_forms.json)."""
    with open(os.path.join(GOLDEN, "closed_forms.json")) as fh:
        cases = json.load(fh)["cases"]
    for case in cases:
        segs = [(np.array(s["cp"], dtype=float), None if s.get("w") is None else np.array(s["w"], dtype=float))
                for s in case["segments"]]
        got, near = _omega(oracle_lib, segs, case["points"])
        want = np.array(case["omega"], dtype=float)
        assert np.all(near == 0), case["name"]
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-14, err_msg=case["name"])


def test_circle_inside_outside_and_arcs(oracle_lib):
    """Circle from four rational quadratic arcs: 1 inside, 0 outside; each
    arc equals its chord angle plus 1 inside its circular segment."""
    rng = np.random.default_rng(5)
    segs = C.circle_arcs(1.0)
    P = rng.uniform(-1.6, 1.6, size=(4000, 2))
    r = np.hypot(P[:, 0], P[:, 1])
    keep = np.abs(r - 1) > 1e-6
    P = P[keep]
    r = r[keep]
    got, near = _omega(oracle_lib, segs, P)
    assert np.all(near == 0)
    np.testing.assert_allclose(got, (r < 1).astype(float), rtol=0, atol=1e-13)
    # per arc closed form
    for cp, w in segs:
        A, B = cp[0], cp[2]
        for x in P[:500]:
            a, b = A - x, B - x
            chord = np.arctan2(a[0] * b[1] - a[1] * b[0], a @ b) / (2 * np.pi)
            in_seg = (np.hypot(*x) < 1) and ((B - A)[0] * (x - A)[1] - (B - A)[1] * (x - A)[0] < 0)
            val, near = oracle_lib.segment_winding(cp, w, x[0], x[1])
            assert abs(val - (chord + (1.0 if in_seg else 0.0))) < 1e-13


def test_circle_center_quarter(oracle_lib):
    for cp, w in C.circle_arcs(2.5, center=(0.3, -0.7)):
        val, near = oracle_lib.segment_winding(cp, w, 0.3, -0.7)
        assert abs(val - 0.25) < 1e-15


def test_reversed_loop_is_minus_one(oracle_lib):
    rng = np.random.default_rng(2)
    P = rng.uniform(-0.9, 0.9, size=(300, 2))
    P = P[np.hypot(P[:, 0], P[:, 1]) < 0.95]
    ccw, _ = _omega(oracle_lib, C.circle_arcs(1.0), P)
    cw, _ = _omega(oracle_lib, C.circle_arcs(1.0, cw=True), P)
    np.testing.assert_allclose(ccw, 1.0, atol=1e-13)
    np.testing.assert_allclose(cw, -1.0, atol=1e-13)


def test_holes_give_zero(oracle_lib):
    """CCW outer loop + CW hole: 1 in the material, 0 in the hole and outside (additivity)."""
    F = W.faces_from_loops([[C.circle_arcs(1.0), C.circle_arcs(0.3, center=(0.2, 0.1), cw=True)]])
    rng = np.random.default_rng(3)
    P = rng.uniform(-1.3, 1.3, size=(3000, 2))
    r_out = np.hypot(P[:, 0], P[:, 1])
    r_in = np.hypot(P[:, 0] - 0.2, P[:, 1] - 0.1)
    ok = (np.abs(r_out - 1) > 1e-6) & (np.abs(r_in - 0.3) > 1e-6)
    P = P[ok]
    want = ((r_out[ok] < 1) & (r_in[ok] > 0.3)).astype(float)
    Q = W.queries_for_faces([P])
    got, near = oracle_lib.query_faces(F, Q)
    np.testing.assert_allclose(got, want, atol=1e-13)


# -- invariants ----------------------------------------------------------------
def _c1_segments():
    f = W.config1_faces()
    segs = []
    for s in range(f.num_segments):
        a, b = f.seg_cp_offsets[s], f.seg_cp_offsets[s + 1]
        segs.append((np.column_stack([f.cp_u[a:b], f.cp_v[a:b]]), None))
    return segs


def test_split_and_elevation_invariance(oracle_lib):
    """Splitting segments at random parameters or elevating their degree does
    not change the curve, so omega is unchanged (additivity; Sec. 5 degree
    elevation experiment)."""
    rng = np.random.default_rng(7)
    segs = _c1_segments()
    split_segs, elev_segs = [], []
    for cp, w in segs:
        t = rng.uniform(0.1, 0.9)
        (l, wl), (r, wr) = C.split(cp, w, t)
        r[0] = l[-1]  # shared point, bit-for-bit
        split_segs += [(l, wl), (r, wr)]
        e, we = C.elevate(cp, w)
        e, we = C.elevate(e, we)
        e[0], e[-1] = cp[0], cp[-1]
        elev_segs.append((e, we))
    P = rng.uniform(-1.5, 1.5, size=(3000, 2))
    base, n0 = _omega(oracle_lib, segs, P)
    sp, n1 = _omega(oracle_lib, split_segs, P)
    el, n2 = _omega(oracle_lib, elev_segs, P)
    ok = (n0 == 0) & (n1 == 0) & (n2 == 0)
    assert ok.mean() > 0.99
    np.testing.assert_allclose(sp[ok], base[ok], atol=1e-14)
    np.testing.assert_allclose(el[ok], base[ok], atol=1e-14)


def test_rational_split_invariance(oracle_lib):
    rng = np.random.default_rng(8)
    faces, _ = W.config2(face_ids=[3])
    segs = []
    for s in range(faces.num_segments):
        a, b = faces.seg_cp_offsets[s], faces.seg_cp_offsets[s + 1]
        segs.append((np.column_stack([faces.cp_u[a:b], faces.cp_v[a:b]]), faces.cp_w[a:b].copy()))
    split_segs = []
    for cp, w in segs:
        (l, wl), (r, wr) = C.split(cp, w, rng.uniform(0.2, 0.8))
        r[0] = l[-1]
        split_segs += [(l, wl), (r, wr)]
    P = rng.uniform(-1.5, 1.5, size=(1500, 2))
    # evaluate loop by loop to keep the same face structure
    lo = faces.loop_seg_offsets
    base = np.zeros(len(P))
    spl = np.zeros(len(P))
    for l in range(faces.num_loops):
        b, n0 = _omega(oracle_lib, segs[lo[l]:lo[l + 1]], P)
        s, n1 = _omega(oracle_lib, split_segs[2 * lo[l]:2 * lo[l + 1]], P)
        base += b
        spl += s
    np.testing.assert_allclose(spl, base, atol=1e-13)


def test_translation_identity(oracle_lib):
    """omega(x, gamma + v) = omega(x - v, gamma) (App. C.1)."""
    rng = np.random.default_rng(9)
    segs = _c1_segments()
    v = np.array([3.25, -1.75])
    moved = [(cp + v, w) for cp, w in segs]
    P = rng.uniform(-1.5, 1.5, size=(2000, 2))
    a, _ = _omega(oracle_lib, moved, P)
    b, _ = _omega(oracle_lib, segs, P - v)
    np.testing.assert_allclose(a, b, atol=1e-14)


def test_closed_loop_integer_and_crossing_number(oracle_lib):
    """Away from the curve a closed loop has an integer winding number equal
    to the crossing number of a dense polygon sampled from the curve."""
    rng = np.random.default_rng(10)
    segs = _c1_segments()
    poly = C.dense_polyline(segs, m=300)
    P = rng.uniform(-1.5, 1.5, size=(3000, 2))
    d = C.polyline_distance(poly, P)
    P = P[d > 1e-3]
    got, near = _omega(oracle_lib, segs, P)
    assert np.all(near == 0)
    assert np.max(np.abs(got - np.round(got))) < 1e-12
    np.testing.assert_array_equal(np.round(got).astype(int), C.crossing_winding(poly, P))


# -- independent numerics ------------------------------------------------------
def test_quadrature_agrees(oracle_lib):
    """Adaptive Gauss-Kronrod quadrature of the defining integral."""
    rng = np.random.default_rng(12)
    faces, _ = W.config2(face_ids=[5])
    for s in rng.choice(faces.num_segments, 12, replace=False):
        a, b = faces.seg_cp_offsets[s], faces.seg_cp_offsets[s + 1]
        cp = np.column_stack([faces.cp_u[a:b], faces.cp_v[a:b]])
        w = faces.cp_w[a:b]
        for x in rng.uniform(-1.5, 1.5, size=(8, 2)):
            q, err = C.winding_quadrature(cp, w, x[0], x[1])
            o, near = oracle_lib.segment_winding(cp, w, x[0], x[1])
            assert near == 0
            assert abs(q - o) < max(1e-12, 10 * err)


def test_long_double_twin_agrees(oracle_lib):
    rng = np.random.default_rng(13)
    faces, q = W.config2(face_ids=[0, 1])
    idx = rng.choice(q.num_points, 400, replace=False)
    pf, u, v = W.subset_queries(q, idx)
    a, na = oracle_lib.query(faces, pf, u, v)
    b, nb = oracle_lib.query(faces, pf, u, v, long_double=True)
    ok = na == 0
    np.testing.assert_allclose(a[ok], b[ok], atol=1e-13)


# -- certified distance ---------------------------------------------------------
def test_near_flag_against_dense_distance(oracle_lib):
    rng = np.random.default_rng(14)
    segs = _c1_segments()
    # points placed at controlled distances along the normal of the curve
    pts, dist = [], []
    for k in range(200):
        cp, w = segs[rng.integers(len(segs))]
        t = rng.uniform(0.05, 0.95)
        p = C.eval_curve(cp, w, t)[0]
        d = C.eval_deriv(cp, w, t)[0]
        nrm = np.array([-d[1], d[0]]) / np.hypot(*d)
        h = 10.0 ** rng.uniform(-12, -6) * rng.choice([-1, 1])
        pts.append(p + h * nrm)
        dist.append(abs(h))
    pts = np.array(pts)
    dist = np.array(dist)
    _, near = _omega(oracle_lib, segs, pts, near_tol=1e-9)
    # normal offsets are (to first order) the distance: far from the threshold the flag is certain
    assert np.all(near[dist < 0.5e-9] == 1)
    assert np.all(near[dist > 2e-9] == 0)
