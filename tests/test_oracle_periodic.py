"""Pins of the oracle's periodic formulation (Sec. 4.3-4.5): closed-form
straight bands on a cylinder and on a torus, lattice translation of the
query, re-cutting the loops at a different seam, window widening, the
pairing negative control (improper pairing gives omega = 2 regions) and the
unlifted negative control; topology errors of the Proposition of Sec. 4.5."""
import numpy as np
import pytest

from paper_2510_25159_amd import workloads as W

T = 2 * np.pi


def _face(curves_and_segs, domain, axes=None):
    axes = axes or ((0,) if domain == W.DOMAIN_CYLINDER_U else (0, 1))
    loops = []
    for cv, nseg in curves_and_segs:
        lp = W.periodic_loop(cv, nseg, (T, T), axes)
        loops.append([(cp, None) for cp in lp.cps])
    return W.faces_from_loops([loops], domains=[domain], periods=[[T, T]])


def _eval(oracle_lib, faces, P):
    q = W.queries_for_faces([np.asarray(P)])
    return oracle_lib.query_faces(faces, q)


def test_cylinder_straight_band_closed_form(oracle_lib):
    rng = np.random.default_rng(0)
    for _ in range(5):
        c1, c2 = np.sort(rng.uniform(-3, 3, 2))
        lo = W.WrappedCurve((rng.uniform(0, T), c1), (T, 0), 0.0, rng)
        hi = W.WrappedCurve((rng.uniform(0, T), c2), (-T, 0), 0.0, rng)
        f = _face([(lo, int(rng.integers(3, 9))), (hi, int(rng.integers(3, 9)))], W.DOMAIN_CYLINDER_U)
        P = np.column_stack([rng.uniform(-T, 2 * T, 2000), rng.uniform(-3.2, 3.2, 2000)])
        P = P[(np.abs(P[:, 1] - c1) > 1e-6) & (np.abs(P[:, 1] - c2) > 1e-6)]
        w, near = _eval(oracle_lib, f, P)
        assert np.all(near == 0)
        want = ((P[:, 1] > c1) & (P[:, 1] < c2)).astype(float)
        np.testing.assert_allclose(w, want, atol=1e-12)


@pytest.mark.parametrize("h", [(1, 0), (0, 1), (1, 1), (2, 3), (5, 2), (3, -4)])
def test_torus_straight_band_closed_form(oracle_lib, h):
    rng = np.random.default_rng(sum(h) + 7)
    vec = np.array([h[0] * T, h[1] * T])
    L = np.hypot(*vec)
    delta = T * T / L
    nrm = np.array([-vec[1], vec[0]]) / L
    width = rng.uniform(0.2, 0.8) * delta
    s0 = rng.uniform(0, T, 2)
    a = W.WrappedCurve(s0, vec, 0.0, rng)
    b = W.WrappedCurve(s0 + width * nrm + rng.uniform(0, 1) * vec, -vec, 0.0, rng)
    f = _face([(a, 7), (b, 5)], W.DOMAIN_TORUS)
    P = rng.uniform(-T, 2 * T, (3000, 2))
    fr = np.mod((P - s0) @ nrm / delta, 1.0)
    ok = (np.abs(fr) > 1e-7) & (np.abs(fr - 1) > 1e-7) & (np.abs(fr - width / delta) > 1e-7)
    P, fr = P[ok], fr[ok]
    w, near = _eval(oracle_lib, f, P)
    want = (fr < width / delta).astype(float)
    np.testing.assert_allclose(w, want, atol=1e-12)


@pytest.mark.parametrize("h", [(1, 0), (2, 3), (1, -2)])
def test_torus_two_straight_bands_closed_form(oracle_lib, h):
    """Two pairs of (h, -h) loops on one torus: each alpha pairs with the
    nearest beta on its left (App. C.2), so omega is 1 inside either band and 0
    in the two gaps, whatever order the loops come in."""
    rng = np.random.default_rng(h[0] * 7 + h[1] + 50)
    vec = np.array([h[0] * T, h[1] * T])
    L = np.hypot(*vec)
    delta = T * T / L
    nrm = np.array([-vec[1], vec[0]]) / L
    s0 = rng.uniform(0, T, 2)
    # bands [0, 0.2) and [0.45, 0.8) of the family spacing, measured from alpha 1
    edges = np.array([0.0, 0.2, 0.45, 0.8]) * delta
    curves = []
    for k, (e, d) in enumerate(zip(edges, (vec, -vec, vec, -vec))):
        curves.append((W.WrappedCurve(s0 + e * nrm + rng.uniform(0, 1) * vec, d, 0.0, rng), 4 + k))
    for order in ([0, 1, 2, 3], [0, 3, 2, 1], [2, 1, 0, 3]):
        f = _face([curves[i] for i in order], W.DOMAIN_TORUS)
        P = rng.uniform(-T, 2 * T, (3000, 2))
        fr = np.mod((P - s0) @ nrm / delta, 1.0)
        ok = np.all(np.abs(fr[:, None] - np.array([0.0, 0.2, 0.45, 0.8, 1.0])[None, :]) > 1e-7, axis=1)
        P, fr = P[ok], fr[ok]
        w, near = _eval(oracle_lib, f, P)
        want = ((fr < 0.2) | ((fr > 0.45) & (fr < 0.8))).astype(float)
        np.testing.assert_allclose(w, want, atol=1e-12)


def test_lattice_translation_and_window_invariance(oracle_lib):
    """Closed loops: omega is lattice periodic.  Open loops (chained by their
    own end-to-start vector, App. C) keep the window invariance exactly.
    Control-point noise opens every joint, so a far copy is then no longer
    exactly its chord and the truncated sum of Sec. 4.4 depends on N at the
    1e-6 level: the windows are part of the definition there."""
    faces, q = W.config3(face_ids=range(6), sigma=0.0, open_frac=0.0)
    w0, n0 = oracle_lib.query_faces(faces, q)
    qs = W.Queries(u=q.u + T, v=q.v.copy(), face_point_offsets=q.face_point_offsets)
    w1, _ = oracle_lib.query_faces(faces, qs)
    np.testing.assert_allclose(w1, w0, atol=1e-11)
    tor = np.repeat(faces.face_domain == W.DOMAIN_TORUS, np.diff(q.face_point_offsets))
    qv = W.Queries(u=q.u.copy(), v=q.v - 2 * T, face_point_offsets=q.face_point_offsets)
    w2, _ = oracle_lib.query_faces(faces, qv)
    np.testing.assert_allclose(w2[tor], w0[tor], atol=1e-11)
    noisy, qn = W.config3(face_ids=range(6), sigma=0.0)  # 20 % open loops, no joint noise
    wn0, _ = oracle_lib.query_faces(noisy, qn)
    oracle_lib.set_periodic_options(extra=3)
    try:
        w3, _ = oracle_lib.query_faces(faces, q)
        wn3, _ = oracle_lib.query_faces(noisy, qn)
    finally:
        oracle_lib.set_periodic_options()
    np.testing.assert_allclose(w3, w0, atol=1e-11)
    np.testing.assert_allclose(wn3, wn0, atol=1e-11)


def test_recut_at_other_seam(oracle_lib):
    """The same loops on the surface, cut at another seam (shifted cell):
    omega(x + delta) is unchanged."""
    rng = np.random.default_rng(5)
    delta = np.array([1.234, -0.77])
    vec = np.array([2 * T, 3 * T])
    L = np.hypot(*vec)
    dl = T * T / L
    nrm = np.array([-vec[1], vec[0]]) / L
    s0 = np.array([0.4, 1.1])
    seeds = rng.integers(0, 1 << 30, 2)

    def build(shift):
        a = W.WrappedCurve(s0 + shift, vec, 0.15 * dl, np.random.default_rng(seeds[0]))
        b = W.WrappedCurve(s0 + shift + 0.5 * dl * nrm + 0.3 * vec, -vec, 0.15 * dl, np.random.default_rng(seeds[1]))
        return _face([(a, 20), (b, 17)], W.DOMAIN_TORUS)

    P = rng.uniform(0, T, (1500, 2))
    w0, n0 = _eval(oracle_lib, build(np.zeros(2)), P)
    w1, n1 = _eval(oracle_lib, build(delta), P + delta)
    ok = (n0 == 0) & (n1 == 0)
    np.testing.assert_allclose(w1[ok], w0[ok], atol=1e-11)
    assert set(np.unique(np.round(w0[ok]))) <= {0.0, 1.0}


def test_contractible_loop_across_seam(oracle_lib):
    """A closed circle-like loop crossing the seam, on a cylinder and a torus."""
    rng = np.random.default_rng(8)
    for dom in (W.DOMAIN_CYLINDER_U, W.DOMAIN_TORUS):
        c = np.array([T - 0.3, T - 0.2 if dom == W.DOMAIN_TORUS else 0.5])
        th = np.linspace(0, 2 * np.pi, 13)
        pts = c + 0.8 * np.column_stack([np.cos(th), np.sin(th)])
        segs = []
        for i in range(12):
            cp = np.stack([pts[i], pts[i + 1]])
            mid = cp.mean(0)
            sh = np.array([-T * np.floor(mid[0] / T), -T * np.floor(mid[1] / T) if dom == W.DOMAIN_TORUS else 0.0])
            segs.append((cp + sh, None))
        f = W.faces_from_loops([[segs]], domains=[dom], periods=[[T, T]])
        P = rng.uniform(0, T, (2000, 2))
        if dom == W.DOMAIN_CYLINDER_U:
            P[:, 1] = rng.uniform(-1, 2, 2000)
        w, near = _eval(oracle_lib, f, P)
        # inside iff some lattice copy of the polygon contains the point
        from tests.curves import crossing_winding

        inside = np.zeros(len(P), dtype=bool)
        for i in (-1, 0, 1):
            for j in ((-1, 0, 1) if dom == W.DOMAIN_TORUS else (0,)):
                inside |= crossing_winding(pts[:-1] + np.array([i * T, j * T]), P) != 0
        np.testing.assert_allclose(w, inside.astype(float), atol=1e-12)


def test_negative_controls(oracle_lib):
    faces, q = W.config3(face_ids=[5], sigma=0.0, open_frac=0.0)  # torus face whose unshifted beta is not the nearest
    w, n = oracle_lib.query_faces(faces, q)
    assert set(np.unique(np.round(w))) <= {0.0, 1.0}
    oracle_lib.set_periodic_options(disable_pairing=True)
    try:
        wb, _ = oracle_lib.query_faces(faces, q)
    finally:
        oracle_lib.set_periodic_options()
    assert np.max(np.round(wb)) >= 2 or np.min(np.round(wb)) <= -1  # overlapping bands (improper pairing)
    planar = W.Faces(faces.face_loop_offsets, faces.loop_seg_offsets, faces.seg_cp_offsets, faces.cp_u, faces.cp_v,
                     faces.cp_w, np.zeros(1, dtype=np.int32), faces.face_period)
    wp, _ = oracle_lib.query_faces(planar, q)
    assert np.mean(np.abs(wp - w) > 0.25) > 0.2  # unlifted evaluation loses the bands


def test_topology_errors(oracle_lib):
    rng = np.random.default_rng(1)
    a = W.WrappedCurve((0.5, 0.5), (2 * T, 3 * T), 0.0, rng)
    f = _face([(a, 9)], W.DOMAIN_TORUS)  # |A| = 1, |B| = 0
    with pytest.raises(oracle_lib.OracleError):
        _eval(oracle_lib, f, [[1.0, 1.0]])
    b = W.WrappedCurve((0.5, 0.5), (2 * T, 4 * T), 0.0, rng)
    c = W.WrappedCurve((0.5, 1.0), (-2 * T, -4 * T), 0.0, rng)
    f2 = _face([(b, 9), (c, 9)], W.DOMAIN_TORUS)  # gcd(2, 4) = 2
    with pytest.raises(oracle_lib.OracleError):
        _eval(oracle_lib, f2, [[1.0, 1.0]])


# -- punctured sphere / cone (Sec. 4.3) -----------------------------------------
def _polyline_loop(us, vs):
    """Degree-1 segments through (us[k], vs[k]); the last vertex is the first
    translated by (+-T, 0), so the loop wraps once around u."""
    return [(np.array([[us[k], vs[k]], [us[k + 1], vs[k + 1]]]), None) for k in range(len(us) - 1)]


def _latitude(c, direction, n=5):
    u = np.linspace(0.0, T, n + 1) if direction > 0 else np.linspace(T, 0.0, n + 1)
    return _polyline_loop(u, np.full(n + 1, c)), (lambda uu: np.full_like(uu, c))


def _zigzag(c, direction, K=8, amp=0.2):
    k = np.arange(K + 1)
    u = T * k / K if direction > 0 else T * (K - k) / K
    v = c + amp * (-1.0) ** k
    uu, vv = (u, v) if direction > 0 else (u[::-1], v[::-1])
    return _polyline_loop(u, v), (lambda x: np.interp(np.mod(x, T), uu, vv))


@pytest.mark.parametrize("domain", [3, 4])
def test_punctured_sphere_closed_forms(oracle_lib, domain):
    """Loops around the poles of a sphere (around the apex of a cone): a cap
    above a +u loop, a cap below a -u loop, a band, both caps (the band's
    complement), a zigzag cap and a cap with a clockwise square hole.  Each
    label follows from comparing v with the loops' heights at u."""
    rng = np.random.default_rng(31 + domain)
    P = np.column_stack([rng.uniform(-T, 2 * T, 4000), rng.uniform(-1.5, 1.5, 4000)])
    hole = _polyline_loop(np.array([2.0, 2.0, 2.6, 2.6, 2.0]), np.array([0.9, 1.3, 1.3, 0.9, 0.9]))
    in_hole = (np.mod(P[:, 0], T) > 2.0) & (np.mod(P[:, 0], T) < 2.6) & (P[:, 1] > 0.9) & (P[:, 1] < 1.3)
    cases = []
    up, f_up = _latitude(0.3, +1)
    cases.append(([up], lambda u, v: v > f_up(u)))
    dn, f_dn = _latitude(0.3, -1)
    cases.append(([dn], lambda u, v: v < f_dn(u)))
    lo, f_lo = _latitude(-0.5, +1)
    hi, f_hi = _latitude(0.4, -1)
    cases.append(([lo, hi], lambda u, v: (v > f_lo(u)) & (v < f_hi(u))))
    lo2, _ = _latitude(-0.5, -1)
    hi2, _ = _latitude(0.4, +1)
    cases.append(([hi2, lo2], lambda u, v: (v < -0.5) | (v > 0.4)))
    zz, f_zz = _zigzag(-0.1, +1)
    cases.append(([zz], lambda u, v: v > f_zz(u)))
    cases.append(([up, hole], lambda u, v: (v > 0.3) & ~in_hole))
    for loops, want_fn in cases:
        f = W.faces_from_loops([loops], domains=[domain], periods=[[T, 0.0]])
        want = want_fn(P[:, 0], P[:, 1]).astype(float)
        w, near = _eval(oracle_lib, f, P)
        clear = near == 0
        assert clear.mean() > 0.99
        np.testing.assert_allclose(w[clear], want[clear], rtol=0, atol=1e-12)


def test_punctured_sphere_inconsistent_face(oracle_lib):
    """Two loops both running +u: the regions' constants span two units."""
    a, _ = _latitude(-0.5, +1)
    b, _ = _latitude(0.4, +1)
    f = W.faces_from_loops([[a, b]], domains=[3], periods=[[T, 0.0]])
    with pytest.raises(oracle_lib.OracleError):
        _eval(oracle_lib, f, [[1.0, 0.0]])
