"""NURBS p-curves: the oracle's plain definitions pinned to closed forms, and
the library's knot-insertion split (a host function, no GPU) against them."""
from math import comb

import numpy as np
import pytest

from oracle import nurbs as O

CIRCLE_KNOTS = [0, 0, 0, 0.25, 0.25, 0.5, 0.5, 0.75, 0.75, 1, 1, 1]
CIRCLE_CP = [[1, 0], [1, 1], [0, 1], [-1, 1], [-1, 0], [-1, -1], [0, -1], [1, -1], [1, 0]]
CIRCLE_W = [1, 2 ** -0.5, 1, 2 ** -0.5, 1, 2 ** -0.5, 1, 2 ** -0.5, 1]


def random_nurbs(rng, p, rational=True):
    spans = rng.integers(1, 6)
    inner = np.sort(rng.uniform(0.05, 0.95, spans - 1)) if spans > 1 else np.zeros(0)
    mult = rng.integers(1, p + 1, len(inner))
    knots = np.concatenate([np.zeros(p + 1), np.repeat(inner, mult), np.ones(p + 1)])
    n = len(knots) - p - 1
    cp = rng.uniform(-1, 1, (n, 2))
    w = rng.uniform(0.5, 2.0, n) if rational else None
    return knots, cp, w


def test_oracle_partition_of_unity_and_bernstein():
    rng = np.random.default_rng(5)
    for p in range(1, 6):
        knots, _, _ = random_nurbs(rng, p)
        for t in np.linspace(0, 1, 37):
            assert abs(np.sum(O.basis(knots, p, t)) - 1.0) < 1e-14
        single = [0.0] * (p + 1) + [1.0] * (p + 1)
        for t in (0.0, 0.2, 0.5, 0.9):
            want = [comb(p, k) * t ** k * (1 - t) ** (p - k) for k in range(p + 1)]
            assert np.allclose(O.basis(single, p, t), want, rtol=0, atol=1e-15)


def test_oracle_circle_and_end_points():
    for t in np.linspace(0, 1, 101):
        x = O.nurbs_point(CIRCLE_KNOTS, 2, CIRCLE_CP, CIRCLE_W, t)
        assert abs(np.hypot(*x) - 1.0) < 1e-14
    rng = np.random.default_rng(6)
    for p in range(1, 6):
        knots, cp, w = random_nurbs(rng, p)
        assert np.allclose(O.nurbs_point(knots, p, cp, w, 0.0), cp[0], atol=1e-15)
        assert np.allclose(O.nurbs_point(knots, p, cp, w, 1.0), cp[-1], atol=1e-15)


@pytest.fixture(scope="module")
def wnlib():
    from paper_2510_25159_amd import wn

    try:
        wn.lib()
    except OSError as exc:  # the library is built by __graft_entry__.build()
        pytest.skip(f"library not built: {exc}")
    return wn


@pytest.mark.parametrize("rational", [True, False])
def test_split_matches_nurbs(wnlib, rational):
    rng = np.random.default_rng(7 + rational)
    for trial in range(60):
        p = int(rng.integers(1, 6))
        knots, cp, w = random_nurbs(rng, p, rational)
        segs = wnlib.nurbs_to_bezier(p, knots, cp, w)
        values = np.unique(knots)
        assert len(segs) == len(values) - 1
        for j, (bcp, bw) in enumerate(segs):
            assert bcp.shape == (p + 1, 2) and (bw is None) == (not rational)
            a, b = values[j], values[j + 1]
            for tau in (0.0, 0.13, 0.5, 0.77, 1.0):
                want = O.nurbs_point(knots, p, cp, w, a + tau * (b - a))
                got = O.bezier_point(bcp, bw, tau)
                assert np.max(np.abs(got - want)) < 1e-13, (trial, p, j, tau)


def test_split_circle(wnlib):
    segs = wnlib.nurbs_to_bezier(2, CIRCLE_KNOTS, CIRCLE_CP, CIRCLE_W)
    assert len(segs) == 4
    for bcp, bw in segs:
        for tau in np.linspace(0, 1, 11):
            assert abs(np.hypot(*O.bezier_point(bcp, bw, tau)) - 1.0) < 1e-14


def test_split_rejects_malformed(wnlib):
    cp = np.zeros((4, 2))
    bad = [
        (0, [0, 0, 0, 0, 1, 1], cp),                      # degree 0
        (3, [0, 0, 0, 1, 1, 1, 1, 1], cp),                # not clamped at the start
        (2, [0, 0, 0, 0.6, 0.4, 1, 1], cp),               # decreasing
        (1, [0, 0, 0.5, 0.5, 1, 1], cp),                  # multiplicity 2 > degree 1: a break
        (2, [0, 0, 0, 0, 0, 0, 0], cp),                   # empty domain
        (2, [0, 0, 0, 0.5, 1, 1, 1, 1], np.zeros((5, 2))),  # end value repeated p + 2 times
        (2, [0, 0, 0, 0, 0.5, 1, 1, 1], np.zeros((5, 2))),  # start value repeated p + 2 times
    ]
    for p, knots, c in bad:
        with pytest.raises(wnlib.WnError):
            wnlib.nurbs_to_bezier(p, knots, c)
    with pytest.raises(wnlib.WnError):
        wnlib.nurbs_to_bezier(2, CIRCLE_KNOTS, CIRCLE_CP, [1, 1, 1, 1, -1, 1, 1, 1, 1])  # weight <= 0


def test_oracle_span_interpolation():
    """The oracle's own span split (interpolation of the homogeneous curve)
    reproduces the curve: each segment's points equal nurbs_point on its span,
    the circle's segments lie on the unit circle, and a single-span curve
    returns its own control points."""
    rng = np.random.default_rng(9)
    for p in range(1, 6):
        for rational in (True, False):
            knots, cp, w = random_nurbs(rng, p, rational)
            U = np.asarray(knots)
            spans = [(U[k], U[k + 1]) for k in range(p, len(U) - p - 1) if U[k + 1] > U[k]]
            segs = O.spans_to_bezier(knots, p, cp, w)
            assert len(segs) == len(spans)
            for (a, b), (scp, sw) in zip(spans, segs):
                for t in np.linspace(0, 1, 9):
                    x = O.bezier_point(scp, sw, t)
                    tt = a + (b - a) * t
                    y = O.nurbs_point(knots, p, cp, w, min(tt, np.nextafter(b, a)) if tt >= b and b < 1 else tt)
                    assert np.allclose(x, y, rtol=0, atol=1e-11), (p, rational, a, b, t)
    for scp, sw in O.spans_to_bezier(CIRCLE_KNOTS, 2, CIRCLE_CP, CIRCLE_W):
        for t in np.linspace(0, 1, 17):
            assert abs(np.hypot(*O.bezier_point(scp, sw, t)) - 1.0) < 1e-13
    single = [0.0] * 4 + [1.0] * 4
    cp = rng.uniform(-1, 1, (4, 2))
    w = rng.uniform(0.5, 2, 4)
    (scp, sw), = O.spans_to_bezier(single, 3, cp, w)
    assert np.allclose(scp, cp, atol=1e-13) and np.allclose(sw, w, atol=1e-13)
