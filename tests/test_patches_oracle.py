"""Pins of the application oracle (Sec. 5.4) against closed forms.

Grid cell centres are checked against hand-computed dyadic values and the
grid invariants; the multi-patch rule (inside when inside any face of the
surface, Sec. 5.4.1) against discs and annuli whose labels follow from the
distance to their centres.  No GPU is involved.
"""
import numpy as np

from paper_2510_25159_amd import workloads as W
from tests import curves as C


def test_grid_samples_dyadic_closed_form(oracle_lib):
    from oracle import patches

    f, u, v = patches.grid_samples([(0.0, -1.0, 0.25, 0.5, 4, 3), (1.0, 2.0, 1.0, 1.0, 0, 5), (-2.0, 0.0, 0.5, 2.0, 2, 1)])
    # face 0: 4 x 3 cells, i along u fastest; face 1 empty; face 2: 2 x 1
    np.testing.assert_array_equal(f, [0] * 12 + [2, 2])
    np.testing.assert_array_equal(u[:12], [0.125, 0.375, 0.625, 0.875] * 3)
    np.testing.assert_array_equal(v[:12], [-0.75] * 4 + [-0.25] * 4 + [0.25] * 4)
    np.testing.assert_array_equal(u[12:], [-1.75, -1.25])
    np.testing.assert_array_equal(v[12:], [1.0, 1.0])


def test_grid_samples_invariants(oracle_lib):
    from oracle import patches

    rng = np.random.default_rng(3)
    grids = [(rng.uniform(-5, 5), rng.uniform(-5, 5), rng.uniform(0.01, 1), rng.uniform(0.01, 1),
              int(rng.integers(1, 40)), int(rng.integers(1, 40))) for _ in range(6)]
    f, u, v = patches.grid_samples(grids)
    assert len(u) == sum(g[4] * g[5] for g in grids)
    for k, (u0, v0, du, dv, nu, nv) in enumerate(grids):
        uu, vv = u[f == k].reshape(nv, nu), v[f == k].reshape(nv, nu)
        # centres strictly inside their cells, spacing du / dv, rows constant in v
        assert np.all(uu > u0) and np.all(uu < u0 + nu * du)
        assert np.all(vv > v0) and np.all(vv < v0 + nv * dv)
        np.testing.assert_allclose(np.diff(uu, axis=1), du, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(np.diff(vv, axis=0), dv, rtol=1e-12, atol=1e-12)
        assert np.all(vv == vv[:, :1])
        np.testing.assert_allclose(uu[:, 0], u0 + du / 2, rtol=0, atol=1e-12)


def _disc_faces():
    """Faces: 0 unit disc at 0, 1 disc r=0.5 at (1.2, 0), 2 clockwise unit
    disc at (5, 0), 3 annulus 0.3 < r < 1 at (10, 0), 4 disc r=0.4 at (10, 0),
    5 a disc no surface references."""
    def disc(r, c, cw=False):
        return [C.circle_arcs(r, center=c, cw=cw)]
    fl = [disc(1.0, (0, 0)), disc(0.5, (1.2, 0)), disc(1.0, (5, 0), cw=True),
          [C.circle_arcs(1.0, center=(10, 0)), C.circle_arcs(0.3, center=(10, 0), cw=True)],
          disc(0.4, (10, 0)), disc(1.0, (0, 0))]
    return W.faces_from_loops(fl)


def test_classify_surfaces_closed_form(oracle_lib):
    from oracle import patches

    faces = _disc_faces()
    rng = np.random.default_rng(8)
    # surface 0: faces 0 and 1 (overlapping discs); 1: face 2 (clockwise);
    # 2: no face; 3: faces 4 and 3 (the annulus's hole covered by face 4)
    sfo = [0, 2, 3, 3, 5]
    sff = [0, 1, 2, 4, 3]
    centres = [(0.5, 0.0), (5.0, 0.0), (0.0, 0.0), (10.0, 0.0)]
    pts = []
    for c in centres:
        P = rng.uniform(-1.5, 1.5, size=(3000, 2)) + np.asarray(c)
        pts.append(P)
    spo = np.cumsum([0] + [len(p) for p in pts])
    P = np.concatenate(pts)
    u, v = P[:, 0].copy(), P[:, 1].copy()
    for rule in (0, 1):
        ins, first, near = patches.classify_surfaces(faces, sfo, sff, u, v, spo, rule=rule)
        for s, c in enumerate(centres):
            a, b = spo[s], spo[s + 1]
            x, y = u[a:b], v[a:b]
            if s == 0:
                r0, r1 = np.hypot(x, y), np.hypot(x - 1.2, y)
                clear = (np.abs(r0 - 1) > 1e-6) & (np.abs(r1 - 0.5) > 1e-6)
                want = (r0 < 1) | (r1 < 0.5)
                want_first = np.where(r0 < 1, 0, np.where(r1 < 0.5, 1, -1))
            elif s == 1:
                r = np.hypot(x - 5, y)
                clear = np.abs(r - 1) > 1e-6
                want = (r < 1) & (rule == 0)  # winding number -1: nonzero rule only
                want_first = np.where(want, 2, -1)
            elif s == 2:
                clear = np.ones(b - a, dtype=bool)
                want = np.zeros(b - a, dtype=bool)
                want_first = np.full(b - a, -1)
            else:
                r = np.hypot(x - 10, y)
                clear = (np.abs(r - 1) > 1e-6) & (np.abs(r - 0.3) > 1e-6) & (np.abs(r - 0.4) > 1e-6)
                want = r < 1
                want_first = np.where(r < 0.4, 4, np.where((r > 0.3) & (r < 1), 3, -1))
            assert not np.any(near[a:b][clear])
            np.testing.assert_array_equal(ins[a:b][clear], want[clear])
            np.testing.assert_array_equal(first[a:b][clear], want_first[clear])
