"""The degree set's generator (inputs of the Sec. 5 degree experiment):
elevation keeps the curve (against the test-local homogeneous elevation
and curve evaluation of tests/curves.py), joints stay shared bit-for-bit,
the queries are the same at every degree, and the oracle's omega is
unchanged by elevation at uniform points.  No GPU involved."""
import numpy as np

from paper_2510_25159_amd import workloads as W
from tests import curves as C


def test_elevate_bezier_keeps_curve():
    rng = np.random.default_rng(3)
    t = np.linspace(0.0, 1.0, 33)
    for n in (1, 2, 3, 4):
        cp = rng.normal(size=(n + 1, 2))
        e1 = W.elevate_bezier(cp, 1)
        ref, _ = C.elevate(cp, None)
        np.testing.assert_allclose(e1, ref, rtol=0, atol=1e-15)
        for times in (1, 2):
            e = W.elevate_bezier(cp, times)
            assert len(e) == n + 1 + times
            assert np.array_equal(e[0], cp[0]) and np.array_equal(e[-1], cp[-1])
            np.testing.assert_allclose(C.eval_curve(e, None, t), C.eval_curve(cp, None, t), rtol=0, atol=1e-14)


def test_degree_set_shapes_and_oracle_invariance(oracle_lib):
    sets = {d: W.degree_set(d, num_faces=3, points_per_face=600) for d in (3, 4, 5)}
    f3, q3 = sets[3]
    w3, n3 = oracle_lib.query_faces(f3, q3)
    for d, (f, q) in sets.items():
        assert np.all(np.diff(f.seg_cp_offsets) == d + 1)
        assert np.array_equal(q.u, q3.u) and np.array_equal(q.v, q3.v)
        # joints: the end point of each segment is the start of the next
        for s in range(f.num_segments):
            a, b = f.seg_cp_offsets[s], f.seg_cp_offsets[s + 1]
            nxt = f.seg_cp_offsets[s + 1] if (s + 1) % 64 else f.seg_cp_offsets[s + 1 - 64]
            assert f.cp_u[b - 1] == f.cp_u[nxt] and f.cp_v[b - 1] == f.cp_v[nxt]
        w, n = oracle_lib.query_faces(f, q)
        far = (n == 0) & (n3 == 0)
        assert far.sum() >= 0.45 * q.num_points  # the uniform half
        assert np.max(np.abs(w[far] - w3[far])) <= 1e-12
