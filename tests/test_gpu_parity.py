"""GPU parity: the HIP library (through the C ABI binding) against the CPU
oracle, element by element on the same seeded inputs.

Bar: inside/outside identical for every point the oracle certifies farther
than 1e-9 from every curve; |omega_gpu - omega_oracle| <= 1e-12 there (FP64).
"""
import numpy as np
import pytest

from paper_2510_25159_amd import workloads as W
from tests import curves as C
from tests.gpu_helpers import compare, run_wn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_25159_amd import wn

    wn.lib()  # fail loudly if the library was not built
    return torch


@pytest.fixture(scope="module")
def c1(oracle_lib):
    f, q = W.config1()
    w, near = oracle_lib.query_faces(f, q)
    return f, q, w, near


@pytest.fixture(scope="module")
def c2_small(oracle_lib):
    # 24 faces of the batched set: every degree, rational weights, holes,
    # ragged query counts (1k..64k, never a multiple of the tile)
    f, q = W.config2(face_ids=range(24))
    w, near = oracle_lib.query_faces(f, q)
    return f, q, w, near


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("qpw", [64, 256, 512])
def test_config1_parity(torch_cuda, c1, schedule, qpw):
    f, q, w_o, n_o = c1
    print(f"config1 schedule={schedule} qpw={qpw}", flush=True)
    w, lab = run_wn(f, q, schedule=schedule, queries_per_wg=qpw)
    st = compare(w, lab, w_o, n_o)
    assert st["compared"] > 65000


@pytest.mark.parametrize("schedule,policy,qpw", [(0, 0, 0), (1, 1, 0), (1, 2, 0), (1, 1, 512), (1, 2, 512),
                                                 (1, 1, 768), (1, 2, 1024)])
def test_config2_subset_parity(torch_cuda, c2_small, schedule, policy, qpw):
    f, q, w_o, n_o = c2_small
    print(f"config2[0:24] schedule={schedule} policy={policy} qpw={qpw} points={q.num_points}", flush=True)
    w, lab = run_wn(f, q, schedule=schedule, queue_policy=policy, queries_per_wg=qpw)
    st = compare(w, lab, w_o, n_o)
    assert st["compared"] > 0.99 * q.num_points


FP32_TOL = 1e-5  # |omega_gpu - omega_oracle| bound for the mixed-precision path


@pytest.mark.parametrize("schedule,qpw", [(0, 256), (1, 64), (1, 256), (2, 0)])
def test_mixed_precision(torch_cuda, c2_small, schedule, qpw):
    """FP32 admission with the FP64 fallback: within the FP32 bound of the
    oracle, and (by construction) equal to the FP64 path bit for bit."""
    f, q, w_o, n_o = c2_small
    print(f"config2[0:24] mixed schedule={schedule} qpw={qpw}", flush=True)
    kw = dict(schedule=schedule, queries_per_wg=qpw, bin_source=1 if schedule == 2 else 0)
    w32, lab32 = run_wn(f, q, precision=1, **kw)
    compare(w32, lab32, w_o, n_o, tol=FP32_TOL)
    w64, lab64 = run_wn(f, q, precision=0, **kw)
    assert np.array_equal(lab32, lab64)
    ok = np.isfinite(w64)
    assert np.array_equal(np.isfinite(w32), ok) and np.array_equal(w32[ok], w64[ok])


@pytest.mark.parametrize("qpw", [256, 512, 768, 1024])
def test_near_queue_overflow_falls_back_in_line(torch_cuda, c2_small, qpw):
    f, q, w_o, n_o = c2_small
    w, lab = run_wn(f, q, schedule=1, near_capacity=1000, queries_per_wg=qpw)
    compare(w, lab, w_o, n_o)


@pytest.mark.parametrize("policy,cap,mode", [(1, 0, 1), (2, 0, 1), (1, 1000, 1), (1, 0, 2)])
def test_path_hierarchy(torch_cuda, c1, c2_small, policy, cap, mode):
    """Path hierarchy (subpath ellipses prune whole subpaths): oracle parity,
    and the same labels and the same near pairs as the flat far pass."""
    for f, q, w_o, n_o in (c1, c2_small):
        print(f"path hierarchy mode={mode} policy={policy} cap={cap} points={q.num_points}", flush=True)
        w, lab = run_wn(f, q, schedule=1, queue_policy=policy, near_capacity=cap, path_hierarchy=mode)
        st = compare(w, lab, w_o, n_o)
        assert st["compared"] > 0.99 * q.num_points
        w0, lab0 = run_wn(f, q, schedule=1, queue_policy=policy, near_capacity=cap)
        far = n_o == 0
        assert np.array_equal(lab[far], lab0[far])
        ok = far & np.isfinite(w0)
        assert np.max(np.abs(w[ok] - w0[ok])) <= 1e-12
    if cap == 0:
        import torch

        from paper_2510_25159_amd import wn

        stats = [torch.zeros(wn.STATS_COUNT, dtype=torch.int64, device="cuda") for _ in range(2)]
        f, q = c2_small[0], c2_small[1]
        run_wn(f, q, schedule=1, queue_policy=policy, stats=stats[0])
        run_wn(f, q, schedule=1, queue_policy=policy, stats=stats[1], path_hierarchy=1)
        s0, s1 = stats[0].cpu().tolist(), stats[1].cpu().tolist()
        assert s0[:6] == s1[:6]  # same near pairs, splits, leaves, evaluations, flops, depth


def test_path_hierarchy_long_path(torch_cuda, oracle_lib):
    """A 4,096-segment star loop: the hierarchy prunes most of it; both far
    passes against the oracle."""
    faces = W.config1_faces(nseg=4096)
    q = W.config1_queries(n=8192)
    w_o, n_o = oracle_lib.query_faces(faces, q)
    for tree in (0, 1, 2):
        print(f"long path tree={tree}", flush=True)
        w, lab = run_wn(faces, q, schedule=1, path_hierarchy=tree)
        st = compare(w, lab, w_o, n_o)
        assert st["compared"] > 0.99 * q.num_points


def test_path_hierarchy_mixed_face_sizes(torch_cuda, oracle_lib):
    """One query over faces on both sides of the spatial-order limit (65,536
    points): the wave walk takes the small faces, the per-lane walk the large
    one, with host offsets (the per-lane pass only when needed) and without
    (both passes always run).  Oracle parity and the flat pass's labels and
    near pairs."""
    import torch

    from paper_2510_25159_amd import wn

    big_face = W.config1_faces(nseg=256)
    f2, q2 = W.config2(face_ids=range(3))
    big_pts = W.config1_queries(n=70000)
    loops = []
    for F in (big_face, f2):
        for f in range(F.num_faces):
            fl = []
            for l in range(F.face_loop_offsets[f], F.face_loop_offsets[f + 1]):
                segs = []
                for s_ in range(F.loop_seg_offsets[l], F.loop_seg_offsets[l + 1]):
                    a, b = F.seg_cp_offsets[s_], F.seg_cp_offsets[s_ + 1]
                    cp = np.column_stack([F.cp_u[a:b], F.cp_v[a:b]])
                    segs.append((cp, None if F.cp_w is None else F.cp_w[a:b]))
                fl.append(segs)
            loops.append(fl)
    faces = W.faces_from_loops(loops)
    pts = [np.column_stack([big_pts.u, big_pts.v])]
    for f in range(3):
        a, b = q2.face_point_offsets[f], q2.face_point_offsets[f + 1]
        pts.append(np.column_stack([q2.u[a:b], q2.v[a:b]]))
    q = W.queries_for_faces(pts)
    w_o, n_o = oracle_lib.query_faces(faces, q)
    w0, lab0 = run_wn(faces, q, schedule=1)
    s0 = torch.zeros(wn.STATS_COUNT, dtype=torch.int64, device="cuda")
    run_wn(faces, q, schedule=1, stats=s0)
    for host in (True, False):
        for tree in (1, 2):
            print(f"mixed face sizes: host offsets {host}, path_hierarchy {tree}", flush=True)
            w, lab = run_wn(faces, q, schedule=1, path_hierarchy=tree, offsets_host=host)
            st = compare(w, lab, w_o, n_o)
            assert st["compared"] > 0.99 * q.num_points
            far = n_o == 0
            assert np.array_equal(lab[far], lab0[far])
            ok = far & np.isfinite(w0)
            assert np.max(np.abs(w[ok] - w0[ok])) <= 1e-12
        s1 = torch.zeros(wn.STATS_COUNT, dtype=torch.int64, device="cuda")
        run_wn(faces, q, schedule=1, stats=s1, path_hierarchy=1, offsets_host=host)
        assert s0.cpu().tolist()[:6] == s1.cpu().tolist()[:6]


def test_interleaved_points_and_device_offsets(torch_cuda, c2_small):
    f, q, w_o, n_o = c2_small
    w, lab = run_wn(f, q, schedule=0, stride=2, offsets_host=False)
    compare(w, lab, w_o, n_o)
    w, lab = run_wn(f, q, schedule=1, stride=2, offsets_host=False)
    compare(w, lab, w_o, n_o)


def test_edge_cases(torch_cuda, oracle_lib):
    """Empty faces, a face without loops, a single point, degree-1 loops,
    points on vertices (on-boundary), non-finite and huge points (invalid)."""
    circ = C.circle_arcs(1.0)
    sq = C.polygon([[-1, -1], [1, -1], [1, 1], [-1, 1]])
    faces = W.faces_from_loops([[circ], [], [sq], [circ, C.circle_arcs(0.3, cw=True)], [sq]])
    rng = np.random.default_rng(0)
    pts = [rng.uniform(-1.5, 1.5, (5, 2)), rng.uniform(-1, 1, (3, 2)), np.zeros((0, 2)),
           rng.uniform(-1.5, 1.5, (257, 2)), np.array([[0.25, 0.5]])]
    q = W.queries_for_faces(pts)
    w_o, n_o = oracle_lib.query_faces(faces, q)
    for sched, qpw, tree in ((0, 0, 0), (1, 0, 0), (1, 512, 0), (1, 0, 1)):
        w, lab = run_wn(faces, q, schedule=sched, queries_per_wg=qpw, path_hierarchy=tree)
        compare(w, lab, w_o, n_o)
        assert np.all(w[5:8] == 0.0)  # face without loops
    # vertices and invalid points on the square face
    special = np.array([[1.0, 1.0], [-1.0, 1.0], [np.nan, 0.0], [np.inf, 1.0], [2e15, 0.0], [0.0, 0.0]])
    q2 = W.queries_for_faces([special])
    f2 = W.faces_from_loops([[sq]])
    for sched, qpw, tree in ((0, 0, 0), (1, 0, 0), (1, 512, 0), (1, 0, 1)):
        w, lab = run_wn(f2, q2, schedule=sched, queries_per_wg=qpw, path_hierarchy=tree)
        assert list(lab) == [2, 2, 3, 3, 3, 1]
        assert np.all(np.isnan(w[:5])) and abs(w[5] - 1.0) < 1e-15


def test_rule_positive(torch_cuda, oracle_lib):
    faces = W.faces_from_loops([[C.circle_arcs(1.0, cw=True)]])
    rng = np.random.default_rng(1)
    P = rng.uniform(-1.5, 1.5, (1000, 2))
    q = W.queries_for_faces([P])
    w_o, n_o = oracle_lib.query_faces(faces, q)
    for sched in (0, 1):
        w, lab = run_wn(faces, q, schedule=sched, rule=1)
        compare(w, lab, w_o, n_o, rule=1)
        assert np.all(lab[np.hypot(P[:, 0], P[:, 1]) < 0.99] == 0)  # omega = -1 is outside under the positive rule


def test_near_boundary_points(torch_cuda, oracle_lib):
    """Points 1e-8..1e-3 from the curve recurse deeply; those within 1e-9 are excluded."""
    rng = np.random.default_rng(4)
    faces, _ = W.config2(face_ids=[7])
    segs = []
    for s in range(faces.num_segments):
        a, b = faces.seg_cp_offsets[s], faces.seg_cp_offsets[s + 1]
        segs.append((np.column_stack([faces.cp_u[a:b], faces.cp_v[a:b]]), faces.cp_w[a:b]))
    P = []
    for _ in range(3000):
        cp, w = segs[rng.integers(len(segs))]
        t = rng.uniform(0, 1)
        p = C.eval_curve(cp, w, t)[0]
        d = C.eval_deriv(cp, w, t)[0]
        nrm = np.array([-d[1], d[0]]) / np.hypot(*d)
        P.append(p + 10.0 ** rng.uniform(-11, -3) * rng.choice([-1, 1]) * nrm)
    q = W.queries_for_faces([np.array(P)])
    w_o, n_o = oracle_lib.query_faces(faces, q)
    for sched, qpw, tree in ((0, 0, 0), (1, 0, 0), (1, 512, 0), (1, 0, 1)):
        w, lab = run_wn(faces, q, schedule=sched, queries_per_wg=qpw, path_hierarchy=tree)
        st = compare(w, lab, w_o, n_o)
        assert st["compared"] > 1500


def test_config2_full_sampled(torch_cuda, oracle_lib):
    """Full batched set (2,000 faces, ~31M points) in the launch configuration
    the benchmark times; sampled points compared with the oracle one by one."""
    import torch

    from paper_2510_25159_amd import wn

    faces, q = W.config2()
    print(f"config2 full: {faces.num_segments} segments, {q.num_points} points", flush=True)
    fs = wn.FaceSet(faces)
    w, lab = run_wn(faces, q, faceset=fs, schedule=1)
    rng = np.random.default_rng(22)
    idx = np.sort(rng.choice(q.num_points, 20000, replace=False))
    pf, u, v = W.subset_queries(q, idx)
    w_o, n_o = oracle_lib.query(faces, pf, u, v)
    st = compare(w[idx], lab[idx], w_o, n_o)
    print(st, flush=True)
    # every label is a valid code and no point is left unwritten
    assert set(np.unique(lab)).issubset({0, 1, 2})
    assert np.isfinite(w[lab != 2]).all()


def _lens(p0, c1, c2, pn, d1, d2, w=None):
    """Closed loop of two cubics p0 -> pn (controls c1, c2) and back (controls d1, d2)."""
    a = np.array([p0, c1, c2, pn], dtype=np.float64)
    b = np.array([pn, d1, d2, p0], dtype=np.float64)
    return [(a, w), (b, None if w is None else w[::-1].copy())]


def test_queries_on_chords_and_ray_ties(torch_cuda, oracle_lib):
    """Queries exactly on the chord of a near segment (horizontal, vertical,
    diagonal chords), on the chords' lines outside the segments, and level
    with vertices: every tie the near-pair bookkeeping breaks must give the
    oracle's winding number."""
    lens_h = _lens((-1, 0), (-0.5, 0.3), (0.5, 0.3), (1, 0), (0.5, -0.3), (-0.5, -0.3))
    lens_v = _lens((0, -1), (-0.3, -0.5), (-0.3, 0.5), (0, 1), (0.3, 0.5), (0.3, -0.5))
    lens_d = _lens((-1, -1), (-1, 0), (0, 1), (1, 1), (1, 0), (0, -1))
    lens_r = _lens((-1, 0), (-0.5, 0.3), (0.5, 0.3), (1, 0), (0.5, -0.3), (-0.5, -0.3),
                   w=np.array([1.0, 2.0, 0.5, 1.0]))
    # one bulge closed by a line: the queries sit between the cubic and its chord
    half = [(np.array([[-1, 0], [-0.5, 0.3], [0.5, 0.3], [1, 0]], dtype=np.float64), None),
            (np.array([[1, 0], [-1, 0]], dtype=np.float64), None)]
    diamond = [(np.array([[1, 0], [0.7, 0.7], [0, 1]], dtype=np.float64), None),
               (np.array([[0, 1], [-0.7, 0.7], [-1, 0]], dtype=np.float64), None),
               (np.array([[-1, 0], [-0.7, -0.7], [0, -1]], dtype=np.float64), None),
               (np.array([[0, -1], [0.7, -0.7], [1, 0]], dtype=np.float64), None)]
    faces = W.faces_from_loops([[lens_h], [lens_v], [lens_d], [lens_r], [half], [diamond],
                                [lens_h, diamond]])
    on_h = [[0, 0], [0.5, 0], [-0.5, 0], [0.25, 0], [0, 0.1], [0, -0.1], [2, 0], [-2, 0], [0.75, 0]]
    on_v = [[y, x] for x, y in on_h]
    on_d = [[0, 0], [0.5, 0.5], [-0.25, -0.25], [2, 2], [-3, -3], [0.5, -0.5]]
    pts = [np.array(on_h, float), np.array(on_v, float), np.array(on_d, float), np.array(on_h, float),
           np.array([[0, 0.05], [0.5, 0.01], [0, 0.1], [-0.5, 0.1], [0.25, 0.2], [0, 0.3], [0.9, 0.01], [2, 0]],
                    float),
           np.array(on_h + [[0.5, 0.5], [-0.5, -0.5]], float),
           np.array(on_h, float)]
    q = W.queries_for_faces(pts)
    w_o, n_o = oracle_lib.query_faces(faces, q)
    assert np.all(n_o == 0)  # every query is well away from the curves
    for sched, qpw, tree in ((0, 0, 0), (1, 0, 0), (1, 512, 0), (1, 0, 1)):
        w, lab = run_wn(faces, q, schedule=sched, queries_per_wg=qpw, path_hierarchy=tree)
        st = compare(w, lab, w_o, n_o)
        assert st["compared"] == q.num_points


def test_nurbs_faces(torch_cuda, oracle_lib):
    """Faces given as NURBS loops: a rational quadratic circle (closed form:
    omega = 1 inside, 0 outside), a closed random quintic with interior knots,
    and the circle as a loop of two half-circle curves.  The library splits
    them by knot insertion (wn_nurbs_to_bezier + wn_create_faces, and
    wn_create_faces_nurbs); the oracle gets its own split (interpolation of
    each span)."""
    from oracle import nurbs as ON
    from paper_2510_25159_amd import wn
    from tests.test_nurbs import CIRCLE_CP, CIRCLE_KNOTS, CIRCLE_W

    rng = np.random.default_rng(12)
    th = np.sort(rng.uniform(0, 2 * np.pi, 11))
    r = rng.uniform(0.6, 1.4, 11)
    cp = np.column_stack([r * np.cos(th), r * np.sin(th)])
    cp = np.vstack([cp, cp[:1]])  # closed: clamped ends at the same point
    knots = np.concatenate([np.zeros(6), [0.3, 0.3, 0.55, 0.7, 0.8, 0.8], np.ones(6)])
    wts = rng.uniform(0.5, 2.0, len(cp))
    s2 = 2 ** -0.5
    half_knots = [0, 0, 0, 0.5, 0.5, 1, 1, 1]
    upper = ([[1, 0], [1, 1], [0, 1], [-1, 1], [-1, 0]], [1, s2, 1, s2, 1])
    lower = ([[-1, 0], [-1, -1], [0, -1], [1, -1], [1, 0]], [1, s2, 1, s2, 1])
    curves = [(2, CIRCLE_KNOTS, CIRCLE_CP, CIRCLE_W), (5, knots, cp, wts), (2, half_knots, *upper),
              (2, half_knots, *lower)]
    loops = [[0], [1], [2, 3]]  # face f = loop f
    # oracle faces from the oracle's split
    o_loops = [[[seg for c in lp for seg in ON.spans_to_bezier(curves[c][1], curves[c][0], curves[c][2],
                                                                 curves[c][3])]] for lp in loops]
    faces_o = W.faces_from_loops(o_loops, rational=True)
    P = rng.uniform(-1.6, 1.6, (20000, 2))
    q = W.queries_for_faces([P, P, P])
    w_o, n_o = oracle_lib.query_faces(faces_o, q)
    rad = np.hypot(P[:, 0], P[:, 1])
    far = np.abs(rad - 1.0) > 1e-6
    for f in (0, 2):
        assert np.allclose(w_o[f * 20000:(f + 1) * 20000][far], (rad[far] < 1.0).astype(float), atol=1e-12)
    # library: split then create, and create from NURBS
    l_loops = [[[seg for c in lp for seg in wn.nurbs_to_bezier(curves[c][0], curves[c][1], curves[c][2],
                                                                curves[c][3])]] for lp in loops]
    faces_l = W.faces_from_loops(l_loops, rational=True)
    fs_n = wn.FaceSet.from_nurbs([0, 1, 2, 3], [0, 1, 2, 4], [c[0] for c in curves],
                                 np.cumsum([0] + [len(c[2]) for c in curves]),
                                 np.concatenate([np.asarray(c[1], dtype=float) for c in curves]),
                                 np.concatenate([np.asarray(c[2], dtype=float)[:, 0] for c in curves]),
                                 np.concatenate([np.asarray(c[2], dtype=float)[:, 1] for c in curves]),
                                 np.concatenate([np.asarray(c[3], dtype=float) for c in curves]))
    for sched in (0, 1):
        w, lab = run_wn(faces_l, q, schedule=sched)
        compare(w, lab, w_o, n_o)
        w2, lab2 = run_wn(None, q, schedule=sched, faceset=fs_n)
        compare(w2, lab2, w_o, n_o)
        assert np.array_equal(lab2, lab)
    with pytest.raises(wn.WnError):  # a curve with too few control points
        wn.FaceSet.from_nurbs([0, 1], [0, 1], [3], [0, 3], np.zeros(7), [0, 1, 2], [0, 1, 0])


@pytest.mark.parametrize("qpw", [512, 1024])
def test_overlapped_far_near_match_serial(torch_cuda, c2_small, qpw):
    """With WN_FLAG_OVERLAP and host offsets the batched FP64 query overlaps
    near passes of early face runs with the far pass of later ones (a side
    stream); by default it runs the passes one after the other.  Same labels,
    omega within rounding of the order of the near pass's additions, and both
    match the oracle."""
    from paper_2510_25159_amd import wn

    f, q, w_o, n_o = c2_small
    w1, l1 = run_wn(f, q, schedule=1, queries_per_wg=qpw, create={"flags": wn.FLAG_OVERLAP})  # overlapped
    w2, l2 = run_wn(f, q, schedule=1, queries_per_wg=qpw)  # serial
    assert np.array_equal(l1, l2)
    ok = l1 < 2
    assert np.max(np.abs(w1[ok] - w2[ok])) <= 1e-12
    compare(w1, l1, w_o, n_o)


def test_overlapped_with_auto_hierarchy(torch_cuda, oracle_lib):
    """Automatic hierarchy with a 720-segment loop (tree walk) beside short
    loops (flat scan): the flat faces' far pass overlaps its near passes, the
    tree face's near entries go to the final near pass; same labels as the
    serial passes, and both match the oracle."""
    k = np.arange(720) * (2 * np.pi / 720)
    r = 1.0 + 0.3 * np.cos(7 * k)
    star = C.polygon(np.column_stack([r * np.cos(k), r * np.sin(k)]))
    sq = C.polygon([[-1, -1], [1, -1], [1, 1], [-1, 1]])
    faces = W.faces_from_loops([[C.circle_arcs(1.0)], [star], [sq], [C.circle_arcs(1.0), C.circle_arcs(0.4, cw=True)],
                                [C.polygon(np.column_stack([np.cos(k[::18]), np.sin(k[::18])]))]])
    rng = np.random.default_rng(21)
    q = W.queries_for_faces([rng.uniform(-1.5, 1.5, (n, 2)) for n in (3000, 5000, 2500, 4000, 1500)])
    w_o, n_o = oracle_lib.query_faces(faces, q)
    from paper_2510_25159_amd import wn

    w1, l1 = run_wn(faces, q, schedule=1, queries_per_wg=1024, path_hierarchy=2, create={"flags": wn.FLAG_OVERLAP})
    w2, l2 = run_wn(faces, q, schedule=1, queries_per_wg=1024, path_hierarchy=2)
    assert np.array_equal(l1, l2)
    ok = l1 < 2
    assert np.max(np.abs(w1[ok] - w2[ok])) <= 1e-12
    st = compare(w1, l1, w_o, n_o)
    assert st["compared"] > 0.99 * q.num_points


def test_concurrent_queries_share_a_handle(torch_cuda, c2_small):
    """Two host threads run overlapped queries on one handle, each on its own
    stream (the handle's side stream is shared, the fork / join events are
    per call): every result equals the single-thread one."""
    import threading

    from paper_2510_25159_amd import wn

    torch = torch_cuda
    f, q, _, _ = c2_small
    fs = wn.FaceSet(f, flags=wn.FLAG_OVERLAP)
    dev = torch.device("cuda:0")
    u = torch.from_numpy(q.u).to(dev)
    v = torch.from_numpy(q.v).to(dev)
    offs = torch.from_numpy(q.face_point_offsets).to(dev)
    w_ref, l_ref = fs.query(u, v, offs, q.face_point_offsets, schedule=1, queries_per_wg=1024)
    torch.cuda.synchronize()
    w_ref, l_ref = w_ref.cpu().numpy(), l_ref.cpu().numpy()
    streams = [torch.cuda.Stream() for _ in range(2)]
    got, errors = [[], []], []

    def work(i):
        try:
            s = streams[i]
            with torch.cuda.stream(s):
                outs = [fs.query(u, v, offs, q.face_point_offsets, schedule=1, queries_per_wg=1024, stream=s)
                        for _ in range(4)]
                s.synchronize()
                got[i] = [(w.cpu().numpy(), lab.cpu().numpy()) for w, lab in outs]
        except Exception as exc:  # reported by the main thread
            errors.append(repr(exc))

    threads = [threading.Thread(target=work, args=(i,)) for i in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    ok = l_ref < 2
    for per in got:
        assert len(per) == 4
        for w, lab in per:
            assert np.array_equal(lab, l_ref)
            assert np.max(np.abs(w[ok] - w_ref[ok])) <= 1e-12
