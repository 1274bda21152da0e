"""The tolerance eps of Alg. 1 (Sec. 4.1) beyond its default.

  * Parity at eps = 1e-9 and 1e-6: with the oracle's certified near band set
    to eps, every point farther than eps from every curve must get the
    oracle's label, and omega within 1e-12 (FP64).  A point the GPU reports
    on-boundary must lie within eps of a curve.
  * The eps sweep of Sec. 5 (Table 3): curve evaluations per point grow
    about linearly in log(1/eps) for points sampled on the curves, and stay
    flat for uniform points.
  * The on-boundary fraction of uniform points (Sec. 5): it falls with eps,
    like 2 eps x perimeter / area, and is 0 at eps = 1e-10 on 2^20 points.
"""
import numpy as np
import pytest

from paper_2510_25159_amd import workloads as W
from tests.gpu_helpers import compare, run_wn

pytestmark = pytest.mark.gpu

SWEEP = [1e-4, 1e-5, 1e-6, 1e-7, 1e-8, 1e-9, 1e-10]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_25159_amd import wn

    wn.lib()
    return torch


@pytest.mark.parametrize("eps", [1e-9, 1e-6])
@pytest.mark.parametrize("schedule", [0, 1])
def test_parity_at_eps(torch_cuda, oracle_lib, eps, schedule):
    for name, (f, q) in (("config1", W.config1()), ("config2[0:16]", W.config2(face_ids=range(16)))):
        print(f"{name} eps={eps} schedule={schedule} points={q.num_points}", flush=True)
        w_o, n_o = oracle_lib.query_faces(f, q, near_tol=eps)
        w, lab = run_wn(f, q, schedule=schedule, create={"eps": eps})
        st = compare(w, lab, w_o, n_o)
        print(f"  {st}", flush=True)
        assert st["compared"] > 0.95 * q.num_points


def _on_curve_points(faces, n, seed):
    """n points on the curves of a planar face set (random segment, t ~ U[0,1])."""
    rng = np.random.default_rng(seed)
    seg = rng.integers(0, faces.num_segments, n)
    t = rng.uniform(0, 1, n)
    out = np.empty((n, 2))
    for s in np.unique(seg):
        m = seg == s
        a, b = faces.seg_cp_offsets[s], faces.seg_cp_offsets[s + 1]
        cp = np.column_stack([faces.cp_u[a:b], faces.cp_v[a:b]])
        w = None if faces.cp_w is None else faces.cp_w[a:b]
        out[m] = W.eval_rational_bezier(cp, w, t[m])
    return out


def _sweep(torch, faces, u, v, eps_list):
    from paper_2510_25159_amd import wn

    dev = torch.device("cuda:0")
    tu, tv = torch.from_numpy(u).to(dev), torch.from_numpy(v).to(dev)
    n = len(u)
    offs = torch.tensor([0, n], dtype=torch.int64, device=dev)
    rows = []
    for eps in eps_list:
        fs = wn.FaceSet(faces, eps=eps)
        stats = torch.zeros(wn.STATS_COUNT, dtype=torch.int64, device=dev)
        _, lab = fs.query(tu, tv, offs, np.array([0, n]), schedule=1, stats=stats)
        torch.cuda.synchronize()
        st = dict(zip(wn.STAT_NAMES, stats.cpu().numpy().tolist()))
        lab = lab.cpu().numpy()
        rows.append({"eps": eps, "splits_per_point": st["splits"] / n, "leaves_per_point": st["leaves"] / n,
                     "near_pairs_per_point": st["near_pairs"] / n, "on_boundary": int(np.sum(lab == 2)),
                     "max_depth": st["max_depth"]})
        print(rows[-1], flush=True)
    return rows


def test_eps_sweep_table3(torch_cuda):
    """Curve evaluations (Alg. 1 splits, one curve point each) per point over
    the sweep of Table 3, on 2^17 points sampled on the curve and 2^17
    uniform points of config 1's face."""
    torch = torch_cuda
    faces = W.config1_faces()
    n = 1 << 17
    pts = _on_curve_points(faces, n, seed=8)
    rows_b = _sweep(torch, faces, pts[:, 0].copy(), pts[:, 1].copy(), SWEEP)
    q = W.config1_queries(seed=9, n=n)
    rows_u = _sweep(torch, faces, q.u, q.v, SWEEP)
    x = np.log10(1.0 / np.array(SWEEP))
    yb = np.array([r["splits_per_point"] for r in rows_b])
    yu = np.array([r["splits_per_point"] for r in rows_u])
    slope, icpt = np.polyfit(x, yb, 1)
    resid = yb - (slope * x + icpt)
    r2 = 1 - np.sum(resid ** 2) / np.sum((yb - yb.mean()) ** 2)
    print(f"on-curve points: {slope:.2f} evaluations per decade of 1/eps (R^2 {r2:.4f}); "
          f"uniform points: {yu.min():.4f}..{yu.max():.4f} per point", flush=True)
    assert np.all(np.diff(yb) > 0)
    assert 2.0 < slope < 40.0 and r2 > 0.99
    # every on-curve point is reported on-boundary at every eps
    assert all(r["on_boundary"] == n for r in rows_b)
    # uniform points: flat (the near pairs of points that are not on a curve
    # do not depend on eps once eps is below their distance)
    assert yu.max() <= 1.05 * yu.min() + 1e-3


def test_on_boundary_fraction(torch_cuda, oracle_lib):
    """2^20 uniform points against config 1's face: the reported on-boundary
    set lies within eps of the curve (oracle), and its size follows
    2 eps x perimeter / area."""
    torch = torch_cuda
    faces = W.config1_faces()
    n = 1 << 20
    q = W.config1_queries(seed=12, n=n)
    # perimeter of the loop (dense sampling of every segment)
    t = np.linspace(0, 1, 2001)
    per = 0.0
    for s in range(faces.num_segments):
        a, b = faces.seg_cp_offsets[s], faces.seg_cp_offsets[s + 1]
        p = W.eval_rational_bezier(np.column_stack([faces.cp_u[a:b], faces.cp_v[a:b]]), None, t)
        per += float(np.sum(np.hypot(*np.diff(p, axis=0).T)))
    area = 9.0  # [-1.5, 1.5]^2
    fr = []
    for eps in (1e-3, 1e-4, 1e-6, 1e-8, 1e-10):
        w, lab = run_wn(faces, q, schedule=1, create={"eps": eps})
        onb = lab == 2
        fr.append(onb.mean())
        expect = 2 * eps * per / area
        print(f"eps={eps:g}: on-boundary {int(onb.sum())} of {n} ({onb.mean():.3e}; band estimate {expect:.3e})",
              flush=True)
        if eps >= 1e-4:
            assert 0.2 * expect <= onb.mean() <= 1.1 * expect
        if eps >= 1e-6:
            # the reported points lie within eps of the curve
            idx = np.nonzero(onb)[0]
            if len(idx):
                pf, u, v = W.subset_queries(q, idx)
                _, near = oracle_lib.query(faces, pf, u, v, near_tol=eps * (1 + 1e-9))
                assert np.all(near == 1)
    assert all(a >= b for a, b in zip(fr, fr[1:]))
    assert fr[-1] == 0.0
