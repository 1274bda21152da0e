"""The subdivided control-point bound variant of the near pass
(WN_BOUND_SUBDIVIDED; Sec. 4.2 / Table 1 contrast control-point bounds with the
ellipse bound): a node's axis is the smaller of B 2^-k and the bound of its
own de Casteljau control points.

  * omega and labels: the oracle's, and the global bound's (the bound never
    changes the answer);
  * depths pair by pair, and split / leaf totals, against the oracle's
    recursive mirror of the same variant (oracle.alg1_pairs(cp_bound=True)),
    except where a node's test lies within rounding of its bound;
  * it splits no more than the global bound, on the same pairs.
"""
import numpy as np
import pytest

from paper_2510_25159_amd import workloads as W
from tests.gpu_helpers import compare

pytestmark = pytest.mark.gpu

EPS = 1e-10
BORDER_REL = 1e-11
BORDER_ABS = 1e-12


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_25159_amd import wn

    wn.lib()
    return torch


def _dev(torch, a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to("cuda:0")


def _sets():
    f4, q4 = W.config4("eval", near_frac=0.3)
    f2, q2 = W.config2(face_ids=range(16))
    return [("config4 near30", f4, q4), ("config2[0:16]", f2, q2)]


@pytest.mark.parametrize("which", [0, 1])
def test_cp_bound_parity_and_depths(torch_cuda, oracle_lib, which):
    torch = torch_cuda
    from paper_2510_25159_amd import wn

    tag, faces, q = _sets()[which]
    fs = wn.FaceSet(faces, eps=EPS)
    u, v = _dev(torch, q.u, np.float64), _dev(torch, q.v, np.float64)
    offs = _dev(torch, q.face_point_offsets, np.int64)
    # results: the oracle's, and equal to the global bound's
    w0, l0 = fs.query(u, v, offs, None, schedule=wn.SCHED_BATCHED)
    w1, l1 = fs.query(u, v, offs, None, schedule=wn.SCHED_BATCHED, bound=wn.BOUND_SUBDIVIDED)
    torch.cuda.synchronize()
    w0, l0, w1, l1 = w0.cpu().numpy(), l0.cpu().numpy(), w1.cpu().numpy(), l1.cpu().numpy()
    w_o, n_o = oracle_lib.query_faces(faces, q)
    st = compare(w1, l1, w_o, n_o)
    assert st["compared"] > 0.9 * q.num_points
    assert np.array_equal(l0, l1)
    fin = np.isfinite(w0)
    assert np.max(np.abs(w0[fin] - w1[fin])) <= 1e-12
    # depths pair by pair against the oracle's mirror of the variant
    pp, ps, pd, _ = wn.near_pairs(fs, u, v, offs, capacity=8 * q.num_points, bound=wn.BOUND_SUBDIVIDED)
    pp, ps, pd = pp.cpu().numpy(), ps.cpu().numpy(), pd.cpu().numpy()
    rng = np.random.default_rng(11)
    idx = np.sort(rng.choice(len(pp), min(len(pp), 20000), replace=False))
    pp, ps, pd = pp[idx], ps[idx], pd[idx]
    o = oracle_lib.alg1_pairs(faces, ps, q.u[pp], q.v[pp], eps=EPS, cp_bound=True)
    g = oracle_lib.alg1_pairs(faces, ps, q.u[pp], q.v[pp], eps=EPS)
    border = (o["margin_rel"] < BORDER_REL) | (o["margin_abs"] < BORDER_ABS)
    use = ~o["onb"] & ~border
    diff = int(np.sum(pd[use] != o["depth"][use]))
    print(f"{tag}: {len(pp)} pairs, {int(use.sum())} compared, {int(border.sum())} borderline, {diff} differences; "
          f"mean depth control-point {o['depth'][use].mean():.3f} vs global {g['depth'][use].mean():.3f}, "
          f"splits {int(o['splits'][use].sum())} vs {int(g['splits'][use].sum())}", flush=True)
    assert diff == 0
    assert border.sum() <= max(1, 1e-4 * len(pp))
    assert np.all(o["depth"][use] <= g["depth"][use]) and np.all(o["splits"][use] <= g["splits"][use])


def test_cp_bound_work_counters(torch_cuda, oracle_lib):
    """Split and leaf totals of the variant's near pass (WN_STAT_SPLITS /
    WN_STAT_LEAVES) on config 4's near30 set against the mirror's, and below
    the global bound's."""
    torch = torch_cuda
    from paper_2510_25159_amd import wn

    faces, q = W.config4("eval", near_frac=0.3)
    fs = wn.FaceSet(faces, eps=EPS)
    u, v = _dev(torch, q.u, np.float64), _dev(torch, q.v, np.float64)
    offs = _dev(torch, q.face_point_offsets, np.int64)
    pp, ps, _, _ = wn.near_pairs(fs, u, v, offs, capacity=8 * q.num_points, bound=wn.BOUND_SUBDIVIDED)
    pp, ps = pp.cpu().numpy(), ps.cpu().numpy()
    stats = {}
    for b in (wn.BOUND_GLOBAL, wn.BOUND_SUBDIVIDED):
        s = torch.zeros(wn.STATS_COUNT, dtype=torch.int64, device="cuda:0")
        fs.query(u, v, offs, None, schedule=1, stats=s, bound=b)
        torch.cuda.synchronize()
        stats[b] = dict(zip(wn.STAT_NAMES, s.cpu().numpy().tolist()))
    o = oracle_lib.alg1_pairs(faces, ps, q.u[pp], q.v[pp], eps=EPS, cp_bound=True)
    border = (o["margin_rel"] < BORDER_REL) | (o["margin_abs"] < BORDER_ABS)
    slack = int(o["splits"][border].sum() + o["leaves"][border].sum()) + 2 * int(border.sum())
    st = stats[wn.BOUND_SUBDIVIDED]
    print(f"splits gpu {st['splits']} oracle {int(o['splits'].sum())} global {stats[wn.BOUND_GLOBAL]['splits']}; "
          f"leaves gpu {st['leaves']} oracle {int(o['leaves'].sum())}; borderline {int(border.sum())}", flush=True)
    assert st["near_pairs"] == len(pp)
    assert abs(st["splits"] - int(o["splits"].sum())) <= slack
    assert abs(st["leaves"] - int(o["leaves"].sum())) <= slack
    assert st["splits"] < stats[wn.BOUND_GLOBAL]["splits"]
