"""Depth parity: the depths the GPU's near pass records (the training labels
of the learned predictor and the measured bin source) against the oracle's
recursive mirror of Alg. 1 (Sec. 4.1, sub-segment bound of Sec. 4.2).

Both the batched near pass (k_near, through wn_near_pairs) and the plain
schedule's in-line recursion (depth_log) are checked pair by pair on sampled
near pairs of config 4 (uniform queries and the 30 % near-curve variant) and
of a config 2 subset (rational segments of degree 1-5).  Depths must be equal
except where some node's ellipse test lies within rounding of its bound
(`borderline`): the GPU inflates each axis by 2^-40 relative plus a few ulps
of the face's scale, and evaluates curve points with another formula.  The
borderline count is reported and must stay below 1e-4 of the pairs.
"""
import numpy as np
import pytest

from paper_2510_25159_amd import workloads as W

pytestmark = pytest.mark.gpu

EPS = 1e-10
BORDER_REL = 1e-11   # relative margin of a node test (GPU inflation 2^-40 = 9.1e-13)
BORDER_ABS = 1e-12   # absolute margin (a few ulps of coordinates of size ~2)


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


def _check(oracle_lib, faces, q, pp, ps, dg, tag):
    o = oracle_lib.alg1_pairs(faces, ps, q.u[pp], q.v[pp], eps=EPS)
    border = (o["margin_rel"] < BORDER_REL) | (o["margin_abs"] < BORDER_ABS)
    use = ~o["onb"] & ~border
    diff = int(np.sum(dg[use] != o["depth"][use]))
    print(f"{tag}: {len(pp)} pairs, {int(use.sum())} compared, {int(border.sum())} borderline, "
          f"{int(o['onb'].sum())} on-boundary, depth range {o['depth'].min()}-{o['depth'].max()}, "
          f"{diff} differences", flush=True)
    assert diff == 0, f"{tag}: {diff} depth differences"
    assert border.sum() <= max(1, 1e-4 * len(pp)), f"{tag}: {int(border.sum())} borderline pairs"
    return o


@pytest.mark.parametrize("variant,near", [("uniform", 0.0), ("near30", 0.3)])
def test_near_pass_depths_config4(torch_cuda, oracle_lib, variant, near):
    torch = torch_cuda
    from paper_2510_25159_amd import wn

    faces, q = W.config4("eval", near_frac=near)
    fs = wn.FaceSet(faces, eps=EPS)
    u, v = _dev(torch, q.u, np.float64), _dev(torch, q.v, np.float64)
    offs = _dev(torch, q.face_point_offsets, np.int64)
    pp, ps, pd, _ = wn.near_pairs(fs, u, v, offs, capacity=8 * q.num_points)
    pp, ps, pd = pp.cpu().numpy(), ps.cpu().numpy(), pd.cpu().numpy()
    assert len(pp) > 500
    # every near pair (uniform) or a seeded sample of 20,000 (near30)
    rng = np.random.default_rng(4)
    idx = np.arange(len(pp)) if len(pp) <= 20000 else np.sort(rng.choice(len(pp), 20000, replace=False))
    o = _check(oracle_lib, faces, q, pp[idx], ps[idx], pd[idx], f"k_near config4 {variant}")
    # the root test failed on every queued pair: the oracle's depth is >= 1 there
    ok = ~o["onb"]
    assert np.all(o["depth"][ok] >= 1)


def test_near_pass_depths_config2_subset(torch_cuda, oracle_lib):
    torch = torch_cuda
    from paper_2510_25159_amd import wn

    faces, q = W.config2(face_ids=range(24))
    fs = wn.FaceSet(faces, eps=EPS)
    u, v = _dev(torch, q.u, np.float64), _dev(torch, q.v, np.float64)
    offs = _dev(torch, q.face_point_offsets, np.int64)
    pp, ps, pd, _ = wn.near_pairs(fs, u, v, offs, capacity=8 * q.num_points)
    pp, ps, pd = pp.cpu().numpy(), ps.cpu().numpy(), pd.cpu().numpy()
    rng = np.random.default_rng(5)
    idx = np.sort(rng.choice(len(pp), min(len(pp), 20000), replace=False))
    _check(oracle_lib, faces, q, pp[idx], ps[idx], pd[idx], "k_near config2 subset")


def test_near_pass_work_counters_match_oracle(torch_cuda, oracle_lib):
    """Splits and leaves summed over every near pair of config 4's near30 set
    (WN_STAT_SPLITS / WN_STAT_LEAVES of the batched schedule) against the
    mirror's counts summed over the same pairs."""
    torch = torch_cuda
    from paper_2510_25159_amd import wn

    faces, q = W.config4("eval", near_frac=0.3)
    fs = wn.FaceSet(faces, eps=EPS)
    u, v = _dev(torch, q.u, np.float64), _dev(torch, q.v, np.float64)
    offs = _dev(torch, q.face_point_offsets, np.int64)
    pp, ps, pd, _ = wn.near_pairs(fs, u, v, offs, capacity=8 * q.num_points)
    pp, ps = pp.cpu().numpy(), ps.cpu().numpy()
    stats = torch.zeros(wn.STATS_COUNT, dtype=torch.int64, device="cuda:0")
    fs.query(u, v, offs, None, schedule=1, stats=stats)
    torch.cuda.synchronize()
    st = dict(zip(wn.STAT_NAMES, stats.cpu().numpy().tolist()))
    o = oracle_lib.alg1_pairs(faces, ps, q.u[pp], q.v[pp], eps=EPS)
    assert st["near_pairs"] == len(pp)
    assert not o["onb"].any()  # no point of this set lies within 1e-10 of the curve
    border = (o["margin_rel"] < BORDER_REL) | (o["margin_abs"] < BORDER_ABS)
    slack = int(o["splits"][border].sum() + o["leaves"][border].sum()) + 2 * int(border.sum())
    print(f"splits gpu {st['splits']} oracle {int(o['splits'].sum())}; leaves gpu {st['leaves']} "
          f"oracle {int(o['leaves'].sum())}; borderline pairs {int(border.sum())}", flush=True)
    assert abs(st["splits"] - int(o["splits"].sum())) <= slack
    assert abs(st["leaves"] - int(o["leaves"].sum())) <= slack
    assert st["max_depth"] == int(o["depth"].max())


def test_plain_depth_log_config4(torch_cuda, oracle_lib):
    """The plain schedule's in-line recursion logs every (point, segment)
    pair: depth 0 where the root test passed, Alg. 1's depth elsewhere."""
    torch = torch_cuda
    from paper_2510_25159_amd import wn

    faces, q = W.config4("eval", near_frac=0.3)
    n = 40000
    fs = wn.FaceSet(faces, eps=EPS)
    info = fs.info()
    S = info.max_segments_per_face
    u, v = _dev(torch, q.u[:n], np.float64), _dev(torch, q.v[:n], np.float64)
    offs = _dev(torch, [0, n], np.int64)
    dl = torch.zeros(n * S, dtype=torch.uint8, device="cuda:0")
    _, lab = fs.query(u, v, offs, np.array([0, n]), schedule=0, depth_log=dl)
    d = dl.cpu().numpy().reshape(n, S)
    lab = lab.cpu().numpy()
    rng = np.random.default_rng(6)
    # all pairs that recursed, plus as many sampled root pairs
    pts, segs = np.nonzero(d > 0)
    keep = lab[pts] != 2
    pts, segs = pts[keep], segs[keep]
    if len(pts) > 15000:
        k = np.sort(rng.choice(len(pts), 15000, replace=False))
        pts, segs = pts[k], segs[k]
    rp = rng.integers(0, n, 15000)
    rs = rng.integers(0, S, 15000)
    pp = np.concatenate([pts, rp])
    ps = np.concatenate([segs, rs]).astype(np.int32)
    ok = lab[pp] != 2
    pp, ps = pp[ok], ps[ok]
    _check(oracle_lib, faces, q, pp, ps, d[pp, ps], "plain depth_log config4 near30")
