"""Boundary degree on the GPU (Sec. 5: cubic curves elevated to higher degree
without changing the geometry, test points sampled on the boundary as the
worst case of the recursion).

  * At degree 3, 4 and 5 the GPU matches the oracle (labels, omega within
    1e-12 away from the curves), and every point sampled on the curve is
    reported on the boundary.
  * Elevation does not change the curve, so the labels are equal across the
    degrees and omega agrees to FP64 rounding at every other point.
  * The recursion's work per on-curve point (splits) stays within a small
    factor across the degrees: Lemma 1's bound of the elevated control
    polygon differs from the cubic's by a bounded factor, and the depth grows
    with log2(B / eps) only.
"""
import numpy as np
import pytest

from paper_2510_25159_amd import workloads as W
from tests.gpu_helpers import compare, run_wn

pytestmark = pytest.mark.gpu

FACES, PPF = 16, 4096


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_25159_amd import wn

    wn.lib()
    return torch


def test_degree_elevation_parity_and_invariance(torch_cuda, oracle_lib):
    torch = torch_cuda
    from paper_2510_25159_amd import wn

    out = {}
    for d in (3, 4, 5):
        faces, q = W.degree_set(d, num_faces=FACES, points_per_face=PPF)
        assert np.all(np.diff(faces.seg_cp_offsets) == d + 1)
        fs = wn.FaceSet(faces)
        s = torch.zeros(wn.STATS_COUNT, dtype=torch.int64, device="cuda:0")
        w, lab = run_wn(faces, q, faceset=fs, schedule=1, stats=s)
        stats = dict(zip(wn.STAT_NAMES, s.cpu().numpy().tolist()))
        w_o, n_o = oracle_lib.query_faces(faces, q)
        st = compare(w, lab, w_o, n_o)
        fid = q.face_ids()
        local = np.arange(q.num_points) - q.face_point_offsets[fid]
        on_curve = local < PPF // 2
        assert np.all(lab[on_curve] == 2), f"degree {d}: {int(np.sum(lab[on_curve] != 2))} on-curve points not flagged"
        print(f"degree {d}: compared {st['compared']}, max err {st['max_abs_err']:.2e}, splits {stats['splits']}, "
              f"leaves {stats['leaves']}, near pairs {stats['near_pairs']}, max depth {stats['max_depth']}", flush=True)
        out[d] = (w, lab, stats)
    w3, l3, s3 = out[3]
    for d in (4, 5):
        w, lab, s = out[d]
        assert np.array_equal(lab, l3), f"degree {d}: {int(np.sum(lab != l3))} labels differ from the cubic's"
        fin = np.isfinite(w3) & np.isfinite(w)
        assert np.array_equal(fin, np.isfinite(w3))
        assert np.max(np.abs(w[fin] - w3[fin])) <= 1e-12
        assert 0.25 * s3["splits"] <= s["splits"] <= 4.0 * s3["splits"]
