"""wn_query_noalloc (the batched query on the library's fixed device scratch)
against wn_query_ex on the same handle and points, two calls in a row with
the second on a smaller input: labels identical, winding within 1e-12, both
also against the oracle.  A planar set (30 % of the points near curves), the
same set under the path hierarchy (its spatial order in the scratch), a
periodic set (cylinders and tori: spatial order and queue shifts in the
scratch), and the limits the entry point rejects."""
import numpy as np
import pytest

from paper_2510_25159_amd import workloads as W
from tests.gpu_helpers import FP64_TOL, compare, translation_tol

pytestmark = pytest.mark.gpu


def _sub(q, keep_every):
    """Every keep_every-th point of each face (offsets recomputed)."""
    fid = q.face_ids()
    idx = np.flatnonzero((np.arange(q.num_points) % keep_every) == 0)
    counts = np.bincount(fid[idx], minlength=len(q.face_point_offsets) - 1)
    offs = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return W.Queries(q.u[idx].copy(), q.v[idx].copy(), offs)


def _run_both(fs, q, **opts):
    import torch

    from paper_2510_25159_amd import wn

    dev = torch.device("cuda:0")
    u = torch.from_numpy(q.u).to(dev)
    v = torch.from_numpy(q.v).to(dev)
    offs = torch.from_numpy(q.face_point_offsets).to(dev)
    n = q.num_points
    w_ref, l_ref = fs.query(u, v, offs, q.face_point_offsets, schedule=wn.SCHED_BATCHED, **opts)
    w_na = torch.full((n,), float("nan"), dtype=torch.float64, device=dev)
    l_na = torch.full((n,), 255, dtype=torch.uint8, device=dev)
    fs.query_noalloc(u, v, offs, w_na, l_na, **opts)
    torch.cuda.synchronize()
    return (w_ref.cpu().numpy(), l_ref.cpu().numpy(), w_na.cpu().numpy(), l_na.cpu().numpy())


def _check(oracle_lib, faces, q, res):
    w_ref, l_ref, w_na, l_na = res
    assert np.array_equal(l_na, l_ref), f"{int(np.sum(l_na != l_ref))} labels differ from wn_query_ex"
    fin = np.isfinite(w_ref)
    assert np.array_equal(fin, np.isfinite(w_na))
    assert np.max(np.abs(w_na[fin] - w_ref[fin]), initial=0.0) <= FP64_TOL
    w_o, n_o = oracle_lib.query_faces(faces, q)
    pf = q.face_ids()
    st = compare(w_na, l_na, w_o, n_o, tol_fn=lambda i: translation_tol(oracle_lib, faces, pf, q.u, q.v, i))
    assert st["compared"] > 0.5 * q.num_points


@pytest.mark.parametrize("kind", ["planar", "planar_hierarchy", "periodic"])
def test_noalloc_matches_query_ex_twice(oracle_lib, kind):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_25159_amd import wn

    opts = {"path_hierarchy": 1} if kind == "planar_hierarchy" else {}
    if kind.startswith("planar"):
        faces, q = W.config2(face_ids=range(24))
    else:
        faces, q = W.config3(face_ids=range(64))
    fs = wn.FaceSet(faces)
    q_small = _sub(q, 3)
    print(f"{kind}: {faces.num_faces} faces, calls of {q.num_points} then {q_small.num_points} points", flush=True)
    assert q.num_points <= wn.NOALLOC_MAX_POINTS
    _check(oracle_lib, faces, q, _run_both(fs, q, **opts))
    _check(oracle_lib, faces, q_small, _run_both(fs, q_small, **opts))


def test_noalloc_rejects_out_of_range():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_25159_amd import wn

    faces, q = W.config1()
    fs = wn.FaceSet(faces)
    dev = torch.device("cuda:0")
    u = torch.zeros(8, dtype=torch.float64, device=dev)
    offs = torch.tensor([0, 8], dtype=torch.int64, device=dev)
    w = torch.empty(8, dtype=torch.float64, device=dev)
    lab = torch.empty(8, dtype=torch.uint8, device=dev)
    with pytest.raises(wn.WnError) as ei:
        fs.query_noalloc(u, u, offs, w, lab, schedule=wn.SCHED_PLAIN)
    assert ei.value.status == wn.WN_E_UNSUPPORTED
    assert wn.lib().wn_query_noalloc_scratch_bytes() == 64 << 20
    # more points than the limit: rejected on the host before anything is launched
    p = wn.wn_points(wn.NOALLOC_MAX_POINTS + 1, u.data_ptr(), u.data_ptr(), 1, offs.data_ptr(), None)
    q = wn._query_opts()
    import ctypes

    st = wn.lib().wn_query_noalloc(fs._h, ctypes.byref(p), w.data_ptr(), lab.data_ptr(), ctypes.byref(q), None)
    assert st == wn.WN_E_INVALID
    fs.query_noalloc(u, u, offs, w, lab)
    torch.cuda.synchronize()
    assert np.all(lab.cpu().numpy() == wn.INSIDE)  # the star r >= 0.7 around the origin contains it
