"""Torus pairing on the GPU (Sec. 4.5, App. C): the pair tables the one-wave
pairing kernel builds at creation equal the host pairing's (WN_FLAG_HOST_PAIRING,
the same rule), loop by loop and shift by shift, on config 3's tori (one pair,
homologies up to (5, 5)), tori with three pairs of a (2, 3) homology, and a
torus with two pairs and a hole; the queries on the GPU-paired faces then match
the oracle, which pairs on its own."""
import numpy as np
import pytest

from paper_2510_25159_amd import workloads as W
from tests.gpu_helpers import compare, run_wn, translation_tol
from tests.test_gpu_periodic import T, _band_loops, _circle_segs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_25159_amd import wn

    wn.lib()
    return torch


def _tables(fs, faces):
    out = {}
    for f in range(faces.num_faces):
        if int(faces.face_domain[f]) == W.DOMAIN_TORUS:
            out[f] = fs.torus_pairs(f)
    return out


def _same_tables(faces):
    from paper_2510_25159_amd import wn

    g = _tables(wn.FaceSet(faces), faces)
    h = _tables(wn.FaceSet(faces, flags=wn.FLAG_HOST_PAIRING), faces)
    assert g.keys() == h.keys()
    npairs = 0
    for f in g:
        (ag, bg, sg), (ah, bh, sh) = g[f], h[f]
        assert np.array_equal(ag, ah), f"face {f}: alpha {ag} vs {ah}"
        assert np.array_equal(bg, bh), f"face {f}: beta {bg} vs {bh}"
        assert np.array_equal(sg, sh), f"face {f}: shifts {sg} vs {sh}"
        npairs += len(ag)
    return len(g), npairs


def _multi_pair_torus(rng, npairs, vec, nrm, width, gap):
    """npairs bands along vec, their lower loops gap apart along the normal."""
    loops = []
    for i in range(npairs):
        loops += _band_loops(rng, vec, np.array([0.2, 0.3]) + i * gap * nrm, width, nrm, amp=0.02)
    return loops


def test_pair_tables_match_host_config3(torch_cuda):
    faces, _ = W.config3()
    nt, npairs = _same_tables(faces)
    print(f"config3: {nt} torus faces, {npairs} pairs, tables identical", flush=True)
    assert nt == 256 and npairs >= 256


def test_pair_tables_match_host_multi_pair_and_holed(torch_cuda, oracle_lib):
    rng = np.random.default_rng(41)
    # three pairs of (2, 3) loops: the normal of h* = (2T, 3T), band width well
    # below the family spacing T^2 / |(2T, 3T)|
    v = np.array([2 * T, 3 * T])
    n = np.array([-v[1], v[0]]) / np.hypot(*v)
    delta = T * T / np.hypot(*v)
    tri = _multi_pair_torus(rng, 3, v, n, 0.12 * delta, 0.3 * delta)
    # two pairs of (1, 0) loops and a hole inside the first band
    nrm = np.array([0.0, 1.0])
    p1 = _band_loops(rng, np.array([T, 0.0]), np.array([0.3, 0.5]), 1.0, nrm)
    p2 = _band_loops(rng, np.array([T, 0.0]), np.array([1.1, 3.5]), 1.1, nrm, amp=0.05)
    thole = [_circle_segs((4.0, 1.0), 0.3, W.DOMAIN_TORUS, cw=True)]
    faces = W.faces_from_loops([tri, p1 + p2 + thole], domains=[W.DOMAIN_TORUS, W.DOMAIN_TORUS],
                               periods=[[T, T], [T, T]])
    nt, npairs = _same_tables(faces)
    print(f"multi-pair / holed tori: {nt} faces, {npairs} pairs, tables identical", flush=True)
    assert nt == 2 and npairs == 5
    P = [rng.uniform(-T, 2 * T, (5000, 2)) for _ in range(2)]
    q = W.queries_for_faces(P)
    w_o, n_o = oracle_lib.query_faces(faces, q)
    pf = q.face_ids()
    for sched in (1, 0):
        w, lab = run_wn(faces, q, schedule=sched)
        st = compare(w, lab, w_o, n_o, tol_fn=lambda i: translation_tol(oracle_lib, faces, pf, q.u, q.v, i))
        assert st["compared"] > 0.97 * q.num_points
