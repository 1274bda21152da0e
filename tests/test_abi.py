"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/wn.h, validates descriptors on the host, and its host
derivative bound B dominates sampled |gamma'(t)| (Lemma 1, App. A.1)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2510_25159_amd import wn
from paper_2510_25159_amd import workloads as W
from tests import curves as C

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "wn.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wn_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    L = wn.lib()
    names = declared_functions()
    assert len(names) >= 10
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(wn.EXPORTS) <= set(names)


def test_status_strings():
    for s in range(7):
        assert len(wn.status_string(s)) > 0


def _desc(faces):
    keep = dict(
        flo=np.ascontiguousarray(faces.face_loop_offsets, dtype=np.int32),
        lso=np.ascontiguousarray(faces.loop_seg_offsets, dtype=np.int32),
        sco=np.ascontiguousarray(faces.seg_cp_offsets, dtype=np.int64),
        cu=np.ascontiguousarray(faces.cp_u), cv=np.ascontiguousarray(faces.cp_v),
        cw=None if faces.cp_w is None else np.ascontiguousarray(faces.cp_w),
        dom=np.ascontiguousarray(faces.face_domain, dtype=np.int32),
        per=np.ascontiguousarray(faces.face_period))
    p = lambda a: None if a is None else a.ctypes.data_as(ctypes.c_void_p)
    d = wn.wn_faces_desc(len(keep["flo"]) - 1, len(keep["lso"]) - 1, len(keep["sco"]) - 1, len(keep["cu"]),
                         p(keep["flo"]), p(keep["lso"]), p(keep["sco"]), p(keep["cu"]), p(keep["cv"]), p(keep["cw"]),
                         p(keep["dom"]), p(keep["per"]))
    return d, keep


def _create_status(faces, **opt):
    d, keep = _desc(faces)
    o = wn.default_options(**opt)
    h = ctypes.c_void_p()
    st = wn.lib().wn_create_faces(ctypes.byref(d), ctypes.byref(o), None, ctypes.byref(h))
    if st == wn.WN_OK:
        wn.lib().wn_destroy_faces(h)
    return st


def test_host_validation_errors():
    good = W.faces_from_loops([[C.circle_arcs(1.0)]])
    bad_deg = W.faces_from_loops([[[(np.zeros((7, 2)), None)]]])
    assert _create_status(bad_deg) == wn.WN_E_INVALID
    nan = W.faces_from_loops([[C.circle_arcs(1.0)]])
    nan.cp_u = nan.cp_u.copy()
    nan.cp_u[3] = np.nan
    assert _create_status(nan) == wn.WN_E_INVALID
    negw = W.faces_from_loops([[C.circle_arcs(1.0)]])
    negw.cp_w = negw.cp_w.copy()
    negw.cp_w[1] = -1.0
    assert _create_status(negw) == wn.WN_E_INVALID
    brk = W.faces_from_loops([[C.circle_arcs(1.0)]])
    brk.loop_seg_offsets = np.array([0, 5], dtype=np.int32)  # more segments than exist
    assert _create_status(brk) == wn.WN_E_INVALID
    assert _create_status(good, eps=0.0) == wn.WN_E_INVALID
    assert _create_status(good, eps=1e-20) == wn.WN_E_INVALID
    assert _create_status(good, stack_cap=99) == wn.WN_E_INVALID


def test_depth_cap_rejects_tiny_eps_on_large_segments():
    big = W.faces_from_loops([[C.circle_arcs(1e6)]])
    # log2(B/eps) + 3 > 52 for B ~ 4e6, eps = 1e-12
    assert _create_status(big, eps=1e-12) == wn.WN_E_DEPTH


def test_segment_bound_dominates_sampled_derivative():
    """B >= max |gamma'(t)| for non-rational (hodograph) and rational
    (min of the two Floater bounds) segments, on random segments."""
    rng = np.random.default_rng(3)
    t = np.linspace(0, 1, 801)
    for trial in range(300):
        n = int(rng.integers(1, 6))
        cp = rng.uniform(-1, 1, (n + 1, 2))
        w = None if trial % 2 == 0 else rng.uniform(0.2, 5.0, n + 1)
        B = wn.segment_bound(cp, w)
        d = C.eval_deriv(cp, w, t)
        assert np.max(np.hypot(d[:, 0], d[:, 1])) <= B * (1 + 1e-12)


def test_segment_bound_closed_forms():
    # straight cubic with uniform speed: B = |P3 - P0| exactly (n * |dP| = 3 * L/3)
    cp = np.array([[0, 0], [1, 0], [2, 0], [3, 0]], dtype=float)
    assert wn.segment_bound(cp) == pytest.approx(3.0, rel=1e-15)
    # quadratic: 2 * max |dP|
    assert wn.segment_bound([[0, 0], [1, 1], [3, 1]]) == pytest.approx(4.0, rel=1e-15)
    with pytest.raises(wn.WnError):
        wn.segment_bound(np.zeros((7, 2)))
    with pytest.raises(wn.WnError):
        wn.segment_bound([[0, 0], [1, 0]], [1.0, 0.0])
