"""CPU oracle (test infrastructure only).

Plain C11 + pthreads in ``wn_oracle.c``; this module compiles it with gcc
and exposes it through ctypes.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it.  It shares no code with the HIP
library and does not import the ``paper_2510_25159_amd`` package.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["wn_oracle.c", "wn_oracle_core.inc", "wn_oracle_periodic.inc", "wn_oracle_alg1.inc"]
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no HIP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-o", tmp,
               os.path.join(_HERE, "wn_oracle.c"), "-lpthread", "-lm"]
        subprocess.run(cmd, check=True, cwd=_HERE)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.wno_query.restype = ctypes.c_int
        lib.wno_query.argtypes = [ctypes.c_int32, P, ctypes.c_int32, P, ctypes.c_int32, P, P, P, P, P, P,
                                  ctypes.c_int64, P, P, P, ctypes.c_double, ctypes.c_int32, ctypes.c_int32, P, P]
        lib.wno_set_periodic_options.argtypes = [ctypes.c_int32, ctypes.c_int32]
        lib.wno_segment_winding.restype = ctypes.c_double
        lib.wno_segment_winding.argtypes = [P, P, P, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_int32, P]
        lib.wno_alg1_pairs.restype = ctypes.c_int
        lib.wno_alg1_pairs.argtypes = [ctypes.c_int32, P, P, P, P, ctypes.c_int64, P, P, P, ctypes.c_double,
                                       ctypes.c_int32, ctypes.c_int32, P]
        lib.wno_alg1_bound.restype = ctypes.c_double
        lib.wno_alg1_bound.argtypes = [P, P, P, ctypes.c_int32]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    pass


def query(faces, point_face, u, v, near_tol: float = 1e-9, nthreads: int | None = None,
          long_double: bool = False):
    """Winding number and certified near flag for each point.

    ``faces`` is any object with the CSR attributes of
    ``paper_2510_25159_amd.workloads.Faces``; ``point_face[i]`` names the face
    of point i.  Returns (omega float64 [N], near int8 [N])."""
    lib = _load()
    flo = np.ascontiguousarray(faces.face_loop_offsets, dtype=np.int32)
    lso = np.ascontiguousarray(faces.loop_seg_offsets, dtype=np.int32)
    sco = np.ascontiguousarray(faces.seg_cp_offsets, dtype=np.int64)
    cu = np.ascontiguousarray(faces.cp_u, dtype=np.float64)
    cv = np.ascontiguousarray(faces.cp_v, dtype=np.float64)
    cw = None if faces.cp_w is None else np.ascontiguousarray(faces.cp_w, dtype=np.float64)
    dom = np.ascontiguousarray(faces.face_domain, dtype=np.int32)
    per = np.ascontiguousarray(faces.face_period, dtype=np.float64)
    pf = np.ascontiguousarray(point_face, dtype=np.int32)
    pu = np.ascontiguousarray(u, dtype=np.float64)
    pv = np.ascontiguousarray(v, dtype=np.float64)
    n = len(pu)
    out_w = np.empty(n, dtype=np.float64)
    out_n = np.empty(n, dtype=np.int8)
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    st = lib.wno_query(len(flo) - 1, _ptr(flo), len(lso) - 1, _ptr(lso), len(sco) - 1, _ptr(sco), _ptr(cu),
                       _ptr(cv), _ptr(cw), _ptr(dom), _ptr(per), n, _ptr(pf), _ptr(pu), _ptr(pv),
                       float(near_tol), int(nthreads), 1 if long_double else 0, _ptr(out_w), _ptr(out_n))
    if st != 0:
        raise OracleError(f"oracle returned status {st}")
    return out_w, out_n


def set_periodic_options(extra: int = 0, disable_pairing: bool = False):
    """Widen periodic windows by ``extra`` copies/families; optionally disable
    the nearest-left pairing (negative control)."""
    _load().wno_set_periodic_options(int(extra), 1 if disable_pairing else 0)


def query_faces(faces, queries, **kw):
    """All points of a ``Queries`` container (grouped by face)."""
    return query(faces, queries.face_ids(), queries.u, queries.v, **kw)


def segment_winding(cp, w, x, y, long_double: bool = False):
    """Winding number (turns) of one Bezier segment seen from (x, y) and its near flag."""
    lib = _load()
    cp = np.asarray(cp, dtype=np.float64)
    cu = np.ascontiguousarray(cp[:, 0])
    cv = np.ascontiguousarray(cp[:, 1])
    cw = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    near = ctypes.c_int32(0)
    r = lib.wno_segment_winding(_ptr(cu), _ptr(cv), _ptr(cw), len(cp) - 1, float(x), float(y),
                                1 if long_double else 0, ctypes.byref(near))
    return r, near.value


def alg1_pairs(faces, seg, x, y, eps: float = 1e-10, nthreads: int | None = None, cp_bound: bool = False):
    """Alg. 1 (Sec. 4.1, sub-segment bound of Sec. 4.2) run recursively on
    (query, segment) pairs: pair i is point (x[i], y[i]) against global
    segment seg[i] of ``faces`` (planar coordinates).  Returns a dict of
    arrays: depth (deepest tested level, root = 0), onb (an evaluated curve
    point within eps), splits, leaves, margin_abs and margin_rel (the
    smallest |d1 + d2 - axis| over the tested nodes, absolute and relative
    to the axis).  cp_bound: the axis of a node is the smaller of B (b - a)
    and the bound of its own (subdivided) control points (the variant that
    Sec. 4.2 / Table 1 contrast with the ellipse bound)."""
    lib = _load()
    sco = np.ascontiguousarray(faces.seg_cp_offsets, dtype=np.int64)
    cu = np.ascontiguousarray(faces.cp_u, dtype=np.float64)
    cv = np.ascontiguousarray(faces.cp_v, dtype=np.float64)
    cw = None if faces.cp_w is None else np.ascontiguousarray(faces.cp_w, dtype=np.float64)
    sg = np.ascontiguousarray(seg, dtype=np.int32)
    px = np.ascontiguousarray(x, dtype=np.float64)
    py = np.ascontiguousarray(y, dtype=np.float64)
    n = len(sg)
    out = np.empty((n, 6), dtype=np.float64)
    if nthreads is None:
        nthreads = os.cpu_count() or 1
    st = lib.wno_alg1_pairs(len(sco) - 1, _ptr(sco), _ptr(cu), _ptr(cv), _ptr(cw), n, _ptr(sg), _ptr(px), _ptr(py),
                            float(eps), 1 if cp_bound else 0, int(nthreads), _ptr(out))
    if st != 0:
        raise OracleError(f"alg1 mirror returned status {st}")
    return {"depth": out[:, 0].astype(np.int32), "onb": out[:, 1] != 0, "splits": out[:, 2].astype(np.int64),
            "leaves": out[:, 3].astype(np.int64), "margin_abs": out[:, 4], "margin_rel": out[:, 5]}


def alg1_segment(cp, w, x, y, eps: float = 1e-10, cp_bound: bool = False):
    """alg1_pairs for one segment given by its control points [n+1, 2] (and
    weights or None) against the points x, y."""
    from types import SimpleNamespace

    cp = np.asarray(cp, dtype=np.float64)
    n = len(cp) - 1
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    y = np.atleast_1d(np.asarray(y, dtype=np.float64))
    f = SimpleNamespace(seg_cp_offsets=np.array([0, n + 1], dtype=np.int64), cp_u=cp[:, 0].copy(),
                        cp_v=cp[:, 1].copy(), cp_w=None if w is None else np.asarray(w, dtype=np.float64))
    return alg1_pairs(f, np.zeros(len(x), dtype=np.int32), x, y, eps, nthreads=1, cp_bound=cp_bound)


def alg1_bound(cp, w=None) -> float:
    """The bound B (Lemma 1, App. A.1) as the depth mirror computes it."""
    lib = _load()
    cp = np.asarray(cp, dtype=np.float64)
    cu = np.ascontiguousarray(cp[:, 0])
    cv = np.ascontiguousarray(cp[:, 1])
    cw = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    return lib.wno_alg1_bound(_ptr(cu), _ptr(cv), _ptr(cw), len(cp) - 1)
