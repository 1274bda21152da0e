"""Python binding of the C ABI in include/wn.h (argument marshalling only).

Every step of the computation runs in the HIP library ``libwn.so``; this
module only converts numpy / torch buffers into pointers.  It fails loudly
when the library has not been built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

from .build import LIB

WN_OK, WN_E_INVALID, WN_E_NOMEM, WN_E_DEVICE, WN_E_TOPOLOGY, WN_E_DEPTH, WN_E_UNSUPPORTED = range(7)
PLANE, CYLINDER_U, TORUS, SPHERE_U, CONE_U = 0, 1, 2, 3, 4
PREC_FP64, PREC_MIXED = 0, 1
RULE_NONZERO, RULE_POSITIVE = 0, 1
SCHED_PLAIN, SCHED_BATCHED, SCHED_BINNED = 0, 1, 2
OUTSIDE, INSIDE, ON_BOUNDARY, INVALID_POINT = 0, 1, 2, 3

EXPORTS = [
    "wn_default_options", "wn_default_query_opts", "wn_create_faces", "wn_query", "wn_query_ex",
    "wn_destroy_faces", "wn_status_string", "wn_segment_bound", "wn_get_faces_info",
    "wn_profile_create", "wn_profile_collect", "wn_profile_destroy",
    "wn_predictor_create", "wn_predictor_destroy", "wn_predictor_train", "wn_predictor_get_params",
    "wn_predictor_set_params", "wn_predictor_loss_grad", "wn_predictor_predict", "wn_pair_features",
    "wn_plan_create", "wn_plan_launch", "wn_plan_autotune", "wn_plan_destroy", "wn_nurbs_to_bezier",
    "wn_classify_grid", "wn_classify_surfaces", "wn_create_faces_nurbs", "wn_near_pairs",
    "wn_query_noalloc", "wn_query_noalloc_scratch_bytes", "wn_torus_pairs", "wn_predictor_predict_mfma",
]
FLAG_HOST_PAIRING, FLAG_OVERLAP = 1, 2
NOALLOC_MAX_POINTS, NOALLOC_MAX_FACES = 1 << 22, 1 << 18
MLP_IN, MLP_HIDDEN = 16, 64
MLP_PARAMS = MLP_IN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN + 1
BIN_PREDICTOR, BIN_HEURISTIC, BIN_MEASURED, BIN_NONE, BIN_PREDICTOR_VALU = 0, 1, 2, 3, 4
BOUND_GLOBAL, BOUND_SUBDIVIDED = 0, 1
KERNEL_ITEMS, KERNEL_FAR, KERNEL_NEAR, KERNEL_FINALIZE, KERNEL_REDO, KERNEL_FAR_PERIODIC = 0, 1, 2, 3, 4, 5
KERNEL_NAMES = {0: "k_build_items", 1: "k_far", 2: "k_near", 3: "k_finalize", 4: "k_redo", 5: "k_far_periodic",
                6: "k_bin"}
KERNEL_KINDS = 8
STAT_NAMES = ["near_pairs", "splits", "leaves", "reevals", "near_flops", "max_depth", "near_steps",
              "near_lane_steps", "periodic_pairs"]
STATS_COUNT = 9

_P = ctypes.c_void_p


class wn_faces_desc(ctypes.Structure):
    _fields_ = [("num_faces", ctypes.c_int32), ("num_loops", ctypes.c_int32), ("num_segments", ctypes.c_int32),
                ("num_cps", ctypes.c_int64), ("face_loop_offsets", _P), ("loop_seg_offsets", _P),
                ("seg_cp_offsets", _P), ("cp_u", _P), ("cp_v", _P), ("cp_w", _P), ("face_domain", _P),
                ("face_period", _P)]


class wn_nurbs_faces_desc(ctypes.Structure):
    _fields_ = [("num_faces", ctypes.c_int32), ("num_loops", ctypes.c_int32), ("num_curves", ctypes.c_int32),
                ("num_cps", ctypes.c_int64), ("num_knots", ctypes.c_int64),
                ("face_loop_offsets", _P), ("loop_curve_offsets", _P), ("curve_degree", _P),
                ("curve_cp_offsets", _P), ("knots", _P), ("cp_u", _P), ("cp_v", _P), ("cp_w", _P),
                ("face_domain", _P), ("face_period", _P)]


class wn_options(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_double), ("precision", ctypes.c_int32), ("rule", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("stack_cap", ctypes.c_int32), ("flags", ctypes.c_int32)]


class wn_points(ctypes.Structure):
    _fields_ = [("num_points", ctypes.c_int64), ("u", _P), ("v", _P), ("stride", ctypes.c_int64),
                ("face_point_offsets", _P), ("face_point_offsets_host", _P)]


class wn_grid(ctypes.Structure):
    _fields_ = [("u0", ctypes.c_double), ("v0", ctypes.c_double), ("du", ctypes.c_double), ("dv", ctypes.c_double),
                ("nu", ctypes.c_int32), ("nv", ctypes.c_int32)]


class wn_query_opts(ctypes.Structure):
    _fields_ = [("schedule", ctypes.c_int32), ("precision", ctypes.c_int32), ("rule", ctypes.c_int32),
                ("queries_per_wg", ctypes.c_int32), ("queue_policy", ctypes.c_int32),
                ("near_capacity", ctypes.c_int64), ("depth_log", _P), ("profile", _P), ("stats", _P),
                ("predictor", _P), ("bin_source", ctypes.c_int32), ("path_hierarchy", ctypes.c_int32),
                ("bound", ctypes.c_int32)]


class wn_train_opts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_float),
                ("weight_decay", ctypes.c_float), ("huber_delta", ctypes.c_float), ("holdout", ctypes.c_float),
                ("seed", ctypes.c_int32), ("max_samples", ctypes.c_int64)]


class wn_train_report(ctypes.Structure):
    _fields_ = [("samples", ctypes.c_int64), ("train_samples", ctypes.c_int64), ("steps", ctypes.c_int32),
                ("final_train_loss", ctypes.c_float), ("holdout_mae", ctypes.c_float),
                ("baseline_mae", ctypes.c_float), ("heuristic_mae", ctypes.c_float), ("mean_depth", ctypes.c_float)]


class wn_faces_info(ctypes.Structure):
    _fields_ = [("num_faces", ctypes.c_int32), ("num_loops", ctypes.c_int32), ("num_segments", ctypes.c_int32),
                ("num_periodic_faces", ctypes.c_int32),
                ("max_segments_per_face", ctypes.c_int32), ("max_depth_bound", ctypes.c_int32),
                ("device_bytes", ctypes.c_int64)]


class WnError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: status {status} ({status_string(status)})")
        self.status = status


_lib = None


def lib():
    """Load libwn.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is missing: build it with paper_2510_25159_amd.build.build()")
        L = ctypes.CDLL(LIB)
        L.wn_status_string.restype = ctypes.c_char_p
        L.wn_status_string.argtypes = [ctypes.c_int]
        L.wn_default_options.argtypes = [ctypes.POINTER(wn_options)]
        L.wn_default_query_opts.argtypes = [ctypes.POINTER(wn_query_opts)]
        L.wn_create_faces.restype = ctypes.c_int
        L.wn_create_faces.argtypes = [ctypes.POINTER(wn_faces_desc), ctypes.POINTER(wn_options), _P,
                                      ctypes.POINTER(_P)]
        L.wn_query.restype = ctypes.c_int
        L.wn_query.argtypes = [_P, ctypes.POINTER(wn_points), _P, _P, _P]
        L.wn_query_ex.restype = ctypes.c_int
        L.wn_query_ex.argtypes = [_P, ctypes.POINTER(wn_points), _P, _P, ctypes.POINTER(wn_query_opts), _P]
        L.wn_query_noalloc.restype = ctypes.c_int
        L.wn_query_noalloc.argtypes = [_P, ctypes.POINTER(wn_points), _P, _P, ctypes.POINTER(wn_query_opts), _P]
        L.wn_query_noalloc_scratch_bytes.restype = ctypes.c_int64
        L.wn_query_noalloc_scratch_bytes.argtypes = []
        L.wn_torus_pairs.restype = ctypes.c_int
        L.wn_torus_pairs.argtypes = [_P, ctypes.c_int32, ctypes.c_int32, _P, _P, _P, ctypes.POINTER(ctypes.c_int32)]
        L.wn_destroy_faces.argtypes = [_P]
        L.wn_segment_bound.restype = ctypes.c_int
        L.wn_segment_bound.argtypes = [_P, _P, _P, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)]
        L.wn_nurbs_to_bezier.restype = ctypes.c_int
        L.wn_nurbs_to_bezier.argtypes = [ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P, ctypes.c_int64, _P, _P, _P,
                                         ctypes.POINTER(ctypes.c_int32)]
        L.wn_profile_create.restype = ctypes.c_int
        L.wn_profile_create.argtypes = [ctypes.c_int32, ctypes.POINTER(_P)]
        L.wn_profile_collect.restype = ctypes.c_int
        L.wn_profile_collect.argtypes = [_P, _P, _P]
        L.wn_profile_destroy.argtypes = [_P]
        L.wn_predictor_create.restype = ctypes.c_int
        L.wn_predictor_create.argtypes = [ctypes.c_int32, ctypes.POINTER(_P)]
        L.wn_predictor_destroy.argtypes = [_P]
        L.wn_predictor_train.restype = ctypes.c_int
        L.wn_predictor_train.argtypes = [_P, _P, ctypes.POINTER(wn_points), ctypes.POINTER(wn_train_opts),
                                         ctypes.POINTER(wn_train_report), _P]
        L.wn_predictor_get_params.restype = ctypes.c_int
        L.wn_predictor_get_params.argtypes = [_P, _P, _P]
        L.wn_predictor_set_params.restype = ctypes.c_int
        L.wn_predictor_set_params.argtypes = [_P, _P, _P]
        L.wn_predictor_loss_grad.restype = ctypes.c_int
        L.wn_predictor_loss_grad.argtypes = [_P, _P, _P, ctypes.c_int64, ctypes.c_float, _P, _P, _P]
        L.wn_predictor_predict.restype = ctypes.c_int
        L.wn_predictor_predict.argtypes = [_P, _P, ctypes.c_int64, _P, _P]
        L.wn_predictor_predict_mfma.argtypes = [_P, _P, ctypes.c_int64, _P, _P]
        L.wn_predictor_predict_mfma.restype = ctypes.c_int
        L.wn_pair_features.restype = ctypes.c_int
        L.wn_pair_features.argtypes = [_P, ctypes.POINTER(wn_points), _P, _P, ctypes.c_int64, _P, _P]
        L.wn_plan_create.restype = ctypes.c_int
        L.wn_plan_create.argtypes = [_P, ctypes.POINTER(wn_points), _P, _P, ctypes.POINTER(wn_query_opts), _P,
                                     ctypes.POINTER(_P)]
        L.wn_plan_launch.restype = ctypes.c_int
        L.wn_plan_launch.argtypes = [_P, _P]
        L.wn_plan_autotune.restype = ctypes.c_int
        L.wn_plan_autotune.argtypes = [_P, ctypes.c_int32, _P, _P]
        L.wn_plan_destroy.argtypes = [_P]
        L.wn_create_faces_nurbs.restype = ctypes.c_int
        L.wn_create_faces_nurbs.argtypes = [ctypes.POINTER(wn_nurbs_faces_desc), ctypes.POINTER(wn_options), _P,
                                            ctypes.POINTER(_P)]
        L.wn_classify_grid.restype = ctypes.c_int
        L.wn_classify_grid.argtypes = [_P, _P, _P, _P, _P, _P, ctypes.POINTER(wn_query_opts), _P]
        L.wn_classify_surfaces.restype = ctypes.c_int
        L.wn_classify_surfaces.argtypes = [_P, ctypes.c_int32, _P, _P, ctypes.POINTER(wn_points), _P, _P,
                                           ctypes.POINTER(wn_query_opts), _P]
        L.wn_near_pairs.restype = ctypes.c_int
        L.wn_near_pairs.argtypes = [_P, ctypes.POINTER(wn_points), ctypes.c_int64, _P, _P, _P, _P,
                                    ctypes.POINTER(ctypes.c_int64), ctypes.c_int32, _P]
        L.wn_get_faces_info.restype = ctypes.c_int
        L.wn_get_faces_info.argtypes = [_P, ctypes.POINTER(wn_faces_info)]
        _lib = L
    return _lib


def status_string(s: int) -> str:
    return lib().wn_status_string(int(s)).decode()


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(_P)


def segment_bound(cp, w=None) -> float:
    """Derivative bound B of one segment (host computation, no GPU)."""
    cp = np.asarray(cp, dtype=np.float64)
    u = np.ascontiguousarray(cp[:, 0])
    v = np.ascontiguousarray(cp[:, 1])
    ww = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    out = ctypes.c_double(0.0)
    st = lib().wn_segment_bound(_np_ptr(u), _np_ptr(v), _np_ptr(ww), len(cp) - 1, ctypes.byref(out))
    if st != WN_OK:
        raise WnError(st, "wn_segment_bound")
    return out.value


def nurbs_to_bezier(degree: int, knots, cp, w=None):
    """Split a clamped NURBS curve into (rational) Bezier segments (host).

    Returns a list of (control points [degree+1, 2], weights [degree+1] or None),
    one per knot span of nonzero length."""
    knots = np.ascontiguousarray(knots, dtype=np.float64)
    cp = np.ascontiguousarray(cp, dtype=np.float64)
    u = np.ascontiguousarray(cp[:, 0])
    v = np.ascontiguousarray(cp[:, 1])
    ww = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
    n = len(cp)
    cap = n + degree * max(len(knots), 1)  # every interior knot raised to multiplicity degree
    ou, ov = np.empty(cap), np.empty(cap)
    ow = None if ww is None else np.empty(cap)
    segs = ctypes.c_int32(0)
    st = lib().wn_nurbs_to_bezier(degree, n, _np_ptr(knots), _np_ptr(u), _np_ptr(v), _np_ptr(ww), cap, _np_ptr(ou),
                                  _np_ptr(ov), _np_ptr(ow), ctypes.byref(segs))
    if st != WN_OK:
        raise WnError(st, "wn_nurbs_to_bezier")
    out = []
    for i in range(segs.value):
        sl = slice(i * degree, i * degree + degree + 1)
        out.append((np.column_stack([ou[sl], ov[sl]]), None if ow is None else ow[sl].copy()))
    return out


def default_options(**kw) -> wn_options:
    o = wn_options()
    lib().wn_default_options(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def _stream_ptr(stream):
    if stream is None:
        import torch

        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


class Profile:
    """HIP-event timing of the library's kernels on the query stream."""

    def __init__(self, capacity: int = 4096):
        self._p = _P()
        st = lib().wn_profile_create(capacity, ctypes.byref(self._p))
        if st != WN_OK:
            raise WnError(st, "wn_profile_create")

    @property
    def handle(self):
        return self._p

    def collect(self):
        """{kernel name: (launches, total ms)}; resets the profile."""
        n = np.zeros(KERNEL_KINDS, dtype=np.int64)
        ms = np.zeros(KERNEL_KINDS, dtype=np.float64)
        st = lib().wn_profile_collect(self._p, _np_ptr(n), _np_ptr(ms))
        if st != WN_OK:
            raise WnError(st, "wn_profile_collect")
        return {KERNEL_NAMES[k]: (int(n[k]), float(ms[k])) for k in KERNEL_NAMES if n[k] > 0}

    def close(self):
        if self._p is not None and self._p.value:
            lib().wn_profile_destroy(self._p)
        self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FaceSet:
    """Owns a ``wn_faces`` handle built from host CSR arrays (see workloads.Faces)."""

    def __init__(self, faces, stream=None, **opts):
        self._h = None
        arrs = dict(
            flo=np.ascontiguousarray(faces.face_loop_offsets, dtype=np.int32),
            lso=np.ascontiguousarray(faces.loop_seg_offsets, dtype=np.int32),
            sco=np.ascontiguousarray(faces.seg_cp_offsets, dtype=np.int64),
            cu=np.ascontiguousarray(faces.cp_u, dtype=np.float64),
            cv=np.ascontiguousarray(faces.cp_v, dtype=np.float64),
            cw=None if faces.cp_w is None else np.ascontiguousarray(faces.cp_w, dtype=np.float64),
            dom=np.ascontiguousarray(faces.face_domain, dtype=np.int32),
            per=np.ascontiguousarray(faces.face_period, dtype=np.float64),
        )
        d = wn_faces_desc(len(arrs["flo"]) - 1, len(arrs["lso"]) - 1, len(arrs["sco"]) - 1, len(arrs["cu"]),
                          _np_ptr(arrs["flo"]), _np_ptr(arrs["lso"]), _np_ptr(arrs["sco"]), _np_ptr(arrs["cu"]),
                          _np_ptr(arrs["cv"]), _np_ptr(arrs["cw"]), _np_ptr(arrs["dom"]), _np_ptr(arrs["per"]))
        o = default_options(**opts)
        h = _P()
        st = lib().wn_create_faces(ctypes.byref(d), ctypes.byref(o), _stream_ptr(stream), ctypes.byref(h))
        if st != WN_OK:
            raise WnError(st, "wn_create_faces")
        self._h = h
        self.num_faces = d.num_faces

    @classmethod
    def from_nurbs(cls, face_loop_offsets, loop_curve_offsets, curve_degree, curve_cp_offsets, knots, cp_u, cp_v,
                   cp_w=None, face_domain=None, face_period=None, stream=None, **opts) -> "FaceSet":
        """Faces whose loops are chains of NURBS curves (host arrays; the
        curves' knot vectors back to back), split by wn_create_faces_nurbs."""
        self = cls.__new__(cls)
        self._h = None
        a = dict(flo=np.ascontiguousarray(face_loop_offsets, dtype=np.int32),
                 lco=np.ascontiguousarray(loop_curve_offsets, dtype=np.int32),
                 deg=np.ascontiguousarray(curve_degree, dtype=np.int32),
                 cco=np.ascontiguousarray(curve_cp_offsets, dtype=np.int64),
                 kn=np.ascontiguousarray(knots, dtype=np.float64),
                 cu=np.ascontiguousarray(cp_u, dtype=np.float64), cv=np.ascontiguousarray(cp_v, dtype=np.float64),
                 cw=None if cp_w is None else np.ascontiguousarray(cp_w, dtype=np.float64),
                 dom=None if face_domain is None else np.ascontiguousarray(face_domain, dtype=np.int32),
                 per=None if face_period is None else np.ascontiguousarray(face_period, dtype=np.float64))
        d = wn_nurbs_faces_desc(len(a["flo"]) - 1, len(a["lco"]) - 1, len(a["deg"]), len(a["cu"]), len(a["kn"]),
                                _np_ptr(a["flo"]),
                                _np_ptr(a["lco"]), _np_ptr(a["deg"]), _np_ptr(a["cco"]), _np_ptr(a["kn"]),
                                _np_ptr(a["cu"]), _np_ptr(a["cv"]), _np_ptr(a["cw"]), _np_ptr(a["dom"]),
                                _np_ptr(a["per"]))
        o = default_options(**opts)
        h = _P()
        st = lib().wn_create_faces_nurbs(ctypes.byref(d), ctypes.byref(o), _stream_ptr(stream), ctypes.byref(h))
        if st != WN_OK:
            raise WnError(st, "wn_create_faces_nurbs")
        self._h = h
        self.num_faces = d.num_faces
        return self

    def info(self) -> wn_faces_info:
        i = wn_faces_info()
        st = lib().wn_get_faces_info(self._h, ctypes.byref(i))
        if st != WN_OK:
            raise WnError(st, "wn_get_faces_info")
        return i

    def close(self):
        if self._h is not None and self._h.value:
            lib().wn_destroy_faces(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def query(self, u, v, offsets, offsets_host=None, out_w=None, out_lab=None, *, stride: int = 1,
              schedule: Optional[int] = None, precision: Optional[int] = None, rule: Optional[int] = None,
              queries_per_wg: int = 0, queue_policy: int = 0, near_capacity: int = 0, depth_log=None,
              profile: Optional[Profile] = None, stats=None, predictor=None, bin_source: int = 0,
              path_hierarchy: int = 0, bound: int = 0, stream=None):
        """Run the query on torch CUDA tensors (float64 u, v; int64 offsets).

        Returns (out_w, out_lab) torch tensors (allocated when not given)."""
        import torch

        n = u.numel() if stride == 1 else u.numel() // stride + (1 if u.numel() % stride else 0)
        assert u.is_cuda and v.is_cuda and offsets.is_cuda
        assert u.dtype == torch.float64 and v.dtype == torch.float64 and offsets.dtype == torch.int64
        if out_w is None:
            out_w = torch.empty(n, dtype=torch.float64, device=u.device)
        if out_lab is None:
            out_lab = torch.empty(n, dtype=torch.uint8, device=u.device)
        hoffs = None
        if offsets_host is not None:
            hoffs = np.ascontiguousarray(offsets_host, dtype=np.int64)
        p = wn_points(n, u.data_ptr(), v.data_ptr(), stride, offsets.data_ptr(), _np_ptr(hoffs))
        q = _query_opts(schedule=schedule, precision=precision, rule=rule, queries_per_wg=queries_per_wg,
                        queue_policy=queue_policy, near_capacity=near_capacity, depth_log=depth_log, profile=profile,
                        stats=stats, predictor=predictor, bin_source=bin_source, path_hierarchy=path_hierarchy,
                        bound=bound)
        st = lib().wn_query_ex(self._h, ctypes.byref(p), out_w.data_ptr(), out_lab.data_ptr(), ctypes.byref(q),
                               _stream_ptr(stream))
        if st != WN_OK:
            raise WnError(st, "wn_query_ex")
        return out_w, out_lab

    def torus_pairs(self, face: int):
        """Pair table of a torus face: (alpha int32 [P], beta int32 [P], shift float64 [P, 2])."""
        cnt = ctypes.c_int32(0)
        st = lib().wn_torus_pairs(self._h, face, 0, None, None, None, ctypes.byref(cnt))
        if st != WN_OK:
            raise WnError(st, "wn_torus_pairs")
        n = cnt.value
        a = np.zeros(n, dtype=np.int32)
        b = np.zeros(n, dtype=np.int32)
        sh = np.zeros((n, 2), dtype=np.float64)
        if n:
            st = lib().wn_torus_pairs(self._h, face, n, _np_ptr(a), _np_ptr(b), _np_ptr(sh), ctypes.byref(cnt))
            if st != WN_OK:
                raise WnError(st, "wn_torus_pairs")
        return a, b, sh

    def query_noalloc(self, u, v, offsets, out_w, out_lab, *, offsets_host=None, stride: int = 1, stream=None,
                      **opts):
        """wn_query_noalloc on torch CUDA tensors: the batched query with the
        library's fixed device scratch (the caller provides both outputs)."""
        import torch

        n = u.numel() if stride == 1 else u.numel() // stride + (1 if u.numel() % stride else 0)
        assert u.is_cuda and v.is_cuda and offsets.is_cuda
        assert u.dtype == torch.float64 and v.dtype == torch.float64 and offsets.dtype == torch.int64
        hoffs = None if offsets_host is None else np.ascontiguousarray(offsets_host, dtype=np.int64)
        p = wn_points(n, u.data_ptr(), v.data_ptr(), stride, offsets.data_ptr(), _np_ptr(hoffs))
        q = _query_opts(**opts)
        st = lib().wn_query_noalloc(self._h, ctypes.byref(p), out_w.data_ptr(), out_lab.data_ptr(), ctypes.byref(q),
                                    _stream_ptr(stream))
        if st != WN_OK:
            raise WnError(st, "wn_query_noalloc")
        return out_w, out_lab

    def classify_grid(self, grids, *, out_uv: bool = True, stream=None, **opts):
        """Tessellation driver: classify the cell centres of one uniform grid
        per face.  ``grids`` is a sequence of (u0, v0, du, dv, nu, nv), one per
        face.  Returns (u, v, omega, label) torch tensors over all cells, face
        by face and row-major inside a face (u and v are None when
        ``out_uv`` is false)."""
        import torch

        assert len(grids) == self.num_faces
        g = (wn_grid * self.num_faces)(*[wn_grid(float(a), float(b), float(c), float(d), int(e), int(f))
                                         for a, b, c, d, e, f in grids])
        n = sum(max(int(e), 0) * max(int(f), 0) for _, _, _, _, e, f in grids)  # the library validates
        dev = torch.device("cuda", torch.cuda.current_device())
        u = torch.empty(n, dtype=torch.float64, device=dev) if out_uv else None
        v = torch.empty(n, dtype=torch.float64, device=dev) if out_uv else None
        w = torch.empty(n, dtype=torch.float64, device=dev)
        lab = torch.empty(n, dtype=torch.uint8, device=dev)
        q = _query_opts(**opts)
        st = lib().wn_classify_grid(self._h, ctypes.cast(g, _P), None if u is None else u.data_ptr(),
                                    None if v is None else v.data_ptr(), w.data_ptr(), lab.data_ptr(),
                                    ctypes.byref(q), _stream_ptr(stream))
        if st != WN_OK:
            raise WnError(st, "wn_classify_grid")
        return u, v, w, lab

    def classify_surfaces(self, surface_face_offsets, surface_faces, u, v, surface_point_offsets, *, stride: int = 1,
                          stream=None, **opts):
        """Multi-patch classification: points on base surfaces (grouped by
        surface; host offsets) against every face that references their
        surface.  Returns (label uint8, first inside face int32) tensors."""
        import torch

        sfo = np.ascontiguousarray(surface_face_offsets, dtype=np.int32)
        sff = np.ascontiguousarray(surface_faces, dtype=np.int32)
        hoffs = np.ascontiguousarray(surface_point_offsets, dtype=np.int64)
        offs = torch.from_numpy(hoffs).to(u.device)
        n = int(hoffs[-1])
        lab = torch.empty(n, dtype=torch.uint8, device=u.device)
        face = torch.empty(n, dtype=torch.int32, device=u.device)
        p = wn_points(n, u.data_ptr(), v.data_ptr(), stride, offs.data_ptr(), _np_ptr(hoffs))
        q = _query_opts(**opts)
        st = lib().wn_classify_surfaces(self._h, len(sfo) - 1, _np_ptr(sfo), _np_ptr(sff), ctypes.byref(p),
                                        lab.data_ptr(), face.data_ptr(), ctypes.byref(q), _stream_ptr(stream))
        if st != WN_OK:
            raise WnError(st, "wn_classify_surfaces")
        return lab, face


def _query_opts(schedule=None, precision=None, rule=None, queries_per_wg=0, queue_policy=0, near_capacity=0,
                depth_log=None, profile=None, stats=None, predictor=None, bin_source=0, path_hierarchy=0, bound=0):
    """wn_query_opts from keyword overrides (None / 0 = default)."""
    q = wn_query_opts()
    lib().wn_default_query_opts(ctypes.byref(q))
    if schedule is not None:
        q.schedule = schedule
    if precision is not None:
        q.precision = precision
    if rule is not None:
        q.rule = rule
    q.queries_per_wg = queries_per_wg
    q.queue_policy = queue_policy
    q.near_capacity = near_capacity
    q.depth_log = None if depth_log is None else depth_log.data_ptr()
    q.profile = None if profile is None else profile.handle
    q.stats = None if stats is None else stats.data_ptr()
    q.predictor = None if predictor is None else predictor.handle
    q.bin_source = bin_source
    q.path_hierarchy = path_hierarchy
    q.bound = bound
    return q


def _points(u, v, offsets, stride=1, n=None):
    n = u.numel() if n is None else n
    return wn_points(n, u.data_ptr(), v.data_ptr(), stride, offsets.data_ptr(), None)


class Predictor:
    """Learned depth predictor (MLP 16-64-64-1, BF16 weights, trained on the GPU)."""

    def __init__(self, seed: int = 0):
        self._p = _P()
        st = lib().wn_predictor_create(int(seed), ctypes.byref(self._p))
        if st != WN_OK:
            raise WnError(st, "wn_predictor_create")

    @property
    def handle(self):
        return self._p

    def close(self):
        if self._p is not None and self._p.value:
            lib().wn_predictor_destroy(self._p)
        self._p = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def train(self, faceset: "FaceSet", u, v, offsets, *, epochs=8, batch=4096, lr=2e-3, weight_decay=1e-4,
              huber_delta=1.0, holdout=0.1, seed=0, max_samples=0, stream=None) -> dict:
        o = wn_train_opts(epochs, batch, lr, weight_decay, huber_delta, holdout, seed, max_samples)
        r = wn_train_report()
        p = _points(u, v, offsets)
        st = lib().wn_predictor_train(self._p, faceset._h, ctypes.byref(p), ctypes.byref(o), ctypes.byref(r),
                                      _stream_ptr(stream))
        if st != WN_OK:
            raise WnError(st, "wn_predictor_train")
        return {k: getattr(r, k) for k, _ in wn_train_report._fields_}

    def get_params(self):
        prm = np.empty(MLP_PARAMS, dtype=np.float32)
        norm = np.empty(2 * MLP_IN, dtype=np.float32)
        st = lib().wn_predictor_get_params(self._p, _np_ptr(prm), _np_ptr(norm))
        if st != WN_OK:
            raise WnError(st, "wn_predictor_get_params")
        return prm, norm

    def set_params(self, params=None, norm=None):
        prm = None if params is None else np.ascontiguousarray(params, dtype=np.float32)
        nm = None if norm is None else np.ascontiguousarray(norm, dtype=np.float32)
        st = lib().wn_predictor_set_params(self._p, _np_ptr(prm), _np_ptr(nm))
        if st != WN_OK:
            raise WnError(st, "wn_predictor_set_params")

    def loss_grad(self, X, Y, huber_delta=1.0, stream=None):
        """X: torch cuda float32 [n,16] (standardised), Y: [n]; returns (loss, grad numpy)."""
        loss = ctypes.c_float(0)
        grad = np.empty(MLP_PARAMS, dtype=np.float32)
        st = lib().wn_predictor_loss_grad(self._p, X.data_ptr(), Y.data_ptr(), X.shape[0], huber_delta,
                                          ctypes.byref(loss), _np_ptr(grad), _stream_ptr(stream))
        if st != WN_OK:
            raise WnError(st, "wn_predictor_loss_grad")
        return loss.value, grad

    @staticmethod
    def _features(X):
        import torch

        if X.dim() != 2 or X.shape[1] != MLP_IN or X.dtype != torch.float32:
            raise ValueError(f"features must be float32 [n][{MLP_IN}], got {tuple(X.shape)} {X.dtype}")
        if not X.is_cuda or not X.is_contiguous():
            raise ValueError("features must be a contiguous device tensor")

    def predict(self, X, stream=None):
        import torch

        self._features(X)
        out = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        st = lib().wn_predictor_predict(self._p, X.data_ptr(), X.shape[0], out.data_ptr(), _stream_ptr(stream))
        if st != WN_OK:
            raise WnError(st, "wn_predictor_predict")
        return out

    def predict_mfma(self, X, stream=None):
        """Predictions on the matrix cores (BF16 inputs and activations)."""
        import torch

        self._features(X)
        out = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        st = lib().wn_predictor_predict_mfma(self._p, X.data_ptr(), X.shape[0], out.data_ptr(),
                                             _stream_ptr(stream))
        if st != WN_OK:
            raise WnError(st, "wn_predictor_predict_mfma")
        return out


def near_pairs(faceset: "FaceSet", u, v, offsets, capacity: int, stream=None, bound: int = 0):
    """Near pairs of a query and the depth the near pass reached on each:
    (point int32 [n], segment int32 [n], depth uint8 [n], shift float64 [n, 2])
    torch cuda tensors, n = min(count, capacity)."""
    import torch

    dev = u.device
    pp = torch.empty(capacity, dtype=torch.int32, device=dev)
    ps = torch.empty(capacity, dtype=torch.int32, device=dev)
    pd = torch.empty(capacity, dtype=torch.uint8, device=dev)
    sh = torch.empty((capacity, 2), dtype=torch.float64, device=dev)
    cnt = ctypes.c_int64(0)
    p = _points(u, v, offsets)
    st = lib().wn_near_pairs(faceset._h, ctypes.byref(p), capacity, pp.data_ptr(), ps.data_ptr(), pd.data_ptr(),
                             sh.data_ptr(), ctypes.byref(cnt), bound, _stream_ptr(stream))
    if st != WN_OK:
        raise WnError(st, "wn_near_pairs")
    n = min(cnt.value, capacity)
    return pp[:n], ps[:n], pd[:n], sh[:n]


def pair_features(faceset: "FaceSet", u, v, offsets, pair_point, pair_segment, stream=None):
    """Raw features [n,16] (torch cuda float32) of (point, global segment) pairs."""
    import torch

    n = pair_point.numel()
    out = torch.empty((n, MLP_IN), dtype=torch.float32, device=u.device)
    p = _points(u, v, offsets)
    st = lib().wn_pair_features(faceset._h, ctypes.byref(p), pair_point.data_ptr(), pair_segment.data_ptr(), n,
                                out.data_ptr(), _stream_ptr(stream))
    if st != WN_OK:
        raise WnError(st, "wn_pair_features")
    return out


class Plan:
    """A batched query captured once into a HIP graph over caller-owned torch
    buffers (capacity = u.numel()); write points/offsets, then launch()."""

    def __init__(self, faceset: "FaceSet", u, v, offsets, out_w, out_lab, *, schedule: int = SCHED_BATCHED,
                 queries_per_wg: int = 0, queue_policy: int = 0, predictor=None, bin_source: int = 0, stream=None):
        self._keep = (faceset, u, v, offsets, out_w, out_lab, predictor)
        self._h = _P()
        p = _points(u, v, offsets)
        q = wn_query_opts()
        lib().wn_default_query_opts(ctypes.byref(q))
        q.schedule = schedule
        q.queries_per_wg = queries_per_wg
        q.queue_policy = queue_policy
        q.predictor = None if predictor is None else predictor.handle
        q.bin_source = bin_source
        st = lib().wn_plan_create(faceset._h, ctypes.byref(p), out_w.data_ptr(), out_lab.data_ptr(), ctypes.byref(q),
                                  _stream_ptr(stream), ctypes.byref(self._h))
        if st != WN_OK:
            raise WnError(st, "wn_plan_create")

    def launch(self, stream=None):
        st = lib().wn_plan_launch(self._h, _stream_ptr(stream))
        if st != WN_OK:
            raise WnError(st, "wn_plan_launch")

    def autotune(self, reps: int = 3, stream=None) -> dict:
        rep = np.zeros(12, dtype=np.float64)
        st = lib().wn_plan_autotune(self._h, reps, _stream_ptr(stream), _np_ptr(rep))
        if st != WN_OK:
            raise WnError(st, "wn_plan_autotune")
        names = [f"{q}/{p}" for q in (64, 128, 256, 512, 1024) for p in ("persistent", "per-item")]
        return {"ms": dict(zip(names, rep[:10].tolist())), "queries_per_wg": int(rep[10]),
                "queue_policy": int(rep[11])}

    def close(self):
        if self._h is not None and self._h.value:
            lib().wn_plan_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
