"""Seeded synthetic inputs: trimmed faces and query points.

This module only *constructs* inputs.  It holds none of the winding-number
arithmetic (no bounds, no angle sums, no recursion, no lifting): the CPU
oracle under ``oracle/`` and the HIP library both consume what it returns,
and neither imports the other.

Shapes follow the workloads of the paper's experiments (Sec. 5): star-shaped
closed C0 Bezier loops standing in for the Bezier-Guarding closed-loop sets,
256x256-style uniform query grids, rational weights (App. A.1 treats the
rational case), and periodic faces whose loops wrap the period cell
(Sec. 4.3-4.5).  Every array is produced from numpy ``PCG64`` streams keyed
by ``(seed, face index)`` so a subset of faces can be rebuilt on its own.

Layout (CSR, host numpy arrays):

* ``face_loop_offsets``  int32  [F+1]   faces -> loops
* ``loop_seg_offsets``   int32  [L+1]   loops -> ordered segments
* ``seg_cp_offsets``     int64  [S+1]   segments -> control points; degree = count-1
* ``cp_u, cp_v``         float64 [C]    control points
* ``cp_w``               float64 [C] or None (non-rational)
* ``face_domain``        int32  [F]     0 plane, 1 cylinder (periodic in u), 2 torus
* ``face_period``        float64 [2F]   (T_u, T_v) per face
"""
from __future__ import annotations

from dataclasses import dataclass, field
from math import comb
from typing import List, Optional, Sequence

import numpy as np

DOMAIN_PLANE = 0
DOMAIN_CYLINDER_U = 1
DOMAIN_TORUS = 2
DOMAIN_SPHERE_U = 3  # periodic in u, poles at both ends of v (punctured)
DOMAIN_CONE_U = 4  # periodic in u, apex at one end of v (punctured)

SEED_C1 = 1
SEED_C2 = 2
SEED_C3 = 3
SEED_C4_TRAIN = 40
SEED_C4_EVAL = 41
SEED_C5 = 5
SEED_BREP = 6
SEED_DEG = 8


@dataclass
class Faces:
    face_loop_offsets: np.ndarray
    loop_seg_offsets: np.ndarray
    seg_cp_offsets: np.ndarray
    cp_u: np.ndarray
    cp_v: np.ndarray
    cp_w: Optional[np.ndarray]
    face_domain: np.ndarray
    face_period: np.ndarray

    @property
    def num_faces(self) -> int:
        return len(self.face_loop_offsets) - 1

    @property
    def num_loops(self) -> int:
        return len(self.loop_seg_offsets) - 1

    @property
    def num_segments(self) -> int:
        return len(self.seg_cp_offsets) - 1

    @property
    def num_cps(self) -> int:
        return len(self.cp_u)

    def face_segment_counts(self) -> np.ndarray:
        lo = self.loop_seg_offsets[self.face_loop_offsets[:-1]]
        hi = self.loop_seg_offsets[self.face_loop_offsets[1:]]
        return (hi - lo).astype(np.int64)


@dataclass
class Queries:
    u: np.ndarray
    v: np.ndarray
    face_point_offsets: np.ndarray  # int64 [F+1]
    near_mask: Optional[np.ndarray] = None  # True where the point was placed near a curve

    @property
    def num_points(self) -> int:
        return len(self.u)

    def face_ids(self) -> np.ndarray:
        counts = np.diff(self.face_point_offsets)
        return np.repeat(np.arange(len(counts), dtype=np.int32), counts)


# --------------------------------------------------------------------------
# loop containers used while building a face
# --------------------------------------------------------------------------
@dataclass
class _Loop:
    # list of per-segment control point arrays, each [(n+1), 2], and weights [(n+1)] or None
    cps: List[np.ndarray] = field(default_factory=list)
    ws: List[Optional[np.ndarray]] = field(default_factory=list)


def _assemble(face_loops: Sequence[Sequence[_Loop]], domains, periods, rational: bool) -> Faces:
    flo = [0]
    lso = [0]
    sco = [0]
    us, vs, wsl = [], [], []
    for loops in face_loops:
        for lp in loops:
            for cp, w in zip(lp.cps, lp.ws):
                us.append(cp[:, 0])
                vs.append(cp[:, 1])
                if rational:
                    wsl.append(w if w is not None else np.ones(len(cp)))
                sco.append(sco[-1] + len(cp))
            lso.append(lso[-1] + len(lp.cps))
        flo.append(flo[-1] + len(loops))
    return Faces(
        face_loop_offsets=np.asarray(flo, dtype=np.int32),
        loop_seg_offsets=np.asarray(lso, dtype=np.int32),
        seg_cp_offsets=np.asarray(sco, dtype=np.int64),
        cp_u=np.ascontiguousarray(np.concatenate(us)).astype(np.float64),
        cp_v=np.ascontiguousarray(np.concatenate(vs)).astype(np.float64),
        cp_w=(np.ascontiguousarray(np.concatenate(wsl)).astype(np.float64) if rational else None),
        face_domain=np.asarray(domains, dtype=np.int32),
        face_period=np.asarray(periods, dtype=np.float64).reshape(-1),
    )


def _face_rng(seed: int, face: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, face])))


# --------------------------------------------------------------------------
# star curves r(theta) = rho * (1 + 0.3 * s(theta)/max|s|), s = 8 Fourier modes
# --------------------------------------------------------------------------
_GRID = np.linspace(0.0, 2.0 * np.pi, 4096, endpoint=False)
_GRID_K = np.arange(1, 9, dtype=np.float64)
_GRID_COS = np.cos(_GRID[:, None] * _GRID_K)
_GRID_SIN = np.sin(_GRID[:, None] * _GRID_K)


class StarCurve:
    """Closed star-shaped curve around ``center`` (counter-clockwise in theta):
    r(theta) = rho (1 + amp s(theta) / max|s|), s = sum_k a_k cos k theta + b_k sin k theta,
    a_k, b_k ~ U[-1, 1] / k, the maximum taken over a 4096-point grid."""

    def __init__(self, rng: np.random.Generator, rho: float = 1.0, center=(0.0, 0.0), modes: int = 8,
                 amp: float = 0.3):
        k = np.arange(1, modes + 1, dtype=np.float64)
        self.k = k
        self.a = rng.uniform(-1.0, 1.0, modes) / k
        self.b = rng.uniform(-1.0, 1.0, modes) / k
        if modes == 8:
            m = np.max(np.abs(_GRID_COS @ self.a + _GRID_SIN @ self.b))
        else:
            m = np.max(np.abs(self._s(_GRID)))
        self.scale = amp / m if m > 0 else 0.0
        self.amp = amp
        self.rho = float(rho)
        self.center = np.asarray(center, dtype=np.float64)

    def _s(self, th):
        th = np.asarray(th, dtype=np.float64)[..., None]
        return np.sum(self.a * np.cos(self.k * th) + self.b * np.sin(self.k * th), axis=-1)

    def _ds(self, th):
        th = np.asarray(th, dtype=np.float64)[..., None]
        return np.sum(self.k * (-self.a * np.sin(self.k * th) + self.b * np.cos(self.k * th)), axis=-1)

    def r(self, th):
        return self.rho * (1.0 + self.scale * self._s(th))

    def point(self, th):
        th = np.asarray(th, dtype=np.float64)
        r = self.r(th)
        return np.stack([self.center[0] + r * np.cos(th), self.center[1] + r * np.sin(th)], axis=-1)

    def tangent(self, th):
        th = np.asarray(th, dtype=np.float64)
        r = self.r(th)
        dr = self.rho * self.scale * self._ds(th)
        c, s = np.cos(th), np.sin(th)
        return np.stack([dr * c - r * s, dr * s + r * c], axis=-1)

    @staticmethod
    def radius_bound(rho: float, amp: float = 0.3) -> float:
        """Upper bound of r(theta) (the grid maximum may miss the true one by a little)."""
        return rho * (1.0 + 1.02 * amp)


def hermite_star_loop(curve: StarCurve, nseg: int) -> _Loop:
    """Closed CCW loop of ``nseg`` cubic Hermite pieces; consecutive pieces share
    their joint bit-for-bit and the last piece ends exactly at the first point."""
    th = 2.0 * np.pi * np.arange(nseg + 1) / nseg
    V = curve.point(th[:-1])
    T = curve.tangent(th[:-1])
    dth = 2.0 * np.pi / nseg
    lp = _Loop()
    for i in range(nseg):
        j = (i + 1) % nseg
        P0, P3 = V[i], V[j]
        P1 = P0 + (dth / 3.0) * T[i]
        P2 = P3 - (dth / 3.0) * T[j]
        lp.cps.append(np.stack([P0, P1, P2, P3]))
        lp.ws.append(None)
    return lp


def sampled_star_loop(curve: StarCurve, nseg: int, degrees: np.ndarray, weights_rng=None,
                      wlo: float = 0.5, whi: float = 2.0) -> _Loop:
    """Closed CCW loop whose segment i has degree ``degrees[i]`` and control points
    sampled on the star at equally spaced angles inside the segment's wedge; the
    joint of consecutive segments is shared bit-for-bit."""
    th = 2.0 * np.pi * np.arange(nseg + 1) / nseg
    degrees = np.asarray(degrees, dtype=np.int64)
    # all interior parameters at once
    inner_th = []
    for i in range(nseg):
        n = int(degrees[i])
        inner_th.append(th[i] + (th[i + 1] - th[i]) * np.arange(1, n) / n)
    inner_all = np.concatenate(inner_th) if nseg else np.zeros(0)
    P_inner = curve.point(inner_all)
    V = curve.point(th[:-1])
    lp = _Loop()
    pos = 0
    wts = weights_rng.uniform(wlo, whi, int(np.sum(degrees + 1))) if weights_rng is not None else None
    wpos = 0
    for i in range(nseg):
        n = int(degrees[i])
        j = (i + 1) % nseg
        cp = np.empty((n + 1, 2))
        cp[0] = V[i]
        cp[1:n] = P_inner[pos:pos + n - 1]
        cp[n] = V[j]
        pos += n - 1
        lp.cps.append(cp)
        if wts is not None:
            lp.ws.append(wts[wpos:wpos + n + 1])
            wpos += n + 1
        else:
            lp.ws.append(None)
    return lp


def reverse_loop(lp: _Loop) -> _Loop:
    out = _Loop()
    for cp, w in zip(reversed(lp.cps), reversed(lp.ws)):
        out.cps.append(cp[::-1].copy())
        out.ws.append(None if w is None else w[::-1].copy())
    return out


def eval_rational_bezier(cp: np.ndarray, w: Optional[np.ndarray], t: np.ndarray) -> np.ndarray:
    """Bernstein-sum evaluation (input placement only)."""
    n = len(cp) - 1
    t = np.asarray(t, dtype=np.float64)[..., None]
    j = np.arange(n + 1)
    binom = np.array([comb(n, int(i)) for i in j], dtype=np.float64)
    basis = binom * t ** j * (1.0 - t) ** (n - j)
    if w is not None:
        basis = basis * w
    den = basis.sum(axis=-1, keepdims=True)
    return (basis @ cp) / den


_BINOM = np.array([[comb(n, j) if j <= n else 0 for j in range(6)] for n in range(6)], dtype=np.float64)


def _eval_many(loops: Sequence[_Loop], li: np.ndarray, si: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Vectorised Bernstein-sum evaluation of segment ``si`` of loop ``li`` at ``t``."""
    segs = [(cp, w) for lp in loops for cp, w in zip(lp.cps, lp.ws)]
    base = np.cumsum([0] + [len(lp.cps) for lp in loops])
    S = len(segs)
    P = np.zeros((S, 6, 2))
    W = np.zeros((S, 6))
    deg = np.zeros(S, dtype=np.int64)
    for k, (cp, w) in enumerate(segs):
        n = len(cp) - 1
        P[k, : n + 1] = cp
        W[k, : n + 1] = 1.0 if w is None else w
        deg[k] = n
    g = base[li] + si
    n = deg[g]
    j = np.arange(6)[None, :]
    tt = t[:, None]
    basis = _BINOM[n] * tt ** j * (1.0 - tt) ** np.maximum(n[:, None] - j, 0) * (j <= n[:, None])
    basis = basis * W[g]
    den = basis.sum(axis=1, keepdims=True)
    return np.einsum("nj,njc->nc", basis, P[g]) / den


# --------------------------------------------------------------------------
# Config 1: one planar face, one closed CCW loop of 64 cubic segments
# --------------------------------------------------------------------------
def config1_faces(seed: int = SEED_C1, nseg: int = 64) -> Faces:
    rng = np.random.Generator(np.random.PCG64(seed))
    curve = StarCurve(rng)
    lp = hermite_star_loop(curve, nseg)
    return _assemble([[lp]], [DOMAIN_PLANE], [[0.0, 0.0]], rational=False)


def config1_queries(seed: int = SEED_C1, n: int = 65536, half: float = 1.5) -> Queries:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 1_000_003])))
    pts = rng.uniform(-half, half, size=(n, 2))
    return Queries(u=np.ascontiguousarray(pts[:, 0]), v=np.ascontiguousarray(pts[:, 1]),
                   face_point_offsets=np.asarray([0, n], dtype=np.int64),
                   near_mask=np.zeros(n, dtype=bool))


def config1(seed: int = SEED_C1):
    return config1_faces(seed), config1_queries(seed)


# --------------------------------------------------------------------------
# Degree set (Sec. 5, runtime against boundary degree): cubic star loops
# elevated to higher degree without changing the curve
# --------------------------------------------------------------------------
def elevate_bezier(cp: np.ndarray, times: int) -> np.ndarray:
    """Control points of the same polynomial Bezier curve at degree n + times
    (repeated degree elevation: P'_i = i/(n+1) P_{i-1} + (1 - i/(n+1)) P_i).
    The end points are kept bit-for-bit, so joints stay shared."""
    cp = np.asarray(cp, dtype=np.float64)
    for _ in range(times):
        n = len(cp) - 1
        a = (np.arange(1, n + 1) / (n + 1))[:, None]
        cp = np.vstack([cp[:1], a * cp[:-1] + (1.0 - a) * cp[1:], cp[-1:]])
    return cp


def degree_set(degree: int, seed: int = SEED_DEG, num_faces: int = 64, nseg: int = 64,
               points_per_face: int = 8192, on_curve_frac: float = 0.5):
    """``num_faces`` cubic star faces (config 1's generator, one per seed) with
    every segment elevated to ``degree`` (3..5), and the same queries for
    every degree: per face, ``on_curve_frac`` of the points on the cubic
    curve (random segment and parameter, evaluated in FP64: within rounding
    of the boundary, the worst case of the recursion) and the rest uniform in
    the face's box [-1.5, 1.5]^2."""
    if not 3 <= degree <= 5:
        raise ValueError("degree_set: degree must be in 3..5 (cubic curves elevated)")
    face_loops, pts = [], []
    for f in range(num_faces):
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, f])))
        lp = hermite_star_loop(StarCurve(rng), nseg)
        k = int(round(on_curve_frac * points_per_face))
        si = rng.integers(0, nseg, k)
        t = rng.uniform(0.0, 1.0, k)
        on = _eval_many([lp], np.zeros(k, dtype=np.int64), si, t)
        uni = rng.uniform(-1.5, 1.5, size=(points_per_face - k, 2))
        pts.append(np.vstack([on, uni]))
        face_loops.append([[(elevate_bezier(c, degree - 3), None) for c in lp.cps]])
    return faces_from_loops(face_loops), queries_for_faces(pts)


# --------------------------------------------------------------------------
# Config 4: pairs of config 1's generator for the learned depth predictor
# --------------------------------------------------------------------------
def config4(split: str = "train", near_frac: float = 0.0):
    """One 64-segment star face (config 1 generator) and its queries:
    train = 78,125 points x 64 segments = 5M pairs (seed 40), eval = 156,250 x 64
    = 10M pairs (seed 41).  ``near_frac`` > 0 places that fraction of the points
    within 1e-3 of the curve (a stress variant outside the configuration)."""
    seed, n = (SEED_C4_TRAIN, 78125) if split == "train" else (SEED_C4_EVAL, 156250)
    faces = config1_faces(seed)
    q = config1_queries(seed, n)
    if near_frac > 0:
        rng = np.random.default_rng(seed + 1000)
        k = int(round(near_frac * n))
        segs = [(np.column_stack([faces.cp_u[faces.seg_cp_offsets[s]:faces.seg_cp_offsets[s + 1]],
                                  faces.cp_v[faces.seg_cp_offsets[s]:faces.seg_cp_offsets[s + 1]]]), None)
                for s in range(faces.num_segments)]
        lp = _Loop([c for c, _ in segs], [None] * len(segs))
        si = rng.integers(0, len(segs), k)
        t = rng.uniform(0, 1, k)
        base = _eval_many([lp], np.zeros(k, dtype=np.int64), si, t)
        rad = 1e-3 * np.sqrt(rng.uniform(0, 1, k))
        phi = rng.uniform(0, 2 * np.pi, k)
        u = q.u.copy()
        v = q.v.copy()
        u[:k] = base[:, 0] + rad * np.cos(phi)
        v[:k] = base[:, 1] + rad * np.sin(phi)
        q = Queries(u=u, v=v, face_point_offsets=q.face_point_offsets, near_mask=np.arange(n) < k)
    return faces, q


# --------------------------------------------------------------------------
# Config 2: batched B-Rep-like planar faces
# --------------------------------------------------------------------------
def _loguniform_int(rng, lo, hi):
    return int(round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))


def _min_hull_radius(lp: _Loop) -> float:
    """Smallest distance from the origin to any segment joining two control
    points of one segment (a lower bound of the distance from the origin to
    every control-point hull of the loop)."""
    A, Bp = [], []
    for cp in lp.cps:
        m = len(cp)
        ii, jj = np.triu_indices(m, 1)
        A.append(cp[ii])
        Bp.append(cp[jj])
    A = np.vstack(A)
    Bp = np.vstack(Bp)
    d = Bp - A
    L2 = np.einsum("ij,ij->i", d, d)
    t = np.where(L2 > 0, np.clip(-np.einsum("ij,ij->i", A, d) / np.where(L2 > 0, L2, 1.0), 0.0, 1.0), 0.0)
    p = A + t[:, None] * d
    return float(np.min(np.hypot(p[:, 0], p[:, 1])))


def config2_face(seed: int, f: int, q_lo: int = 1024, q_hi: int = 65536, near_frac: float = 0.3,
                 seg_lo: int = 4, seg_hi: int = 256, max_holes: int = 7, near_offset: float = 1e-3):
    """One face of the batched set: loops (outer first) and its queries."""
    rng = _face_rng(seed, f)
    outer_curve = StarCurve(rng, rho=1.0)
    nseg = _loguniform_int(rng, seg_lo, seg_hi)
    outer = sampled_star_loop(outer_curve, nseg, rng.integers(1, 6, nseg), weights_rng=rng)
    loops = [outer]
    r_safe = min(0.6, 0.95 * _min_hull_radius(outer))
    K = int(rng.integers(0, max_holes + 1))
    discs = []
    for _ in range(K):
        for _try in range(200):
            rho = rng.uniform(0.05, 0.15)
            rmax = StarCurve.radius_bound(rho)
            c = rng.uniform(-r_safe, r_safe, 2)
            if np.hypot(*c) + rmax > r_safe:
                continue
            if any(np.hypot(*(c - c2)) <= rmax + r2 for c2, r2 in discs):
                continue
            hc = StarCurve(rng, rho=rho, center=c)
            discs.append((c, rmax))
            ns = _loguniform_int(rng, seg_lo, seg_hi)
            hole = sampled_star_loop(hc, ns, rng.integers(1, 6, ns), weights_rng=rng)
            loops.append(reverse_loop(hole))
            break
    nq = _loguniform_int(rng, q_lo, q_hi)
    n_near = int(round(near_frac * nq))
    pts = rng.uniform(-1.5, 1.5, size=(nq, 2))
    near = np.zeros(nq, dtype=bool)
    if n_near > 0:
        li = rng.integers(0, len(loops), n_near)
        seg_counts = np.array([len(lp.cps) for lp in loops])
        si = (rng.uniform(0, 1, n_near) * seg_counts[li]).astype(np.int64)
        si = np.minimum(si, seg_counts[li] - 1)
        t = rng.uniform(0, 1, n_near)
        rad = near_offset * np.sqrt(rng.uniform(0, 1, n_near))
        phi = rng.uniform(0, 2 * np.pi, n_near)
        base = _eval_many(loops, li, si, t)
        pts[:n_near] = base + np.stack([rad * np.cos(phi), rad * np.sin(phi)], axis=-1)
        near[:n_near] = True
        perm = rng.permutation(nq)
        pts = pts[perm]
        near = near[perm]
    return loops, pts, near


def config2(seed: int = SEED_C2, num_faces: int = 2000, face_ids: Optional[Sequence[int]] = None, **kw):
    ids = list(range(num_faces)) if face_ids is None else list(face_ids)
    face_loops, pts_all, near_all, offs = [], [], [], [0]
    for f in ids:
        loops, pts, near = config2_face(seed, f, **kw)
        face_loops.append(loops)
        pts_all.append(pts)
        near_all.append(near)
        offs.append(offs[-1] + len(pts))
    faces = _assemble(face_loops, [DOMAIN_PLANE] * len(ids), [[0.0, 0.0]] * len(ids), rational=True)
    P = np.concatenate(pts_all)
    q = Queries(u=np.ascontiguousarray(P[:, 0]), v=np.ascontiguousarray(P[:, 1]),
                face_point_offsets=np.asarray(offs, dtype=np.int64), near_mask=np.concatenate(near_all))
    return faces, q


# --------------------------------------------------------------------------
# Config 3: periodic faces (cylinder / torus parameter domains)
# --------------------------------------------------------------------------
TWO_PI = 2.0 * np.pi


class WrappedCurve:
    """alpha(t) = s0 + t * vec + A * nrm * f(t), t in [0, 1], on the covering
    space; f is a 4-mode periodic Fourier series, so alpha(1) = alpha(0) + vec."""

    def __init__(self, s0, vec, amp, rng, modes: int = 4):
        self.s0 = np.asarray(s0, dtype=np.float64)
        self.vec = np.asarray(vec, dtype=np.float64)
        L = np.hypot(*self.vec)
        self.nrm = np.array([-self.vec[1], self.vec[0]]) / L
        k = np.arange(1, modes + 1, dtype=np.float64)
        self.k = k
        c = rng.uniform(-1, 1, modes) / k
        d = rng.uniform(-1, 1, modes) / k
        grid = np.linspace(0, 1, 2048, endpoint=False)
        m = np.max(np.abs(np.cos(TWO_PI * grid[:, None] * k) @ c + np.sin(TWO_PI * grid[:, None] * k) @ d))
        self.c = c * (amp / m if m > 0 else 0.0)
        self.d = d * (amp / m if m > 0 else 0.0)

    def f(self, t):
        t = np.asarray(t, dtype=np.float64)[..., None]
        return np.sum(self.c * np.cos(TWO_PI * self.k * t) + self.d * np.sin(TWO_PI * self.k * t), axis=-1)

    def df(self, t):
        t = np.asarray(t, dtype=np.float64)[..., None]
        return np.sum(TWO_PI * self.k * (-self.c * np.sin(TWO_PI * self.k * t) + self.d * np.cos(TWO_PI * self.k * t)),
                      axis=-1)

    def point(self, t):
        t = np.asarray(t, dtype=np.float64)
        return self.s0 + t[..., None] * self.vec + self.f(t)[..., None] * self.nrm

    def deriv(self, t):
        t = np.asarray(t, dtype=np.float64)
        return self.vec + self.df(t)[..., None] * self.nrm


def _seam_crossings(curve: WrappedCurve, t0: float, t1: float, axis: int, T: float, tol: float = 1e-15):
    """Parameters in (t0, t1) where coordinate ``axis`` crosses a multiple of T (bisection)."""
    out = []
    ts = np.linspace(t0, t1, 65)
    vals = curve.point(ts)[:, axis] / T
    for a, b, fa, fb in zip(ts[:-1], ts[1:], vals[:-1], vals[1:]):
        ka, kb = np.floor(fa), np.floor(fb)
        if ka == kb:
            continue
        # possibly several lines between a and b: handle each
        lo_line, hi_line = (ka + 1, kb) if kb > ka else (kb + 1, ka)
        for line in np.arange(lo_line, hi_line + 1):
            lo, hi = a, b
            glo = curve.point(lo)[axis] / T - line
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                gm = curve.point(mid)[axis] / T - line
                if (gm > 0) == (glo > 0):
                    lo, glo = mid, gm
                else:
                    hi = mid
                if hi - lo < tol:
                    break
            out.append(0.5 * (lo + hi))
    return sorted(out)


def periodic_loop(curve: WrappedCurve, nseg: int, periods, axes) -> _Loop:
    """Cubic Hermite pieces of ``curve`` between the segment parameters i/nseg
    and every seam crossing; each piece translated by a lattice vector into
    the base cell (so the loop is discontinuous at the seams)."""
    breaks = [i / nseg for i in range(nseg + 1)]
    cuts = set(breaks)
    for ax in axes:
        for i in range(nseg):
            for t in _seam_crossings(curve, breaks[i], breaks[i + 1], ax, periods[ax]):
                cuts.add(t)
    ts = np.array(sorted(cuts))
    ts = ts[np.concatenate([[True], np.diff(ts) > 1e-12])]
    P = curve.point(ts)
    D = curve.deriv(ts)
    lp = _Loop()
    for i in range(len(ts) - 1):
        h = ts[i + 1] - ts[i]
        cp = np.stack([P[i], P[i] + (h / 3) * D[i], P[i + 1] - (h / 3) * D[i + 1], P[i + 1]])
        mid = curve.point(0.5 * (ts[i] + ts[i + 1]))
        shift = np.zeros(2)
        for ax in axes:
            shift[ax] = -periods[ax] * np.floor(mid[ax] / periods[ax])
        lp.cps.append(cp + shift)
        lp.ws.append(None)
    return lp


def _open_and_noise(lp: _Loop, rng, open_loop: bool, gap_lo: float, gap_hi: float, sigma: float):
    if open_loop:
        g = rng.uniform(gap_lo, gap_hi)
        phi = rng.uniform(0, TWO_PI)
        lp.cps[-1] = lp.cps[-1].copy()
        lp.cps[-1][-1] += g * np.array([np.cos(phi), np.sin(phi)])
    if sigma > 0:
        lp.cps = [cp + rng.normal(0.0, sigma, cp.shape) for cp in lp.cps]


def _coprime_pair(rng):
    while True:
        h1, h2 = int(rng.integers(2, 6)), int(rng.integers(2, 6))
        if np.gcd(h1, h2) == 1:
            return h1, h2


def config3_face(seed: int, f: int, queries: int = 2048, open_frac: float = 0.2, gap=(1e-4, 1e-2),
                 sigma: float = 1e-5, seg_lo: int = 16, seg_hi: int = 64):
    """Face f of the periodic set: even f cylinder (period 2pi in u, cell
    [0,2pi) x [-pi,pi)), odd f torus (period 2pi in u and v)."""
    rng = _face_rng(seed, f)
    T = TWO_PI
    loops = []
    if f % 2 == 0:
        domain, periods, axes = DOMAIN_CYLINDER_U, (T, 0.0), (0,)
        nb = int(rng.integers(1, 3))
        # disjoint bands [c1, c2] inside (-pi, pi)
        edges = np.sort(rng.uniform(-0.85 * np.pi, 0.85 * np.pi, 2 * nb))
        for b in range(nb):
            c1, c2 = edges[2 * b], edges[2 * b + 1]
            if c2 - c1 < 0.2:
                c2 = c1 + 0.2
            amp = min(0.2, 0.2 * (c2 - c1))
            u0 = rng.uniform(0, T)
            lo = WrappedCurve((u0, c1), (T, 0.0), amp, rng)
            hi = WrappedCurve((u0 + rng.uniform(0, T), c2), (-T, 0.0), amp, rng)
            for cv in (lo, hi):
                lp = periodic_loop(cv, int(rng.integers(seg_lo, seg_hi + 1)), (T, T), axes)
                _open_and_noise(lp, rng, rng.uniform() < open_frac, gap[0], gap[1], sigma)
                loops.append(lp)
        lo_v, hi_v = -np.pi, np.pi
    else:
        domain, periods, axes = DOMAIN_TORUS, (T, T), (0, 1)
        kind = (f // 2) % 2
        if kind == 0:
            h1, h2 = _coprime_pair(rng)
        else:
            h1, h2 = [(1, 0), (0, 1), (1, 1)][int(rng.integers(0, 3))]
        vec = np.array([h1 * T, h2 * T])
        L = np.hypot(*vec)
        delta = T * T / L
        nrm = np.array([-vec[1], vec[0]]) / L
        s0 = rng.uniform(0, T, 2)
        amp = rng.uniform(0.05, 0.2) * delta
        a = WrappedCurve(s0, vec, amp, rng)
        b = WrappedCurve(s0 + 0.5 * delta * nrm + rng.uniform(0, 1) * vec, -vec, amp, rng)
        for cv in (a, b):
            lp = periodic_loop(cv, int(rng.integers(seg_lo, seg_hi + 1)), (T, T), axes)
            _open_and_noise(lp, rng, rng.uniform() < open_frac, gap[0], gap[1], sigma)
            loops.append(lp)
        lo_v, hi_v = 0.0, T
    pts = np.column_stack([rng.uniform(0, T, queries), rng.uniform(lo_v, hi_v, queries)])
    return loops, pts, domain, (T, T)


def config3(seed: int = SEED_C3, num_faces: int = 512, face_ids: Optional[Sequence[int]] = None, **kw):
    ids = list(range(num_faces)) if face_ids is None else list(face_ids)
    face_loops, pts_all, doms, pers, offs = [], [], [], [], [0]
    for f in ids:
        loops, pts, dom, per = config3_face(seed, f, **kw)
        face_loops.append(loops)
        pts_all.append(pts)
        doms.append(dom)
        pers.append(per)
        offs.append(offs[-1] + len(pts))
    faces = _assemble(face_loops, doms, pers, rational=False)
    P = np.concatenate(pts_all)
    q = Queries(u=np.ascontiguousarray(P[:, 0]), v=np.ascontiguousarray(P[:, 1]),
                face_point_offsets=np.asarray(offs, dtype=np.int64))
    return faces, q


# --------------------------------------------------------------------------
# Sphere- and cone-like faces (Sec. 4.3: the singular points are punctured)
# --------------------------------------------------------------------------
SEED_SPHERE = 7


def sphere_face(seed: int, f: int, queries: int = 2048, open_frac: float = 0.2, gap=(1e-4, 1e-2),
                sigma: float = 1e-5, seg_lo: int = 16, seg_hi: int = 64):
    """Face f of a sphere/cone set: cell [0, 2pi) x [-pi/2, pi/2], periodic
    in u, even f sphere (poles at v = -+pi/2), odd f cone (apex at v = -pi/2).
    The face is one of: a cap above a +u loop, a cap below a -u loop (a cone's
    apex region), a band, or both caps (spheres only); loops are wavy
    (amplitude <= 0.12), at least 0.5 apart in height, opened and perturbed
    like the periodic set; half of the faces get a contractible star hole in
    their inside region."""
    rng = _face_rng(seed, f)
    T = TWO_PI
    domain = DOMAIN_SPHERE_U if f % 2 == 0 else DOMAIN_CONE_U
    kinds = ["cap_up", "cap_down", "band", "both"] if domain == DOMAIN_SPHERE_U else ["cap_down", "band"]
    kind = kinds[int(rng.integers(0, len(kinds)))]
    c1 = rng.uniform(-0.9, -0.1)
    c2 = c1 + rng.uniform(0.5, 1.0)
    specs = {"cap_up": [(c1, +1)], "cap_down": [(c2, -1)], "band": [(c1, +1), (c2, -1)],
             "both": [(c1, -1), (c2, +1)]}[kind]
    loops = []
    for c, d in specs:
        cv = WrappedCurve((rng.uniform(0, T), c), (d * T, 0.0), rng.uniform(0.02, 0.12), rng)
        lp = periodic_loop(cv, int(rng.integers(seg_lo, seg_hi + 1)), (T, T), (0,))
        _open_and_noise(lp, rng, rng.uniform() < open_frac, gap[0], gap[1], sigma)
        loops.append(lp)
    if rng.uniform() < 0.5:
        # a clockwise star hole inside the face's inside region
        vc = {"cap_up": c1 + 0.45, "cap_down": c2 - 0.45, "band": 0.5 * (c1 + c2), "both": c2 + 0.45}[kind]
        hc = StarCurve(rng, rho=0.08, center=(rng.uniform(0.5, T - 0.5), vc))
        ns = int(rng.integers(6, 17))
        loops.append(reverse_loop(sampled_star_loop(hc, ns, rng.integers(1, 4, ns))))
    pts = np.column_stack([rng.uniform(0, T, queries), rng.uniform(-0.5 * np.pi, 0.5 * np.pi, queries)])
    return loops, pts, domain, (T, 0.0)


def sphere_set(seed: int = SEED_SPHERE, num_faces: int = 64, face_ids: Optional[Sequence[int]] = None, **kw):
    ids = list(range(num_faces)) if face_ids is None else list(face_ids)
    face_loops, pts_all, doms, pers, offs = [], [], [], [], [0]
    for f in ids:
        loops, pts, dom, per = sphere_face(seed, f, **kw)
        face_loops.append(loops)
        pts_all.append(pts)
        doms.append(dom)
        pers.append(per)
        offs.append(offs[-1] + len(pts))
    faces = _assemble(face_loops, doms, pers, rational=False)
    P = np.concatenate(pts_all)
    q = Queries(u=np.ascontiguousarray(P[:, 0]), v=np.ascontiguousarray(P[:, 1]),
                face_point_offsets=np.asarray(offs, dtype=np.int64))
    return faces, q


# --------------------------------------------------------------------------
# Applications (Sec. 5.4): multi-patch surfaces and tessellation grids
# --------------------------------------------------------------------------
@dataclass
class Patches:
    """Faces grouped by base surface, with sample points on each surface."""
    faces: "Faces"
    surface_face_offsets: np.ndarray  # int32 [S+1]
    surface_faces: np.ndarray  # int32 [K]
    u: np.ndarray  # float64 [N], grouped by surface
    v: np.ndarray
    surface_point_offsets: np.ndarray  # int64 [S+1]

    @property
    def num_surfaces(self) -> int:
        return len(self.surface_face_offsets) - 1


def _moved(lp: _Loop, scale: float, center) -> _Loop:
    out = _Loop()
    for cp, w in zip(lp.cps, lp.ws):
        out.cps.append(cp * scale + np.asarray(center, dtype=np.float64))
        out.ws.append(None if w is None else w.copy())
    return out


def brep_patches(seed: int = SEED_BREP, num_surfaces: int = 64, points_per_surface: int = 16384,
                 faces_lo: int = 2, faces_hi: int = 6, periodic_every: int = 4, seg_hi: int = 256,
                 unreferenced: int = 0) -> Patches:
    """A synthetic multi-patch B-Rep (the Boolean-union models of Sec. 5.4.1):
    each base surface is referenced by several trimmed faces and sampled
    uniformly over its parameter rectangle.

    * planar surfaces ([-2, 2]^2): faces_lo..faces_hi faces, each a batched-set
      face (star outer loop with holes) scaled by U(0.35, 0.9) and moved to a
      centre in U(-1.2, 1.2)^2; faces may overlap;
    * every ``periodic_every``-th surface is a cylinder ([0, 2 pi) x [-pi, pi))
      referenced by two faces of the periodic set (bands with open, noisy
      loops);
    * ``unreferenced`` extra faces at the end belong to no surface."""
    face_loops, doms, pers = [], [], []
    sfo, sff, pts, spo = [0], [], [], [0]
    for s in range(num_surfaces):
        rng = _face_rng(seed, s)
        periodic = periodic_every > 0 and s % periodic_every == periodic_every - 1
        if periodic:
            for j in range(2):
                loops, _, dom, per = config3_face(seed, 2 * (2 * s + j), queries=1)
                sff.append(len(face_loops))
                face_loops.append(loops)
                doms.append(dom)
                pers.append(list(per))
            P = np.column_stack([rng.uniform(0, TWO_PI, points_per_surface),
                                 rng.uniform(-np.pi, np.pi, points_per_surface)])
        else:
            k = int(rng.integers(faces_lo, faces_hi + 1))
            for j in range(k):
                loops, _, _ = config2_face(seed, 64 * s + j, q_lo=1, q_hi=1, near_frac=0.0, seg_hi=seg_hi)
                scale = rng.uniform(0.35, 0.9)
                c = rng.uniform(-1.2, 1.2, 2)
                sff.append(len(face_loops))
                face_loops.append([_moved(lp, scale, c) for lp in loops])
                doms.append(DOMAIN_PLANE)
                pers.append([0.0, 0.0])
            P = rng.uniform(-2.0, 2.0, size=(points_per_surface, 2))
        sfo.append(len(sff))
        pts.append(P)
        spo.append(spo[-1] + len(P))
    for j in range(unreferenced):
        loops, _, _ = config2_face(seed, 10 ** 6 + j, q_lo=1, q_hi=1, near_frac=0.0, seg_hi=seg_hi)
        face_loops.append(loops)
        doms.append(DOMAIN_PLANE)
        pers.append([0.0, 0.0])
    faces = _assemble(face_loops, doms, pers, rational=True)
    P = np.concatenate(pts) if pts else np.zeros((0, 2))
    return Patches(faces, np.asarray(sfo, dtype=np.int32), np.asarray(sff, dtype=np.int32),
                   np.ascontiguousarray(P[:, 0]), np.ascontiguousarray(P[:, 1]), np.asarray(spo, dtype=np.int64))


def tessellation_grids(faces: "Faces", n: int, margin: float = 0.05):
    """One n x n grid per face (u0, v0, du, dv, nu, nv): the period cell of a
    periodic face (cylinder [0, T_u) x [-pi, pi), torus [0, T_u) x [0, T_v),
    as the periodic set lays them out), the control points' bounding box
    widened by ``margin`` of its size for a planar face."""
    grids = []
    F = len(faces.face_loop_offsets) - 1
    for f in range(F):
        dom = int(faces.face_domain[f])
        Tu, Tv = float(faces.face_period[2 * f]), float(faces.face_period[2 * f + 1])
        if dom == DOMAIN_TORUS:
            grids.append((0.0, 0.0, Tu / n, Tv / n, n, n))
        elif dom == DOMAIN_CYLINDER_U:
            grids.append((0.0, -np.pi, Tu / n, TWO_PI / n, n, n))
        else:
            l0, l1 = faces.face_loop_offsets[f], faces.face_loop_offsets[f + 1]
            s0, s1 = faces.loop_seg_offsets[l0], faces.loop_seg_offsets[l1]
            c0, c1 = faces.seg_cp_offsets[s0], faces.seg_cp_offsets[s1]
            u, v = faces.cp_u[c0:c1], faces.cp_v[c0:c1]
            w, h = u.max() - u.min(), v.max() - v.min()
            u0, v0 = u.min() - margin * w, v.min() - margin * h
            grids.append((float(u0), float(v0), (1 + 2 * margin) * w / n, (1 + 2 * margin) * h / n, n, n))
    return grids


# --------------------------------------------------------------------------
# helpers for tests
# --------------------------------------------------------------------------
def faces_from_loops(face_loops, domains=None, periods=None, rational=None) -> Faces:
    """Build a Faces container from explicit python loops.

    ``face_loops``: list (faces) of list (loops) of list (segments) of
    (cps [(n+1),2], weights or None)."""
    fl = []
    any_rat = False
    for loops in face_loops:
        lps = []
        for segs in loops:
            lp = _Loop()
            for cp, w in segs:
                lp.cps.append(np.asarray(cp, dtype=np.float64))
                lp.ws.append(None if w is None else np.asarray(w, dtype=np.float64))
                any_rat |= w is not None
            lps.append(lp)
        fl.append(lps)
    F = len(fl)
    domains = [DOMAIN_PLANE] * F if domains is None else domains
    periods = [[0.0, 0.0]] * F if periods is None else periods
    return _assemble(fl, domains, periods, rational=any_rat if rational is None else rational)


def queries_for_faces(per_face_points: Sequence[np.ndarray]) -> Queries:
    offs = [0]
    for p in per_face_points:
        offs.append(offs[-1] + len(p))
    P = np.concatenate([np.asarray(p, dtype=np.float64).reshape(-1, 2) for p in per_face_points]) \
        if per_face_points else np.zeros((0, 2))
    return Queries(u=np.ascontiguousarray(P[:, 0]), v=np.ascontiguousarray(P[:, 1]),
                   face_point_offsets=np.asarray(offs, dtype=np.int64))


def subset_queries(q: Queries, idx: np.ndarray):
    """Pick queries ``idx`` (global indices).  Returns (face id per point, u, v)."""
    fid = q.face_ids()[idx]
    return fid, q.u[idx].copy(), q.v[idx].copy()
