"""Oracle of the application drivers of Sec. 5.4 (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
may import it.  Both functions are plain compositions of the winding-number
oracle (``oracle.query``) with the definitions below; nothing is shared with
the HIP library.

* Tessellation (Sec. 5.4.3): sample points of a uniform grid in a face's
  parameter domain are classified.  The samples here are the cell centres,
  u0 + (i + 1/2) du and v0 + (j + 1/2) dv (each product and each sum rounded
  once, as numpy does), face by face and row-major (i along u fastest).
* Multiple patches (Sec. 5.4.1): a point sampled on a base surface is inside
  when it lies inside any trimmed face that references the surface, and
  outside otherwise.
"""
from __future__ import annotations

import numpy as np

from . import query


def grid_samples(grids):
    """(face id, u, v) of every cell centre of ``grids`` (a sequence of
    (u0, v0, du, dv, nu, nv), one per face), face by face, row-major."""
    fids, us, vs = [], [], []
    for f, (u0, v0, du, dv, nu, nv) in enumerate(grids):
        i = np.tile(np.arange(nu, dtype=np.float64), nv)
        j = np.repeat(np.arange(nv, dtype=np.float64), nu)
        us.append(np.float64(u0) + (i + 0.5) * np.float64(du))
        vs.append(np.float64(v0) + (j + 0.5) * np.float64(dv))
        fids.append(np.full(nu * nv, f, dtype=np.int32))
    if not us:
        return np.zeros(0, np.int32), np.zeros(0), np.zeros(0)
    return np.concatenate(fids), np.concatenate(us), np.concatenate(vs)


def inside_label(omega, rule: int = 0):
    """Label from a winding number: nonzero rule |omega| > 1/2, positive
    rule omega > 1/2 (the winding number of a closed loop is an integer; the
    half-way threshold reads it off an open or noisy one)."""
    omega = np.asarray(omega)
    return (np.abs(omega) > 0.5) if rule == 0 else (omega > 0.5)


def classify_surfaces(faces, surface_face_offsets, surface_faces, u, v, surface_point_offsets, rule: int = 0,
                      near_tol: float = 1e-9, nthreads=None):
    """Multi-patch labels.  Returns (inside bool [N], first inside face int32
    [N] (-1: none), near bool [N]).  ``near`` marks points within ``near_tol``
    of a curve of some face of their surface, where the oracle does not
    decide a face's label; ``inside`` and ``first`` hold the label the other
    faces decide for them, and are exact elsewhere."""
    sfo = np.asarray(surface_face_offsets)
    sff = np.asarray(surface_faces)
    spo = np.asarray(surface_point_offsets)
    n = int(spo[-1])
    inside = np.zeros(n, dtype=bool)
    first = np.full(n, -1, dtype=np.int32)
    near = np.zeros(n, dtype=bool)
    for s in range(len(sfo) - 1):
        a, b = int(spo[s]), int(spo[s + 1])
        if a == b:
            continue
        for k in range(int(sfo[s]), int(sfo[s + 1])):
            f = int(sff[k])
            w, nr = query(faces, np.full(b - a, f, dtype=np.int32), u[a:b], v[a:b], near_tol=near_tol,
                          nthreads=nthreads)
            ins = inside_label(w, rule) & (nr == 0)
            near[a:b] |= nr != 0
            take = ins & (first[a:b] < 0)
            first[a:b][take] = f
            inside[a:b] |= ins
    return inside, first, near
