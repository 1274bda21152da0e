"""Helpers shared by the GPU tests: run the HIP library through its binding
and compare with the CPU oracle."""
import numpy as np

FP64_TOL = 1e-12  # |omega_gpu - omega_oracle| bound for FP64 (far from curves)
# Periodic copies are evaluated at translated queries x - t (translation
# identity of App. C.1), and |t| reaches a few tens on the test domains
# (torus homologies up to 5 on a 2 pi cell).  The FP64 rounding of x - t then
# moves the query by up to a few units in the last place of |t|; a bound of
# SHIFT_ROUNDING = 2^-44 (8 ulps of 32) covers it.  At such a point the
# winding number itself is only determined to |grad omega| * SHIFT_ROUNDING
# by its FP64 input, so the FP64 bound there is FP64_TOL plus that amount.
SHIFT_ROUNDING = 2.0 ** -44
GRAD_STEP = 1e-7  # central-difference step of the oracle's gradient estimate


def run_wn(faces, queries, *, offsets_host=True, stride=1, **kw):
    import torch

    from paper_2510_25159_amd import wn

    fs = kw.pop("faceset", None)
    if fs is None:
        fs = wn.FaceSet(faces, **kw.pop("create", {}))
    dev = torch.device("cuda:0")
    if stride == 1:
        u = torch.from_numpy(np.ascontiguousarray(queries.u)).to(dev)
        v = torch.from_numpy(np.ascontiguousarray(queries.v)).to(dev)
    else:
        inter = np.empty(2 * queries.num_points)
        inter[0::2], inter[1::2] = queries.u, queries.v
        t = torch.from_numpy(inter).to(dev)
        u = t  # element i at u[2 i]
        v = t[1:]  # element i at v[2 i]
    offs = torch.from_numpy(np.ascontiguousarray(queries.face_point_offsets, dtype=np.int64)).to(dev)
    if stride != 1:
        n = queries.num_points
        out_w = torch.empty(n, dtype=torch.float64, device=dev)
        out_l = torch.empty(n, dtype=torch.uint8, device=dev)
        fs.query(u, v, offs, queries.face_point_offsets if offsets_host else None, out_w, out_l, stride=stride, **kw)
    else:
        out_w, out_l = fs.query(u, v, offs, queries.face_point_offsets if offsets_host else None, **kw)
    torch.cuda.synchronize()
    return out_w.cpu().numpy(), out_l.cpu().numpy()


def translation_tol(oracle_lib, faces, point_face, u, v, idx, tol=FP64_TOL):
    """Per-point FP64 bounds for points idx of periodic faces: tol plus
    |grad omega| * SHIFT_ROUNDING, the gradient estimated by the oracle with
    central differences (its own arithmetic, independent of the GPU).
    Points of planar faces keep tol (no translation is applied to them)."""
    idx = np.asarray(idx, dtype=np.int64)
    out = np.full(idx.size, tol)
    per = np.asarray(faces.face_domain)[np.asarray(point_face)[idx]] != 0
    if not per.any():
        return out
    j = idx[per]
    pf = np.asarray(point_face, dtype=np.int32)[j]
    x = np.asarray(u, dtype=np.float64)[j]
    y = np.asarray(v, dtype=np.float64)[j]
    h = GRAD_STEP
    xs = np.concatenate([x + h, x - h, x, x])
    ys = np.concatenate([y, y, y + h, y - h])
    w, _ = oracle_lib.query(faces, np.tile(pf, 4), xs, ys)
    n = j.size
    gx = (w[:n] - w[n:2 * n]) / (2 * h)
    gy = (w[2 * n:3 * n] - w[3 * n:]) / (2 * h)
    out[per] = tol + np.hypot(gx, gy) * SHIFT_ROUNDING
    return out


def compare(w_gpu, lab_gpu, w_orc, near_orc, tol=FP64_TOL, rule=0, tol_fn=None):
    """Return a dict of parity statistics; raises AssertionError on failure.

    tol_fn(indices) -> per-point bounds, consulted only for the compared
    points whose error exceeds tol (e.g. translation_tol for periodic faces)."""
    w_gpu = np.asarray(w_gpu)
    lab_gpu = np.asarray(lab_gpu)
    far = near_orc == 0
    # on-boundary may only be reported for points the oracle puts within 1e-9 of a curve
    onb = lab_gpu == 2
    assert not np.any(onb & far), f"{int(np.sum(onb & far))} on-boundary labels on certified-far points"
    assert not np.any(lab_gpu == 3), "unexpected invalid labels"
    if rule == 0:
        want = (np.abs(w_orc) > 0.5).astype(np.uint8)
    else:
        want = (w_orc > 0.5).astype(np.uint8)
    # ambiguous (omega within 1e-9 of a half integer) points are reported separately
    amb = np.abs(np.abs(w_orc) - np.round(np.abs(w_orc) - 0.5) - 0.5) < 1e-9
    cmp = far & ~amb
    mism = int(np.sum(lab_gpu[cmp] != want[cmp]))
    err = np.abs(w_gpu[cmp] - w_orc[cmp])
    maxerr = float(err.max()) if err.size else 0.0
    assert mism == 0, f"{mism} inside/outside mismatches"
    n_cond = 0
    if maxerr > tol and tol_fn is not None:
        big = np.flatnonzero(cmp)[err > tol]
        bound = tol_fn(big)
        e = np.abs(w_gpu[big] - w_orc[big])
        worst = int(np.argmax(e / bound))
        assert np.all(e <= bound), (f"max |domega| = {e[worst]:.3e} > conditioned bound {bound[worst]:.3e} "
                                    f"at point {int(big[worst])}")
        n_cond = int(big.size)
    else:
        assert maxerr <= tol, f"max |domega| = {maxerr:.3e} > {tol:.1e}"
    return {"compared": int(cmp.sum()), "excluded_near": int((~far).sum()), "ambiguous": int((far & amb).sum()),
            "mismatches": mism, "max_abs_err": maxerr, "conditioned": n_cond}
