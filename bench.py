"""Benchmark: batched generalized-winding-number containment on one MI355X.

A step is one pass of the whole query path (work-item build, far-field pair
pass, near-pair recursion pass, finalize) over the batched planar set:
2,000 faces, 1 outer + 0-7 hole loops, 4-256 segments per loop of degree
1-5 with rational weights, 1k-64k points per face, 30% of them within 1e-3
of a curve.  Inputs sit in HBM before the timed region starts.

Prints one JSON line (rank 0).  `value` is point x segment pair evaluations
per second of the batched schedule; the plain schedule (one launch per face,
in-line recursion) is reported beside it, together with queries/s, the
CPU oracle's throughput on a bounded sample (and single-threaded on config
1), and per-kernel roofline positions.  The timed steps run the far and
near passes in series (the library's default); `roofline` is the dominant
kernel of those steps: algorithmic flops per launch over its HIP-event
launch duration on the stream it runs on, against the FP64 VALU peak, and
its measured HBM bytes per launch against 8 TB/s.  The overlapped form
(WN_FLAG_OVERLAP) is timed beside it for reference (rooflines_overlapped).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "point×segment winding evals/s & queries/s, plain vs batched form, 0 mismatches"
# Algorithmic FP64 work of one (query, segment) pair at the root of Alg. 1
# (FMA = 2 flops, sqrt/atan2/compare = 1): two distances (2 x 6), the ellipse
# comparison (2), the chord angle (cross 3 + dot 3 + atan2 1 + accumulate 1).
FLOPS_PER_PAIR = 22
PEAK_FP64_VALU = 78.6e12   # MI355X vector FP64, FLOP/s
PEAK_HBM = 8.0e12          # B/s
# HBM traffic per launch measured with rocprofv3 counters (FETCH_SIZE and
# WRITE_SIZE, each scaled by a plain copy's reading); valid only while the
# library sources are the ones the counters were taken on.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_config2.txt")
LIB_SOURCES = os.path.join(ROOT, "paper_2510_25159_amd", "csrc")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash() -> str:
    """sha256 over the library's kernel and host sources (sorted by name)."""
    import hashlib

    h = hashlib.sha256()
    for name in sorted(os.listdir(LIB_SOURCES)):
        if name.endswith((".hip", ".h")):
            h.update(name.encode())
            with open(os.path.join(LIB_SOURCES, name), "rb") as f:
                h.update(f.read())
    return h.hexdigest()


def measured_traffic() -> dict:
    """{kernel: HBM bytes per launch} from the committed counter summary, or
    {} when it is missing or was taken on other sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            lines = f.read().splitlines()
    except OSError:
        return {}
    kv = {}
    for ln in lines:
        if "=" in ln and not ln.startswith((" ", "#", "$")):
            k, v = ln.split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != source_hash():
        return {}
    out = {}
    for k, v in kv.items():
        if k.startswith("traffic_bytes_per_launch "):
            out[k.split()[1]] = float(v)
    return out


def measured_copy_rate(torch, gib: int = 2, reps: int = 10) -> float:
    """HBM rate of a plain device copy (bytes read + written per second):
    the measured counterpart of the published 8 TB/s."""
    n = gib * (1 << 30) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    rate = 2.0 * 8 * n * reps / (a.elapsed_time(b) / 1e3)
    del src, dst
    torch.cuda.empty_cache()
    return rate


def host_cpu() -> dict:
    """CPU model and logical CPU count of the host (from /proc/cpuinfo)."""
    model, n = None, 0
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    n += 1
                    model = model or ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return {"model": model, "nproc": n or os.cpu_count()}


def _dev_queries(torch, q):
    dev = torch.device("cuda:0")
    return (torch.from_numpy(q.u).to(dev), torch.from_numpy(q.v).to(dev),
            torch.from_numpy(q.face_point_offsets).to(dev))


def _time_query(torch, fs, tens, offs_host, reps, **kw):
    from paper_2510_25159_amd import wn

    prof = wn.Profile(64 * (reps + 1))
    fs.query(*tens, offs_host, **kw)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        fs.query(*tens, offs_host, profile=prof, **kw)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3 / reps
    return ms, {k: t_ / max(n, 1) for k, (n, t_) in prof.collect().items()}


def section_config1(args):
    """One planar face, 64 cubic segments, 65,536 uniform points."""
    import torch

    from paper_2510_25159_amd import wn
    from paper_2510_25159_amd import workloads as W

    faces, q = W.config1()
    fs = wn.FaceSet(faces)
    tens = _dev_queries(torch, q)
    pairs = faces.num_segments * q.num_points
    out = {"pairs": pairs, "points": q.num_points}
    for name, sched in (("plain", 0), ("batched", 1)):
        ms, k = _time_query(torch, fs, tens, q.face_point_offsets, 50, schedule=sched)
        out[name] = {"ms_per_step": ms, "evals_per_s": pairs / (ms / 1e3), "queries_per_s": q.num_points / (ms / 1e3),
                     "kernel_ms": k}
    kf = out["plain"]["kernel_ms"].get("k_far", float("nan"))
    out["plain"]["far_roofline_frac"] = FLOPS_PER_PAIR * pairs / (kf / 1e3) / PEAK_FP64_VALU
    # wall time per query without the per-kernel events, and the batched query
    # as an autotuned plan (one graph replay per query: no host work per call)
    reps = 200
    for name, sched in (("plain", 0), ("batched", 1)):
        ow, ol = fs.query(*tens, q.face_point_offsets, schedule=sched)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            fs.query(*tens, q.face_point_offsets, ow, ol, schedule=sched)
        torch.cuda.synchronize()
        out[name]["ms_per_step_unprofiled"] = (time.perf_counter() - t) * 1e3 / reps
    lab_plain = fs.query(*tens, q.face_point_offsets, schedule=0)[1].cpu().numpy()
    ow = torch.empty(q.num_points, dtype=torch.float64, device="cuda:0")
    ol = torch.empty(q.num_points, dtype=torch.uint8, device="cuda:0")
    plan = wn.Plan(fs, *tens, ow, ol)
    rep = plan.autotune(reps=5)
    plan.launch()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(reps):
        plan.launch()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3 / reps
    out["batched_plan"] = {"ms_per_step": ms, "evals_per_s": pairs / (ms / 1e3), "autotune": rep,
                           "labels_equal_plain": bool(np.array_equal(ol.cpu().numpy(), lab_plain))}
    # where the plain kernel's time goes: the same face with the points whose
    # pairs recurse removed (found from the kernel's own depth log) leaves the
    # far scan alone; the difference is the tail of the in-line recursions
    spf = fs.info().max_segments_per_face
    dl = torch.zeros(q.num_points * spf, dtype=torch.uint8, device="cuda:0")
    fs.query(*tens, q.face_point_offsets, schedule=0, depth_log=dl)
    torch.cuda.synchronize()
    deep = dl.view(q.num_points, spf).amax(dim=1).cpu().numpy()
    keep = np.flatnonzero(deep == 0)
    qf = W.queries_for_faces([np.column_stack([q.u[keep], q.v[keep]])])
    msf, kff = _time_query(torch, fs, _dev_queries(torch, qf), qf.face_point_offsets, 50, schedule=0)
    out["plain"]["recursion"] = {"points_with_near_pairs": int(q.num_points - keep.size),
                                 "max_depth": int(deep.max()),
                                 "far_only_points": int(keep.size), "far_only_k_far_ms": kff.get("k_far"),
                                 "far_only_ms_per_step": msf}
    return out


def section_long_path(args):
    """Path hierarchy on a long path: one star face of 16,384 cubic segments
    (config 1's generator) and 2^20 uniform points, flat far pass against the
    hierarchy (labels compared)."""
    import torch

    from paper_2510_25159_amd import wn
    from paper_2510_25159_amd import workloads as W

    faces = W.config1_faces(nseg=16384)
    q = W.config1_queries(n=1 << 20)
    fs = wn.FaceSet(faces)
    tens = _dev_queries(torch, q)
    pairs = faces.num_segments * q.num_points
    out = {"segments": faces.num_segments, "points": q.num_points, "pairs": pairs}
    labs = {}
    for name, tree in (("flat", 0), ("hierarchy", 1), ("auto", 2)):
        ms, k = _time_query(torch, fs, tens, q.face_point_offsets, 5, schedule=1, path_hierarchy=tree)
        w, lab = fs.query(*tens, q.face_point_offsets, schedule=1, path_hierarchy=tree)
        labs[name] = lab.cpu().numpy()
        out[name] = {"ms_per_step": ms, "queries_per_s": q.num_points / (ms / 1e3), "kernel_ms": k}
    both = (labs["flat"] != 2) & (labs["hierarchy"] != 2) & (labs["auto"] != 2)
    out["label_differences"] = int(np.sum(labs["flat"][both] != labs["hierarchy"][both]) +
                                   np.sum(labs["flat"][both] != labs["auto"][both]))
    out["speedup_hierarchy"] = out["flat"]["ms_per_step"] / out["hierarchy"]["ms_per_step"]
    return out


def _seg_counts(faces):
    lso = np.asarray(faces.loop_seg_offsets)
    flo = np.asarray(faces.face_loop_offsets)
    return lso[flo[1:]] - lso[flo[:-1]]


def section_spheres(args):
    """512 sphere- and cone-like faces (punctured, u-periodic), 2^20 points."""
    import torch

    from paper_2510_25159_amd import wn
    from paper_2510_25159_amd import workloads as W

    faces, q = W.sphere_set(num_faces=512)
    fs = wn.FaceSet(faces)
    tens = _dev_queries(torch, q)
    out = {"faces": faces.num_faces, "segments": faces.num_segments, "points": q.num_points}
    ms, k = _time_query(torch, fs, tens, q.face_point_offsets, 10, schedule=1)
    out["batched"] = {"ms_per_step": ms, "queries_per_s": q.num_points / (ms / 1e3), "kernel_ms": k}
    return out


def section_tessellation(args):
    """Tessellation driver (wn_classify_grid): the cell centres of a 128 x 128
    grid over the period cell of each of the 512 periodic faces (8.4M
    samples), generated on the device and classified."""
    import torch

    from paper_2510_25159_amd import wn
    from paper_2510_25159_amd import workloads as W

    faces, _ = W.config3()
    grids = W.tessellation_grids(faces, 128)
    fs = wn.FaceSet(faces)
    n = sum(g[4] * g[5] for g in grids)
    pairs = int(np.sum(_seg_counts(faces) * np.array([g[4] * g[5] for g in grids])))
    out = {"faces": faces.num_faces, "samples": n, "segment_pairs": pairs}
    for name, sched in (("batched", 1),):
        fs.classify_grid(grids, schedule=sched)
        torch.cuda.synchronize()
        reps = 5
        prof = wn.Profile(64 * (reps + 1))
        t = time.perf_counter()
        for _ in range(reps):
            u, v, w, lab = fs.classify_grid(grids, schedule=sched, profile=prof)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3 / reps
        k = {a: b / max(m, 1) for a, (m, b) in prof.collect().items()}
        lab = lab.cpu().numpy()
        out[name] = {"ms_per_call": ms, "samples_per_s": n / (ms / 1e3), "kernel_ms": k,
                     "inside_fraction": float(np.mean(lab == 1))}
    return out


def section_multipatch(args):
    """Multi-patch driver (wn_classify_surfaces): 128 base surfaces (every
    fourth a cylinder with two periodic faces, the others planar with 2-6
    trimmed faces) and 32,768 uniform samples per surface."""
    import torch

    from paper_2510_25159_amd import wn
    from paper_2510_25159_amd import workloads as W

    p = W.brep_patches(num_surfaces=128, points_per_surface=32768)
    fs = wn.FaceSet(p.faces)
    dev = torch.device("cuda:0")
    u, v = torch.from_numpy(p.u).to(dev), torch.from_numpy(p.v).to(dev)
    spo = p.surface_point_offsets
    nps = np.diff(spo)
    segs = _seg_counts(p.faces)
    copies, pairs = 0, 0
    for s in range(p.num_surfaces):
        fl = p.surface_faces[p.surface_face_offsets[s]:p.surface_face_offsets[s + 1]]
        copies += int(nps[s]) * len(fl)
        pairs += int(nps[s]) * int(segs[fl].sum())
    out = {"surfaces": p.num_surfaces, "faces": p.faces.num_faces, "points": int(spo[-1]), "face_copies": copies,
           "segment_pairs": pairs}
    fs.classify_surfaces(p.surface_face_offsets, p.surface_faces, u, v, spo)
    torch.cuda.synchronize()
    reps = 5
    prof = wn.Profile(64 * (reps + 1))
    t = time.perf_counter()
    for _ in range(reps):
        lab, face = fs.classify_surfaces(p.surface_face_offsets, p.surface_faces, u, v, spo, profile=prof)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t) * 1e3 / reps
    k = {a: b / max(m, 1) for a, (m, b) in prof.collect().items()}
    lab = lab.cpu().numpy()
    out["batched"] = {"ms_per_call": ms, "points_per_s": int(spo[-1]) / (ms / 1e3), "kernel_ms": k,
                      "inside_fraction": float(np.mean(lab == 1))}
    return out


def section_config3(args):
    """512 periodic faces (cylinder / torus), 2^20 points."""
    import torch

    from paper_2510_25159_amd import wn
    from paper_2510_25159_amd import workloads as W

    faces, q = W.config3()
    fs = wn.FaceSet(faces)
    tens = _dev_queries(torch, q)
    out = {"faces": faces.num_faces, "segments": faces.num_segments, "points": q.num_points}
    for name, sched in (("plain", 0), ("batched", 1)):
        ms, k = _time_query(torch, fs, tens, q.face_point_offsets, 10 if sched else 3, schedule=sched)
        out[name] = {"ms_per_step": ms, "queries_per_s": q.num_points / (ms / 1e3), "kernel_ms": k}
    # the (query, segment copy) pairs of the copy windows, counted by the
    # periodic far pass itself in one more (untimed) query
    st = torch.zeros(wn.STATS_COUNT, dtype=torch.int64, device="cuda:0")
    fs.query(*tens, q.face_point_offsets, schedule=1, stats=st)
    torch.cuda.synchronize()
    pairs = int(st[wn.STAT_NAMES.index("periodic_pairs")].item())
    b = out["batched"]
    kp = b["kernel_ms"].get("k_far_periodic", float("nan"))
    out["pairs"] = pairs
    b["evals_per_s"] = pairs / (b["ms_per_step"] / 1e3)
    out["plain"]["evals_per_s"] = pairs / (out["plain"]["ms_per_step"] / 1e3)
    b["far_periodic_roofline_frac"] = FLOPS_PER_PAIR * pairs / (kp / 1e3) / PEAK_FP64_VALU
    return out


def section_config4(args):
    """Learned depth predictor: train on 5M pairs (seed 40), evaluate 10M pairs (seed 41)."""
    import torch

    from paper_2510_25159_amd import wn
    from paper_2510_25159_amd import workloads as W

    out = {}
    for variant, near in (("uniform", 0.0), ("near30", 0.3)):
        ft, qt = W.config4("train", near_frac=near)
        fe, qe = W.config4("eval", near_frac=near)
        pr = wn.Predictor(seed=7)
        t = time.perf_counter()
        rep = pr.train(wn.FaceSet(ft), *_dev_queries(torch, qt), epochs=60, lr=3e-3, seed=1)
        rep["train_s"] = time.perf_counter() - t
        fs = wn.FaceSet(fe)
        tens = _dev_queries(torch, qe)
        res = {"train": rep}
        for name, sched, src in (("unbinned", 1, 3), ("mlp_binned", 2, 0), ("mlp_valu_binned", 2, 4),
                                 ("heuristic_binned", 2, 1), ("measured_binned", 2, 2)):
            ms, k = _time_query(torch, fs, tens, qe.face_point_offsets, 20, schedule=sched, predictor=pr,
                                bin_source=src)
            res[name] = {"ms_per_step": ms, "k_near_ms": k.get("k_near"), "k_bin_ms": k.get("k_bin")}
        out[variant] = res
    # the network alone: 8M standardised feature rows, matrix cores vs VALU
    n = 8 << 20
    X = torch.randn(n, wn.MLP_IN, dtype=torch.float32, device="cuda:0")
    fwd = {}
    for name, fn in (("mfma", pr.predict_mfma), ("valu", pr.predict)):
        fn(X)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(20):
            fn(X)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / 20
        flop = 2.0 * n * (wn.MLP_IN * wn.MLP_HIDDEN + wn.MLP_HIDDEN * wn.MLP_HIDDEN + wn.MLP_HIDDEN)
        fwd[name] = {"ms": ms, "rows_per_s": n / (ms / 1e3), "tflops": flop / (ms / 1e3) / 1e12}
    out["mlp_forward_8M_rows"] = fwd
    return out


def section_degree(args):
    """Runtime against boundary degree (Sec. 5): 512 cubic star faces (64
    segments each) elevated to degree 4 and 5 without changing the curves,
    4096 points per face, all on the curves (the recursion's worst case) or
    all uniform."""
    import torch

    from paper_2510_25159_amd import wn
    from paper_2510_25159_amd import workloads as W

    out = {}
    for sampling, frac in (("on_curve", 1.0), ("uniform", 0.0)):
        res = {}
        for d in (3, 4, 5):
            faces, q = W.degree_set(d, num_faces=512, points_per_face=4096, on_curve_frac=frac)
            fs = wn.FaceSet(faces)
            tens = _dev_queries(torch, q)
            ms, k = _time_query(torch, fs, tens, q.face_point_offsets, 10, schedule=1)
            st = torch.zeros(wn.STATS_COUNT, dtype=torch.int64, device="cuda:0")
            fs.query(*tens, q.face_point_offsets, schedule=1, stats=st)
            torch.cuda.synchronize()
            stats = dict(zip(wn.STAT_NAMES, st.cpu().numpy().tolist()))
            res[f"degree{d}"] = {"ms_per_step": ms, "queries_per_s": q.num_points / (ms / 1e3),
                                 "kernel_ms": k, "splits_per_point": stats["splits"] / q.num_points,
                                 "near_pairs_per_point": stats["near_pairs"] / q.num_points,
                                 "max_depth": stats["max_depth"]}
        out[sampling] = res
    out["points"] = 512 * 4096
    return out


def section_config5(args):
    """Serving loop: Poisson arrivals, resident faces, graph replays."""
    from paper_2510_25159_amd import serving

    return serving.run(duration=args.serving_duration)


SECTIONS = (("config1", section_config1), ("long_path", section_long_path), ("config3", section_config3),
            ("config4", section_config4), ("config5", section_config5), ("spheres", section_spheres),
            ("tessellation", section_tessellation), ("multipatch", section_multipatch), ("degree", section_degree))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--faces", type=int, default=2000, help="faces of the batched set (default: the full set)")
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--mixed-steps", type=int, default=5)
    ap.add_argument("--tree-steps", type=int, default=10, help="timed steps with the path hierarchy")
    ap.add_argument("--cp-steps", type=int, default=3, help="timed steps with the subdivided control-point bound")
    ap.add_argument("--cpu-sample", type=int, default=15000000, help="points of the oracle sample (about 15 s on 16 threads)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--schedule", type=int, default=1)
    ap.add_argument("--qpw", type=int, default=0)
    ap.add_argument("--policy", type=int, default=0)
    ap.add_argument("--no-extra", action="store_true", help="skip the extra sections")
    ap.add_argument("--serial-steps", type=int, default=10,
                    help="timed steps with the far and near passes in series (each kernel alone on the GPU): "
                         "the per-kernel rooflines")
    ap.add_argument("--overlap", type=int, default=0,
                    help="0: the timed steps run the far and near passes in series (default, the faster form); "
                         "1: the face set is created with WN_FLAG_OVERLAP and the timed steps overlap near and far "
                         "passes of different face runs")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the timed batched steps and the work counters (profiling runs)")
    ap.add_argument("--sections", default="", help="comma list of the extra sections to run (default: all)")
    ap.add_argument("--sections-only", action="store_true",
                    help="run only the extra sections named by --sections (profiling runs of other workloads)")
    ap.add_argument("--serving-duration", type=float, default=10.0)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device copy of this size first (counter calibration under rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(queries and faces shard across GPUs without any exchange).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2510_25159_amd import wn
    from paper_2510_25159_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.sections_only:
        only = {x for x in args.sections.split(",") if x}
        res = {}
        for name, fn in SECTIONS:
            if name in only:
                t = time.time()
                res[name] = fn(args)
                log(f"{name}: {time.time() - t:.1f}s")
        print(json.dumps({"sections": res}), flush=True)
        return
    t0 = time.time()
    faces, q = W.config2(face_ids=range(args.faces))
    S_f = faces.face_segment_counts()
    Q_f = np.diff(q.face_point_offsets)
    pairs = int(np.sum(S_f * Q_f))
    N = q.num_points
    log(f"generated {args.faces} faces, {faces.num_segments} segments, {N} points, {pairs:.3e} pairs "
        f"in {time.time() - t0:.1f}s")

    u = torch.from_numpy(q.u).to(dev)
    v = torch.from_numpy(q.v).to(dev)
    offs = torch.from_numpy(q.face_point_offsets).to(dev)
    out_w = torch.empty(N, dtype=torch.float64, device=dev)
    out_l = torch.empty(N, dtype=torch.uint8, device=dev)
    fs = wn.FaceSet(faces, flags=wn.FLAG_OVERLAP if args.overlap else 0)
    stream = torch.cuda.current_stream()
    prof = wn.Profile(capacity=16 * (args.steps + args.warmup) + 64)

    # host offsets: with WN_FLAG_OVERLAP they let the library overlap the near
    # passes of early face runs with the far pass of later ones
    offs_overlap = q.face_point_offsets

    def step(schedule, profile=None):
        fs.query(u, v, offs, offs_overlap, out_w, out_l, schedule=schedule, queries_per_wg=args.qpw,
                 queue_policy=args.policy, profile=profile, stream=stream)

    if args.copy_calibration_mib > 0:
        # a plain copy of known size: reads and writes exactly copy_calibration_mib MiB
        n = args.copy_calibration_mib * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # warmup
    for _ in range(args.warmup):
        step(args.schedule)
    torch.cuda.synchronize()
    prof.collect()
    # timed region (batched schedule): events recorded around each library kernel
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step(args.schedule, prof)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    kern = prof.collect()
    ms_step = (t2 - t1) * 1e3 / args.steps
    value = pairs / (ms_step / 1e3)
    log(f"batched: {ms_step:.3f} ms/step, {value:.3e} evals/s; kernels {kern}")
    w_b = out_w.cpu().numpy()
    lab_b = out_l.cpu().numpy()

    # the overlapped form for reference (a handle with WN_FLAG_OVERLAP)
    ms_ovl_ref = None
    if not args.overlap and not args.headline_only and args.serial_steps > 0:
        fs_ovl = wn.FaceSet(faces, flags=wn.FLAG_OVERLAP)
        fs_ovl.query(u, v, offs, q.face_point_offsets, out_w, out_l, schedule=args.schedule, stream=stream)
        torch.cuda.synchronize()
        to1 = time.perf_counter()
        for _ in range(args.serial_steps):
            fs_ovl.query(u, v, offs, q.face_point_offsets, out_w, out_l, schedule=args.schedule, stream=stream)
        torch.cuda.synchronize()
        ms_ovl_ref = (time.perf_counter() - to1) * 1e3 / args.serial_steps
        ovl_same = bool(np.array_equal(out_l.cpu().numpy(), lab_b))
        del fs_ovl
        log(f"overlapped far/near passes (reference): {ms_ovl_ref:.3f} ms/step; labels equal: {ovl_same}")

    # the same steps without the far/near overlap (no host offsets: the passes
    # run one after the other), for rooflines of each kernel on its own
    kern_serial, ms_serial = {}, None
    if args.serial_steps > 0 and not args.headline_only and args.overlap:
        def step_serial(profile=None):
            fs.query(u, v, offs, None, out_w, out_l, schedule=args.schedule, queries_per_wg=args.qpw,
                     queue_policy=args.policy, profile=profile, stream=stream)

        step_serial()
        torch.cuda.synchronize()
        ps_ = wn.Profile(capacity=16 * args.serial_steps + 64)
        ts1 = time.perf_counter()
        for _ in range(args.serial_steps):
            step_serial(ps_)
        torch.cuda.synchronize()
        ms_serial = (time.perf_counter() - ts1) * 1e3 / args.serial_steps
        kern_serial = ps_.collect()
        log(f"batched, passes in series: {ms_serial:.3f} ms/step; kernels {kern_serial}")

    ms_mixed = ms_tree = ms_plain = ms_cp = ms_combo = float("nan")
    kern_mixed = kern_tree = kern_cp = work_cp = kern_combo = rep_tr = {}
    combo_same = None
    cp_diff = cp_onb = None
    mixed_same = plain_agree = None
    tree_diff = tree_onb = None

    if not args.headline_only:
        # batched schedule with the FP32 far-field admission (same results, see the header)
        def step_mixed(profile=None):
            fs.query(u, v, offs, q.face_point_offsets, out_w, out_l, schedule=args.schedule, precision=1,
                     queries_per_wg=args.qpw, queue_policy=args.policy, profile=profile, stream=stream)

        step_mixed()
        torch.cuda.synchronize()
        pm = wn.Profile(capacity=8 * args.mixed_steps + 64)
        tm1 = time.perf_counter()
        for _ in range(args.mixed_steps):
            step_mixed(pm)
        torch.cuda.synchronize()
        ms_mixed = (time.perf_counter() - tm1) * 1e3 / max(args.mixed_steps, 1)
        kern_mixed = {k: t_ / max(n, 1) for k, (n, t_) in pm.collect().items()}
        mixed_same = bool(np.array_equal(out_l.cpu().numpy(), lab_b))
        log(f"batched mixed: {ms_mixed:.3f} ms/step; kernels {kern_mixed}; labels equal to FP64: {mixed_same}")

        # path hierarchy (Sec. 4.2): subpath ellipses prune whole subpaths, so fewer
        # pairs are tested; reported on its own row (queries/s), not as evals/s
        def step_tree(profile=None):
            fs.query(u, v, offs, q.face_point_offsets, out_w, out_l, schedule=args.schedule, queries_per_wg=args.qpw,
                     queue_policy=args.policy, profile=profile, stream=stream, path_hierarchy=1)

        step_tree()
        torch.cuda.synchronize()
        ptree = wn.Profile(capacity=8 * args.tree_steps + 64)
        tt1 = time.perf_counter()
        for _ in range(args.tree_steps):
            step_tree(ptree)
        torch.cuda.synchronize()
        ms_tree = (time.perf_counter() - tt1) * 1e3 / max(args.tree_steps, 1)
        kern_tree = {k: t_ / max(n, 1) for k, (n, t_) in ptree.collect().items()}
        lab_t = out_l.cpu().numpy()
        both = (lab_t != 2) & (lab_b != 2)
        tree_diff = int(np.sum(lab_t[both] != lab_b[both]))
        tree_onb = int(np.sum((lab_t == 2) != (lab_b == 2)))
        log(f"path hierarchy: {ms_tree:.3f} ms/step, {N / (ms_tree / 1e3):.3e} queries/s; kernels {kern_tree}; "
            f"label differences vs flat {tree_diff}, on-boundary differences {tree_onb}")

        # the subdivided control-point bound in the near pass (Sec. 4.2 / Table 1
        # contrast): fewer splits, the same results, O(n^2) per split
        def step_cp(profile=None, stats=None):
            fs.query(u, v, offs, None, out_w, out_l, schedule=args.schedule, queries_per_wg=args.qpw,
                     queue_policy=args.policy, profile=profile, stats=stats, stream=stream,
                     bound=wn.BOUND_SUBDIVIDED)

        step_cp()
        torch.cuda.synchronize()
        pc = wn.Profile(capacity=8 * args.cp_steps + 64)
        tc1 = time.perf_counter()
        for _ in range(args.cp_steps):
            step_cp(pc)
        torch.cuda.synchronize()
        ms_cp = (time.perf_counter() - tc1) * 1e3 / max(args.cp_steps, 1)
        kern_cp = {k: t_ / max(n, 1) for k, (n, t_) in pc.collect().items()}
        lab_c = out_l.cpu().numpy()
        both_c = (lab_c != 2) & (lab_b != 2)
        cp_diff = int(np.sum(lab_c[both_c] != lab_b[both_c]))
        cp_onb = int(np.sum((lab_c == 2) != (lab_b == 2)))
        st_cp = torch.zeros(wn.STATS_COUNT, dtype=torch.int64, device=dev)
        step_cp(stats=st_cp)
        torch.cuda.synchronize()
        work_cp = dict(zip(wn.STAT_NAMES, (int(x) for x in st_cp.cpu().numpy())))
        log(f"subdivided control-point bound: {ms_cp:.3f} ms/step; kernels {kern_cp}; label differences {cp_diff}, "
            f"on-boundary differences {cp_onb}; work {work_cp}")

        # all three of the method's accelerations together: batched schedule,
        # FP32 far-field admission and near pairs binned by the learned depth
        # predictor (MLP on the matrix cores), trained on 100 faces of the same
        # generator outside the timed set; compared with the plain FP64 kernel below
        t_tr = time.perf_counter()
        f_tr, q_tr = W.config2(face_ids=range(args.faces, args.faces + 100))
        pr = wn.Predictor(seed=7)
        rep_tr = pr.train(wn.FaceSet(f_tr), *_dev_queries(torch, q_tr), epochs=20, lr=3e-3, seed=1,
                          max_samples=400000)
        rep_tr["train_s"] = time.perf_counter() - t_tr

        def step_combo(profile=None):
            fs.query(u, v, offs, q.face_point_offsets, out_w, out_l, schedule=wn.SCHED_BINNED, precision=1,
                     predictor=pr, bin_source=wn.BIN_PREDICTOR, queries_per_wg=args.qpw, profile=profile,
                     stream=stream)

        step_combo()
        torch.cuda.synchronize()
        pcb = wn.Profile(capacity=8 * args.mixed_steps + 64)
        tcb = time.perf_counter()
        for _ in range(args.mixed_steps):
            step_combo(pcb)
        torch.cuda.synchronize()
        ms_combo = (time.perf_counter() - tcb) * 1e3 / max(args.mixed_steps, 1)
        kern_combo = {k: t_ / max(n, 1) for k, (n, t_) in pcb.collect().items()}
        combo_same = bool(np.array_equal(out_l.cpu().numpy(), lab_b))
        log(f"batched + FP32 admission + learned binning: {ms_combo:.3f} ms/step; kernels {kern_combo}; "
            f"labels equal to FP64 batched: {combo_same}; predictor {rep_tr}")

        # plain schedule beside it (one launch per face, in-line recursion)
        step(0)
        torch.cuda.synchronize()
        tp1 = time.perf_counter()
        for _ in range(args.plain_steps):
            step(0)
        torch.cuda.synchronize()
        tp2 = time.perf_counter()
        ms_plain = (tp2 - tp1) * 1e3 / args.plain_steps
        lab_p = out_l.cpu().numpy()
        w_p = out_w.cpu().numpy()
        log(f"plain: {ms_plain:.3f} ms/step, {pairs / (ms_plain / 1e3):.3e} evals/s")
        plain_agree = bool(np.array_equal(lab_p, lab_b))

    # work counters of one (untimed) instrumented pass
    stats = torch.zeros(wn.STATS_COUNT, dtype=torch.int64, device=dev)
    fs.query(u, v, offs, q.face_point_offsets, out_w, out_l, schedule=args.schedule, queries_per_wg=args.qpw,
             queue_policy=args.policy, stats=stats, stream=stream)
    torch.cuda.synchronize()
    st = dict(zip(wn.STAT_NAMES, (int(x) for x in stats.cpu().numpy())))
    log(f"work counters: {st}")

    kernels = {k: {"launches": n, "avg_ms": t / max(n, 1)} for k, (n, t) in kern.items()}
    traffic = measured_traffic()
    work = {"k_far": (FLOPS_PER_PAIR * pairs, f"{pairs} pairs x {FLOPS_PER_PAIR} flops (root test + chord) per step"),
            "k_near": (st["near_flops"], f"{st['near_pairs']} near pairs, {st['splits']} splits x (6n+15) + "
                                         f"{st['leaves']} leaves x 11 = {st['near_flops']} flops per step")}

    def rooflines_of(kern_avg, nsteps):
        """Per-kernel roofline entries: algorithmic flops per launch (the
        step's work / launches per step) over the average HIP-event launch
        duration; HBM bytes per launch from the committed counters."""
        res = {}
        for k, (flops, desc) in work.items():
            if k not in kern_avg:
                continue
            n, t = kern_avg[k]
            ms = t / max(n, 1)
            per = n / nsteps
            a = flops / per / (ms / 1e3)
            tb = traffic.get(k)
            res[k] = {"bound": "alu", "achieved": a / 1e12, "peak": PEAK_FP64_VALU / 1e12, "unit": "TFLOP/s",
                      "frac": a / PEAK_FP64_VALU, "traffic": tb,
                      "hbm_achieved_GBps": None if tb is None else tb / (ms / 1e3) / 1e9,
                      "hbm_frac": None if tb is None else tb / (ms / 1e3) / PEAK_HBM,
                      "avg_launch_ms": ms, "launches_per_step": per, "ms_per_step": ms * per, "work": desc}
        return res

    # Each kernel alone on the GPU: the steps with the passes in series (with
    # --overlap 0 these are the timed steps themselves).  The headline entry
    # is the kernel with the most time per such step, so its launches never
    # share the GPU with another kernel of the path.
    if args.overlap:
        rooflines_serial = rooflines_of(kern_serial, args.serial_steps) if kern_serial else {}
        rooflines_overlapped = rooflines_of(kern, args.steps)
    else:
        rooflines_serial = rooflines_of(kern, args.steps)
        rooflines_overlapped = {}
        ms_serial = ms_step
    roofline = None
    if rooflines_serial:
        dom = max(rooflines_serial, key=lambda k: rooflines_serial[k]["ms_per_step"])
        roofline = dict(rooflines_serial[dom], kernel=dom)
        roofline["note"] = ("kernel alone on the GPU (far and near passes in series, the default and faster "
                            "form); the overlapped form's step time is under rooflines_overlapped")
        # measured counterpart of the HBM peak (context; the fractions use the published peak)
        roofline["measured_copy_GBps"] = measured_copy_rate(torch) / 1e9

    # CPU oracle on a bounded sample of the same workload; also the parity check
    cpu = None
    mism = None
    if not args.no_cpu:
        import oracle

        rng = np.random.default_rng(1234)
        ns = min(args.cpu_sample, N)
        idx = np.sort(rng.choice(N, ns, replace=False))
        pf, su, sv = W.subset_queries(q, idx)
        # the process's CPU set, at most the 16 cores one GPU's share of a host has
        avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
        cores = min(16, avail)
        tc = time.perf_counter()
        w_o, near = oracle.query(faces, pf, su, sv, nthreads=cores)
        tcpu = time.perf_counter() - tc
        sample_pairs = int(np.sum(S_f[pf]))
        cpu = {"value": sample_pairs / tcpu, "unit": "evals/s", "cores": cores, "kind": "oracle",
               "sample": f"{ns} points drawn uniformly from the timed set ({sample_pairs:.3e} pairs), "
                         f"{tcpu:.1f} s",
               "host": host_cpu(), "cpus_available": avail}
        # single thread on config 1 (one face of 64 cubics, 65,536 points): the
        # paper's per-shape costs (Sec. 5, Table 2) are single-thread timings
        # of 65,536 samples per shape, on other shapes and another CPU
        f1, q1 = W.config1()
        tc = time.perf_counter()
        oracle.query_faces(f1, q1, nthreads=1)
        t1 = time.perf_counter() - tc
        cpu["single_thread_config1"] = {"s_per_shape": t1, "points": q1.num_points, "segments": f1.num_segments,
                                        "evals_per_s": q1.num_points * f1.num_segments / t1,
                                        "paper_table2_s_per_shape": {"BG A": 0.095, "OpenClipArt20K": 0.407}}
        far = near == 0
        want = (np.abs(w_o) > 0.5).astype(np.uint8)
        mism = int(np.sum(lab_b[idx][far] != want[far]))
        maxerr = float(np.max(np.abs(w_b[idx][far] - w_o[far])))
        log(f"oracle sample: {ns} points in {tcpu:.1f}s on {cores} threads; mismatches {mism}, max err {maxerr:.2e}")

    sections = {}
    if not args.no_extra:
        only = {x for x in args.sections.split(",") if x}
        for name, fn in SECTIONS:
            if only and name not in only:
                continue
            t = time.time()
            try:
                sections[name] = fn(args)
            except Exception as exc:  # report, keep the headline line
                sections[name] = {"error": repr(exc)}
            log(f"{name}: {time.time() - t:.1f}s {json.dumps(sections[name])[:400]}")

    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "batched planar set: 2000 faces, 1 outer + 0-7 hole loops, 4-256 segments/loop "
                               "(degree 1-5, rational weights U[0.5,2]), 1k-64k points/face, 30% within 1e-3 "
                               "of a curve",
                   "faces": args.faces, "segments": faces.num_segments, "points": N, "pairs": pairs,
                   "schedule": {0: "plain", 1: "batched"}.get(args.schedule, str(args.schedule)), "eps": 1e-10,
                   "overlap": bool(args.overlap)},
        "queries_per_s": N / (ms_step / 1e3),
        "plain": {"ms_per_step": ms_plain, "evals_per_s": pairs / (ms_plain / 1e3),
                  "queries_per_s": N / (ms_plain / 1e3), "labels_equal_batched": plain_agree},
        "speedup_batched_vs_plain": ms_plain / ms_step,
        "batched_mixed": {"ms_per_step": ms_mixed, "evals_per_s": pairs / (ms_mixed / 1e3), "kernel_ms": kern_mixed,
                          "labels_equal_fp64": mixed_same},
        "path_hierarchy": {"ms_per_step": ms_tree, "queries_per_s": N / (ms_tree / 1e3), "kernel_ms": kern_tree,
                           "speedup_vs_flat": ms_step / ms_tree, "label_differences_vs_flat": tree_diff,
                           "on_boundary_differences_vs_flat": tree_onb},
        "subdivided_bound": {"ms_per_step": ms_cp, "kernel_ms": kern_cp, "label_differences_vs_global": cp_diff,
                             "on_boundary_differences_vs_global": cp_onb,
                             "splits": work_cp.get("splits"), "leaves": work_cp.get("leaves"),
                             "max_depth": work_cp.get("max_depth"),
                             "note": "near pass with the smaller of B 2^-k and the node's control-point bound "
                                     "(passes in series); compare rooflines_serial's k_near and work.splits"},
        "batched_mixed_binned": {"ms_per_step": ms_combo, "evals_per_s": pairs / (ms_combo / 1e3),
                                 "kernel_ms": kern_combo, "labels_equal_fp64": combo_same,
                                 "speedup_vs_plain_fp64": ms_plain / ms_combo,
                                 "predictor": {k: v for k, v in rep_tr.items()
                                               if k in ("samples", "holdout_mae", "baseline_mae", "train_s")},
                                 "note": "batched schedule + FP32 far-field admission + near pairs binned by the "
                                         "learned depth predictor (MLP on the matrix cores, trained on faces "
                                         f"{args.faces}..{args.faces + 99} of the generator) vs the plain FP64 kernel"},
        "mismatches": mism,
        "kernels": kernels,
        "work": st,
        "roofline": roofline,
        "rooflines_serial": {"ms_per_step": ms_serial, "kernels": rooflines_serial},
        "rooflines_overlapped": {"ms_per_step": ms_step if args.overlap else ms_ovl_ref,
                                 "kernels": rooflines_overlapped},
        "cpu_baseline": cpu,
        "configs": sections,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
