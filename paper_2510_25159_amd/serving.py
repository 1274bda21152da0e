"""Serving loop: containment requests against resident faces, batched into
replays of one captured query graph.

Open-loop Poisson arrivals (default 2,000 requests/s for 10 s).  Each request
names one face of a resident pool (512 faces of the single-star generator,
512 periodic faces) and carries Q fresh points, Q log-uniform in [256, 262144].
A request is admitted when its point and output buffers fit in a device
memory budget (default 4 GiB, FIFO otherwise); whenever the GPU is idle the
dispatcher packs every admitted request (up to the plan capacity) into one
batch, copies its points from pinned host memory and replays the graph.
Latency = device completion event - arrival.  Reports p50/p99 latency and
queries/s.
"""
from __future__ import annotations

import argparse
import json
import time
from collections import deque

import numpy as np

from . import wn
from . import workloads as W

BYTES_PER_POINT = 16 + 9  # (u, v) in, (winding, label) out


def build_pool(n_star: int = 512, n_periodic: int = 512, seed: int = W.SEED_C5):
    """Resident faces: star faces (config 1 generator, one seed each) then
    periodic faces (config 3 generator)."""
    loops, doms, pers, kinds = [], [], [], []
    for i in range(n_star):
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 7, i])))
        lp = W.hermite_star_loop(W.StarCurve(rng), 64)
        loops.append([lp])
        doms.append(W.DOMAIN_PLANE)
        pers.append([0.0, 0.0])
        kinds.append(0)
    for i in range(n_periodic):
        lps, _, dom, per = W.config3_face(seed, i, queries=1)
        loops.append(lps)
        doms.append(dom)
        pers.append(list(per))
        kinds.append(dom)
    faces = W._assemble(loops, doms, pers, rational=False)
    return faces, np.array(kinds)


def run(rate: float = 2000.0, duration: float = 10.0, budget_gib: float = 4.0, capacity: int = 1 << 23,
        seed: int = W.SEED_C5, pool_points: int = 1 << 24, verbose: bool = False, sample_every: int = 0,
        sample_points: int = 4096) -> dict:
    """Run the serving loop.  With sample_every = k > 0, one seeded request of
    every k-th batch is kept for checking: its face, its first sample_points
    points and the served winding numbers and labels, copied back once the
    batch has completed (before the next replay overwrites them); they are
    returned under "samples" (host arrays, not part of the timing report)."""
    import torch

    dev = torch.device("cuda:0")
    faces, kinds = build_pool(seed=seed)
    F = faces.num_faces
    fs = wn.FaceSet(faces)
    rng = np.random.default_rng(seed)
    # requests
    n_req = int(rng.poisson(rate * duration))
    t_arr = np.sort(rng.uniform(0.0, duration, n_req))
    face = rng.integers(0, F, n_req)
    Q = np.round(np.exp(rng.uniform(np.log(256), np.log(262144), n_req))).astype(np.int64)
    # pinned point pools, one per domain kind (fresh uniform points of the face's box)
    pools = {}
    for kind, (lo, hi) in {0: ((-1.5, -1.5), (1.5, 1.5)), 1: ((0, -np.pi), (2 * np.pi, np.pi)),
                           2: ((0, 0), (2 * np.pi, 2 * np.pi))}.items():
        pu = torch.empty(pool_points, dtype=torch.float64).pin_memory()
        pv = torch.empty(pool_points, dtype=torch.float64).pin_memory()
        pu.numpy()[:] = rng.uniform(lo[0], hi[0], pool_points)
        pv.numpy()[:] = rng.uniform(lo[1], hi[1], pool_points)
        pools[kind] = (pu.numpy(), pv.numpy())
    start = rng.integers(0, pool_points - Q.max(), n_req)
    # plan over device buffers of `capacity` points
    u = torch.zeros(capacity, dtype=torch.float64, device=dev)
    v = torch.zeros(capacity, dtype=torch.float64, device=dev)
    offs = torch.zeros(F + 1, dtype=torch.int64, device=dev)
    ow = torch.zeros(capacity, dtype=torch.float64, device=dev)
    ol = torch.zeros(capacity, dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    plan = wn.Plan(fs, u, v, offs, ow, ol, schedule=wn.SCHED_BATCHED, stream=stream)
    stage_u = torch.empty(capacity, dtype=torch.float64).pin_memory()
    stage_v = torch.empty(capacity, dtype=torch.float64).pin_memory()
    stage_o = torch.empty(F + 1, dtype=torch.int64).pin_memory()
    su, sv, so = stage_u.numpy(), stage_v.numpy(), stage_o.numpy()
    budget = int(budget_gib * (1 << 30))
    # warm the graph once
    so[:] = 0
    offs.copy_(stage_o, non_blocking=True)
    plan.launch(stream)
    torch.cuda.synchronize()

    lat = np.full(n_req, np.nan)
    batches = []
    samples = []
    srng = np.random.default_rng(seed + 17)
    pending, admitted = deque(), deque()
    used = 0
    nxt = 0
    busy = None  # (done_event, request ids, bytes)
    t0_ev = torch.cuda.Event(enable_timing=True)
    t0_ev.record(stream)
    t0 = time.perf_counter()
    done = 0
    while done < n_req:
        now = time.perf_counter() - t0
        while nxt < n_req and t_arr[nxt] <= now:
            pending.append(nxt)
            nxt += 1
        while pending and used + Q[pending[0]] * BYTES_PER_POINT <= budget:
            i = pending.popleft()
            used += Q[i] * BYTES_PER_POINT
            admitted.append(i)
        if busy is not None and busy[0].query():
            ev, ids, nbytes, pick = busy
            t_done = t0_ev.elapsed_time(ev) / 1e3
            if pick is not None:
                i, pos, k = pick
                pu, pv = pools[kinds[face[i]]]
                samples.append({"face": int(face[i]), "u": pu[start[i]:start[i] + k].copy(),
                                "v": pv[start[i]:start[i] + k].copy(),
                                "w": ow[pos:pos + k].cpu().numpy(), "lab": ol[pos:pos + k].cpu().numpy()})
            lat[ids] = t_done - t_arr[ids]
            used -= nbytes
            done += len(ids)
            busy = None
        if busy is None and admitted:
            ids, tot = [], 0
            while admitted and tot + Q[admitted[0]] <= capacity:
                i = admitted.popleft()
                ids.append(i)
                tot += Q[i]
            if not ids:  # a single request larger than the capacity is split by the caller (not generated)
                raise RuntimeError("request exceeds plan capacity")
            ids = np.array(ids)
            order = ids[np.argsort(face[ids], kind="stable")]
            pick = None
            pick_req = order[srng.integers(0, len(order))] if sample_every and len(batches) % sample_every == 0 else -1
            pos = 0
            for i in order:
                if i == pick_req:
                    pick = (int(i), pos, int(min(Q[i], sample_points)))
                pu, pv = pools[kinds[face[i]]]
                su[pos:pos + Q[i]] = pu[start[i]:start[i] + Q[i]]
                sv[pos:pos + Q[i]] = pv[start[i]:start[i] + Q[i]]
                pos += Q[i]
            cnt = np.bincount(face[order], weights=Q[order], minlength=F).astype(np.int64)
            so[0] = 0
            np.cumsum(cnt, out=so[1:])
            u[:pos].copy_(stage_u[:pos], non_blocking=True)
            v[:pos].copy_(stage_v[:pos], non_blocking=True)
            offs.copy_(stage_o, non_blocking=True)
            plan.launch(stream)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(stream)
            busy = (ev, order, int(np.sum(Q[order])) * BYTES_PER_POINT, pick)
            batches.append((len(order), pos))
            continue
        if busy is None and not admitted and nxt < n_req:
            time.sleep(max(0.0, min(t_arr[nxt] - (time.perf_counter() - t0), 0.002)))
        elif busy is not None:
            time.sleep(0.0002)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.close()
    total_q = int(Q.sum())
    span = float(np.nanmax(lat + t_arr) - t_arr[0]) if n_req else 0.0
    res = {
        "requests": int(n_req), "rate_req_per_s": rate, "duration_s": duration,
        "queries": total_q, "offered_queries_per_s": total_q / duration,
        "queries_per_s": total_q / span if span > 0 else 0.0,
        "p50_ms": float(np.nanpercentile(lat, 50) * 1e3), "p99_ms": float(np.nanpercentile(lat, 99) * 1e3),
        "max_ms": float(np.nanmax(lat) * 1e3), "batches": len(batches),
        "mean_batch_requests": float(np.mean([b[0] for b in batches])) if batches else 0.0,
        "mean_batch_points": float(np.mean([b[1] for b in batches])) if batches else 0.0,
        "budget_gib": budget_gib, "capacity_points": capacity, "wall_s": wall,
        "pool": "512 star faces (64 cubic segments) + 512 periodic faces (cylinder/torus)",
    }
    if verbose:
        print(json.dumps(res), flush=True)
    if sample_every:
        res["samples"] = samples
        res["pool_faces"] = faces
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--rate", type=float, default=2000.0)
    ap.add_argument("--duration", type=float, default=10.0)
    ap.add_argument("--budget-gib", type=float, default=4.0)
    args = ap.parse_args()
    run(args.rate, args.duration, args.budget_gib, verbose=True)


if __name__ == "__main__":
    main()
