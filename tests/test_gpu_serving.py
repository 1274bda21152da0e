"""Serving loop (config 5): every request completes with a finite latency,
and sampled served results equal the oracle's.

One seeded request of every second batch is copied back after its replay
(its first 4,096 points) and checked against the CPU oracle on the same face
and points: labels identical for every point farther than 1e-9 from the
face's curves, winding within 1e-12 (on periodic faces, whose copies are
evaluated at translated queries, plus the winding number's own FP64
conditioning at the point: see gpu_helpers.translation_tol).  The pool mixes star faces and
periodic (cylinder / torus) faces, and batches of several request sizes go
through the same captured graph.
"""
import numpy as np
import pytest

from tests.gpu_helpers import compare, translation_tol

pytestmark = pytest.mark.gpu


def test_serving_short_run(oracle_lib):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_25159_amd import serving

    res = serving.run(rate=500.0, duration=0.5, budget_gib=0.25, capacity=1 << 21, pool_points=1 << 20,
                      sample_every=2, sample_points=4096)
    assert res["requests"] > 100
    assert res["p99_ms"] > 0 and res["p99_ms"] < 60000
    assert res["queries_per_s"] > 0
    samples = res["samples"]
    faces = res["pool_faces"]
    assert len(samples) >= 10
    kinds = set()
    checked = 0
    for s in samples:
        k = len(s["u"])
        pf = np.full(k, s["face"], dtype=np.int32)
        w_o, n_o = oracle_lib.query(faces, pf, s["u"], s["v"])
        ok = (n_o == 0) & np.isfinite(s["w"])
        if ok.any():
            i = int(np.argmax(np.where(ok, np.abs(s["w"] - w_o), 0)))
            w_ld, _ = oracle_lib.query(faces, pf[i:i + 1], s["u"][i:i + 1], s["v"][i:i + 1], long_double=True)
            print(f"face {s['face']} domain {int(faces.face_domain[s['face']])}: worst point "
                  f"({s['u'][i]!r}, {s['v'][i]!r}) gpu {s['w'][i]!r} oracle {w_o[i]!r} "
                  f"long double {w_ld[0]!r}", flush=True)
        st = compare(s["w"], s["lab"], w_o, n_o,
                     tol_fn=lambda i: translation_tol(oracle_lib, faces, pf, s["u"], s["v"], i))
        checked += st["compared"]
        kinds.add(int(faces.face_domain[s["face"]]))
    print(f"{len(samples)} sampled requests, {checked} points compared, domains {sorted(kinds)}", flush=True)
    assert checked > 0.95 * sum(len(s["u"]) for s in samples)
