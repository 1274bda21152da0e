"""Plans: the batched pipeline captured in a HIP graph, replayed with
different point counts; every replay (with eager work and synchronisations
between replays) must equal the eager query; the autotuner keeps it equal."""
import numpy as np
import pytest

from paper_2510_25159_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_25159_amd import wn

    wn.lib()
    return torch


def _batch(q, face_ids, n_faces, rng, frac):
    """A request batch: a random fraction of each chosen face's points."""
    us, vs, offs = [], [], [0]
    for f in range(n_faces):
        a, b = q.face_point_offsets[f], q.face_point_offsets[f + 1]
        if f in face_ids:
            k = max(1, int(frac * (b - a)))
            sel = np.sort(rng.choice(np.arange(a, b), k, replace=False))
            us.append(q.u[sel])
            vs.append(q.v[sel])
            offs.append(offs[-1] + k)
        else:
            offs.append(offs[-1])
    return np.concatenate(us), np.concatenate(vs), np.array(offs, dtype=np.int64)


@pytest.mark.parametrize("schedule,source", [(1, 0), (2, 1)])
def test_graph_replays_match_eager(torch_cuda, schedule, source):
    torch = torch_cuda
    from paper_2510_25159_amd import wn

    fp, qp = W.config2(face_ids=range(6))
    fs = wn.FaceSet(fp)
    dev = "cuda:0"
    cap = qp.num_points
    u = torch.zeros(cap, dtype=torch.float64, device=dev)
    v = torch.zeros(cap, dtype=torch.float64, device=dev)
    offs = torch.zeros(fp.num_faces + 1, dtype=torch.int64, device=dev)
    ow = torch.zeros(cap, dtype=torch.float64, device=dev)
    ol = torch.zeros(cap, dtype=torch.uint8, device=dev)
    plan = wn.Plan(fs, u, v, offs, ow, ol, schedule=schedule, bin_source=source)
    rng = np.random.default_rng(0)
    batches = [_batch(qp, {0, 1, 2, 3, 4, 5}, 6, rng, 1.0), _batch(qp, {1, 4}, 6, rng, 0.3),
               _batch(qp, {0, 2, 5}, 6, rng, 0.6)]
    for it, (bu, bv, bo) in enumerate(batches * 2):
        n = len(bu)
        u[:n].copy_(torch.from_numpy(bu))
        v[:n].copy_(torch.from_numpy(bv))
        offs.copy_(torch.from_numpy(bo))
        torch.cuda.synchronize()
        plan.launch()
        torch.cuda.synchronize()
        w_g, l_g = ow[:n].cpu().numpy().copy(), ol[:n].cpu().numpy().copy()
        # eager reference on fresh tensors, plus unrelated eager work in between
        eu, ev, eo = (torch.from_numpy(x).to(dev) for x in (bu, bv, bo))
        w_e, l_e = fs.query(eu, ev, eo, bo, schedule=1)
        _ = (torch.randn(1 << 20, device=dev) * 2).sum().item()
        torch.cuda.synchronize()
        w_e, l_e = w_e.cpu().numpy(), l_e.cpu().numpy()
        assert np.array_equal(l_g, l_e), f"replay {it}"
        ok = l_e < 2
        assert np.max(np.abs(w_g[ok] - w_e[ok])) <= 1e-12, f"replay {it}"
    rep = plan.autotune(reps=2)
    assert rep["queries_per_wg"] in (64, 128, 256, 512, 1024)
    bu, bv, bo = batches[1]
    n = len(bu)
    u[:n].copy_(torch.from_numpy(bu))
    v[:n].copy_(torch.from_numpy(bv))
    offs.copy_(torch.from_numpy(bo))
    plan.launch()
    torch.cuda.synchronize()
    eu, ev, eo = (torch.from_numpy(x).to(dev) for x in (bu, bv, bo))
    w_e, l_e = fs.query(eu, ev, eo, bo, schedule=1)
    torch.cuda.synchronize()
    assert np.array_equal(ol[:n].cpu().numpy(), l_e.cpu().numpy())
    plan.close()
