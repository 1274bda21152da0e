"""Learned depth predictor on the GPU: gradients against the FP64 CPU
reference, features against a test-local computation, training on config 4
(the network must beat predicting the mean depth), and binned scheduling
leaving every answer unchanged."""
import numpy as np
import pytest

from oracle import mlp_ref
from paper_2510_25159_amd import workloads as W
from tests.gpu_helpers import compare, run_wn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_25159_amd import wn

    wn.lib()
    return torch


def _dev(torch, a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to("cuda:0")


def test_gradient_and_forward_vs_cpu_reference(torch_cuda):
    torch = torch_cuda
    from paper_2510_25159_amd import wn

    rng = np.random.default_rng(0)
    pr = wn.Predictor(seed=3)
    params, norm = pr.get_params()
    params = params + rng.normal(0, 0.05, params.shape).astype(np.float32)  # nonzero biases too
    pr.set_params(params)
    X = rng.normal(0, 1, (2000, 16)).astype(np.float32)
    Y = rng.uniform(0, 12, 2000).astype(np.float32)
    for delta in (1.0, 50.0):
        loss, g = pr.loss_grad(_dev(torch, X, np.float32), _dev(torch, Y, np.float32), huber_delta=delta)
        loss_r, g_r = mlp_ref.loss_grad(params, X, Y, delta, bf16=True)
        assert abs(loss - loss_r) <= 1e-4 * (1 + abs(loss_r))
        scale = np.max(np.abs(g_r))
        assert np.max(np.abs(g - g_r)) <= 2e-4 * scale, (np.max(np.abs(g - g_r)), scale)
    pred = pr.predict(_dev(torch, X, np.float32)).cpu().numpy()
    np.testing.assert_allclose(pred, mlp_ref.predict(params, X, bf16=True), rtol=0, atol=1e-4 * (1 + np.abs(pred).max()))


def test_predict_mfma_vs_bf16_reference(torch_cuda):
    """The matrix-core forward pass (BF16 inputs, weights and layer-1
    activations, FP32 accumulation) against the FP64 reference with the same
    roundings.  The two sides may round a layer-1 activation to neighbouring
    BF16 values when its FP32 sum lies within rounding of a tie; one such
    step moves y by at most 2^-7 |h1_k| |W2[:, k]| |w3|, so every row stays
    within the sum of those, and nearly every row agrees to FP32 rounding.
    4133 rows: whole waves and a ragged tail."""
    torch = torch_cuda
    from paper_2510_25159_amd import wn

    rng = np.random.default_rng(5)
    pr = wn.Predictor(seed=11)
    params, _ = pr.get_params()
    params = params + rng.normal(0, 0.05, params.shape).astype(np.float32)
    pr.set_params(params)
    X = rng.normal(0, 1.5, (4133, 16)).astype(np.float32)
    y = pr.predict_mfma(_dev(torch, X, np.float32)).cpu().numpy().astype(np.float64)
    y_ref, h1 = mlp_ref.predict(params, X, bf16=True, bf16_act=True, return_hidden=True)
    q = mlp_ref.unpack(mlp_ref.bf16_round(params))
    flip = 2.0 ** -7 * (np.abs(h1) @ np.abs(q["W2"]).T) @ np.abs(q["w3"])
    h2 = np.maximum(h1 @ q["W2"].T + q["b2"], 0.0)
    fp32 = 1e-5 * (1.0 + np.abs(h2) @ np.abs(q["w3"]) + np.abs(h1) @ np.abs(q["W2"]).T @ np.abs(q["w3"]))
    d = np.abs(y - y_ref)
    print(f"mfma vs reference: max |d| {d.max():.3e}, rows beyond FP32 rounding {int(np.sum(d > fp32))}", flush=True)
    assert np.all(d <= flip + fp32)
    assert np.sum(d > fp32) <= 0.01 * len(y)
    # the VALU version keeps FP32 activations: the two differ by activation rounding only
    yv = pr.predict(_dev(torch, X, np.float32)).cpu().numpy().astype(np.float64)
    assert np.all(np.abs(yv - mlp_ref.predict(params, X, bf16=True)) <= fp32 + 1e-4 * (1 + np.abs(yv)))
    # empty input
    assert pr.predict_mfma(torch.zeros((0, 16), dtype=torch.float32, device="cuda:0")).numel() == 0


def test_pair_features_vs_numpy(torch_cuda):
    torch = torch_cuda
    from paper_2510_25159_amd import wn

    faces, q = W.config2(face_ids=[0])
    fs = wn.FaceSet(faces)
    rng = np.random.default_rng(1)
    n = 500
    pp = rng.integers(0, q.num_points, n).astype(np.int32)
    ps = rng.integers(0, faces.num_segments, n).astype(np.int32)
    u, v = _dev(torch, q.u, np.float64), _dev(torch, q.v, np.float64)
    offs = _dev(torch, q.face_point_offsets, np.int64)
    F = wn.pair_features(fs, u, v, offs, _dev(torch, pp, np.int32), _dev(torch, ps, np.int32)).cpu().numpy()
    for k in range(n):
        s = ps[k]
        a, b = faces.seg_cp_offsets[s], faces.seg_cp_offsets[s + 1]
        cp = np.column_stack([faces.cp_u[a:b], faces.cp_v[a:b]])
        w = faces.cp_w[a:b]
        x = np.array([q.u[pp[k]], q.v[pp[k]]])
        B = wn.segment_bound(cp, w)
        P0, Pn = cp[0], cp[-1]
        L = np.hypot(*(Pn - P0))
        uax = (Pn - P0) / L
        r = x - (P0 + Pn) / 2
        lo, hi = cp.min(0), cp.max(0)
        dbox = np.hypot(*np.maximum(np.maximum(lo - x, x - hi), 0))
        d1, d2 = np.hypot(*(x - P0)), np.hypot(*(x - Pn))
        e2 = -r[0] * uax[1] + r[1] * uax[0]
        want = [(r @ uax) / (B / 2), e2 / (B / 2), B / 2, np.sqrt(max((B / 2) ** 2 - (L / 2) ** 2, 0)), len(cp) - 1,
                w.min(), w.max(), L, dbox, d1, d2, (d1 + d2) / B, np.log2(B / max(1e-10, dbox)), B, L / 2,
                1.0 if e2 >= 0 else -1.0]
        np.testing.assert_allclose(F[k], np.array(want, dtype=np.float32), rtol=2e-5, atol=1e-6)


@pytest.fixture(scope="module")
def trained(torch_cuda):
    torch = torch_cuda
    from paper_2510_25159_amd import wn

    faces, q = W.config4("train", near_frac=0.3)
    fs = wn.FaceSet(faces)
    pr = wn.Predictor(seed=7)
    rep = pr.train(fs, _dev(torch, q.u, np.float64), _dev(torch, q.v, np.float64),
                   _dev(torch, q.face_point_offsets, np.int64), epochs=60, lr=3e-3, seed=1)
    print("training report", rep, flush=True)
    return pr, rep


def test_training_beats_mean_predictor(trained):
    pr, rep = trained
    assert rep["samples"] > 10000
    assert rep["holdout_mae"] < 0.8 * rep["baseline_mae"], rep


@pytest.mark.parametrize("source", [0, 1, 2, 3, 4])
def test_binned_schedule_changes_nothing(torch_cuda, trained, oracle_lib, source):
    pr, _ = trained
    faces, q = W.config4("eval", near_frac=0.3)
    idx = np.arange(0, q.num_points, 7)
    w_ref, lab_ref = run_wn(faces, q, schedule=1)
    w, lab = run_wn(faces, q, schedule=2, predictor=pr, bin_source=source)
    assert np.array_equal(lab, lab_ref)
    ok = lab < 2
    assert np.max(np.abs(w[ok] - w_ref[ok])) <= 1e-12
    pf, u, v = W.subset_queries(q, idx)
    w_o, n_o = oracle_lib.query(faces, pf, u, v)
    compare(w[idx], lab[idx], w_o, n_o)


def test_binned_periodic_and_rational(torch_cuda, trained, oracle_lib):
    pr, _ = trained
    for faces, q in (W.config2(face_ids=range(4)), W.config3(face_ids=range(8))):
        w_o, n_o = oracle_lib.query_faces(faces, q)
        for source in (0, 1, 2, 4):
            w, lab = run_wn(faces, q, schedule=2, predictor=pr, bin_source=source)
            compare(w, lab, w_o, n_o)


def test_depth_log_within_termination_bound(torch_cuda):
    torch = torch_cuda
    from paper_2510_25159_amd import wn

    faces, q = W.config4("train", near_frac=0.3)
    fs = wn.FaceSet(faces)
    info = fs.info()
    n = 20000
    u, v = _dev(torch, q.u[:n], np.float64), _dev(torch, q.v[:n], np.float64)
    offs = _dev(torch, [0, n], np.int64)
    dl = torch.zeros(n * info.max_segments_per_face, dtype=torch.uint8, device="cuda:0")
    fs.query(u, v, offs, np.array([0, n]), schedule=0, depth_log=dl)
    d = dl.cpu().numpy()
    assert d.max() <= info.max_depth_bound
    assert (d > 0).mean() > 0.01  # near pairs recurse
