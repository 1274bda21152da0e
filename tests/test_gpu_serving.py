"""Serving loop smoke: every request completes with a finite latency."""
import pytest

pytestmark = pytest.mark.gpu


def test_serving_short_run():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_25159_amd import serving

    res = serving.run(rate=500.0, duration=0.5, budget_gib=0.25, capacity=1 << 21, pool_points=1 << 20)
    assert res["requests"] > 100
    assert res["p99_ms"] > 0 and res["p99_ms"] < 60000
    assert res["queries_per_s"] > 0
