"""Pin of the FP64 MLP reference used for the predictor's gradient checks:
analytic gradient vs central finite differences (no BF16 rounding), and
the BF16 rounding helper vs hand-computed bit patterns."""
import numpy as np

from oracle import mlp_ref


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    p = rng.normal(0, 0.3, mlp_ref.PARAMS)
    X = rng.normal(0, 1, (40, 16))
    Y = rng.uniform(0, 8, 40)
    for delta in (0.5, 100.0):  # Huber in both regimes
        loss, g = mlp_ref.loss_grad(p, X, Y, delta)
        idx = rng.choice(mlp_ref.PARAMS, 60, replace=False)
        h = 1e-6
        for i in idx:
            e = np.zeros_like(p)
            e[i] = h
            fd = (mlp_ref.loss_grad(p + e, X, Y, delta)[0] - mlp_ref.loss_grad(p - e, X, Y, delta)[0]) / (2 * h)
            assert abs(fd - g[i]) <= 1e-6 * (1 + abs(fd))


def test_bf16_rounding_bits():
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: round to even -> 1.0
    assert mlp_ref.bf16_round(np.float32(1.0 + 2 ** -8)) == 1.0
    # 1 + 3 * 2^-8 ties up to 1 + 2^-6 (even mantissa)
    assert mlp_ref.bf16_round(np.float32(1.0 + 3 * 2 ** -8)) == 1.0 + 2 ** -6
    # exactly representable values are unchanged
    for v in (0.5, -3.0, 1.0 + 2 ** -7, 2.0 ** -20):
        assert mlp_ref.bf16_round(np.float32(v)) == v
