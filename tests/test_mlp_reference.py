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


def _small_integer_net():
    """W1 picks h1[0] = x0 + x1 and h1[1] = x2, W2 copies h1[0:2] into h2,
    w3 = (1, 1000); every weight is BF16-exact."""
    q = {name: np.zeros(shape) for name, shape in mlp_ref.SIZES}
    q["W1"][0, 0] = q["W1"][0, 1] = 1.0
    q["W1"][1, 2] = 1.0
    q["W2"][0, 0] = q["W2"][1, 1] = 1.0
    q["w3"][0], q["w3"][1] = 1.0, 1000.0
    return np.concatenate([q[name].ravel() for name, _ in mlp_ref.SIZES])


def test_bf16_activation_rounding():
    p = _small_integer_net()
    # BF16-exact inputs and activations: rounding changes nothing
    X = np.zeros((1, 16))
    X[0, :3] = (100.0, 28.0, 3.0)
    assert mlp_ref.predict(p, X, bf16_act=True)[0] == mlp_ref.predict(p, X, bf16=False)[0] == 128.0 + 3000.0
    # h1[0] = 256 + 1 = 257 lies halfway between 256 and 258 (even: 256);
    # x2 = 1 + 2^-8 rounds to 1 on the way in
    X[0, :3] = (256.0, 1.0, 1.0 + 2 ** -8)
    y, h1 = mlp_ref.predict(p, X, bf16_act=True, return_hidden=True)
    assert h1[0, 0] == 256.0 and h1[0, 1] == 1.0
    assert y[0] == 256.0 + 1000.0
    assert mlp_ref.predict(p, X, bf16=True)[0] == 257.0 + 1000.0 * (1.0 + 2 ** -8)
    # ReLU before the rounding: a negative pre-activation stays zero
    X[0, :3] = (-300.0, 1.0, 0.0)
    assert mlp_ref.predict(p, X, bf16_act=True)[0] == 0.0
