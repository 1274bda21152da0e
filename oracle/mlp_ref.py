"""FP64 CPU reference of the depth predictor's MLP (test infrastructure).

Network 16 -> 64 -> 64 -> 1 with ReLU, parameter layout W1[64][16], b1[64],
W2[64][64], b2[64], w3[64], b3; mean Huber loss.  ``bf16=True`` rounds the
weights to BF16 (round to nearest even) in the forward pass, as the GPU
kernels do; the gradient is then taken with respect to the unrounded
parameters with the rounding treated as the identity.  Pinned by central
finite differences in the tests (``bf16=False``).

``predict(..., bf16_act=True)`` also rounds the inputs and the layer-1
activations to BF16 before they are multiplied, as the matrix-core version of
the kernels does (BF16 operands, wide accumulation).  Pinned on small-integer
networks whose activations are BF16-exact (no change) or fall between two
BF16 values (round to nearest even).
"""
import numpy as np

IN, H = 16, 64
SIZES = [("W1", (H, IN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", (1,))]
PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(p):
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = np.asarray(p[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def bf16_round(x):
    a = np.asarray(x, dtype=np.float32).copy()
    u = a.view(np.uint32)
    u += np.uint32(0x7FFF) + ((u >> np.uint32(16)) & np.uint32(1))
    u &= np.uint32(0xFFFF0000)
    return a.astype(np.float64)


def loss_grad(params, X, Y, delta=1.0, bf16=False):
    """Mean Huber loss and its gradient (FP64)."""
    p = np.asarray(params, dtype=np.float64)
    q = unpack(bf16_round(p) if bf16 else p)
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    n = len(Y)
    a1 = X @ q["W1"].T + q["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ q["W2"].T + q["b2"]
    h2 = np.maximum(a2, 0.0)
    y = h2 @ q["w3"] + q["b3"][0]
    r = y - Y
    ar = np.abs(r)
    loss = np.where(ar <= delta, 0.5 * r * r, delta * (ar - 0.5 * delta)).mean()
    g = np.where(ar <= delta, r, delta * np.sign(r)) / n
    gw3 = h2.T @ g
    gb3 = np.array([g.sum()])
    d2 = np.outer(g, q["w3"]) * (a2 > 0)
    gW2 = d2.T @ h1
    gb2 = d2.sum(0)
    d1 = (d2 @ q["W2"]) * (a1 > 0)
    gW1 = d1.T @ X
    gb1 = d1.sum(0)
    grad = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gw3, gb3])
    return loss, grad


def predict(params, X, bf16=True, bf16_act=False, return_hidden=False):
    """Network output per row of X (FP64 arithmetic).  bf16: weights rounded
    to BF16; bf16_act: inputs and layer-1 activations rounded to BF16 too.
    return_hidden: also the layer-1 activations (after any rounding)."""
    p = np.asarray(params, dtype=np.float64)
    q = unpack(bf16_round(p) if bf16 else p)
    X = np.asarray(X, dtype=np.float64)
    if bf16_act:
        X = bf16_round(X)
    h1 = np.maximum(X @ q["W1"].T + q["b1"], 0.0)
    if bf16_act:
        h1 = bf16_round(h1)
    h2 = np.maximum(h1 @ q["W2"].T + q["b2"], 0.0)
    y = h2 @ q["w3"] + q["b3"][0]
    return (y, h1) if return_hidden else y
