"""FP64 reference of the learned closure's network (test infrastructure only).

Not part of the paper's method: a per-node multilayer perceptron
8 -> 64 -> 64 -> 9 with tanh-form GELU (Hendrycks & Gimpel) predicts a
residual added to the recursive a1^(3), a1^(4).  This module writes the
forward pass, the analytic backward pass (MSE loss), Adam (Kingma & Ba) and
the bfloat16 rounding points of the GPU kernels, so that the GPU's outputs
and gradients can be compared with a plain computation.

Flat parameter vector (float32 on the device, float64 here), row-major
[in][out] matrices:
    W1 (8 x 64) | b1 (64) | W2 (64 x 64) | b2 (64) | W3 (64 x 16) | b3 (16)
Outputs 9..15 of the last layer are padding and stay zero.
"""
from __future__ import annotations

import numpy as np

NIN, NH, NOUT, NOUT_PAD = 8, 64, 9, 16
SHAPES = [("W1", (NIN, NH)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)),
          ("W3", (NH, NOUT_PAD)), ("b3", (NOUT_PAD,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)  # 5776
GELU_C = np.sqrt(2.0 / np.pi)
GELU_A = 0.044715


def unpack(theta):
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(p) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def init_params(seed: int) -> np.ndarray:
    """He-style initialisation; padding outputs zero."""
    rng = np.random.default_rng(seed)
    p = {
        "W1": rng.normal(0, np.sqrt(2.0 / NIN), (NIN, NH)), "b1": np.zeros(NH),
        "W2": rng.normal(0, np.sqrt(2.0 / NH), (NH, NH)), "b2": np.zeros(NH),
        "W3": np.zeros((NH, NOUT_PAD)), "b3": np.zeros(NOUT_PAD),
    }
    p["W3"][:, :NOUT] = rng.normal(0, np.sqrt(1.0 / NH), (NH, NOUT))
    return pack(p)


def gelu(z):
    return 0.5 * z * (1.0 + np.tanh(GELU_C * (z + GELU_A * z ** 3)))


def gelu_prime(z):
    t = np.tanh(GELU_C * (z + GELU_A * z ** 3))
    return 0.5 * (1.0 + t) + 0.5 * z * (1.0 - t * t) * GELU_C * (1.0 + 3.0 * GELU_A * z * z)


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(theta, X, emulate_bf16=True):
    """X (B, 8) -> Y (B, 9) and the cache of pre-activations.  With
    emulate_bf16 the inputs, weights and hidden activations are rounded to
    bfloat16 where the GPU rounds them (accumulation stays float64)."""
    p = unpack(theta)
    r = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    Xb = r(X)
    W1, W2, W3 = r(p["W1"]), r(p["W2"]), r(p["W3"][:, :NOUT])
    Z1 = Xb @ W1 + p["b1"]
    H1 = r(gelu(Z1))
    Z2 = H1 @ W2 + p["b2"]
    H2 = r(gelu(Z2))
    Y = H2 @ W3 + p["b3"][:NOUT]
    return Y, dict(Xb=Xb, Z1=Z1, H1=H1, Z2=Z2, H2=H2, W1=W1, W2=W2, W3=W3)


def loss_and_grad(theta, X, T, emulate_bf16=True):
    """Mean squared error over the batch and the 9 outputs, and its gradient
    with respect to the parameters (the bfloat16 roundings pass gradients
    through unchanged)."""
    Y, c = forward(theta, X, emulate_bf16)
    B = X.shape[0]
    diff = Y - T
    loss = float(np.mean(diff ** 2))
    dY = 2.0 * diff / (B * NOUT)
    g = {name: np.zeros(shape) for name, shape in SHAPES}
    g["W3"][:, :NOUT] = c["H2"].T @ dY
    g["b3"][:NOUT] = dY.sum(0)
    dZ2 = (dY @ c["W3"].T) * gelu_prime(c["Z2"])
    g["W2"] = c["H1"].T @ dZ2
    g["b2"] = dZ2.sum(0)
    dZ1 = (dZ2 @ c["W2"].T) * gelu_prime(c["Z1"])
    g["W1"] = c["Xb"].T @ dZ1
    g["b1"] = dZ1.sum(0)
    return loss, pack(g)


def adam(theta, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
