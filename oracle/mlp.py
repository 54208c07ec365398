"""FP64 reference of the surrogate network (test infrastructure only).

An ensemble member maps 5 droplet parameters to 3 outputs:

    z1 = W1 x + b1,  h1 = gelu(z1)          (128 units)
    z2 = W2 h1 + b2, h2 = gelu(z2)          (128 units)
    y  = W3 h2 + b3                         (3 outputs)

with the exact GELU, gelu(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2.  The
training loss of a batch of n samples is

    L = sum_j w_j sum_s mask_sj (y_sj - t_sj)^2 / n

(mask 0 drops a target that is undefined for a sample).  Parameters are one
flat FP32 vector per member in the order W1 (128x5, row-major), b1, W2
(128x128), b2, W3 (3x128), b3.  `bf16=True` rounds the matrix operands to
BF16 (round to nearest even from FP32) at the points where the GPU kernels
feed the matrix cores: x and the weights, h1 and h2 in the forward pass, the
output gradient dY and dZ2 in the backward pass, and the stored activations
and gradients of the weight-gradient products.
"""
from __future__ import annotations

import math
from typing import Dict, Tuple

import numpy as np

IN, HID, OUT = 5, 128, 3
SHAPES = (("W1", (HID, IN)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)), ("W3", (OUT, HID)), ("b3", (OUT,)))
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(flat: np.ndarray) -> Dict[str, np.ndarray]:
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(p: Dict[str, np.ndarray]) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SHAPES])


def bf16(a: np.ndarray) -> np.ndarray:
    """Round to BF16 (nearest, ties to even) through FP32."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + np.vectorize(math.erf)(z / math.sqrt(2.0)))


def gelu_prime(z):
    Phi = 0.5 * (1.0 + np.vectorize(math.erf)(z / math.sqrt(2.0)))
    return Phi + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(flat: np.ndarray, x: np.ndarray, bf: bool = False):
    """Outputs y (n, 3) and the intermediates (z1, h1, z2, h2)."""
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    p = unpack(flat)
    x = r(x)
    z1 = x @ r(p["W1"]).T + p["b1"]
    h1 = gelu(z1)
    z2 = r(h1) @ r(p["W2"]).T + p["b2"]
    h2 = gelu(z2)
    y = r(h2) @ r(p["W3"]).T + p["b3"]
    return y, (x, z1, h1, z2, h2)


def loss_and_grad(flat: np.ndarray, x: np.ndarray, t: np.ndarray, mask: np.ndarray, w, bf: bool = False
                  ) -> Tuple[float, np.ndarray]:
    """L and dL/dparams (flat, same layout) by the chain rule."""
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    p = unpack(flat)
    n = x.shape[0]
    w = np.asarray(w, dtype=np.float64)
    y, (xr, z1, h1, z2, h2) = forward(flat, x, bf)
    res = (y - t) * mask
    L = float(np.sum(w * res * res) / n)
    dy = 2.0 * w * res / n                        # (n, 3)
    dW3 = r(dy).T @ r(h2)
    db3 = dy.sum(axis=0)
    dz2 = (r(dy) @ r(p["W3"])) * gelu_prime(z2)  # (n, 128)
    dW2 = r(dz2).T @ r(h1)
    db2 = dz2.sum(axis=0)
    dz1 = (r(dz2) @ r(p["W2"])) * gelu_prime(z1)
    dW1 = r(dz1).T @ xr
    db1 = dz1.sum(axis=0)
    return L, pack(dict(W1=dW1, b1=db1, W2=dW2, b2=db2, W3=dW3, b3=db3))


def loss(flat, x, t, mask, w) -> float:
    return loss_and_grad(flat, x, t, mask, w)[0]


def adam(flat, grad, m, v, step: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma & Ba, 2015), bias-corrected; returns new (flat, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v


def init(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in SHAPES:
        if name.startswith("W"):
            bound = math.sqrt(6.0 / shape[1])
            p[name] = rng.uniform(-bound, bound, shape)
        else:
            p[name] = np.zeros(shape)
    return pack(p)
