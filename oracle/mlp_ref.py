"""FP64 reference of the histogram -> centroid network (test infrastructure only).

Network: input the 256-bin grey-level histogram normalised to sum 1;
h1 = relu(x W1 + b1) (128 units), h2 = relu(h1 W2 + b2) (64 units),
y = h2 W3 + b3 (C outputs: the centroids divided by 255).  Loss: mean squared
error over the batch and the C outputs, L = sum (y - t)^2 / (B C).
Parameters are kept as one flat vector in the order W1 (256 x 128, row-major),
b1, W2 (128 x 64), b2, W3 (64 x C), b3.  Adam: the standard update with bias
correction (beta1 = 0.9, beta2 = 0.999, eps = 1e-8).

BF16 inference: bfloat16 keeps 8 significant bits (1 implicit + 7 stored)
and the FP32 exponent range; values are rounded to nearest, ties to even.
`forward_bf16` rounds the input, every weight and bias, and every hidden
activation to BF16 and sums exactly (FP64), so it differs from a BF16 kernel
with FP32 accumulation only by that accumulation's rounding.
"""
from __future__ import annotations

import numpy as np

SIZES = (256, 128, 64)


def shapes(C: int):
    return [(256, 128), (128,), (128, 64), (64,), (64, C), (C,)]


def n_params(C: int) -> int:
    return int(sum(np.prod(s) for s in shapes(C)))


def unpack(theta: np.ndarray, C: int):
    out, o = [], 0
    for s in shapes(C):
        k = int(np.prod(s))
        out.append(theta[o:o + k].reshape(s))
        o += k
    return out


def forward(theta, X, C):
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(theta, dtype=np.float64), C)
    X = np.asarray(X, dtype=np.float64)
    z1 = X @ W1 + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2 + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ W3 + b3
    return y, (X, z1, h1, z2, h2)


def loss(theta, X, T, C):
    y, _ = forward(theta, X, C)
    return float(((y - T) ** 2).sum() / (y.shape[0] * C))


def grad(theta, X, T, C):
    """Analytic gradient of `loss` by the chain rule (flat, same layout)."""
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(theta, dtype=np.float64), C)
    y, (X, z1, h1, z2, h2) = forward(theta, X, C)
    B = y.shape[0]
    dy = 2.0 * (y - T) / (B * C)
    gW3 = h2.T @ dy
    gb3 = dy.sum(axis=0)
    dh2 = dy @ W3.T
    dz2 = dh2 * (z2 > 0)
    gW2 = h1.T @ dz2
    gb2 = dz2.sum(axis=0)
    dh1 = dz2 @ W2.T
    dz1 = dh1 * (z1 > 0)
    gW1 = X.T @ dz1
    gb1 = dz1.sum(axis=0)
    return np.concatenate([g.ravel() for g in (gW1, gb1, gW2, gb2, gW3, gb3)])


def adam_step(theta, g, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(v):
    """Round to the nearest BF16 value, ties to even (finite, normal inputs)."""
    v = np.asarray(v, dtype=np.float64)
    m, e = np.frexp(v)                 # v = m 2^e, |m| in [0.5, 1)
    return np.ldexp(np.rint(m * 256.0) / 256.0, e)   # 8 significant bits; rint ties to even


def forward_bf16(theta, X, C):
    W1, b1, W2, b2, W3, b3 = (bf16_round(w) for w in unpack(np.asarray(theta, dtype=np.float64), C))
    a0 = bf16_round(np.asarray(X, dtype=np.float64))
    a1 = bf16_round(np.maximum(a0 @ W1 + b1, 0.0))
    a2 = bf16_round(np.maximum(a1 @ W2 + b2, 0.0))
    return a2 @ W3 + b3
