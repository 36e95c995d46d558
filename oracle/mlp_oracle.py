"""FP64 CPU oracle of the edge-screener MLP (test infrastructure only).

Only the test suite may import this module.  The network is 4 -> 64 -> 64 ->
1 with ReLU, on per-(stage, edge) features (the edge's robot-frame endpoints
scaled by 1/FEATURE_SCALE).  The GPU kernels multiply BF16 operands with
FP32 accumulation; this oracle evaluates the same network in float64 and,
with ``bf16=True``, rounds to BF16 exactly where the kernels feed a matrix
unit: the features and the first-layer weights, the first hidden layer
(input of layer 2) and the second-layer weights, and in the backward pass the
second-layer output gradient (input of the weight-gradient and input-gradient
products) and the first-layer output gradient.  Layer 3 and the biases stay
in full precision, as in the kernels.  With ``bf16=False`` it is the plain
float64 network, which finite differences pin.

Loss: mean squared error over the batch, L = mean((y - t)^2).
Parameter vector layout (float32 master copy, 4545 entries):
W1[64][4], b1[64], W2[64][64], b2[64], w3[64], b3[1].
"""
from __future__ import annotations

import numpy as np

H = 64
N_IN = 4
FEATURE_SCALE = 4.0
N_PARAMS = H * N_IN + H + H * H + H + H + 1


def unpack(theta):
    t = np.asarray(theta, dtype=np.float64)
    o = 0
    W1 = t[o:o + H * N_IN].reshape(H, N_IN); o += H * N_IN
    b1 = t[o:o + H]; o += H
    W2 = t[o:o + H * H].reshape(H, H); o += H * H
    b2 = t[o:o + H]; o += H
    w3 = t[o:o + H]; o += H
    b3 = t[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([np.ravel(W1), b1, np.ravel(W2), b2, w3, [b3]])


def bf16(x):
    """Round float32-representable values to bfloat16, nearest-even, as float64."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(np.isnan(a), np.nan, out)


def _r(x, on):
    return bf16(x) if on else np.asarray(x, dtype=np.float64)


def forward(theta, X, bf16_on=True):
    """y (B,) and the intermediates for backward."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    Xr = _r(X, bf16_on)
    h1pre = Xr @ _r(W1, bf16_on).T + b1
    h1 = np.maximum(h1pre, 0.0)
    h1r = _r(h1, bf16_on)
    h2pre = h1r @ _r(W2, bf16_on).T + b2
    h2 = np.maximum(h2pre, 0.0)
    y = h2 @ w3 + b3
    return y, dict(Xr=Xr, h1pre=h1pre, h1r=h1r, h2pre=h2pre, h2=h2)


def loss(theta, X, t, bf16_on=True):
    y, _ = forward(theta, X, bf16_on)
    return float(np.mean((y - np.asarray(t, dtype=np.float64)) ** 2))


def backward(theta, X, t, bf16_on=True):
    """Gradient of the mean squared error with respect to the parameter
    vector (same layout as theta).  ReLU'(0) = 0."""
    W1, b1, W2, b2, w3, b3 = unpack(theta)
    y, c = forward(theta, X, bf16_on)
    B = len(y)
    dy = 2.0 * (y - np.asarray(t, dtype=np.float64)) / B
    dw3 = c["h2"].T @ dy
    db3 = dy.sum()
    dh2 = (dy[:, None] * w3[None, :]) * (c["h2pre"] > 0)
    dh2r = _r(dh2, bf16_on)
    dW2 = dh2r.T @ c["h1r"]
    db2 = dh2.sum(0)
    dh1 = (dh2r @ _r(W2, bf16_on)) * (c["h1pre"] > 0)
    dh1r = _r(dh1, bf16_on)
    dW1 = dh1r.T @ c["Xr"]
    db1 = dh1.sum(0)
    return pack(dW1, db1, dW2, db2, dw3, db3)


def adam(theta, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (step counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
