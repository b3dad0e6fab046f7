"""Reference of the candidate-filter MLP (test infrastructure).

The network scores a candidate window from its 64 seed-hit features:
    z1 = x W1 + b1,  a1 = relu(z1)         W1: 64 x 128
    z2 = a1 W2 + b2, a2 = relu(z2)         W2: 128 x 128
    z = a2 w3 + b3,  p = sigmoid(z)        w3: 128
trained with the mean binary cross-entropy on logits and Adam on float32
master weights.  The GPU kernels multiply bfloat16 operands with float32
accumulation; `rounding=True` reproduces their rounding points (weights,
inputs, a1, a2 and the back-propagated dz2/dz1 rounded to bfloat16 before they
enter a product), `rounding=False` is the plain float64 network used to pin
the gradients against finite differences.

Parameter vector layout (float32, 24,961 values): W1 row-major [in][out], b1,
W2 row-major, b2, w3, b3.
"""
from __future__ import annotations

import numpy as np

from oracle.features_ref import bf16_round

D_IN, D_H = 64, 128
SIZES = [("W1", (D_IN, D_H)), ("b1", (D_H,)), ("W2", (D_H, D_H)), ("b2", (D_H,)),
         ("w3", (D_H,)), ("b3", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    out, k = {}, 0
    for name, shape in SIZES:
        size = int(np.prod(shape))
        out[name] = np.asarray(theta[k:k + size]).reshape(shape)
        k += size
    return out


def pack(p) -> np.ndarray:
    return np.concatenate([np.asarray(p[name]).reshape(-1) for name, _ in SIZES])


def init(seed: int) -> np.ndarray:
    """He-normal weights, zero biases (float32)."""
    g = np.random.default_rng(seed)
    p = {"W1": g.normal(0, np.sqrt(2 / D_IN), (D_IN, D_H)),
         "b1": np.zeros(D_H), "W2": g.normal(0, np.sqrt(2 / D_H), (D_H, D_H)),
         "b2": np.zeros(D_H), "w3": g.normal(0, np.sqrt(1 / D_H), D_H), "b3": np.zeros(1)}
    return pack(p).astype(np.float32)


def _r(x, rounding):
    return bf16_round(x).astype(np.float64) if rounding else np.asarray(x, dtype=np.float64)


def forward(theta, X, rounding=True):
    """Returns dict of z1, a1, z2, a2, z (logits), p for inputs X [B, 64]."""
    P = unpack(np.asarray(theta, dtype=np.float64 if not rounding else np.float32))
    dt = np.float32 if rounding else np.float64
    X = _r(X, rounding)
    W1, W2, w3 = _r(P["W1"], rounding), _r(P["W2"], rounding), _r(P["w3"], rounding)
    z1 = (X @ W1).astype(dt) + P["b1"].astype(dt)
    a1 = _r(np.maximum(z1, 0), rounding)
    z2 = (a1 @ W2).astype(dt) + P["b2"].astype(dt)
    a2 = _r(np.maximum(z2, 0), rounding)
    z = (a2 @ w3).astype(dt) + P["b3"].astype(dt)[0]
    p = 1.0 / (1.0 + np.exp(-z.astype(np.float64)))
    return dict(X=X, z1=z1, a1=a1, z2=z2, a2=a2, z=z, p=p)


def bce_with_logits(z, y) -> float:
    z = np.asarray(z, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    return float(np.mean(np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z)))))


def loss(theta, X, y, rounding=False) -> float:
    return bce_with_logits(forward(theta, X, rounding)["z"], y)


def grads(theta, X, y, rounding=True):
    """Loss and gradient vector (same layout as theta) of the mean BCE."""
    f = forward(theta, X, rounding)
    P = unpack(np.asarray(theta, dtype=np.float64))
    B = len(y)
    W2 = _r(P["W2"], rounding)
    w3 = _r(P["w3"], rounding)
    dz = (f["p"] - np.asarray(y, dtype=np.float64)) / B             # dL/dz
    dw3 = f["a2"].T @ dz
    db3 = np.array([dz.sum()])
    dz2 = np.outer(dz, w3) * (f["z2"] > 0)
    dz2 = _r(dz2, rounding)
    dW2 = f["a1"].T @ dz2
    db2 = dz2.sum(axis=0)
    dz1 = (dz2 @ W2.T) * (f["z1"] > 0)
    dz1 = _r(dz1, rounding)
    dW1 = f["X"].T @ dz1
    db1 = dz1.sum(axis=0)
    g = pack({"W1": dW1, "b1": db1, "W2": dW2, "b2": db2, "w3": dw3, "b3": db3})
    return bce_with_logits(f["z"], y), g


def adam(theta, m, v, g, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update in float32; returns (theta, m, v)."""
    f32 = np.float32
    m = (f32(b1) * m + f32(1 - b1) * g).astype(f32)
    v = (f32(b2) * v + f32(1 - b2) * g * g).astype(f32)
    mh = m / f32(1 - b1 ** step)
    vh = v / f32(1 - b2 ** step)
    theta = (theta - f32(lr) * mh / (np.sqrt(vh) + f32(eps))).astype(f32)
    return theta, m, v
