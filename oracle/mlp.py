"""Oracle: the learned surrogate (set-plus-position MLP), float64 reference.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The surrogate maps a kernel set and a launch order to a predicted makespan
(normalised by the set's area lower bound).  Each kernel contributes one token:
its 8 features and the one-hot of its launch position (16 positions plus one
"unplaced" slot for partial orders), zero-padded to 32 inputs.

  Z1 = X W1^T + b1            per token          (32 -> 256)
  S  = sum over tokens of relu(Z1)               (set pooling)
  Z2 = S W2^T + b2,  A2 = relu(Z2)               (256 -> 256)
  Z3 = A2 W3^T + b3, A3 = relu(Z3)               (256 -> 256)
  y  = A3 . w4 + b4                              (256 -> 1)
  loss = mean (y - t)^2

The device computes matrix products on BF16 operands with float32
accumulation.  This reference computes in float64 and rounds to BF16 (round
to nearest even, through float32) exactly where the device feeds an MFMA
operand: X, W1, W2, W3, w4, S, A2, A3 in the forward pass and dZ1, dZ2, dZ3
in the backward pass.  With ``bf16=False`` it is the plain float64 model, used
for central finite-difference checks.

Adam (Kingma & Ba 2015) with bias correction updates float32 master weights.
"""

from __future__ import annotations

import numpy as np

N_FEAT = 8
N_POS = 17          # 16 launch positions + "unplaced"
UNPLACED = 16
D_IN = 32
D_HID = 256

SHAPES = (("W1", (D_HID, D_IN)), ("b1", (D_HID,)), ("W2", (D_HID, D_HID)), ("b2", (D_HID,)),
          ("W3", (D_HID, D_HID)), ("b3", (D_HID,)), ("w4", (D_HID,)), ("b4", (1,)))


def n_params() -> int:
    return sum(int(np.prod(s)) for _, s in SHAPES)


def unflatten(vec):
    out, off = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = np.asarray(vec[off:off + size], dtype=np.float64).reshape(shape)
        off += size
    return out


def flatten(params) -> np.ndarray:
    return np.concatenate([np.asarray(params[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (through float32, round to nearest even); returned as float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    bits = (bits + 0x7FFF + lsb) & 0xFFFF0000
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)


def _r(x, on):
    return bf16(x) if on else np.asarray(x, dtype=np.float64)


def forward(params, X, bf16_points: bool = True):
    """X: [B, n, 32].  Returns (y [B], cache)."""
    p = params
    X = _r(X, bf16_points)
    W1, W2, W3, w4 = (_r(p[k], bf16_points) for k in ("W1", "W2", "W3", "w4"))
    Z1 = X @ W1.T + p["b1"]
    S = np.maximum(Z1, 0.0).sum(axis=1)
    y, cache = from_pooled(params, S, bf16_points)
    cache.update(X=X, W1=W1, Z1=Z1)
    return y, cache


def from_pooled(params, S, bf16_points: bool = True):
    """The layers after pooling, from S [B, 256] (the sum over tokens of
    relu(Z1)).  Returns (y [B], cache)."""
    p = params
    W2, W3, w4 = (_r(p[k], bf16_points) for k in ("W2", "W3", "w4"))
    Sb = _r(S, bf16_points)
    Z2 = Sb @ W2.T + p["b2"]
    A2b = _r(np.maximum(Z2, 0.0), bf16_points)
    Z3 = A2b @ W3.T + p["b3"]
    A3b = _r(np.maximum(Z3, 0.0), bf16_points)
    y = A3b @ w4 + p["b4"][0]
    return y, dict(W2=W2, W3=W3, w4=w4, Sb=Sb, Z2=Z2, A2b=A2b, Z3=Z3, A3b=A3b)


def loss_and_grads(params, X, t, bf16_points: bool = True):
    """Mean squared error and its gradient with respect to every parameter."""
    y, c = forward(params, X, bf16_points)
    t = np.asarray(t, dtype=np.float64)
    B = len(t)
    loss = float(np.mean((y - t) ** 2))
    dy = 2.0 * (y - t) / B
    g = {}
    g["w4"] = c["A3b"].T @ dy
    g["b4"] = np.array([dy.sum()])
    dZ3 = np.outer(dy, c["w4"]) * (c["Z3"] > 0)
    g["b3"] = dZ3.sum(axis=0)
    dZ3b = _r(dZ3, bf16_points)
    g["W3"] = dZ3b.T @ c["A2b"]
    dZ2 = (dZ3b @ c["W3"]) * (c["Z2"] > 0)
    g["b2"] = dZ2.sum(axis=0)
    dZ2b = _r(dZ2, bf16_points)
    g["W2"] = dZ2b.T @ c["Sb"]
    dS = dZ2b @ c["W2"]
    dZ1 = dS[:, None, :] * (c["Z1"] > 0)
    g["b1"] = dZ1.sum(axis=(0, 1))
    dZ1b = _r(dZ1, bf16_points)
    g["W1"] = dZ1b.reshape(-1, D_HID).T @ c["X"].reshape(-1, D_IN)
    return loss, y, g


def adam_step(theta, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update of flat float64 arrays (returns new theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    theta = theta - lr * mhat / (np.sqrt(vhat) + eps)
    return theta, m, v
