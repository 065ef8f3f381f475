"""FP64 reference of the warm-start MLP (test infrastructure only: only the
tests, the smoke check and the benchmark's CPU leg use it; the library never
imports it).

Network in -> hidden (ReLU) -> hidden (ReLU) -> out with mean-squared-error
loss; flat parameters [W1, b1, W2, b2, W3, b3], W_l stored out_l x in_l.

`bf16=True` is the network of the warm-start configuration, a bfloat16 network
with float32 accumulation: every matrix product takes bfloat16 operands (the
input, the weights, the activations of the forward pass and the gradients
propagated back through the products), so those operands are rounded to the
nearest bfloat16 (ties to even) and the products and everything else are
evaluated in float64.  Biases, the ReLU masks, the loss and the bias gradients
use the unrounded values.  `bf16=False` is the plain network, whose gradient
is pinned by finite differences in the tests; on data for which every rounded
operand is already a bfloat16 value the two modes agree exactly.

`adam_step` is the Adam update (Kingma and Ba, "Adam: a method for
stochastic optimization", 2015, Algorithm 1) in float64.
"""
from __future__ import annotations

import numpy as np


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(theta: np.ndarray, dims):
    i, h, o = dims
    shapes = [(h, i), (h,), (h, h), (h,), (o, h), (o,)]
    out, k = [], 0
    for s in shapes:
        size = int(np.prod(s))
        out.append(np.asarray(theta[k:k + size], dtype=np.float64).reshape(s))
        k += size
    return out


def loss_and_grad(theta, x, t, dims, bf16: bool = True):
    """Return (loss, flat gradient) of mean((y - t)^2)."""
    r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(theta, dims)
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    xb = r(x)
    a1 = np.maximum(xb @ r(W1).T + b1, 0.0)
    a1b = r(a1)
    a2 = np.maximum(a1b @ r(W2).T + b2, 0.0)
    a2b = r(a2)
    y = a2b @ r(W3).T + b3
    count = y.size
    loss = float(((y - t) ** 2).sum() / count)
    dy = 2.0 * (y - t) / count
    dyb = r(dy)
    gW3 = dyb.T @ a2b
    gb3 = dy.sum(0)
    dz2 = (dyb @ r(W3)) * (a2 > 0)
    dz2b = r(dz2)
    gW2 = dz2b.T @ a1b
    gb2 = dz2.sum(0)
    dz1 = (dz2b @ r(W2)) * (a1 > 0)
    dz1b = r(dz1)
    gW1 = dz1b.T @ xb
    gb1 = dz1.sum(0)
    grad = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, grad


def forward(theta, x, dims, bf16: bool = True):
    r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(theta, dims)
    a1 = np.maximum(r(x) @ r(W1).T + b1, 0.0)
    a2 = np.maximum(r(a1) @ r(W2).T + b2, 0.0)
    return r(a2) @ r(W3).T + b3


def adam_step(theta, grad, m, v, step: int, lr: float, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8):
    """One Adam step on flat float64 arrays; `step` counts from 1.  Returns
    (theta, m, v) after the step: biased first and second moment estimates,
    their bias corrections by 1 - beta^step, and the update
    lr * m_hat / (sqrt(v_hat) + eps)."""
    theta = np.asarray(theta, dtype=np.float64)
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = v / (1.0 - beta2 ** step)
    return theta - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
