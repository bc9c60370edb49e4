"""CPU oracle of the join cost model -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may use
this module.  The paper has no learned component; the model is the cost
predictor of the mining pipeline, and this file writes out its definition in
float64 numpy so that the device kernels can be checked against it:

* parameters: W1 (D x H), b1 (H), W2 (H x O), b2 (O); the forward and
  backward passes read them as bfloat16 values (``bf16``), the optimiser
  keeps float32 master copies;
* forward: ``h = relu(x W1 + b1)``, ``y = h W2 + b2``;
* loss over a batch of B rows: ``L = sum((y - t)^2) / (2 B)``;
* backward: the chain rule of the two lines above, no other terms;
* optimiser: Adam as defined by Kingma and Ba (2015), Algorithm 1, with
  bias-corrected moments, applied to the float32 master copies.

The flat parameter layout (W1 row-major, b1, W2 row-major, b2) is the one
the device library exchanges with its callers.
"""
from __future__ import annotations

import numpy as np


def bf16(a):
    """Round float32 values to bfloat16 (round to nearest, ties to even) and
    return them as float64.  bfloat16 is the upper half of an IEEE binary32
    word; NaN and infinity do not occur in the model."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def sizes(D, H, O):
    return [(D, H), (H,), (H, O), (O,)]


def count(D, H, O):
    return D * H + H + H * O + O


def unpack(theta, D, H, O):
    """Flat parameter vector -> [W1, b1, W2, b2] (views)."""
    out, off = [], 0
    for shp in sizes(D, H, O):
        k = int(np.prod(shp))
        out.append(np.asarray(theta[off:off + k]).reshape(shp))
        off += k
    return out


def forward(theta, x, D, H, O):
    """Predictions y (B x O) and the hidden pre-activations, from the
    bfloat16 view of the parameters."""
    W1, b1, W2, b2 = unpack(bf16(theta), D, H, O)
    x = np.asarray(x, np.float64)
    z = x @ W1 + b1
    h = np.maximum(z, 0.0)
    return h @ W2 + b2, z


def loss(theta, x, t, D, H, O):
    y, _ = forward(theta, x, D, H, O)
    return float(np.sum((y - np.asarray(t, np.float64)) ** 2) / (2 * len(x)))


def loss_at(values, x, t, D, H, O):
    """Loss at parameter values used as they are (no bfloat16 rounding)."""
    W1, b1, W2, b2 = unpack(np.asarray(values, np.float64), D, H, O)
    h = np.maximum(np.asarray(x, np.float64) @ W1 + b1, 0.0)
    return float(np.sum((h @ W2 + b2 - np.asarray(t, np.float64)) ** 2) / (2 * len(x)))


def grad(theta, x, t, D, H, O):
    """Gradient of ``loss`` with respect to the bfloat16 parameter values,
    flattened in the parameter layout."""
    return grad_at(bf16(theta), x, t, D, H, O)


def grad_at(values, x, t, D, H, O):
    """Gradient of ``loss_at`` at the given parameter values."""
    W1, b1, W2, b2 = unpack(np.asarray(values, np.float64), D, H, O)
    x = np.asarray(x, np.float64)
    B = len(x)
    z = x @ W1 + b1
    h = np.maximum(z, 0.0)
    y = h @ W2 + b2
    dy = (y - np.asarray(t, np.float64)) / B
    gW2 = h.T @ dy
    gb2 = dy.sum(axis=0)
    dz = (dy @ W2.T) * (z > 0)
    gW1 = x.T @ dz
    gb1 = dz.sum(axis=0)
    return np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2])


def adam(theta, x, t, D, H, O, steps, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """``steps`` full-batch Adam steps from float32 master parameters
    ``theta``; returns the float32 master parameters after the last step."""
    p = np.asarray(theta, np.float64).astype(np.float32).astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for k in range(1, steps + 1):
        g = grad(p, x, t, D, H, O)
        m = beta1 * m + (1 - beta1) * g
        v = beta2 * v + (1 - beta2) * g * g
        mh = m / (1 - beta1 ** k)
        vh = v / (1 - beta2 ** k)
        p = p - lr * mh / (np.sqrt(vh) + eps)
        p = p.astype(np.float32).astype(np.float64)   # master copies are float32
    return p
