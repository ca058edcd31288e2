"""Plain numpy reference of the band-proposal network (test infrastructure only).

The network maps 1,088 input features to 64 band logits through two hidden
ReLU layers of 512 and 256 units: z1 = x W1 + b1, h1 = relu(z1), z2 = h1 W2 + b2,
h2 = relu(z2), logits = h2 W3 + b3, trained with softmax cross-entropy and Adam.
This file states that arithmetic in FP64 with no blocking or fusion; with
``bf16=True`` it rounds to BF16 at the points where the GPU kernels store BF16
(inputs, weights, hidden activations, back-propagated gradients), so that a
GPU result can be compared tightly.  It shares no code with the HIP path.
"""
from __future__ import annotations

import numpy as np

DIMS = (1088, 512, 256, 64)


def bf16_round(x):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_bits(x):
    """BF16 bit patterns (uint16) of x, rounded to nearest even."""
    f = bf16_round(x).astype(np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


def from_bf16_bits(h):
    return (np.asarray(h, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)


def _r(x, on):
    return bf16_round(x) if on else np.asarray(x, dtype=np.float64)


def forward(params, x, bf16=False):
    """Returns (logits, cache).  params = [W1, b1, W2, b2, W3, b3]."""
    W1, b1, W2, b2, W3, b3 = params
    x = _r(x, bf16)
    z1 = x @ _r(W1, bf16) + b1
    h1 = _r(np.maximum(z1, 0.0), bf16)
    z2 = h1 @ _r(W2, bf16) + b2
    h2 = _r(np.maximum(z2, 0.0), bf16)
    logits = h2 @ _r(W3, bf16) + b3
    return logits, (x, h1, h2)


def softmax_xent(logits, labels):
    """Cross-entropy averaged over all n rows, and its gradient with respect to
    the logits.  A row whose label is outside [0, c) is ignored: it adds 0 to
    the loss sum and gets a zero gradient (the divisor stays n)."""
    z = logits - logits.max(axis=1, keepdims=True)
    p = np.exp(z)
    p /= p.sum(axis=1, keepdims=True)
    n, c = logits.shape
    labels = np.asarray(labels)
    keep = (labels >= 0) & (labels < c)
    rows = np.arange(n)[keep]
    loss = -np.log(p[rows, labels[keep]]).sum() / n
    g = p.copy()
    g[rows, labels[keep]] -= 1.0
    g[~keep] = 0.0
    return loss, g / n


def backward(params, cache, dlogits, bf16=False):
    """Gradients [dW1, db1, dW2, db2, dW3, db3] of the loss given dL/dlogits."""
    W1, b1, W2, b2, W3, b3 = params
    x, h1, h2 = cache
    g3 = _r(dlogits, bf16)
    dW3 = h2.T @ g3
    db3 = dlogits.sum(axis=0)
    dz2 = (g3 @ _r(W3, bf16).T) * (h2 > 0)
    db2 = dz2.sum(axis=0)
    dz2 = _r(dz2, bf16)
    dW2 = h1.T @ dz2
    dz1 = (dz2 @ _r(W2, bf16).T) * (h1 > 0)
    db1 = dz1.sum(axis=0)
    dz1 = _r(dz1, bf16)
    dW1 = x.T @ dz1
    return [dW1, db1, dW2, db2, dW3, db3]


def loss(params, x, labels, bf16=False):
    logits, _ = forward(params, x, bf16)
    return softmax_xent(logits, labels)[0]


def adam_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One bias-corrected Adam step; returns (p, m, v)."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed, dims=DIMS):
    """He-normal weights, zero biases."""
    rng = np.random.default_rng(seed)
    out = []
    for a, b in zip(dims[:-1], dims[1:]):
        out.append(rng.normal(0.0, np.sqrt(2.0 / a), size=(a, b)))
        out.append(np.zeros(b))
    return out
