"""FP64 oracle of the direction-conditioned surrogate -- TEST INFRASTRUCTURE ONLY.

Only the tests and the benchmark may import this module; it shares no code
with the GPU library.  The surrogate predicts a direction's reflection
filters (the sparse factor of Eq. (1)) from (sin az, cos az, sin el, cos el)
through ReLU hidden layers and a linear output layer (the taps are the
largest positive outputs); activations are stored as bfloat16 between layers, so
the oracle rounds at the same points (round to nearest, ties to even, on the
FP64 value) and computes everything else in FP64.

Parameters are a list of (W [k_in][k_out], b [k_out]) pairs; the loss is the
mean squared error over every output; the optimiser is Adam with bias
correction.  Parity status: bf16 rounding pinned by its definition's
boundary cases and by torch's own float32 -> bfloat16 conversion; the
backward pass by central finite differences of the forward pass; one Adam
step by its closed form at step 1 (tests/test_oracle_mlp.py).
"""
from __future__ import annotations

import numpy as np


def bf16(x) -> np.ndarray:
    """Round to the nearest bfloat16 (8 significant bits), ties to even.
    Values stay float64; zeros and non-finite values pass through."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                       # x = m 2^e, 0.5 <= |m| < 1
    r = np.ldexp(np.rint(np.ldexp(m, 8)), e - 8)
    return np.where(np.isfinite(x), r, x)


def features(az, el) -> np.ndarray:
    """Network input of a direction (angles in radians):
    (sin az, cos az, sin el, cos el)."""
    az = np.asarray(az, dtype=np.float64)
    el = np.asarray(el, dtype=np.float64)
    return np.stack([np.sin(az), np.cos(az), np.sin(el), np.cos(el)], axis=-1)


def forward(params, X, rounding: bool = True):
    """Returns (y, cache).  cache holds each layer's bf16 input activations
    and pre-activations, for backward.  rounding=False skips the bf16
    rounding (used to check the backward pass by finite differences)."""
    rnd = bf16 if rounding else (lambda v: np.asarray(v, dtype=np.float64))
    h = rnd(X)
    cache = []
    for li, (W, b) in enumerate(params):
        z = h @ W + b
        cache.append((h, z))
        last = li + 1 == len(params)
        h = z if last else rnd(np.maximum(z, 0.0))     # ReLU hidden layers, linear output
    return h, cache


def loss_and_grads(params, X, T, rounding: bool = True):
    """Mean squared error over all outputs and its gradients (the rounding
    passes gradients straight through)."""
    y, cache = forward(params, X, rounding)
    n_el = y.size
    loss = float(np.sum((y - T) ** 2) / n_el)
    dh = 2.0 * (y - T) / n_el
    grads = [None] * len(params)
    for li in range(len(params) - 1, -1, -1):
        W, _ = params[li]
        h_in, z = cache[li]
        dz = dh if li + 1 == len(params) else dh * (z > 0)
        grads[li] = (h_in.T @ dz, dz.sum(axis=0))
        dh = dz @ W.T
    return loss, grads


def adam_step(params, grads, state, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam step (t counts from 1); state is a list of (mW, vW, mb, vb)."""
    out, new_state = [], []
    for (W, b), (gW, gb), (mW, vW, mb, vb) in zip(params, grads, state):
        res = []
        for p, g, m, v in ((W, gW, mW, vW), (b, gb, mb, vb)):
            m = beta1 * m + (1 - beta1) * g
            v = beta2 * v + (1 - beta2) * g * g
            mh = m / (1 - beta1 ** t)
            vh = v / (1 - beta2 ** t)
            res.append((p - lr * mh / (np.sqrt(vh) + eps), m, v))
        out.append((res[0][0], res[1][0]))
        new_state.append((res[0][1], res[0][2], res[1][1], res[1][2]))
    return out, new_state


def zero_state(params):
    return [(np.zeros_like(W), np.zeros_like(W), np.zeros_like(b), np.zeros_like(b)) for W, b in params]
