"""Float64 reference of the depth-order network (forward, loss, backward).

Test infrastructure only: imported by the tests, smoke() and the benchmark's CPU baseline, never
by the library.

The network predicts a target's minimal T-count from its canonical channel
representation: x (4^n * 4^n features) -> [Linear -> GELU] x depth -> Linear ->
softmax over T-counts 0..classes-1, trained with cross-entropy.  Weights and
inputs are taken as given (already rounded to BF16 by the caller when comparing
against the BF16 GPU path); everything here is float64.

GELU is the exact erf form, gelu(z) = z/2 (1 + erf(z / sqrt2)), with derivative
gelu'(z) = (1 + erf(z / sqrt2))/2 + z exp(-z^2 / 2) / sqrt(2 pi).
The loss is the mean over the batch of -log softmax(logits)[label].
"""

from __future__ import annotations

import math
from typing import Dict, List

import numpy as np

_erf = np.vectorize(math.erf)


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float32."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(a)
    out = (r & 0xFFFFFFFF).astype(np.uint32).view(np.float32)
    out = np.where(nan, a, out)
    return out


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(params: Dict[str, np.ndarray], x: np.ndarray, depth: int):
    """Returns (logits, cache).  params: W0..W{depth} (in x out), b0..b{depth}."""
    h = np.asarray(x, dtype=np.float64)
    cache = {"h0": h}
    for l in range(depth):
        z = h @ params[f"W{l}"].astype(np.float64) + params[f"b{l}"].astype(np.float64)
        h = gelu(z)
        cache[f"z{l}"] = z
        cache[f"h{l + 1}"] = h
    logits = h @ params[f"W{depth}"].astype(np.float64) + params[f"b{depth}"].astype(np.float64)
    return logits, cache


def softmax(logits):
    m = logits.max(axis=1, keepdims=True)
    e = np.exp(logits - m)
    return e / e.sum(axis=1, keepdims=True)


def loss(params, x, labels, depth: int) -> float:
    logits, _ = forward(params, x, depth)
    p = softmax(logits)
    return float(-np.mean(np.log(p[np.arange(len(labels)), labels])))


def gradients(params, x, labels, depth: int) -> Dict[str, np.ndarray]:
    """Gradients of the mean cross-entropy with respect to every weight and bias."""
    logits, cache = forward(params, x, depth)
    b = len(labels)
    g = softmax(logits)
    g[np.arange(b), labels] -= 1.0
    g /= b
    grads = {}
    for l in range(depth, -1, -1):
        h = cache[f"h{l}"]
        grads[f"W{l}"] = h.T @ g
        grads[f"b{l}"] = g.sum(axis=0)
        if l > 0:
            dh = g @ params[f"W{l}"].astype(np.float64).T
            g = dh * gelu_grad(cache[f"z{l - 1}"])
    return grads


def layer_sizes(inp: int, hidden: int, depth: int, classes: int) -> List[tuple]:
    sizes = [inp] + [hidden] * depth + [classes]
    return [(sizes[i], sizes[i + 1]) for i in range(depth + 1)]


SQRT2 = 1.4142135623730951      # the double nearest sqrt(2)
SQRT1_2 = 0.7071067811865476    # the double nearest 1/sqrt(2)


def features(m) -> np.ndarray:
    """FP32 features of a channel rep: its exact canonical form (zmat.canonical_form: minimal
    exponent e, rows sign-normalised and sorted as integer tuples), each entry
    (a + b sqrt2) 2^(-e/2) evaluated in float64 as t = a + (b * SQRT2), t = t * SQRT1_2 if e is
    odd, t = t * 2^(-floor(e/2)), then rounded to float32 (nearest even)."""
    from . import zmat
    e, rows = zmat.canonical_form(m)
    r = len(rows)
    out = np.empty(r * r, dtype=np.float32)
    scale = math.ldexp(1.0, -(e // 2))
    for i, row in enumerate(rows):
        for q in range(r):
            a, b = row[2 * q], row[2 * q + 1]
            t = float(a) + float(b) * SQRT2
            if e % 2:
                t = t * SQRT1_2
            out[i * r + q] = np.float32(t * scale)
    return out
