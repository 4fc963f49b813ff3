"""Seeded synthetic inputs for the U-Net: initial parameters and BF16-exact
test tensors.  Random draws only; no step of the network is computed here.

Draws use the counter-based SplitMix64 stream of `inputs.uniform01`, one
stream per tensor (seed + 1000003 * tensor index).
"""
from __future__ import annotations

import numpy as np

from .inputs import splitmix64, uniform01


def bf16_exact(seed: int, shape, exp: int = 7, kmax: int = 255) -> np.ndarray:
    """float32 array of k * 2^-exp with integer k uniform in [-kmax, kmax]:
    at most 8 significant bits, so every value is exact in BF16."""
    n = int(np.prod(shape))
    k = (splitmix64(seed, np.arange(n)) % np.uint64(2 * kmax + 1)).astype(np.int64) - kmax
    return (k.astype(np.float64) * 2.0 ** -exp).astype(np.float32).reshape(shape)


def _uniform(seed: int, n: int, lo: float, hi: float) -> np.ndarray:
    return lo + (hi - lo) * uniform01(seed, np.arange(n))


def init_params(entries, seed: int = 0, head_gamma: float = 0.05, bf16_weights: bool = False) -> dict:
    """Initial parameters {name: float32 array} for the entries (name, dims)
    of the flat parameter array.  Convolution weights ~ U(-b, b) with
    b = 1/sqrt(fan_in); GN gamma = 1 (head: head_gamma), beta = 0; MLP
    first layer ~ U(-1, 1), later layers and biases ~ U(-b, b); projections
    ~ U(-b, b) with b = 1/sqrt(basis).  bf16_weights rounds the convolution
    weights to the nearest 8-significant-bit value (so a BF16 copy is exact)."""
    out = {}
    for idx, (name, dims) in enumerate(entries):
        n = int(np.prod(dims))
        s = seed + 1000003 * (idx + 1)
        if name.endswith(".gamma"):
            v = np.full(n, head_gamma if name.startswith("head") else 1.0)
        elif name.endswith(".beta"):
            v = np.zeros(n)
        elif name.startswith("mlp.w0") or name.startswith("mlp.b0"):
            v = _uniform(s, n, -1.0, 1.0)
        elif name.startswith("mlp."):
            b = 1.0 / np.sqrt(dims[-1]) if name.startswith("mlp.w") else 1.0 / np.sqrt(n)
            v = _uniform(s, n, -b, b)
        elif name.startswith("film"):
            b = 1.0 / np.sqrt(dims[-1])
            v = _uniform(s, n, -b, b)
        else:  # enc/mid/dec/head conv [9][Cout][Cin] or up [4][Cout][Cin]
            fan_in = dims[0] * dims[2] if dims[0] == 9 else dims[2]
            b = 1.0 / np.sqrt(fan_in)
            v = _uniform(s, n, -b, b)
            if bf16_weights:
                e = np.floor(np.log2(np.maximum(np.abs(v), 1e-30)))
                q = 2.0 ** (e - 7)
                v = np.round(v / q) * q
        out[name] = v.astype(np.float32).reshape(dims)
    return out
