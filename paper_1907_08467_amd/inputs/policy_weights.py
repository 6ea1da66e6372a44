"""Seeded random weights for the policy network (an input: the throughput
measurements need no trained weights).  He-uniform weights and small uniform
biases, rounded to bf16; returned both as bf16 bit patterns in the layouts the
library takes and as the float64 values of those bf16 numbers.

Layer l has N_l outputs and K_l reduction inputs: (32, 256), (64, 512),
(64, 576), (512, 3136), (19, 512).  Layer 1's reduction index is
(channel * 8 + ky) * 8 + kx; the others' (ky * KW + kx) * Cin + channel.
"""
from __future__ import annotations

import numpy as np

SHAPES = [(32, 256), (64, 512), (64, 576), (512, 3136), (19, 512)]


def to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """float32 -> bf16 bit patterns, round to nearest even (finite inputs)."""
    u = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return r.astype(np.uint16)


def bf16_bits_to_f64(b: np.ndarray) -> np.ndarray:
    return (b.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def policy_weights(seed: int = 7):
    """[(w_bits [N][K] uint16, w [N][K] float64, b [N] float32)] for the 5 layers."""
    g = np.random.Generator(np.random.PCG64(seed))
    out = []
    for n, k in SHAPES:
        lim = np.sqrt(6.0 / k)
        w = g.uniform(-lim, lim, (n, k)).astype(np.float32)
        bits = to_bf16_bits(w)
        b = g.uniform(-0.05, 0.05, n).astype(np.float32)
        out.append((bits, bf16_bits_to_f64(bits), b))
    return out
