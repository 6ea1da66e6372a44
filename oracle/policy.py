"""Policy-network oracle (test infrastructure only; the library never uses it).

The network of the inference path, stated as its plain definition in float64
with no intermediate rounding: x = stack / 255 (channels = the 4 stacked
observations); three valid convolutions with ReLU, out[y, x, o] = b[o] +
sum over (ky, kx, c) of w[o, ky, kx, c] * in[s*y + ky, s*x + kx, c]
(32 filters 8x8 stride 4, 64 4x4 stride 2, 64 3x3 stride 1); a dense layer on
the 7x7x64 map flattened in (y, x, c) order with ReLU; a dense head whose
first 18 outputs are the action logits (the 19th a value).  The greedy
action is the first maximal logit.
"""
from __future__ import annotations

import numpy as np

CONVS = [(4, 8, 4), (32, 4, 2), (64, 3, 1)]   # (input channels, kernel, stride)


def conv_relu(x: np.ndarray, w: np.ndarray, b: np.ndarray, stride: int) -> np.ndarray:
    """x [n][H][W][C], w [O][k][k][C] -> relu(conv) [n][OH][OW][O], float64."""
    n, h, wd, c = x.shape
    o, k = w.shape[0], w.shape[1]
    oh, ow = (h - k) // stride + 1, (wd - k) // stride + 1
    out = np.broadcast_to(b.astype(np.float64), (n, oh, ow, o)).copy()
    for ky in range(k):
        for kx in range(k):
            patch = x[:, ky:ky + stride * (oh - 1) + 1:stride, kx:kx + stride * (ow - 1) + 1:stride, :]
            out += patch @ w[:, ky, kx, :].T
    return np.maximum(out, 0.0)


def unpack_weights(layers):
    """The library layouts (see inputs.policy_weights) -> natural float64 arrays."""
    w1 = layers[0][1].reshape(32, 4, 8, 8).transpose(0, 2, 3, 1)        # (o, ci, ky, kx) -> (o, ky, kx, ci)
    w2 = layers[1][1].reshape(64, 4, 4, 32)
    w3 = layers[2][1].reshape(64, 3, 3, 64)
    w4 = layers[3][1]                                                   # [512][3136], (y, x, c) order
    w5 = layers[4][1]                                                   # [19][512]
    bs = [l[2].astype(np.float64) for l in layers]
    return [w1, w2, w3, w4, w5], bs


def forward(stack: np.ndarray, layers) -> np.ndarray:
    """stack u8 [n][4][84][84] -> outputs [n][19] float64 (18 logits, value)."""
    ws, bs = unpack_weights(layers)
    x = stack.astype(np.float64).transpose(0, 2, 3, 1) / 255.0
    for (cin, k, s), w, b in zip(CONVS, ws[:3], bs[:3]):
        x = conv_relu(x, w, b, s)
    h = np.maximum(x.reshape(x.shape[0], -1) @ ws[3].T + bs[3], 0.0)
    return h @ ws[4].T + bs[4]


def greedy(logits: np.ndarray) -> np.ndarray:
    return np.argmax(logits[:, :18], axis=1).astype(np.uint8)
