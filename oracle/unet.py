"""Oracle of the learned-stage network: a plain numpy U-Net forward pass.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The network is the 4-level 3D U-Net of the learned preconditioner stage:
3x3x3 convolutions with zero padding, ReLU after every convolution but the
last, 2x2x2 average pooling, nearest upsampling, additive skip connections
(added before the ReLU), channels 16/32/48/64, 3 input features padded to 16,
output channel 0.  Parameters are one flat FP32 array: all weights layer by
layer as [c_out][27 taps][c_in] (tap = 9 dz + 3 dy + dx, offsets -1..1), then
all biases.  Arrays are channel-last: [z][y][x][c].  Arithmetic is float64;
``round_bf16`` emulates the BF16 storage of inputs, weights and activations.
"""
from __future__ import annotations

import numpy as np

SPEC = [(0, 16, 16, 1), (0, 16, 16, 1), (1, 16, 32, 1), (1, 32, 32, 1), (2, 32, 48, 1), (2, 48, 48, 1),
        (3, 48, 64, 1), (3, 64, 64, 1), (2, 64, 48, 1), (2, 48, 48, 1), (1, 48, 32, 1), (1, 32, 32, 1),
        (0, 32, 16, 1), (0, 16, 16, 1), (0, 16, 16, 0)]


def param_count():
    return sum(co * 27 * ci for _, ci, co, _ in SPEC) + sum(co for _, _, co, _ in SPEC)


def split_params(p):
    ws, bs, off = [], [], 0
    for _, ci, co, _ in SPEC:
        ws.append(p[off:off + co * 27 * ci].reshape(co, 27, ci))
        off += co * 27 * ci
    for _, _, co, _ in SPEC:
        bs.append(p[off:off + co])
        off += co
    return ws, bs


def round_bf16(a):
    """Round float values to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def conv3(x, w, b):
    """3x3x3 convolution, zero padding: out[v][co] = sum_tap,ci w[co,tap,ci] x[v+off(tap)][ci] + b."""
    n = x.shape[0]
    xp = np.zeros((n + 2, n + 2, n + 2, x.shape[3]))
    xp[1:-1, 1:-1, 1:-1] = x
    out = np.zeros((n, n, n, w.shape[0]))
    for tap in range(27):
        dz, dy, dx = tap // 9, (tap // 3) % 3, tap % 3
        out += xp[dz:dz + n, dy:dy + n, dx:dx + n] @ w[:, tap, :].T
    return out + b


def pool(x):
    n = x.shape[0] // 2
    return x.reshape(n, 2, n, 2, n, 2, -1).mean(axis=(1, 3, 5))


def up(x):
    return x.repeat(2, axis=0).repeat(2, axis=1).repeat(2, axis=2)


def forward(params, feats, bf16=True):
    """Prediction (n^3, channel 0 of the output) for planar features (3, n, n, n)."""
    r = round_bf16 if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    ws, bs = split_params(np.asarray(params, dtype=np.float64))
    ws = [r(w) for w in ws]
    n = feats.shape[1]
    x = np.zeros((n, n, n, 16))
    for c in range(3):
        x[..., c] = feats[c]
    x = r(x)
    relu = lambda a: np.maximum(a, 0.0)
    L = lambda i, inp, skip=None: r(relu(conv3(inp, ws[i], bs[i]) + (0 if skip is None else skip)))
    a0 = L(0, x); s0 = L(1, a0)
    a1 = L(2, r(pool(s0))); s1 = L(3, a1)
    a2 = L(4, r(pool(s1))); s2 = L(5, a2)
    a3 = L(6, r(pool(s2))); d3 = L(7, a3)
    x2 = L(8, up(d3), s2); d2 = L(9, x2)
    x1 = L(10, up(d2), s1); d1 = L(11, x1)
    x0 = L(12, up(d1), s0); d0 = L(13, x0)
    y = conv3(d0, ws[14], bs[14])
    return y[..., 0]


def loss(params, feats, target, bf16=False):
    d = forward(params, feats, bf16=bf16) - target
    return float(np.mean(d * d))
