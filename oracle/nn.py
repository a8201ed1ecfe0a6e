"""FP64 reference of the small 3D convolutional network used as a learned preconditioner.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Layers (the network is not from the paper, which uses only the diagonal-block preconditioner
of eqs (2.31)-(2.32); its shape comes from the task: three 3x3x3 convolutions, 32 hidden
channels):
    h1 = act(conv(x, W1) + b1), h2 = act(conv(h1, W2) + b2), y = conv(h2, W3) + b3
with periodic (circular) padding, since the fields live on the periodic unit cell, and
act(t) = t for t > 0, slope * t otherwise (leaky ReLU).

Arrays: activations (C, N, N, N) indexed [c][z][y][x]; weights (Cout, Cin, 3, 3, 3) indexed
[co][ci][dz][dy][dx] with tap offsets d - 1.  Every function is a direct summation of the
definition.
"""
from __future__ import annotations

import numpy as np

SLOPE = 0.01


def conv3d(x: np.ndarray, w: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[co,z,y,x] = b[co] + sum_{ci,dz,dy,dx} w[co,ci,dz,dy,dx] x[ci, z+dz-1, y+dy-1, x+dx-1]
    (indices modulo N)."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    co = w.shape[0]
    out = np.zeros((co,) + x.shape[1:], dtype=np.float64)
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                xs = np.roll(x, shift=(-(dz - 1), -(dy - 1), -(dx - 1)), axis=(1, 2, 3))
                out += np.einsum("oc,czyx->ozyx", w[:, :, dz, dy, dx], xs)
    return out + np.asarray(b, dtype=np.float64)[:, None, None, None]


def conv3d_backward(x: np.ndarray, w: np.ndarray, gy: np.ndarray):
    """Gradients of sum(gy * conv3d(x, w, b)) with respect to x, w and b."""
    gx = np.zeros_like(x, dtype=np.float64)
    gw = np.zeros_like(w, dtype=np.float64)
    for dz in range(3):
        for dy in range(3):
            for dx in range(3):
                sh = (-(dz - 1), -(dy - 1), -(dx - 1))
                xs = np.roll(x, shift=sh, axis=(1, 2, 3))
                gw[:, :, dz, dy, dx] = np.einsum("ozyx,czyx->oc", gy, xs)
                g = np.einsum("oc,ozyx->czyx", w[:, :, dz, dy, dx], gy)
                gx += np.roll(g, shift=tuple(-s for s in sh), axis=(1, 2, 3))
    gb = gy.sum(axis=(1, 2, 3))
    return gx, gw, gb


def act(t: np.ndarray) -> np.ndarray:
    return np.where(t > 0, t, SLOPE * t)


def act_grad(t: np.ndarray, g: np.ndarray) -> np.ndarray:
    return np.where(t > 0, g, SLOPE * g)


def forward(params, x: np.ndarray):
    """params = [(W1, b1), (W2, b2), (W3, b3)]; returns output and the pre-activations."""
    (w1, b1), (w2, b2), (w3, b3) = params
    z1 = conv3d(x, w1, b1)
    h1 = act(z1)
    z2 = conv3d(h1, w2, b2)
    h2 = act(z2)
    y = conv3d(h2, w3, b3)
    return y, (z1, h1, z2, h2)


def loss(y: np.ndarray, target: np.ndarray) -> float:
    """Mean squared error over all entries."""
    d = y - target
    return float(np.mean(d * d))


def loss_grad(y: np.ndarray, target: np.ndarray) -> np.ndarray:
    return 2.0 * (y - target) / y.size


def backward(params, x: np.ndarray, cache, gy: np.ndarray):
    """Gradients of sum(gy * forward(params, x)) for every weight and bias, and for x."""
    (w1, b1), (w2, b2), (w3, b3) = params
    z1, h1, z2, h2 = cache
    gh2, gw3, gb3 = conv3d_backward(h2, w3, gy)
    gz2 = act_grad(z2, gh2)
    gh1, gw2, gb2 = conv3d_backward(h1, w2, gz2)
    gz1 = act_grad(z1, gh1)
    gx, gw1, gb1 = conv3d_backward(x, w1, gz1)
    return [(gw1, gb1), (gw2, gb2), (gw3, gb3)], gx


def adam_step(p: np.ndarray, g: np.ndarray, m: np.ndarray, v: np.ndarray, step: int, lr: float,
              b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round FP32 values to the nearest BF16 (ties to even), returned as float32."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    rounding = 0x7FFF + ((u >> 16) & 1)
    r = ((u + rounding) >> 16) << 16
    return r.astype(np.uint32).view(np.float32)
