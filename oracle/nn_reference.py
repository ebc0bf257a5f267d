"""FP64 CPU reference for the warm-start network's layers (test infrastructure).

Plain numpy definitions, channels-last arrays (n, d, h, w, c), periodic
3x3x3 convolutions with weights w[co, tap, ci], tap = (dz+1)*9 + (dy+1)*3 +
(dx+1).  Shares no code with the GPU kernels; the tests pin these
definitions to scipy's periodic correlation and to finite differences.
"""
from __future__ import annotations

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def shifted(x: np.ndarray, off) -> np.ndarray:
    """x[m + off] with periodic wrap (axes 1..3 are z, y, x)."""
    dz, dy, dx = off
    return np.roll(x, shift=(-dz, -dy, -dx), axis=(1, 2, 3))


def conv3d(x, w, bias=None):
    """y[.., co] = bias[co] + sum_{tap, ci} x[m + off(tap), ci] w[co, tap, ci]."""
    y = np.zeros(x.shape[:4] + (w.shape[0],))
    for t, off in enumerate(TAPS):
        y += shifted(x, off) @ w[:, t, :].T
    if bias is not None:
        y += bias
    return y


def conv3d_backward(x, w, dy):
    """(dx, dw, db) of conv3d for upstream gradient dy."""
    dx = np.zeros_like(x, dtype=np.float64)
    dw = np.zeros(w.shape)
    for t, off in enumerate(TAPS):
        xs = shifted(x, off)
        dw[:, t, :] = dy.reshape(-1, dy.shape[-1]).T @ xs.reshape(-1, xs.shape[-1])
        # x[m + off] feeds y[m]: its gradient is dy shifted back by off
        dx += shifted(dy @ w[:, t, :], tuple(-o for o in off))
    db = dy.reshape(-1, dy.shape[-1]).sum(axis=0)
    return dx, dw, db


def pool2(x):
    n, d, h, w, c = x.shape
    return x.reshape(n, d // 2, 2, h // 2, 2, w // 2, 2, c).mean(axis=(2, 4, 6))


def pool2_backward(dy):
    return np.repeat(np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2), 2, axis=3) / 8.0


def up2(x):
    return np.repeat(np.repeat(np.repeat(x, 2, axis=1), 2, axis=2), 2, axis=3)


def up2_backward(dy):
    n, d, h, w, c = dy.shape
    return dy.reshape(n, d // 2, 2, h // 2, 2, w // 2, 2, c).sum(axis=(2, 4, 6))


def bf16(a: np.ndarray) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) >> 16 << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)
