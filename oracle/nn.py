"""Reference 3-D convolution network pieces for the learned preconditioner
(test infrastructure only; the product path never imports this module).

Tensors are channels-last ``(D, H, W, C)`` arrays.  A 3x3x3 convolution with
zero padding ("same" size, stride 1) is

    Y[v, o] = sum_{t in taps} sum_i W[t, o, i] X[v + t, i]

with taps t = (dz, dy, dx) in {-1, 0, 1}^3 enumerated as t = (dz+1)*9 + (dy+1)*3 + (dx+1).
Operands are rounded to bfloat16 (round to nearest, ties to even) exactly as the
GPU kernels do and the sums are taken in float64, so the GPU's FP32 accumulation
is the only difference.
"""
from __future__ import annotations

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def bf16_round(a) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64.

    The value is first rounded to float32 (the GPU keeps float32 master copies),
    then the low 16 bits of the float32 pattern are rounded away."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) >> 16 << 16
    return (u.astype(np.uint32)).view(np.float32).astype(np.float64)


def _shift(X: np.ndarray, t) -> np.ndarray:
    """Z[v] = X[v + t] with zeros outside (X: D, H, W, C)."""
    D, H, W = X.shape[:3]
    Z = np.zeros_like(X)
    dz, dy, dx = t
    zs = slice(max(0, -dz), min(D, D - dz))
    ys = slice(max(0, -dy), min(H, H - dy))
    xs = slice(max(0, -dx), min(W, W - dx))
    zs2 = slice(zs.start + dz, zs.stop + dz)
    ys2 = slice(ys.start + dy, ys.stop + dy)
    xs2 = slice(xs.start + dx, xs.stop + dx)
    Z[zs, ys, xs] = X[zs2, ys2, xs2]
    return Z


def conv3d(X: np.ndarray, Wt: np.ndarray, relu: bool = False, round_inputs: bool = True) -> np.ndarray:
    """Forward: X (D,H,W,Ci), Wt (27 or 1, Co, Ci) -> (D,H,W,Co), FP64 accumulation."""
    Xr = bf16_round(X) if round_inputs else np.asarray(X, np.float64)
    Wr = bf16_round(Wt) if round_inputs else np.asarray(Wt, np.float64)
    taps = TAPS if Wr.shape[0] == 27 else [(0, 0, 0)]
    Y = np.zeros(X.shape[:3] + (Wr.shape[1],))
    for ti, t in enumerate(taps):
        Y += _shift(Xr, t) @ Wr[ti].T
    return np.maximum(Y, 0.0) if relu else Y


def conv3d_dgrad(dY: np.ndarray, Wt: np.ndarray, round_inputs: bool = True) -> np.ndarray:
    """dX[v, i] = sum_t sum_o W[t, o, i] dY[v - t, o]."""
    dYr = bf16_round(dY) if round_inputs else np.asarray(dY, np.float64)
    Wr = bf16_round(Wt) if round_inputs else np.asarray(Wt, np.float64)
    taps = TAPS if Wr.shape[0] == 27 else [(0, 0, 0)]
    dX = np.zeros(dY.shape[:3] + (Wr.shape[2],))
    for ti, t in enumerate(taps):
        dX += _shift(dYr, (-t[0], -t[1], -t[2])) @ Wr[ti]
    return dX


def conv3d_wgrad(X: np.ndarray, dY: np.ndarray, ntaps: int = 27, round_inputs: bool = True) -> np.ndarray:
    """dW[t, o, i] = sum_v dY[v, o] X[v + t, i]."""
    Xr = bf16_round(X) if round_inputs else np.asarray(X, np.float64)
    dYr = bf16_round(dY) if round_inputs else np.asarray(dY, np.float64)
    taps = TAPS if ntaps == 27 else [(0, 0, 0)]
    Co, Ci = dY.shape[3], X.shape[3]
    dW = np.zeros((len(taps), Co, Ci))
    A = dYr.reshape(-1, Co)
    for ti, t in enumerate(taps):
        dW[ti] = A.T @ _shift(Xr, t).reshape(-1, Ci)
    return dW


def avgpool2(X: np.ndarray) -> np.ndarray:
    D, H, W, C = X.shape
    return X.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).mean(axis=(1, 3, 5))


def avgpool2_grad(dY: np.ndarray) -> np.ndarray:
    return np.repeat(np.repeat(np.repeat(dY, 2, 0), 2, 1), 2, 2) / 8.0


def upsample2(X: np.ndarray) -> np.ndarray:
    return np.repeat(np.repeat(np.repeat(X, 2, 0), 2, 1), 2, 2)


def upsample2_grad(dY: np.ndarray) -> np.ndarray:
    D, H, W, C = dY.shape
    return dY.reshape(D // 2, 2, H // 2, 2, W // 2, 2, C).sum(axis=(1, 3, 5))


def adam_step(w, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba): returns (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
