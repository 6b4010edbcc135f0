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


# ---------------------------------------------------------------------------
# The whole network, composed from the layer table of the library's C header
# (4 levels, 3x3x3 convolutions, channels 16/32/48/64, average pooling, nearest
# upsampling, skip concatenations [upsampled, skip], a final 1x1x1 layer).  Every
# stored activation is rounded to bfloat16 where the network stores one; the
# convolution sums are float64.
# ---------------------------------------------------------------------------

# (taps, cin, cout, cin_real) of L0..L14, channel counts padded to multiples of 16
LAYERS = [(27, 16, 16, 14), (27, 16, 16, 16), (27, 16, 32, 16), (27, 32, 32, 32), (27, 32, 48, 32),
          (27, 48, 48, 48), (27, 48, 64, 48), (27, 64, 64, 64), (27, 112, 48, 112), (27, 48, 48, 48),
          (27, 80, 32, 80), (27, 32, 32, 32), (27, 48, 16, 48), (27, 16, 16, 16), (1, 16, 16, 16)]


def split_params(flat: np.ndarray) -> list:
    """The flat FP32 parameter vector as the 15 weight arrays [taps][cout][cin]."""
    out, off = [], 0
    for taps, cin, cout, _ in LAYERS:
        n = taps * cout * cin
        out.append(np.asarray(flat[off:off + n], np.float64).reshape(taps, cout, cin))
        off += n
    assert off == len(flat)
    return out


def pack_input(r: np.ndarray, chi: np.ndarray, bf16: bool = True, w: np.ndarray | None = None):
    """X0 (n1, n2, n3, 16): Re, Im of r_x, r_y, r_z times s, Re, Im of chi, then Re, Im
    of w_x, w_y, w_z times s when a base vector w is given (zeros otherwise), zeros;
    rounded to bfloat16 (bf16 = True); s = sqrt(3N / ||r||^2)."""
    n = r.shape[1:]
    N = int(np.prod(n))
    s = np.sqrt(3.0 * N / np.sum(np.abs(r) ** 2))
    X = np.zeros(n + (16,))
    for c in range(3):
        X[..., 2 * c] = (r[c] * s).real
        X[..., 2 * c + 1] = (r[c] * s).imag
        if w is not None:
            X[..., 8 + 2 * c] = (w[c] * s).real
            X[..., 9 + 2 * c] = (w[c] * s).imag
    X[..., 6] = chi.real
    X[..., 7] = chi.imag
    return (bf16_round(X) if bf16 else X), s


def unet_forward(W: list, X0: np.ndarray, bf16: bool = True) -> dict:
    """All activations of one forward pass; 'out' is the FP64 sum of the last layer.
    bf16 = False: exact FP64 throughout (no rounding of weights or activations)."""
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    conv = lambda X, w: conv3d(X, w, round_inputs=bf16)
    relu = lambda Y: rnd(np.maximum(Y, 0.0))
    a = {"X0": X0}
    a["E1a"] = relu(conv(X0, W[0]))
    a["E1b"] = relu(conv(a["E1a"], W[1]))
    a["P1"] = rnd(avgpool2(a["E1b"]))
    a["E2a"] = relu(conv(a["P1"], W[2]))
    a["E2b"] = relu(conv(a["E2a"], W[3]))
    a["P2"] = rnd(avgpool2(a["E2b"]))
    a["E3a"] = relu(conv(a["P2"], W[4]))
    a["E3b"] = relu(conv(a["E3a"], W[5]))
    a["P3"] = rnd(avgpool2(a["E3b"]))
    a["E4a"] = relu(conv(a["P3"], W[6]))
    a["E4b"] = relu(conv(a["E4a"], W[7]))
    a["C3"] = np.concatenate([upsample2(a["E4b"]), a["E3b"]], axis=3)
    a["D3a"] = relu(conv(a["C3"], W[8]))
    a["D3b"] = relu(conv(a["D3a"], W[9]))
    a["C2"] = np.concatenate([upsample2(a["D3b"]), a["E2b"]], axis=3)
    a["D2a"] = relu(conv(a["C2"], W[10]))
    a["D2b"] = relu(conv(a["D2a"], W[11]))
    a["C1"] = np.concatenate([upsample2(a["D2b"]), a["E1b"]], axis=3)
    a["D1a"] = relu(conv(a["C1"], W[12]))
    a["D1b"] = relu(conv(a["D1a"], W[13]))
    a["out"] = conv(a["D1b"], W[14])
    return a


def unpack_output(r: np.ndarray, out: np.ndarray, s: float) -> np.ndarray:
    """z_c = r_c + (out[2c] + i out[2c+1]) / s."""
    z = np.array(r, dtype=np.complex128)
    for c in range(3):
        z[c] += (out[..., 2 * c] + 1j * out[..., 2 * c + 1]) / s
    return z


def unet_apply(W: list, r: np.ndarray, chi: np.ndarray, bf16: bool = True, w: np.ndarray | None = None) -> np.ndarray:
    """The preconditioner's action: the network's correction added to the base vector
    (w when given, else r)."""
    X0, s = pack_input(r, chi, bf16, w)
    return unpack_output(r if w is None else w, unet_forward(W, X0, bf16)["out"], s)


def unet_loss_grads(W: list, samples, bf16: bool = True) -> tuple:
    """Mean squared error of out[0:6] against (target - base) s over the six channels and
    all voxels, averaged over the samples (r, chi, target[, base]; base = r when
    absent), and its gradient with
    respect to every layer's weights: backpropagation through the composition of
    unet_forward (chain rule layer by layer: weight gradient, input gradient masked
    by the ReLU of the layer's input, adjoints of upsampling and pooling, the skip
    and pooling paths of a level added).  With bf16 = True every stored gradient is
    rounded to bfloat16 where the network stores one."""
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    grads = [np.zeros_like(w) for w in W]
    total = 0.0
    count = len(samples)
    for smp in samples:
        r, chi, target = smp[:3]
        base = smp[3] if len(smp) > 3 else None
        X0, s = pack_input(r, chi, bf16, base)
        a = unet_forward(W, X0, bf16)
        n = r.shape[1:]
        V = int(np.prod(n))
        ref = r if base is None else base
        want = np.zeros(n + (16,))
        for c in range(3):
            d = (target[c] - ref[c]) * s
            want[..., 2 * c] = d.real
            want[..., 2 * c + 1] = d.imag
        diff = np.zeros(n + (16,))
        diff[..., :6] = a["out"][..., :6] - want[..., :6]
        total += np.sum(diff[..., :6] ** 2) / (6.0 * V)
        g = rnd(diff * (2.0 / (6.0 * V * count)))

        def back(i, X, dY, mask=None):
            grads[i] += conv3d_wgrad(X, dY, ntaps=W[i].shape[0], round_inputs=bf16)
            dX = conv3d_dgrad(dY, W[i], round_inputs=bf16)
            if mask is not None:
                dX = np.where(mask > 0, dX, 0.0)
            return dX

        gD1b = rnd(back(14, a["D1b"], g, a["D1b"]))
        gD1a = rnd(back(13, a["D1a"], gD1b, a["D1a"]))
        gC1 = rnd(back(12, a["C1"], gD1a, a["C1"]))
        gD2b = rnd(upsample2_grad(gC1[..., :32]))
        gD2a = rnd(back(11, a["D2a"], gD2b, a["D2a"]))
        gC2 = rnd(back(10, a["C2"], gD2a, a["C2"]))
        gD3b = rnd(upsample2_grad(gC2[..., :48]))
        gD3a = rnd(back(9, a["D3a"], gD3b, a["D3a"]))
        gC3 = rnd(back(8, a["C3"], gD3a, a["C3"]))
        gE4b = rnd(upsample2_grad(gC3[..., :64]))
        gE4a = rnd(back(7, a["E4a"], gE4b, a["E4a"]))
        gP3 = rnd(back(6, a["P3"], gE4a))
        gE3b = rnd(gC3[..., 64:] + np.where(a["E3b"] > 0, avgpool2_grad(gP3), 0.0))
        gE3a = rnd(back(5, a["E3a"], gE3b, a["E3a"]))
        gP2 = rnd(back(4, a["P2"], gE3a))
        gE2b = rnd(gC2[..., 48:] + np.where(a["E2b"] > 0, avgpool2_grad(gP2), 0.0))
        gE2a = rnd(back(3, a["E2a"], gE2b, a["E2a"]))
        gP1 = rnd(back(2, a["P1"], gE2a))
        gE1b = rnd(gC1[..., 32:] + np.where(a["E1b"] > 0, avgpool2_grad(gP1), 0.0))
        gE1a = rnd(back(1, a["E1a"], gE1b, a["E1a"]))
        back(0, X0, gE1a)
    return total / count, grads


def unet_loss(W: list, samples, bf16: bool = True) -> float:
    """The loss of unet_loss_grads alone (forward passes only)."""
    total = 0.0
    for smp in samples:
        r, chi, target = smp[:3]
        base = smp[3] if len(smp) > 3 else None
        X0, s = pack_input(r, chi, bf16, base)
        out = unet_forward(W, X0, bf16)["out"]
        V = int(np.prod(r.shape[1:]))
        ref = r if base is None else base
        for c in range(3):
            d = (target[c] - ref[c]) * s
            total += (np.sum((out[..., 2 * c] - d.real) ** 2) + np.sum((out[..., 2 * c + 1] - d.imag) ** 2)) / (6.0 * V)
    return total / len(samples)
