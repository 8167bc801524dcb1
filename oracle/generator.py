"""Plain float64 CPU oracle of the learned factor/map generator — TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this
module; it shares no code with the HIP library.

The network follows the paper's pipeline (Sec. "Preliminary": context from a resized
image, Eq. backbone; supplementary Table backbone: bilinear downsample to 256x256, then
stride-2 3x3 convolutions; Table gen_lut: a fully connected head emitting the U, S, V
components of nine 2D LUTs), sized as a small CNN:

    downsample to 256x256 (bilinear, half-pixel centres, no antialias)
    5 x [conv3x3 stride 2 pad 1 + ReLU]: 3 -> 16 -> 32 -> 64 -> 128 -> 128
    global average pool -> FC 128 -> 9 * (D*R + R + D*R)        (factors, linear)
    conv3x3 stride 1 pad 1, 64 -> 9, on the 32x32 third-layer features (spatial map, linear)

Layouts (shared interface with the library, stated here in full): activations NHWC;
conv weights [Cout][3][3][Cin]; FC weight [out][in]; FC output per LUT l (l = 3c + p) is
the block [U (D x R, row-major) | s (R) | V (D x R)].

Precision mirror (``mixed=True``): convolution operands (activations, weights and, in the
backward, the output gradients) are rounded to bfloat16 (round to nearest even) and
products are accumulated in float64, standing in for bf16 matrix-core products with fp32
accumulation; post-ReLU activations are stored rounded to bf16; bias adds, the map head's
output, pooling, the FC layer and all bias gradients stay in full precision.  With
``mixed=False`` everything is float64 (used for finite-difference pins).
"""
from __future__ import annotations

import numpy as np

CONV_CH = (3, 16, 32, 64, 128, 128)
HEAD_IN = 64          # the map head reads the third conv layer's output
N_MAP = 9
GAP_DIM = 128
NET_IN = 256


def bf16_round(a):
    """Round float values to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    rounded = (bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000
    return rounded.astype(np.uint32).view(np.float32).astype(np.float64)


def param_shapes(D: int = 33, R: int = 8):
    """Ordered (name, shape) list of the flat parameter vector."""
    out = []
    for i in range(5):
        out.append((f"conv{i + 1}.w", (CONV_CH[i + 1], 3, 3, CONV_CH[i])))
        out.append((f"conv{i + 1}.b", (CONV_CH[i + 1],)))
    out.append(("head.w", (N_MAP, 3, 3, HEAD_IN)))
    out.append(("head.b", (N_MAP,)))
    n_fc = 9 * (2 * D * R + R)
    out.append(("fc.w", (n_fc, GAP_DIM)))
    out.append(("fc.b", (n_fc,)))
    return out


def unflatten(theta, D=33, R=8):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for name, shp in param_shapes(D, R):
        n = int(np.prod(shp))
        out[name] = theta[o:o + n].reshape(shp)
        o += n
    assert o == theta.size, (o, theta.size)
    return out


def flatten(d, D=33, R=8):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in param_shapes(D, R)])


# ---------------------------------------------------------------- downsample
def _src_axis(n_out: int, n_in: int):
    """Half-pixel source coordinate: src = max((dst + 0.5) * n_in / n_out - 0.5, 0)."""
    dst = np.arange(n_out, dtype=np.float64)
    src = np.maximum((dst + 0.5) * (n_in / n_out) - 0.5, 0.0)
    i0 = np.floor(src).astype(np.int64)
    i0 = np.minimum(i0, n_in - 1)
    i1 = np.minimum(i0 + 1, n_in - 1)
    return i0, i1, src - i0


def downsample(x, out_h: int = NET_IN, out_w: int = NET_IN):
    """Bilinear resize of planar [B][3][H][W] to NHWC [B][out_h][out_w][3] (supp. Table backbone)."""
    x = np.asarray(x, dtype=np.float64)
    y0, y1, ly = _src_axis(out_h, x.shape[2])
    x0, x1, lx = _src_axis(out_w, x.shape[3])
    ly = ly[:, None]
    lx = lx[None, :]
    top = x[:, :, y0][:, :, :, x0] * (1 - lx) + x[:, :, y0][:, :, :, x1] * lx
    bot = x[:, :, y1][:, :, :, x0] * (1 - lx) + x[:, :, y1][:, :, :, x1] * lx
    out = top * (1 - ly) + bot * ly
    return np.transpose(out, (0, 2, 3, 1))


# ---------------------------------------------------------------- convolution
def _pad(a, p):
    return np.pad(a, ((0, 0), (p, p), (p, p), (0, 0)))


def conv2d(a, w, b, stride: int):
    """3x3 convolution, zero padding 1, NHWC input a, weight [Cout][3][3][Cin] -> NHWC."""
    a = np.asarray(a, np.float64)
    w = np.asarray(w, np.float64)
    N, H, W, _ = a.shape
    Ho, Wo = (H - 1) // stride + 1, (W - 1) // stride + 1
    ap = _pad(a, 1)
    out = np.zeros((N, Ho, Wo, w.shape[0]))
    for ky in range(3):
        for kx in range(3):
            patch = ap[:, ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride, :]
            out += patch @ w[:, ky, kx, :].T
    return out + np.asarray(b, np.float64)


def conv2d_dgrad(dz, w, in_shape, stride: int):
    """Gradient of conv2d's input: scatter each output gradient back through its 3x3 taps."""
    dz = np.asarray(dz, np.float64)
    w = np.asarray(w, np.float64)
    N, H, W, Cin = in_shape
    Ho, Wo = dz.shape[1], dz.shape[2]
    dap = np.zeros((N, H + 2, W + 2, Cin))
    for ky in range(3):
        for kx in range(3):
            dap[:, ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride, :] += dz @ w[:, ky, kx, :]
    return dap[:, 1:H + 1, 1:W + 1, :]


def conv2d_wgrad(dz, a, stride: int):
    """Gradient of conv2d's weight [Cout][3][3][Cin]."""
    dz = np.asarray(dz, np.float64)
    a = np.asarray(a, np.float64)
    Ho, Wo = dz.shape[1], dz.shape[2]
    ap = _pad(a, 1)
    dw = np.zeros((dz.shape[3], 3, 3, a.shape[3]))
    dzf = dz.reshape(-1, dz.shape[3])
    for ky in range(3):
        for kx in range(3):
            patch = ap[:, ky:ky + stride * (Ho - 1) + 1:stride, kx:kx + stride * (Wo - 1) + 1:stride, :]
            dw[:, ky, kx, :] = dzf.T @ patch.reshape(-1, a.shape[3])
    return dw


# ---------------------------------------------------------------- network
def forward(params, x_full, D=33, R=8, mixed=True):
    """Generator forward.  Returns (U, s, V, map [B][9][32][32], cache for backward)."""
    q = bf16_round if mixed else (lambda v: np.asarray(v, np.float64))
    P = params
    a = q(downsample(x_full))
    acts = [a]
    a3 = None
    for i in range(5):
        z = conv2d(a, q(P[f"conv{i + 1}.w"]), P[f"conv{i + 1}.b"], 2)
        a = q(np.maximum(z, 0.0))
        acts.append(a)
        if i == 2:
            a3 = a
    smap = conv2d(a3, q(P["head.w"]), P["head.b"], 1)              # [B][32][32][9]
    g = acts[5].mean(axis=(1, 2))                                   # [B][128]
    o = g @ np.asarray(P["fc.w"], np.float64).T + np.asarray(P["fc.b"], np.float64)
    U, s, V = split_fc(o, D, R)
    cache = {"acts": acts, "g": g}
    return U, s, V, np.transpose(smap, (0, 3, 1, 2)), cache


def split_fc(o, D, R):
    B = o.shape[0]
    blk = o.reshape(B, 9, 2 * D * R + R)
    U = blk[:, :, :D * R].reshape(B, 9, D, R)
    s = blk[:, :, D * R:D * R + R]
    V = blk[:, :, D * R + R:].reshape(B, 9, D, R)
    return U, s, V


def join_fc(dU, ds, dV):
    B = dU.shape[0]
    return np.concatenate([np.asarray(dU).reshape(B, 9, -1), np.asarray(ds).reshape(B, 9, -1),
                           np.asarray(dV).reshape(B, 9, -1)], axis=2).reshape(B, -1)


def backward(params, cache, dU, ds, dV, dmap, mixed=True):
    """Gradients of every parameter given dL/dU, dL/ds, dL/dV and dL/dmap ([B][9][32][32])."""
    q = bf16_round if mixed else (lambda v: np.asarray(v, np.float64))
    P = params
    acts, g = cache["acts"], cache["g"]
    grads = {}
    do = join_fc(dU, ds, dV)
    grads["fc.w"] = do.T @ g
    grads["fc.b"] = do.sum(axis=0)
    dg = do @ np.asarray(P["fc.w"], np.float64)
    a5 = acts[5]
    da = np.broadcast_to(dg[:, None, None, :] / (a5.shape[1] * a5.shape[2]), a5.shape)
    dmap_nhwc = np.transpose(np.asarray(dmap, np.float64), (0, 2, 3, 1))
    for i in range(4, -1, -1):
        a_out = acts[i + 1]
        dz = np.where(a_out > 0, da, 0.0)
        a_in = acts[i]
        grads[f"conv{i + 1}.w"] = conv2d_wgrad(q(dz), a_in, 2)
        grads[f"conv{i + 1}.b"] = dz.sum(axis=(0, 1, 2))
        if i == 0:
            break
        da = conv2d_dgrad(q(dz), q(P[f"conv{i + 1}.w"]), a_in.shape, 2)
        if i == 3:          # a_in is the third layer's output: add the map head's gradient
            grads["head.w"] = conv2d_wgrad(q(dmap_nhwc), a_in, 1)
            grads["head.b"] = dmap_nhwc.sum(axis=(0, 1, 2))
            da = da + conv2d_dgrad(q(dmap_nhwc), q(P["head.w"]), a_in.shape, 1)
    return grads


# ---------------------------------------------------------------- optimiser
def adam(theta, grad, m, v, t, lr=1e-4, b1=0.9, b2=0.999, eps=1e-8):
    """One step of standard Adam (Kingma & Ba), t counted from 1; returns new (theta, m, v)."""
    theta = np.asarray(theta, np.float64)
    g = np.asarray(grad, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
