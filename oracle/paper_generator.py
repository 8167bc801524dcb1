"""Plain float64 CPU oracle of the paper's own generator network — TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this
module; it shares no code with the HIP library.  It follows the supplementary Sec.
"Details of Network Structure": Table backbone (bilinear downsample to 256x256, five 3x3
stride-2 convolution blocks with m = 8, LeakyReLU and instance normalisation, dropout 0.5,
average pooling to 2x2, reshape to 32m = 256 features), Tables gen_lut / gen_lut_weight /
gen_bilateral / gen_bilateral_weight (two fully connected layers per generator with a hidden
width of 8), and the main paper's Sec. "Preliminary" (context from the downsampled image).

Readings where the tables are silent (also listed in the design notes):
  * block = conv3x3 (stride 2, zero padding 1, with bias) -> LeakyReLU (negative slope 0.2)
    -> instance normalisation (per image and channel over H x W, biased variance, eps 1e-5,
    learned scale and shift); the fifth block has no normalisation;
  * dropout is a caller-supplied keep mask [B][64][8][8] (NCHW order, values 0 or 1), kept
    values scaled by 2; no mask means evaluation (identity);
  * average pooling over 4x4 windows with stride 4; the 256 features are the pooled map
    flattened in NCHW order (index 4c + 2py + px);
  * each generator is FC(256 -> 8) followed by FC(8 -> n) with no activation in between
    (the rank factorisation the supplement motivates the two layers with);
  * H_t emits [U (9 x D x R) | S (9 x R) | V (9 x D x R)] with LUT index l = 3c + p, p in
    order (rg, rb, gb); H_tw emits, per output channel c, (w_rg, w_rb, w_gb, b^c); H_s emits
    the grids [K][3][Ds][Ds] with planes (xy, xc, yc); H_sw emits, per grid k,
    (w_xy, w_xc, w_yc, b^k).  The tables print an extra factor 3 in the widths of H_tw and
    H_sw; the widths above (12 and 4K) with affine instance normalisation give exactly the
    parameter counts of the component ablation (160,478 for the full model, 109,332 for the
    LUT-only model), which the tables' widths do not;
  * the LUT weights w^c_p of supp. Eq. weighted sum become a 9 x 1 x 1 spatial map
    (map[3c + p]) and b^c the per-channel bias of the fused transform.

Precision mirror (``mixed=True``): convolution operands (activations, weights and, in the
backward, the pre-activation gradients) are rounded to bfloat16 and products accumulated in
float64, standing in for bf16 matrix-core products with fp32 accumulation; the normalised
activations that feed the next convolution are stored rounded to bf16.  Biases, LeakyReLU,
normalisation statistics, pooling, the fully connected layers and every bias, scale and
shift gradient stay in full precision.  ``mixed=False`` is float64 throughout.
"""
from __future__ import annotations

import numpy as np

from .generator import bf16_round, conv2d, conv2d_dgrad, conv2d_wgrad, downsample

CH = (3, 8, 16, 32, 64, 64)    # m = 8: 3 -> m -> 2m -> 4m -> 8m -> 8m
HID = 8                        # hidden width of every generator
FEAT = 256                     # 32m pooled features
SLOPE = 0.2
EPS = 1e-5


def head_sizes(D: int = 33, R: int = 8, K: int = 6, Ds: int = 17):
    """(name, output width) of the generators; K = 0 is the LUT-only model."""
    out = [("t", 9 * (2 * D * R + R)), ("tw", 12)]
    if K:
        out += [("s", K * 3 * Ds * Ds), ("sw", 4 * K)]
    return out


def param_shapes(D: int = 33, R: int = 8, K: int = 6, Ds: int = 17):
    """Ordered (name, shape) list of the flat parameter vector.  Convolution weights are
    [Cout][3][3][Cin]; FC weights [out][in]."""
    out = []
    for i in range(5):
        co, ci = CH[i + 1], CH[i]
        out += [(f"conv{i + 1}.w", (co, 3, 3, ci)), (f"conv{i + 1}.b", (co,))]
        if i < 4:
            out += [(f"in{i + 1}.g", (co,)), (f"in{i + 1}.b", (co,))]
    for h, n in head_sizes(D, R, K, Ds):
        out += [(f"{h}.fc1.w", (HID, FEAT)), (f"{h}.fc1.b", (HID,)), (f"{h}.fc2.w", (n, HID)), (f"{h}.fc2.b", (n,))]
    return out


def param_count(D=33, R=8, K=6, Ds=17) -> int:
    return int(sum(np.prod(s) for _, s in param_shapes(D, R, K, Ds)))


def unflatten(theta, D=33, R=8, K=6, Ds=17):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for name, shp in param_shapes(D, R, K, Ds):
        n = int(np.prod(shp))
        out[name] = theta[o:o + n].reshape(shp)
        o += n
    assert o == theta.size, (o, theta.size)
    return out


def flatten(d, D=33, R=8, K=6, Ds=17):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in param_shapes(D, R, K, Ds)])


def _lrelu(z):
    return np.where(z > 0, z, SLOPE * z)


def _keep(mask, shape_nhwc):
    """Dropout factor in NHWC order: 2 * mask, or 1 without a mask."""
    if mask is None:
        return np.ones(shape_nhwc)
    return 2.0 * np.transpose(np.asarray(mask, np.float64), (0, 2, 3, 1))


def forward(P, x, D=33, R=8, K=6, Ds=17, mask=None, mixed=True):
    """The paper's generator on a batch x [B][3][H][W].

    Returns (out, cache); out holds U, V [B][9][D][R], s [B][9][R], lut_w [B][9] (the
    9 x 1 x 1 map), lut_b [B][3] and, for K > 0, grids [B][K][3][Ds][Ds], gw [B][K][3],
    gb [B][K]."""
    q = bf16_round if mixed else (lambda v: np.asarray(v, np.float64))
    a = q(downsample(x))
    acts, hs, stats = [a], [], []
    for i in range(5):
        z = conv2d(a, q(P[f"conv{i + 1}.w"]), P[f"conv{i + 1}.b"], 2)
        h = _lrelu(z)
        hs.append(h)
        if i < 4:
            mu = h.mean(axis=(1, 2), keepdims=True)
            var = ((h - mu) ** 2).mean(axis=(1, 2), keepdims=True)
            rstd = 1.0 / np.sqrt(var + EPS)
            a = q(P[f"in{i + 1}.g"] * (h - mu) * rstd + P[f"in{i + 1}.b"])
            acts.append(a)
            stats.append((mu, rstd))
    h5 = hs[4]                                            # [B][8][8][64]
    B, Hh, Wh, C = h5.shape
    d = h5 * _keep(mask, h5.shape)
    pooled = d.reshape(B, 2, Hh // 2, 2, Wh // 2, C).mean(axis=(2, 4))     # [B][2][2][C]
    f = np.transpose(pooled, (0, 3, 1, 2)).reshape(B, -1)                # NCHW flatten
    hid, outs = {}, {}
    for h, _ in head_sizes(D, R, K, Ds):
        hid[h] = f @ P[f"{h}.fc1.w"].T + P[f"{h}.fc1.b"]
        outs[h] = hid[h] @ P[f"{h}.fc2.w"].T + P[f"{h}.fc2.b"]
    out = split_outputs(outs, B, D, R, K, Ds)
    cache = {"acts": acts, "hs": hs, "stats": stats, "f": f, "hid": hid}
    return out, cache


def split_outputs(outs, B, D, R, K, Ds):
    o = outs["t"]
    nU = 9 * D * R
    out = {"U": o[:, :nU].reshape(B, 9, D, R), "s": o[:, nU:nU + 9 * R].reshape(B, 9, R),
           "V": o[:, nU + 9 * R:].reshape(B, 9, D, R)}
    tw = outs["tw"].reshape(B, 3, 4)
    out["lut_w"] = tw[:, :, :3].reshape(B, 9)
    out["lut_b"] = tw[:, :, 3]
    if K:
        out["grids"] = outs["s"].reshape(B, K, 3, Ds, Ds)
        sw = outs["sw"].reshape(B, K, 4)
        out["gw"] = sw[:, :, :3]
        out["gb"] = sw[:, :, 3]
    return out


def join_outputs(g, B, K):
    """Inverse of split_outputs for upstream gradients (same keys)."""
    outs = {"t": np.concatenate([np.asarray(g["U"], np.float64).reshape(B, -1),
                                 np.asarray(g["s"], np.float64).reshape(B, -1),
                                 np.asarray(g["V"], np.float64).reshape(B, -1)], axis=1)}
    tw = np.concatenate([np.asarray(g["lut_w"], np.float64).reshape(B, 3, 3),
                         np.asarray(g["lut_b"], np.float64).reshape(B, 3, 1)], axis=2)
    outs["tw"] = tw.reshape(B, 12)
    if K:
        outs["s"] = np.asarray(g["grids"], np.float64).reshape(B, -1)
        sw = np.concatenate([np.asarray(g["gw"], np.float64).reshape(B, K, 3),
                             np.asarray(g["gb"], np.float64).reshape(B, K, 1)], axis=2)
        outs["sw"] = sw.reshape(B, 4 * K)
    return outs


def backward(P, cache, dout, D=33, R=8, K=6, Ds=17, mask=None, mixed=True, abs_sums=None):
    """Gradients of every parameter given the upstream gradients dout (keys of forward's out).

    When abs_sums is a dict it receives, for each convolution bias, the per-channel sum of
    |dz| over the terms that make up that bias's gradient (the scale against which a
    rounding-level result is judged); the gradients themselves do not depend on it."""
    q = bf16_round if mixed else (lambda v: np.asarray(v, np.float64))
    acts, hs, stats, f, hid = cache["acts"], cache["hs"], cache["stats"], cache["f"], cache["hid"]
    B = f.shape[0]
    douts = join_outputs(dout, B, K)
    G = {}
    df = np.zeros_like(f)
    for h, _ in head_sizes(D, R, K, Ds):
        do = douts[h]
        G[f"{h}.fc2.w"] = do.T @ hid[h]
        G[f"{h}.fc2.b"] = do.sum(axis=0)
        dh = do @ P[f"{h}.fc2.w"]
        G[f"{h}.fc1.w"] = dh.T @ f
        G[f"{h}.fc1.b"] = dh.sum(axis=0)
        df += dh @ P[f"{h}.fc1.w"]
    h5 = hs[4]
    _, Hh, Wh, C = h5.shape
    dpool = np.transpose(df.reshape(B, C, 2, 2), (0, 2, 3, 1))                    # [B][2][2][C]
    dd = np.repeat(np.repeat(dpool, Hh // 2, axis=1), Wh // 2, axis=2) / ((Hh // 2) * (Wh // 2))
    dz = dd * _keep(mask, h5.shape) * np.where(h5 > 0, 1.0, SLOPE)
    for i in range(4, -1, -1):
        a_in = acts[i]
        dzq = q(dz)
        G[f"conv{i + 1}.w"] = conv2d_wgrad(dzq, a_in, 2)
        G[f"conv{i + 1}.b"] = dz.sum(axis=(0, 1, 2))
        if abs_sums is not None:
            abs_sums[f"conv{i + 1}.b"] = np.abs(dz).sum(axis=(0, 1, 2))
        if i == 0:
            break
        da = conv2d_dgrad(dzq, q(P[f"conv{i + 1}.w"]), a_in.shape, 2)
        h = hs[i - 1]
        mu, rstd = stats[i - 1]
        xh = (h - mu) * rstd
        G[f"in{i}.g"] = (da * xh).sum(axis=(0, 1, 2))
        G[f"in{i}.b"] = da.sum(axis=(0, 1, 2))
        dxh = da * P[f"in{i}.g"]
        dh = rstd * (dxh - dxh.mean(axis=(1, 2), keepdims=True) - xh * (dxh * xh).mean(axis=(1, 2), keepdims=True))
        dz = dh * np.where(h > 0, 1.0, SLOPE)
    return G
