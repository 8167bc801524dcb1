"""Plain float64 CPU oracle of the 2D-LUT hot path — TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this
module.  It shares no code with the HIP library and imports nothing from it.  Every
function is the plain definition of what the method computes, written from the paper
(Kim, Lee & Cho, "Lightweight and Fast Real-time Image Enhancement via Decomposition of
the Spatial-aware Lookup Tables", arXiv 2508.16121); the section or equation it follows
is named in each docstring.

Notation.  Colour channels a in {0: r, 1: g, 2: b}.  Colour pairs p in {0: rg, 1: rb,
2: gb} with (alpha_p, beta_p) = (0, 1), (0, 2), (1, 2).  The nine LUTs (and the nine
spatial-map channels) are indexed l = 3*c + p for output channel c.  D is the number of
vertices per LUT axis and R the rank of the factorisation.

Readings where the paper is silent or garbled (each also listed in the design notes):
  * a LUT is indexed T[alpha][beta]: row = first channel of the pair, column = second;
    T = U diag(s) V^T with U along alpha;
  * inputs are clamped to [0, 1] with fmin/fmax semantics (NaN -> 0); the cell index is
    taken from q = p*(D-1) rounded to float32, then clamped to D-2 so p = 1 lands in the
    last cell with delta = 1;
  * the spatial map is upsampled corner-aligned (x' = x/(W-1), the rule of the paper's
    2D slicing query), a size-1 axis is constant;
  * Y_c = sum_p S_{3c+p} * phi_{3c+p} + b_c, no output clamp; the paper's scalar weights
    are the constant-map special case (its repeated w_rb term is read as w_gb).
"""
from __future__ import annotations

import numpy as np

PAIRS = ((0, 1), (0, 2), (1, 2))   # (alpha, beta) for p = rg, rb, gb


def lut_id(c: int, p: int) -> int:
    return 3 * c + p


# ---------------------------------------------------------------- O1 reconstruction
def reconstruct(U, s, V):
    """T = U . diag(s) . V^T for every LUT (Sec. "Singular Value Decomposition", Eq. gen_LUT_SVD).

    U, V: [..., D, R]; s: [..., R]  ->  T: [..., D, D] in float64.  No orthogonality, sign
    or ordering constraint is placed on the factors.
    """
    U = np.asarray(U, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    return np.matmul(U * s[..., None, :], np.swapaxes(V, -1, -2))


# ---------------------------------------------------------------- O2 decode
def clamp01_f32(x):
    """p = min(max(x, 0), 1) in float32 with fmin/fmax semantics (NaN -> 0)."""
    x = np.asarray(x, dtype=np.float32)
    return np.fmin(np.fmax(x, np.float32(0.0)), np.float32(1.0))


def decode(x, D: int):
    """Left vertex and fractional offset on one LUT axis (supplementary Eq. lookup).

    p^l = floor(p (D-1)) / (D-1) and delta = (p - p^l) / (p^r - p^l) = q - floor(q) with
    q = p (D-1).  q is rounded to float32; the cell index is clamped to D-2 so that p = 1
    uses the last cell with delta = 1.  Returns (i int64, delta float64).
    """
    p = clamp01_f32(x)
    q = (p * np.float32(D - 1)).astype(np.float32)
    i = np.minimum(np.floor(q), D - 2).astype(np.int64)
    i = np.maximum(i, 0)
    delta = q.astype(np.float64) - i
    return i, delta


# ---------------------------------------------------------------- O3 bilinear lookup
def bilinear(T, ia, da, ib, db):
    """phi = bilinear interpolation of 2D LUT T at (p_alpha, p_beta) (supp. Eqs. adjacent, bilinear).

    V00 = T[ia][ib], V10 = T[ia+1][ib], V01 = T[ia][ib+1], V11 = T[ia+1][ib+1].
    """
    T = np.asarray(T, dtype=np.float64)
    return ((1 - da) * (1 - db) * T[ia, ib] + da * (1 - db) * T[ia + 1, ib]
            + (1 - da) * db * T[ia, ib + 1] + da * db * T[ia + 1, ib + 1])


# ---------------------------------------------------------------- O4 map upsample
def axis_coords(n_out: int, n_in: int):
    """Corner-aligned source index and weight for each of n_out positions on an n_in axis.

    u = (x / (n_out - 1)) * (n_in - 1), the 2D-slicing query rule x' = x/(W-1) of the
    supplementary Eq. query_grid applied to a spatial grid of n_in vertices; computed as
    x*(n_in-1)/(n_out-1) so that exact knots stay exact.  A size-1 input axis is constant.
    """
    xs = np.arange(n_out, dtype=np.float64)
    if n_in == 1:
        return np.zeros(n_out, np.int64), np.zeros(n_out)
    u = xs * (n_in - 1) / (n_out - 1) if n_out > 1 else np.zeros(n_out)
    i = np.minimum(np.floor(u), n_in - 2).astype(np.int64)
    return i, u - i


def upsample(smap, H: int, W: int):
    """Corner-aligned bilinear upsample of a [C][h][w] map to [C][H][W] (float64)."""
    m = np.asarray(smap, dtype=np.float64)
    C, h, w = m.shape
    iv, dv = axis_coords(H, h)
    iu, du = axis_coords(W, w)
    iv1 = np.minimum(iv + 1, h - 1)
    iu1 = np.minimum(iu + 1, w - 1)
    dv = dv[:, None]
    du = du[None, :]
    r0 = m[:, iv][:, :, iu] * (1 - du) + m[:, iv][:, :, iu1] * du
    r1 = m[:, iv1][:, :, iu] * (1 - du) + m[:, iv1][:, :, iu1] * du
    return r0 * (1 - dv) + r1 * dv


# ---------------------------------------------------------------- O5 fusion
def transform(x, T, smap, bias=None):
    """Spatially weighted 2D-LUT transform of one image.

    x [3][H][W] (values used as given: float32 or the decoded float16), T [9][D][D],
    smap [9][h][w], bias [3] or None.  Y_c = sum_p S_{3c+p} * phi_{3c+p} + b_c with phi the
    bilinear lookup (supp. Eq. bilinear) and S the upsampled map; with a constant map this
    is the paper's weighted sum (Eq. LUTdecompose_out, supp. Eq. weighte_sum).
    Returns float64 [3][H][W].
    """
    x = np.asarray(x)
    T = np.asarray(T, dtype=np.float64)
    _, H, W = x.shape
    D = T.shape[-1]
    dec = [decode(x[a], D) for a in range(3)]
    S = upsample(smap, H, W)
    Y = np.zeros((3, H, W))
    for c in range(3):
        for p, (al, be) in enumerate(PAIRS):
            l = lut_id(c, p)
            (ia, da), (ib, db) = dec[al], dec[be]
            Y[c] += S[l] * bilinear(T[l], ia, da, ib, db)
        if bias is not None:
            Y[c] += float(bias[c])
    return Y


def transform_at(x, T, smap, ys, xs, bias=None):
    """The same transform evaluated only at pixels (ys[k], xs[k]) of an image of size x.shape.

    Uses the image's full-size coordinates for the map upsample, so the values equal the
    corresponding entries of transform(); for sampled checks of large images.
    Returns float64 [3][len(ys)].
    """
    x = np.asarray(x)
    T = np.asarray(T, dtype=np.float64)
    m = np.asarray(smap, dtype=np.float64)
    _, H, W = x.shape
    D = T.shape[-1]
    C, h, w = m.shape
    ys = np.asarray(ys, np.int64)
    xs = np.asarray(xs, np.int64)
    ivs, dvs = axis_coords(H, h)
    ius, dus = axis_coords(W, w)
    iv, dv = ivs[ys], dvs[ys]
    iu, du = ius[xs], dus[xs]
    iv1 = np.minimum(iv + 1, h - 1)
    iu1 = np.minimum(iu + 1, w - 1)
    S = ((1 - dv) * ((1 - du) * m[:, iv, iu] + du * m[:, iv, iu1])
         + dv * ((1 - du) * m[:, iv1, iu] + du * m[:, iv1, iu1]))
    px = x[:, ys, xs]
    dec = [decode(px[a], D) for a in range(3)]
    Y = np.zeros((3, ys.size))
    for c in range(3):
        for p, (al, be) in enumerate(PAIRS):
            l = lut_id(c, p)
            (ia, da), (ib, db) = dec[al], dec[be]
            Y[c] += S[l] * bilinear(T[l], ia, da, ib, db)
        if bias is not None:
            Y[c] += float(bias[c])
    return Y


def apply(x, U, s, V, smap, bias=None):
    """Batched forward: x [B][3][H][W], U/V [B][9][D][R], s [B][9][R], smap [B][9][h][w]."""
    T = reconstruct(U, s, V)
    B = x.shape[0]
    return np.stack([transform(x[b], T[b], smap[b], None if bias is None else bias[b])
                     for b in range(B)])


def phi_all(x, T):
    """The nine lookups phi_l for one image, [9][H][W] float64 (supp. Eq. bilinear)."""
    D = T.shape[-1]
    dec = [decode(x[a], D) for a in range(3)]
    out = np.zeros((9,) + x.shape[1:])
    for c in range(3):
        for p, (al, be) in enumerate(PAIRS):
            (ia, da), (ib, db) = dec[al], dec[be]
            out[lut_id(c, p)] = bilinear(T[lut_id(c, p)], ia, da, ib, db)
    return out


# ---------------------------------------------------------------- O6 trilinear 3D LUT
def trilinear(x, T3):
    """Trilinear interpolation of a 3D LUT T3[i_r][i_g][i_b] at the pixel colours (Eq. coloren).

    x [3][H][W]; the same per-axis decode as the 2D lookups.  Returns float64 [H][W].
    """
    T3 = np.asarray(T3, dtype=np.float64)
    D = T3.shape[0]
    (ir, dr), (ig, dg), (ib, db) = (decode(x[a], D) for a in range(3))
    out = 0.0
    for a in (0, 1):
        wr = dr if a else 1 - dr
        for b in (0, 1):
            wg = dg if b else 1 - dg
            for c in (0, 1):
                wb = db if c else 1 - db
                out = out + wr * wg * wb * T3[ir + a, ig + b, ib + c]
    return out


def lut1d(x, T1):
    """Per-channel 1D LUT (the lowest LUT dimension of the paper's LUT-dimension analysis):
    Y_c = linear interpolation of the curve T1[c] (D vertices) at the decoded X_c.

    x [3][H][W], T1 [3][D].  Returns float64 [3][H][W].
    """
    T1 = np.asarray(T1, dtype=np.float64)
    D = T1.shape[1]
    out = np.zeros(np.shape(x), dtype=np.float64)
    for c in range(3):
        i, d = decode(x[c], D)
        out[c] = (1 - d) * T1[c][i] + d * T1[c][i + 1]
    return out


# ---------------------------------------------------------------- O7 backward
def transform_bwd(x, T, smap, G):
    """Gradients of sum(G * Y) for one image by the chain rule of the forward above.

    Returns dict with dT [9][D][D], dmap [9][h][w], dx [3][H][W], db [3] (float64).
    dT_l[ia+a][ib+b] += G_c S_l w_alpha(a) w_beta(b);  dmap_l[iv+a][iu+b] += G_c phi_l wv(a) wu(b);
    dx_a = sum_{l: a in pair(l)} G_c S_l dphi_l/dp_a, times 1 where 0 <= x_a <= 1, else 0.
    """
    x = np.asarray(x)
    T = np.asarray(T, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    m = np.asarray(smap, dtype=np.float64)
    _, H, W = x.shape
    D = T.shape[-1]
    C, h, w = m.shape
    dec = [decode(x[a], D) for a in range(3)]
    S = upsample(m, H, W)
    dT = np.zeros_like(T)
    dmap = np.zeros_like(m)
    dx = np.zeros((3, H, W))
    iv, dv = axis_coords(H, h)
    iu, du = axis_coords(W, w)
    IV = np.broadcast_to(iv[:, None], (H, W))
    IU = np.broadcast_to(iu[None, :], (H, W))
    DV = np.broadcast_to(dv[:, None], (H, W))
    DU = np.broadcast_to(du[None, :], (H, W))
    for c in range(3):
        for p, (al, be) in enumerate(PAIRS):
            l = lut_id(c, p)
            (ia, da), (ib, db) = dec[al], dec[be]
            g = G[c] * S[l]
            for a in (0, 1):
                wa = da if a else 1 - da
                for b in (0, 1):
                    wb = db if b else 1 - db
                    np.add.at(dT[l], (ia + a, ib + b), g * wa * wb)
            t = T[l]
            dphi_da = (D - 1) * ((1 - db) * (t[ia + 1, ib] - t[ia, ib]) + db * (t[ia + 1, ib + 1] - t[ia, ib + 1]))
            dphi_db = (D - 1) * ((1 - da) * (t[ia, ib + 1] - t[ia, ib]) + da * (t[ia + 1, ib + 1] - t[ia + 1, ib]))
            dx[al] += g * dphi_da
            dx[be] += g * dphi_db
            phi = bilinear(t, ia, da, ib, db)
            gp = G[c] * phi
            for a in (0, 1):
                if a and h == 1:
                    continue
                wv = DV if a else 1 - DV
                for b in (0, 1):
                    if b and w == 1:
                        continue
                    wu = DU if b else 1 - DU
                    np.add.at(dmap[l], (IV + a, IU + b), gp * wv * wu)
    xf = np.asarray(x, dtype=np.float64)
    inside = (xf >= 0.0) & (xf <= 1.0)      # NaN compares False -> zero gradient
    dx = np.where(inside, dx, 0.0)
    db_ = G.reshape(3, -1).sum(axis=1)
    return {"dT": dT, "dmap": dmap, "dx": dx, "db": db_}


def factor_grads(dT, U, s, V):
    """Gradients of the factors from dL/dT by the chain rule of T = U diag(s) V^T.

    dU = dT V diag(s);  dV = dT^T U diag(s);  ds_k = sum_ij dT_ij U_ik V_jk.
    """
    dT = np.asarray(dT, dtype=np.float64)
    U = np.asarray(U, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    dU = np.matmul(dT, V) * s[..., None, :]
    dV = np.matmul(np.swapaxes(dT, -1, -2), U) * s[..., None, :]
    ds = np.einsum("...ij,...ik,...jk->...k", dT, U, V)
    return dU, ds, dV


def apply_bwd(x, U, s, V, smap, G):
    """Batched backward: returns dU, ds, dV, dmap, dx, db for upstream gradient G [B][3][H][W]."""
    T = reconstruct(U, s, V)
    out = {k: [] for k in ("dT", "dmap", "dx", "db")}
    for b in range(x.shape[0]):
        r = transform_bwd(x[b], T[b], smap[b], G[b])
        for k in out:
            out[k].append(r[k])
    dT = np.stack(out["dT"])
    dU, ds, dV = factor_grads(dT, U, s, V)
    return {"dU": dU, "ds": ds, "dV": dV, "dT": dT, "dmap": np.stack(out["dmap"]),
            "dx": np.stack(out["dx"]), "db": np.stack(out["db"])}


# ---------------------------------------------------------------- losses (C4 / C5)
def l1_loss(Y, Yt):
    """Mean absolute error and its gradient sign(Y - Yt)/N with sign(0) = 0."""
    d = np.asarray(Y, np.float64) - np.asarray(Yt, np.float64)
    n = d.size
    return np.abs(d).mean(), np.sign(d) / n


def mse_loss(Y, Yt):
    """Mean squared error (the fidelity term of the paper's loss, Sec. "Loss Function") and 2(Y-Yt)/N."""
    d = np.asarray(Y, np.float64) - np.asarray(Yt, np.float64)
    n = d.size
    return (d * d).mean(), 2.0 * d / n
