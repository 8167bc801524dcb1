"""Plain float64 CPU oracle of 2D bilateral-grid slicing — TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this
module; it shares no code with the HIP library.  It follows the supplementary material of
arXiv 2508.16121: Sec. "2D Slicing" (Eqs. query_grid, lookup_grid, adjacent_grid,
bilinear_grid and the weighted sum of the three planes) and Sec. "Slicing and LUT
Transform" (Eq. slicing_transform), with the decomposition of a 3D bilateral grid into
three 2D planes of the main paper (Eq. Griddecompose).

Readings where the paper is silent (also listed in the design notes):
  * K grids; grid k queries colour channel c = k mod 3 and adds to output channel c
    (K = 6: two grids per channel);
  * every grid has three planes in the order (xy, xc, yc), each indexed
    [alpha][beta] with (alpha, beta) = (x, y), (x, c), (y, c);
  * the spatial query x' = x/(W-1) is evaluated exactly as x*(Ds-1)/(W-1) (the same
    corner-aligned rule as the spatial map; a size-1 image axis queries 0); the colour
    query is the LUT decode of the clamped channel with Ds vertices (float32 q);
  * Psi^k = w_xy psi_xy + w_xc psi_xc + w_yc psi_yc + b^k;
    Y_c = (LUT transform)_c + sum over k with k mod 3 = c of Psi^k.
"""
from __future__ import annotations

import numpy as np

from .lut import axis_coords, bilinear, decode, transform

PLANES = ("xy", "xc", "yc")


def _spatial(H: int, W: int, Ds: int):
    """Per-pixel grid coordinates along x and y (supp. Eqs. query_grid, lookup_grid)."""
    ix, dx = axis_coords(W, Ds)
    iy, dy = axis_coords(H, Ds)
    IX = np.broadcast_to(ix[None, :], (H, W))
    DX = np.broadcast_to(dx[None, :], (H, W))
    IY = np.broadcast_to(iy[:, None], (H, W))
    DY = np.broadcast_to(dy[:, None], (H, W))
    return IX, DX, IY, DY


def plane_values(x, g):
    """psi for every grid and plane of one image: [K][3][H][W] (supp. Eq. bilinear_grid).

    x [3][H][W]; g [K][3][Ds][Ds] with planes (xy, xc, yc) indexed [alpha][beta].
    """
    x = np.asarray(x)
    g = np.asarray(g, dtype=np.float64)
    K, _, Ds, _ = g.shape
    _, H, W = x.shape
    IX, DX, IY, DY = _spatial(H, W, Ds)
    dec = [decode(x[c], Ds) for c in range(3)]
    psi = np.zeros((K, 3, H, W))
    for k in range(K):
        ic, dc = dec[k % 3]
        psi[k, 0] = bilinear(g[k, 0], IX, DX, IY, DY)
        psi[k, 1] = bilinear(g[k, 1], IX, DX, ic, dc)
        psi[k, 2] = bilinear(g[k, 2], IY, DY, ic, dc)
    return psi


def slice_grids(x, g, gw, gb):
    """Psi^k of one image, [K][H][W] (supp. weighted sum of the three 2D slicings).

    gw [K][3] plane weights (w_xy, w_xc, w_yc), gb [K] biases.
    """
    psi = plane_values(x, g)
    gw = np.asarray(gw, dtype=np.float64)
    gb = np.asarray(gb, dtype=np.float64)
    return np.einsum("kp,kphw->khw", gw, psi) + gb[:, None, None]


def slice_grids_at(x, g, gw, gb, ys, xs):
    """The same Psi^k evaluated only at pixels (ys[n], xs[n]) of an image of size x.shape:
    [K][len(ys)] (for sampled checks of large frames)."""
    x = np.asarray(x)
    g = np.asarray(g, dtype=np.float64)
    gw = np.asarray(gw, dtype=np.float64)
    gb = np.asarray(gb, dtype=np.float64)
    K, _, Ds, _ = g.shape
    _, H, W = x.shape
    ys = np.asarray(ys)
    xs = np.asarray(xs)
    ix_all, dx_all = axis_coords(W, Ds)
    iy_all, dy_all = axis_coords(H, Ds)
    IX, DX, IY, DY = ix_all[xs], dx_all[xs], iy_all[ys], dy_all[ys]
    out = np.zeros((K, ys.size))
    for k in range(K):
        ic, dc = decode(x[k % 3][ys, xs], Ds)
        out[k] = (gw[k, 0] * bilinear(g[k, 0], IX, DX, IY, DY) + gw[k, 1] * bilinear(g[k, 1], IX, DX, ic, dc)
                  + gw[k, 2] * bilinear(g[k, 2], IY, DY, ic, dc) + gb[k])
    return out


def transform_grid(x, T, smap, g, gw, gb, bias=None):
    """Fused slicing and LUT transform of one image (supp. Eq. slicing_transform).

    Y_c = sum_p S_{3c+p} phi_{3c+p} + b_c + sum_{k mod 3 = c} Psi^k, float64 [3][H][W].
    """
    Y = transform(x, T, smap, bias)
    Psi = slice_grids(x, g, gw, gb)
    for k in range(Psi.shape[0]):
        Y[k % 3] += Psi[k]
    return Y


def apply_grid(x, U, s, V, smap, g, gw, gb, bias=None):
    """Batched forward with grids: g [B][K][3][Ds][Ds], gw [B][K][3], gb [B][K]."""
    from .lut import reconstruct
    T = reconstruct(U, s, V)
    return np.stack([transform_grid(x[b], T[b], smap[b], g[b], gw[b], gb[b],
                                    None if bias is None else bias[b]) for b in range(x.shape[0])])


def slice_bwd(x, g, gw, G):
    """Gradients of sum_c sum G_c * (sum_{k mod 3 = c} Psi^k) for one image.

    Returns dict dg [K][3][Ds][Ds], dgw [K][3], dgb [K], dx [3][H][W] (float64):
    dg_plane[a+i][b+j] += G_c w_plane w_alpha(i) w_beta(j);  dgw = sum G_c psi;  dgb = sum G_c;
    dx_c = sum over the grids of channel c of G_c (w_xc dpsi_xc/dp_c + w_yc dpsi_yc/dp_c),
    times 1 where 0 <= x_c <= 1, else 0.
    """
    x = np.asarray(x)
    g = np.asarray(g, dtype=np.float64)
    gw = np.asarray(gw, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    K, _, Ds, _ = g.shape
    _, H, W = x.shape
    IX, DX, IY, DY = _spatial(H, W, Ds)
    dec = [decode(x[c], Ds) for c in range(3)]
    psi = plane_values(x, g)
    dg = np.zeros_like(g)
    dgw = np.zeros((K, 3))
    dgb = np.zeros(K)
    dx = np.zeros((3, H, W))
    for k in range(K):
        c = k % 3
        ic, dc = dec[c]
        Gc = G[c]
        dgb[k] = Gc.sum()
        for pl in range(3):
            dgw[k, pl] = (Gc * psi[k, pl]).sum()
        axes = ((IX, DX, IY, DY), (IX, DX, ic, dc), (IY, DY, ic, dc))
        for pl, (ia, da, ib, db) in enumerate(axes):
            gg = Gc * gw[k, pl]
            for a in (0, 1):
                wa = da if a else 1 - da
                for b in (0, 1):
                    wb = db if b else 1 - db
                    np.add.at(dg[k, pl], (ia + a, ib + b), gg * wa * wb)
        for pl, (ia, da) in ((1, (IX, DX)), (2, (IY, DY))):
            t = g[k, pl]
            dpsi_dc = (Ds - 1) * ((1 - da) * (t[ia, ic + 1] - t[ia, ic]) + da * (t[ia + 1, ic + 1] - t[ia + 1, ic]))
            dx[c] += Gc * gw[k, pl] * dpsi_dc
    xf = np.asarray(x, dtype=np.float64)
    dx = np.where((xf >= 0.0) & (xf <= 1.0), dx, 0.0)
    return {"dg": dg, "dgw": dgw, "dgb": dgb, "dx": dx}
