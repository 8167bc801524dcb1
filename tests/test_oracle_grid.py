"""Pins of the bilateral-grid slicing oracle (oracle/grid.py) against the paper's equations
and independent routines: torch interpolate for the spatial plane, SciPy for the colour
planes and for the 3D grid the three planes decompose (Eq. Griddecompose), closed forms,
scalar brute force, adjoint identities and finite differences.  CPU only."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F
from scipy.interpolate import RegularGridInterpolator

import synth
from oracle import grid as og
from oracle import lut as ol


def _case(seed=21, H=9, W=13, K=6, Ds=5):
    g = np.random.default_rng(seed)
    x = g.uniform(-0.05, 1.05, size=(3, H, W)).astype(np.float32)
    gr = g.normal(size=(K, 3, Ds, Ds))
    gw = g.uniform(0.2, 1.0, size=(K, 3))
    gb = g.normal(size=K)
    return x, gr, gw, gb


def _only(gw, plane):
    w = np.zeros_like(gw)
    w[:, plane] = gw[:, plane]
    return w


def test_xy_plane_is_corner_aligned_upsample():
    # the xy plane depends on position only: slicing = align_corners bilinear resize of the
    # plane (indexed [x][y]) to the image size
    x, gr, gw, gb = _case()
    K, _, Ds, _ = gr.shape
    H, W = x.shape[1:]
    Psi = og.slice_grids(x, gr, _only(gw, 0), np.zeros(K))
    for k in range(K):
        plane_yx = torch.from_numpy(np.ascontiguousarray(gr[k, 0].T))[None, None]
        ref = F.interpolate(plane_yx, size=(H, W), mode="bilinear", align_corners=True)[0, 0].numpy()
        np.testing.assert_allclose(Psi[k], gw[k, 0] * ref, atol=1e-12)


@pytest.mark.parametrize("plane", [1, 2])
def test_colour_planes_match_scipy(plane):
    x, gr, gw, gb = _case(seed=22)
    K, _, Ds, _ = gr.shape
    H, W = x.shape[1:]
    Psi = og.slice_grids(x, gr, _only(gw, plane), np.zeros(K))
    knots = np.linspace(0.0, 1.0, Ds)
    ys, xs = np.meshgrid(np.arange(H) / (H - 1), np.arange(W) / (W - 1), indexing="ij")
    for k in range(K):
        c = np.clip(x[k % 3].astype(np.float64), 0.0, 1.0)
        spatial = xs if plane == 1 else ys
        f = RegularGridInterpolator((knots, knots), gr[k, plane], method="linear")
        ref = f(np.stack([spatial.ravel(), c.ravel()], axis=1)).reshape(H, W)
        # the oracle rounds q = p (Ds-1) to float32 as the decode does: tolerance 1e-6
        np.testing.assert_allclose(Psi[k], gw[k, plane] * ref, atol=1e-6)


def test_three_planes_equal_the_3d_grid_they_decompose():
    # Eq. Griddecompose: G3[x][y][c] = w_xy g_xy[x][y] + w_xc g_xc[x][c] + w_yc g_yc[y][c] + b;
    # trilinear slicing of G3 at (x', y', X_c) equals the weighted sum of the 2D slicings
    x, gr, gw, gb = _case(seed=23, H=7, W=11, Ds=4)
    K, _, Ds, _ = gr.shape
    H, W = x.shape[1:]
    Psi = og.slice_grids(x, gr, gw, gb)
    knots = np.linspace(0.0, 1.0, Ds)
    ys, xs = np.meshgrid(np.arange(H) / (H - 1), np.arange(W) / (W - 1), indexing="ij")
    for k in range(K):
        G3 = (gw[k, 0] * gr[k, 0][:, :, None] + gw[k, 1] * gr[k, 1][:, None, :]
              + gw[k, 2] * gr[k, 2][None, :, :] + gb[k])
        c = np.clip(x[k % 3].astype(np.float64), 0.0, 1.0)
        f = RegularGridInterpolator((knots, knots, knots), G3, method="linear")
        ref = f(np.stack([xs.ravel(), ys.ravel(), c.ravel()], axis=1)).reshape(H, W)
        np.testing.assert_allclose(Psi[k], ref, atol=1e-6)


def test_bilinear_functions_reproduced_exactly():
    # planes sampled from a + b u + c v + d u v are reproduced at every query point
    H, W, Ds = 6, 9, 5
    g = np.random.default_rng(24)
    x = g.uniform(0, 1, size=(3, H, W)).astype(np.float32)
    t = np.linspace(0.0, 1.0, Ds)
    coef = g.normal(size=(3, 4))
    gr = np.stack([np.stack([a + b * t[:, None] + c * t[None, :] + d * t[:, None] * t[None, :]
                             for (a, b, c, d) in coef])] * 3)     # [K=3][3][Ds][Ds]
    gw = np.ones((3, 3))
    Psi = og.slice_grids(x, gr, gw, np.zeros(3))
    xq = np.arange(W) / (W - 1)
    yq = np.arange(H) / (H - 1)
    for k in range(3):
        q = np.float32(np.float32(np.clip(x[k], 0, 1)) * np.float32(Ds - 1)).astype(np.float64) / (Ds - 1)
        f = lambda u, v, cf: cf[0] + cf[1] * u + cf[2] * v + cf[3] * u * v
        ref = (f(xq[None, :], yq[:, None], coef[0]) + f(xq[None, :], q, coef[1]) + f(yq[:, None], q, coef[2]))
        np.testing.assert_allclose(Psi[k], ref, atol=1e-12)


def test_scalar_brute_force():
    # the supplementary equations written out as scalar loops on a tiny image
    x, gr, gw, gb = _case(seed=25, H=3, W=4, K=3, Ds=4)
    K, _, Ds, _ = gr.shape
    H, W = x.shape[1:]

    def left(p):
        q = float(np.float32(np.float32(p) * np.float32(Ds - 1)))
        i = min(int(np.floor(q)), Ds - 2)
        return i, q - i

    def spatial(v, n):
        u = v * (Ds - 1) / (n - 1)
        i = min(int(np.floor(u)), Ds - 2)
        return i, u - i

    def bil(t, ia, da, ib, db):
        return ((1 - da) * (1 - db) * t[ia][ib] + da * (1 - db) * t[ia + 1][ib]
                + (1 - da) * db * t[ia][ib + 1] + da * db * t[ia + 1][ib + 1])

    Psi = og.slice_grids(x, gr, gw, gb)
    for k in range(K):
        for yy in range(H):
            for xx in range(W):
                p = min(max(float(x[k % 3, yy, xx]), 0.0), 1.0)
                ic, dc = left(p)
                ix, dx = spatial(xx, W)
                iy, dy = spatial(yy, H)
                v = (gw[k, 0] * bil(gr[k, 0], ix, dx, iy, dy) + gw[k, 1] * bil(gr[k, 1], ix, dx, ic, dc)
                     + gw[k, 2] * bil(gr[k, 2], iy, dy, ic, dc) + gb[k])
                assert abs(Psi[k, yy, xx] - v) < 1e-12


def test_fused_output_adds_each_grid_to_its_channel():
    c, gr, gw, gb = synth.grid_case(26, 8, 12, 5, 2, 3, 4, K=6, Ds=5)
    T = ol.reconstruct(c.U, c.s, c.V)[0]
    Y = og.transform_grid(c.x[0], T, c.smap[0], gr[0], gw[0], gb[0])
    Y0 = ol.transform(c.x[0], T, c.smap[0])
    Psi = og.slice_grids(c.x[0], gr[0], gw[0], gb[0])
    for ch in range(3):
        np.testing.assert_allclose(Y[ch] - Y0[ch], Psi[ch] + Psi[ch + 3], atol=1e-12)


def test_adjoint_grids_weights_bias():
    # Psi is linear in the planes (weights fixed) and in (weights, bias): dot tests
    x, gr, gw, gb = _case(seed=27)
    K = gr.shape[0]
    g = np.random.default_rng(28)
    G = g.normal(size=x.shape)

    def L(gr_, gw_, gb_):
        Psi = og.slice_grids(x, gr_, gw_, gb_)
        return sum((G[k % 3] * Psi[k]).sum() for k in range(K))

    r = og.slice_bwd(x, gr, gw, G)
    dgr = g.normal(size=gr.shape)
    np.testing.assert_allclose(L(gr + dgr, gw, gb) - L(gr, gw, gb), (r["dg"] * dgr).sum(), rtol=1e-10)
    dgw = g.normal(size=gw.shape)
    np.testing.assert_allclose(L(gr, gw + dgw, gb) - L(gr, gw, gb), (r["dgw"] * dgw).sum(), rtol=1e-10)
    dgb = g.normal(size=gb.shape)
    np.testing.assert_allclose(L(gr, gw, gb + dgb) - L(gr, gw, gb), (r["dgb"] * dgb).sum(), rtol=1e-10)


def test_input_gradient_finite_differences():
    x, gr, gw, gb = _case(seed=29, H=5, W=6, K=6, Ds=6)
    K, _, Ds, _ = gr.shape
    g = np.random.default_rng(30)
    G = g.normal(size=x.shape)
    r = og.slice_bwd(x, gr, gw, G)
    h = 1e-3
    checked = 0
    for (c, yy, xx) in [(c, yy, xx) for c in range(3) for yy in range(5) for xx in range(6)]:
        v = float(x[c, yy, xx])
        q = v * (Ds - 1)
        if not (2 * h < v < 1 - 2 * h) or abs(q - round(q)) < 2 * h * (Ds - 1):
            continue
        xp, xm = x.copy(), x.copy()
        xp[c, yy, xx] = np.float32(v + h)
        xm[c, yy, xx] = np.float32(v - h)
        step = float(xp[c, yy, xx]) - float(xm[c, yy, xx])

        def L(xx_):
            Psi = og.slice_grids(xx_, gr, gw, gb)
            return sum((G[k % 3] * Psi[k]).sum() for k in range(K))
        fd = (L(xp) - L(xm)) / step
        assert abs(fd - r["dx"][c, yy, xx]) <= 1e-3 * abs(fd) + 1e-6
        checked += 1
    assert checked > 40


def test_sampled_slicing_matches_full():
    x, gr, gw, gb = _case(seed=31, H=11, W=17)
    Psi = og.slice_grids(x, gr, gw, gb)
    g = np.random.default_rng(32)
    ys = g.integers(0, 11, 50)
    xs = g.integers(0, 17, 50)
    np.testing.assert_allclose(og.slice_grids_at(x, gr, gw, gb, ys, xs), Psi[:, ys, xs], atol=0)
