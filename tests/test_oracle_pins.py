"""Pins of the CPU oracle to what the paper and mathematics fix (no GPU needed).

Each test checks the oracle against something other than itself: a closed form, an
invariant the paper states, an independent scalar brute force written from the paper's
equations, or a library routine (NumPy SVD, SciPy's grid interpolator, torch's
grid_sample / interpolate / conv2d / autograd / Adam).
"""
import math

import numpy as np
import pytest
import torch
import torch.nn.functional as F
from scipy.interpolate import RegularGridInterpolator

import synth
from oracle import generator as og
from oracle import lut as ol
from oracle import pairs as op

RNG = np.random.default_rng(12345)


def rand_image(g, H, W, lo=0.0, hi=1.0):
    return g.uniform(lo, hi, size=(3, H, W)).astype(np.float32)


def identity_factors(D):
    """Rank-1 identity: t^r_rg[i][j] = i/(D-1), t^g_rg[i][j] = j/(D-1), t^b_rb[i][j] = j/(D-1)."""
    ramp = np.arange(D) / (D - 1)
    one = np.ones(D)
    U = np.zeros((9, D, 1)); V = np.zeros((9, D, 1)); s = np.zeros((9, 1))
    U[ol.lut_id(0, 0), :, 0], V[ol.lut_id(0, 0), :, 0] = ramp, one   # r from (r, g) rows
    U[ol.lut_id(1, 0), :, 0], V[ol.lut_id(1, 0), :, 0] = one, ramp   # g from (r, g) columns
    U[ol.lut_id(2, 1), :, 0], V[ol.lut_id(2, 1), :, 0] = one, ramp   # b from (r, b) columns
    s[[0, 3, 7], 0] = 1.0
    return U, s, V


# ------------------------------------------------------------------ P1 identity
@pytest.mark.parametrize("D", [2, 17, 33])
def test_identity_lut_returns_input(D):
    g = np.random.default_rng(D)
    x = rand_image(g, 9, 13, -0.2, 1.2)
    x[0, 0, :4] = [0.0, 1.0, np.nan, 0.5]
    U, s, V = identity_factors(D)
    m = np.ones((9, 2, 3))
    y = ol.transform(x, ol.reconstruct(U, s, V), m)
    expect = np.fmin(np.fmax(x.astype(np.float64), 0.0), 1.0)
    assert np.nanmax(np.abs(y - expect)) <= 1e-6
    assert y[0, 0, 2] == 0.0                       # NaN input -> 0


def test_identity_dense_lut():
    D = 9
    ramp = np.arange(D) / (D - 1)
    T = np.zeros((9, D, D))
    T[ol.lut_id(0, 0)] = ramp[:, None] + 0 * ramp[None]
    T[ol.lut_id(1, 2)] = ramp[:, None] + 0 * ramp[None]     # g as the row of (g, b)
    T[ol.lut_id(2, 2)] = 0 * ramp[:, None] + ramp[None]     # b as the column of (g, b)
    x = rand_image(np.random.default_rng(1), 6, 7)
    y = ol.transform(x, T, np.ones((9, 1, 1)))
    assert np.abs(y - x).max() <= 1e-6


# ------------------------------------------------------------------ P2 SVD reconstruction
@pytest.mark.parametrize("D", [5, 17, 33])
def test_full_rank_svd_reproduces_dense_lut(D):
    A = np.random.default_rng(D).normal(size=(D, D))
    u, sig, vt = np.linalg.svd(A)
    T = ol.reconstruct(u, sig, vt.T)
    assert np.abs(T - A).max() <= 1e-12


def test_truncated_svd_eckart_young():
    D = 33
    A = np.random.default_rng(7).normal(size=(D, D))
    u, sig, vt = np.linalg.svd(A)
    for r in (1, 4, 8, 16):
        T = ol.reconstruct(u[:, :r], sig[:r], vt[:r].T)
        err = np.linalg.norm(A - T)
        assert abs(err - math.sqrt((sig[r:] ** 2).sum())) <= 1e-10 * np.linalg.norm(A)


def test_reconstruct_orientation_asymmetric():
    U = np.array([[1.0], [0.0], [0.0]]); V = np.array([[0.0], [0.0], [1.0]]); s = np.array([2.0])
    T = ol.reconstruct(U, s, V)
    assert T[0, 2] == 2.0 and T[2, 0] == 0.0        # U indexes rows (alpha), V columns (beta)


# ------------------------------------------------------------------ P3 sum of pairwise terms
@pytest.mark.parametrize("D", [5, 33])
def test_sum_of_pairs_equals_trilinear(D):
    g = np.random.default_rng(100 + D)
    A, B, C = (g.normal(size=(D, D)) for _ in range(3))
    T3 = A[:, :, None] + B[:, None, :] + C[None, :, :]
    x = rand_image(g, 11, 9)
    T = np.zeros((9, D, D))
    T[ol.lut_id(0, 0)], T[ol.lut_id(0, 1)], T[ol.lut_id(0, 2)] = A, B, C
    y = ol.transform(x, T, np.ones((9, 1, 1)))
    assert np.abs(y[0] - ol.trilinear(x, T3)).max() <= 1e-12
    assert np.abs(y[1:]).max() == 0.0


# ------------------------------------------------------------------ P4 brute force + libraries
def _brute_transform(x, T, m):
    """Scalar loops written directly from the supplementary equations (query, lookup, adjacent,
    bilinear, weighted sum) and the corner-aligned map rule x' = x/(W-1)."""
    _, H, W = x.shape
    D = T.shape[-1]
    C, h, w = m.shape
    pairs = {0: (0, 1), 1: (0, 2), 2: (1, 2)}

    def left_and_delta(v):
        p = min(max(float(v), 0.0), 1.0)
        q = float(np.float32(np.float32(p) * np.float32(D - 1)))
        i = min(int(math.floor(q)), D - 2)
        return i, q - i

    def mapcoord(k, n_out, n_in):
        if n_in == 1:
            return 0, 0, 0.0
        u = (k / (n_out - 1)) * (n_in - 1) if n_out > 1 else 0.0
        i = min(int(math.floor(u + 1e-12)), n_in - 2)
        return i, i + 1, u - i

    Y = np.zeros((3, H, W))
    for yy in range(H):
        a0, a1, dv = mapcoord(yy, H, h)
        for xx in range(W):
            b0, b1, du = mapcoord(xx, W, w)
            dec = [left_and_delta(x[ch, yy, xx]) for ch in range(3)]
            for c in range(3):
                tot = 0.0
                for p in range(3):
                    l = 3 * c + p
                    (ia, da), (ib, db) = dec[pairs[p][0]], dec[pairs[p][1]]
                    t = T[l]
                    phi = ((1 - da) * (1 - db) * t[ia][ib] + da * (1 - db) * t[ia + 1][ib]
                           + (1 - da) * db * t[ia][ib + 1] + da * db * t[ia + 1][ib + 1])
                    S = ((1 - dv) * ((1 - du) * m[l][a0][b0] + du * m[l][a0][b1])
                         + dv * ((1 - du) * m[l][a1][b0] + du * m[l][a1][b1]))
                    tot += S * phi
                Y[c, yy, xx] = tot
    return Y


@pytest.mark.parametrize("shape", [(4, 4, 5, 2, 2), (4, 4, 3, 1, 3), (5, 3, 17, 3, 1), (1, 1, 2, 1, 1)])
def test_brute_force_small_images(shape):
    H, W, D, h, w = shape
    g = np.random.default_rng(H * 100 + W * 10 + D)
    x = rand_image(g, H, W, -0.1, 1.1)
    x[:, 0, 0] = [0.0, 1.0, 0.5]
    T = g.normal(size=(9, D, D))
    m = g.uniform(size=(9, h, w))
    assert np.abs(ol.transform(x, T, m) - _brute_transform(x, T, m)).max() <= 1e-12


def test_bilinear_matches_scipy_and_grid_sample():
    D = 17
    g = np.random.default_rng(3)
    T = g.normal(size=(D, D))
    pa = g.uniform(size=500).astype(np.float32)
    pb = g.uniform(size=500).astype(np.float32)
    ia, da = ol.decode(pa, D)
    ib, db = ol.decode(pb, D)
    ours = ol.bilinear(T, ia, da, ib, db)
    grid = np.linspace(0.0, 1.0, D)
    sp = RegularGridInterpolator((grid, grid), T, method="linear")(np.stack([pa, pb], 1).astype(np.float64))
    tol = 1e-6 * np.abs(T).max() * D
    assert np.abs(ours - sp).max() <= tol
    inp = torch.from_numpy(T)[None, None]
    gr = torch.from_numpy(np.stack([2 * pb.astype(np.float64) - 1, 2 * pa.astype(np.float64) - 1], -1))[None, None]
    ts = F.grid_sample(inp, gr, mode="bilinear", padding_mode="border", align_corners=True)[0, 0, 0].numpy()
    assert np.abs(ours - ts).max() <= tol


def test_trilinear_matches_scipy():
    D = 9
    g = np.random.default_rng(4)
    T3 = g.normal(size=(D, D, D))
    x = rand_image(g, 7, 8)
    grid = np.linspace(0.0, 1.0, D)
    sp = RegularGridInterpolator((grid, grid, grid), T3, method="linear")(
        np.stack([x[0].ravel(), x[1].ravel(), x[2].ravel()], 1).astype(np.float64)).reshape(7, 8)
    assert np.abs(ol.trilinear(x, T3) - sp).max() <= 1e-6 * np.abs(T3).max() * D


@pytest.mark.parametrize("sizes", [((9, 5, 7), (40, 33)), ((9, 1, 4), (5, 16)), ((9, 32, 32), (256, 256))])
def test_map_upsample_matches_interpolate(sizes):
    (C, h, w), (H, W) = sizes
    m = np.random.default_rng(h * w).uniform(size=(C, h, w))
    ours = ol.upsample(m, H, W)
    ref = F.interpolate(torch.from_numpy(m)[None], size=(H, W), mode="bilinear", align_corners=True)[0].numpy()
    assert np.abs(ours - ref).max() <= 1e-12


# ------------------------------------------------------------------ P5 closed forms
def test_bilinear_polynomial_lut_and_map_reproduced():
    D, H, W, h, w = 33, 23, 31, 4, 5
    g = np.random.default_rng(5)
    co = g.normal(size=(9, 4))
    grid = np.arange(D) / (D - 1)
    T = np.stack([co[l, 0] + co[l, 1] * grid[:, None] + co[l, 2] * grid[None, :]
                  + co[l, 3] * grid[:, None] * grid[None, :] for l in range(9)])
    mc = g.normal(size=(9, 4))
    vv = (np.arange(h) / (h - 1))[:, None]
    uu = (np.arange(w) / (w - 1))[None, :]
    m = np.stack([mc[l, 0] + mc[l, 1] * vv + mc[l, 2] * uu + mc[l, 3] * vv * uu for l in range(9)])
    x = rand_image(g, H, W)
    y = ol.transform(x, T, m)
    yp = (np.arange(H) / (H - 1))[:, None]
    xp = (np.arange(W) / (W - 1))[None, :]
    for c in range(3):
        ref = 0.0
        for p, (a, b) in enumerate(ol.PAIRS):
            l = 3 * c + p
            pa, pb = x[a].astype(np.float64), x[b].astype(np.float64)
            phi = co[l, 0] + co[l, 1] * pa + co[l, 2] * pb + co[l, 3] * pa * pb
            S = mc[l, 0] + mc[l, 1] * yp + mc[l, 2] * xp + mc[l, 3] * yp * xp
            ref = ref + S * phi
        assert np.abs(y[c] - ref).max() <= 1e-5


# ------------------------------------------------------------------ P6 scalar weights (paper's weighted sum)
def test_constant_map_is_scalar_weighted_sum():
    D = 33
    g = np.random.default_rng(6)
    T = g.normal(size=(9, D, D))
    wts = g.uniform(size=9)
    bias = g.normal(size=3)
    x = rand_image(g, 8, 8)
    y = ol.transform(x, T, np.broadcast_to(wts[:, None, None], (9, 3, 3)), bias)
    grid = np.linspace(0.0, 1.0, D)
    pts = lambda a, b: np.stack([x[a].ravel(), x[b].ravel()], 1).astype(np.float64)
    for c in range(3):
        w_rg, w_rb, w_gb = wts[3 * c:3 * c + 3]
        phi = [RegularGridInterpolator((grid, grid), T[3 * c + p])(pts(*ol.PAIRS[p])).reshape(8, 8) for p in range(3)]
        ref = w_rg * phi[0] + w_rb * phi[1] + w_gb * phi[2] + bias[c]
        assert np.abs(y[c] - ref).max() <= 1e-5


# ------------------------------------------------------------------ P7 adjoints and factor gradients
def _small_case(seed=8, H=12, W=10, D=5, R=3, h=4, w=3):
    g = np.random.default_rng(seed)
    x = rand_image(g, H, W, -0.05, 1.05)
    U = g.normal(size=(9, D, R)); s = g.uniform(size=(9, R)); V = g.normal(size=(9, D, R))
    m = g.uniform(size=(9, h, w))
    G = g.normal(size=(3, H, W))
    return g, x, U, s, V, m, G


def test_adjoint_lut_and_map():
    g, x, U, s, V, m, G = _small_case()
    T = ol.reconstruct(U, s, V)
    r = ol.transform_bwd(x, T, m, G)
    T2 = g.normal(size=T.shape)
    assert abs((ol.transform(x, T2, m) * G).sum() - (T2 * r["dT"]).sum()) <= 1e-10
    m2 = g.normal(size=m.shape)
    assert abs((ol.transform(x, T, m2) * G).sum() - (m2 * r["dmap"]).sum()) <= 1e-10
    assert np.allclose(r["db"], G.reshape(3, -1).sum(1))


def test_factor_gradients_euler_identity():
    g, x, U, s, V, m, G = _small_case(9)
    dT = g.normal(size=(9, 5, 5))
    dU, ds, dV = ol.factor_grads(dT, U, s, V)
    f = (ol.reconstruct(U, s, V) * dT).sum()      # T is linear in each factor separately
    for a, da in ((U, dU), (s, ds), (V, dV)):
        assert abs((a * da).sum() - f) <= 1e-10


def _fd_factor(fun, arr, idx, h=1e-6):
    a1 = arr.copy(); a1[idx] += h
    a2 = arr.copy(); a2[idx] -= h
    return (fun(a1) - fun(a2)) / (2 * h)


def test_finite_differences_factors_and_map():
    g, x, U, s, V, m, G = _small_case(10)
    res = ol.apply_bwd(x[None], U[None], s[None], V[None], m[None], G[None])
    loss = lambda U_, s_, V_, m_: (ol.apply(x[None], U_[None], s_[None], V_[None], m_[None]) * G[None]).sum()
    for _ in range(6):
        i = tuple(int(g.integers(0, n)) for n in U.shape)
        assert abs(_fd_factor(lambda a: loss(a, s, V, m), U, i) - res["dU"][0][i]) <= 1e-6
        i = tuple(int(g.integers(0, n)) for n in V.shape)
        assert abs(_fd_factor(lambda a: loss(U, s, a, m), V, i) - res["dV"][0][i]) <= 1e-6
        i = tuple(int(g.integers(0, n)) for n in s.shape)
        assert abs(_fd_factor(lambda a: loss(U, a, V, m), s, i) - res["ds"][0][i]) <= 1e-6
        i = tuple(int(g.integers(0, n)) for n in m.shape)
        assert abs(_fd_factor(lambda a: loss(U, s, V, a), m, i) - res["dmap"][0][i]) <= 1e-6


def test_finite_differences_input():
    D = 5
    g, x, U, s, V, m, G = _small_case(11, D=D)
    x = x.astype(np.float64)
    T = ol.reconstruct(U, s, V)
    r = ol.transform_bwd(x, T, m, G)
    h = 1e-3
    checked = 0
    for _ in range(200):
        a, yy, xx = (int(g.integers(0, n)) for n in x.shape)
        v = x[a, yy, xx]
        knot_dist = abs(v * (D - 1) - round(v * (D - 1)))
        if not (0.01 < v < 0.99) or knot_dist < 2 * h * (D - 1):
            continue
        def L(val):
            x2 = x.copy(); x2[a, yy, xx] = val
            return (ol.transform(x2, T, m) * G).sum()
        # the lookup is linear in each colour inside a cell, so the central difference is exact;
        # divide by the step actually taken after the float32 decode
        v1, v2 = float(np.float32(v + h)), float(np.float32(v - h))
        fd = (L(v1) - L(v2)) / (v1 - v2)
        assert abs(fd - r["dx"][a, yy, xx]) <= 1e-5 * max(1.0, abs(fd))
        checked += 1
    assert checked > 50
    outside = (x < 0) | (x > 1)
    assert outside.any() and np.all(r["dx"][outside] == 0.0)


def test_l1_and_mse_gradients():
    g = np.random.default_rng(12)
    Y = g.normal(size=(2, 3, 4, 4)); Yt = g.normal(size=Y.shape)
    Yt[0, 0, 0, 0] = Y[0, 0, 0, 0]
    v, d = ol.l1_loss(Y, Yt)
    assert np.isclose(v, np.abs(Y - Yt).mean()) and d[0, 0, 0, 0] == 0.0
    tY = torch.from_numpy(Y).requires_grad_()
    torch.nn.functional.l1_loss(tY, torch.from_numpy(Yt)).backward()
    mask = Y != Yt
    assert np.allclose(d[mask], tY.grad.numpy()[mask])
    v, d = ol.mse_loss(Y, Yt)
    tY = torch.from_numpy(Y).requires_grad_()
    lt = torch.nn.functional.mse_loss(tY, torch.from_numpy(Yt)); lt.backward()
    assert np.isclose(v, lt.item()) and np.allclose(d, tY.grad.numpy())


# ------------------------------------------------------------------ generator pins
def test_bf16_round_matches_torch():
    v = np.random.default_rng(13).normal(size=10000).astype(np.float32) * 10.0 ** np.random.default_rng(14).integers(-6, 6, 10000)
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(og.bf16_round(v), ref)


@pytest.mark.parametrize("stride", [1, 2])
def test_conv_matches_torch(stride):
    g = np.random.default_rng(15 + stride)
    a = g.normal(size=(2, 9, 11, 5)); w = g.normal(size=(7, 3, 3, 5)); b = g.normal(size=7)
    ours = og.conv2d(a, w, b, stride)
    ta = torch.from_numpy(a).permute(0, 3, 1, 2).requires_grad_()
    tw = torch.from_numpy(w).permute(0, 3, 1, 2).contiguous().requires_grad_()
    ref = F.conv2d(ta, tw, torch.from_numpy(b), stride=stride, padding=1)
    assert np.abs(ours - ref.permute(0, 2, 3, 1).detach().numpy()).max() <= 1e-12
    dz = g.normal(size=ours.shape)
    ref.backward(torch.from_numpy(dz).permute(0, 3, 1, 2))
    assert np.abs(og.conv2d_dgrad(dz, w, a.shape, stride) - ta.grad.permute(0, 2, 3, 1).numpy()).max() <= 1e-12
    assert np.abs(og.conv2d_wgrad(dz, a, stride) - tw.grad.permute(0, 2, 3, 1).numpy()).max() <= 1e-12


@pytest.mark.parametrize("hw", [(256, 256), (480, 640), (2160, 3840 // 8), (100, 37)])
def test_downsample_matches_interpolate(hw):
    H, W = hw
    x = np.random.default_rng(H + W).uniform(size=(1, 3, H, W))
    ours = og.downsample(x)
    ref = F.interpolate(torch.from_numpy(x), size=(256, 256), mode="bilinear", align_corners=False,
                        antialias=False).permute(0, 2, 3, 1).numpy()
    assert np.abs(ours - ref).max() <= 1e-12


def _torch_generator(P, x, D, R):
    t = {k: torch.tensor(v, requires_grad=True) for k, v in P.items()}
    a = F.interpolate(torch.from_numpy(x), size=(256, 256), mode="bilinear", align_corners=False)
    a3 = None
    for i in range(5):
        w = t[f"conv{i + 1}.w"].permute(0, 3, 1, 2)
        a = torch.relu(F.conv2d(a, w, t[f"conv{i + 1}.b"], stride=2, padding=1))
        if i == 2:
            a3 = a
    smap = F.conv2d(a3, t["head.w"].permute(0, 3, 1, 2), t["head.b"], padding=1)
    o = a.mean(dim=(2, 3)) @ t["fc.w"].T + t["fc.b"]
    blk = o.reshape(x.shape[0], 9, 2 * D * R + R)
    return t, blk[:, :, :D * R].reshape(-1, 9, D, R), blk[:, :, D * R:D * R + R], blk[:, :, D * R + R:].reshape(-1, 9, D, R), smap


def _init_params(g, D, R):
    P = {}
    for name, shp in og.param_shapes(D, R):
        fan = np.prod(shp[1:]) if len(shp) > 1 else 1
        P[name] = g.normal(0, 1.0 / math.sqrt(fan), size=shp) if len(shp) > 1 else g.normal(0, 0.1, size=shp)
    return P


def test_generator_exact_backward_matches_torch_autograd():
    D, R = 5, 2
    g = np.random.default_rng(16)
    P = _init_params(g, D, R)
    x = g.uniform(size=(2, 3, 300, 280))
    U, s, V, smap, cache = og.forward(P, x, D, R, mixed=False)
    t, tU, ts, tV, tmap = _torch_generator(P, x, D, R)
    assert np.abs(U - tU.detach().numpy()).max() <= 1e-10
    assert np.abs(smap - tmap.detach().numpy()).max() <= 1e-10
    GU, Gs, GV, Gm = (g.normal(size=a.shape) for a in (U, s, V, smap))
    grads = og.backward(P, cache, GU, Gs, GV, Gm, mixed=False)
    L = (tU * torch.from_numpy(GU)).sum() + (ts * torch.from_numpy(Gs)).sum() + \
        (tV * torch.from_numpy(GV)).sum() + (tmap * torch.from_numpy(Gm)).sum()
    L.backward()
    for k in P:
        ref = t[k].grad.numpy()
        assert np.abs(grads[k] - ref).max() <= 1e-9 * max(1.0, np.abs(ref).max()), k


def test_generator_exact_backward_finite_differences():
    D, R = 4, 2
    g = np.random.default_rng(17)
    P = _init_params(g, D, R)
    x = g.uniform(size=(1, 3, 256, 256))
    U, s, V, smap, cache = og.forward(P, x, D, R, mixed=False)
    GU, Gs, GV, Gm = (g.normal(size=a.shape) for a in (U, s, V, smap))
    grads = og.backward(P, cache, GU, Gs, GV, Gm, mixed=False)

    def L(P2):
        U2, s2, V2, m2, _ = og.forward(P2, x, D, R, mixed=False)
        return (U2 * GU).sum() + (s2 * Gs).sum() + (V2 * GV).sum() + (m2 * Gm).sum()

    h = 1e-6
    for name in ("conv1.w", "conv3.b", "conv5.w", "head.w", "fc.w", "fc.b", "conv2.w"):
        for _ in range(2):
            idx = tuple(int(g.integers(0, n)) for n in P[name].shape)
            P1 = dict(P); P1[name] = P[name].copy(); P1[name][idx] += h
            P2 = dict(P); P2[name] = P[name].copy(); P2[name][idx] -= h
            fd = (L(P1) - L(P2)) / (2 * h)
            assert abs(fd - grads[name][idx]) <= 1e-5 * max(1.0, abs(fd)), (name, idx)


def test_param_count_and_fc_width():
    shapes = og.param_shapes(33, 8)
    assert sum(int(np.prod(s)) for _, s in shapes) == 872513
    # supplementary Table gen_lut: the LUT head emits 3*3*(D_t*N_S + N_S + D_t*N_S) values
    assert dict(shapes)["fc.b"] == (3 * 3 * (33 * 8 + 8 + 33 * 8),)


def test_adam_matches_torch():
    g = np.random.default_rng(18)
    th = g.normal(size=50)
    p = torch.tensor(th, requires_grad=True)
    opt = torch.optim.Adam([p], lr=1e-4, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(50); v = np.zeros(50)
    for t in range(1, 6):
        gr = g.normal(size=50)
        p.grad = torch.from_numpy(gr.copy()); opt.step()
        th, m, v = og.adam(th, gr, m, v, t)
    assert np.abs(th - p.detach().numpy()).max() <= 1e-12


# ------------------------------------------------------------------ training pairs
def test_identity_degradation_returns_base():
    base = synth.image(np.random.default_rng(19), 32, 40)
    D = 33
    ramp = np.arange(D) / (D - 1)
    ident = np.stack(np.meshgrid(ramp, ramp, ramp, indexing="ij"))
    out = op.degrade(base, ident, (0.3, -0.2, 0.1, 0.0))
    assert np.abs(out - base).max() <= 1e-6


def test_pair_is_degraded_and_deterministic():
    x1, t1 = op.make_pair(3, 64, 64)
    x2, t2 = op.make_pair(3, 64, 64)
    assert np.array_equal(x1, x2) and np.array_equal(t1, t2)
    assert 0.005 < np.abs(x1 - t1).mean() < 0.3


def test_transform_at_matches_full_transform():
    g = np.random.default_rng(20)
    x = rand_image(g, 37, 53, -0.1, 1.1)
    T = g.normal(size=(9, 9, 9))
    m = g.uniform(size=(9, 5, 7))
    full = ol.transform(x, T, m, [0.1, 0.2, 0.3])
    ys = g.integers(0, 37, 200); xs = g.integers(0, 53, 200)
    ys[:2] = [0, 36]; xs[:2] = [0, 52]
    assert np.array_equal(ol.transform_at(x, T, m, ys, xs, [0.1, 0.2, 0.3]), full[:, ys, xs])


def test_lut1d_matches_numpy_interp():
    """The 1D-LUT oracle is numpy's piecewise-linear interpolation of the curve at the clamped
    input (away from the float32 rounding of the cell index)."""
    g = np.random.default_rng(61)
    D = 33
    T1 = g.normal(0, 1, (3, D))
    x = g.uniform(-0.1, 1.1, (3, 20, 30))
    got = ol.lut1d(x, T1)
    knots = np.linspace(0, 1, D)
    for c in range(3):
        ref = np.interp(np.clip(x[c], 0, 1), knots, T1[c])
        assert np.abs(got[c] - ref).max() <= 1e-6 * np.abs(T1).max()
    # identity curve returns the clamped input
    ident = np.tile(knots, (3, 1))
    assert np.abs(ol.lut1d(x, ident) - np.clip(x, 0, 1)).max() <= 1e-7


# ---------------------------------------------------------------- generator: bf16 mirror placement
def _bf16(t):
    """Round to bfloat16 (nearest even) through float32, as the mirror mode does, back to float64."""
    return t.detach().float().to(torch.bfloat16).to(torch.float64)


def _st(t):
    """Value rounded to bf16, gradient passed straight through (a stored bf16 copy)."""
    return t + (_bf16(t) - t).detach()


def _round_grad(t):
    """Identity forward; the gradient flowing back through t is rounded to bf16."""
    t.register_hook(lambda g: _bf16(g))
    return t


def _torch_generator_mixed(P, x, D, R):
    """The small CNN from torch primitives with bf16 casts where the mirror mode places them:
    the downsampled input, every convolution weight and the post-ReLU activations are stored
    as bf16; the gradient of each convolution's output is rounded to bf16 before it reaches
    the convolution's weight and input gradients (bias gradients see the unrounded one); the
    map head, pooling and the FC layer are full precision."""
    t = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in P.items()}
    a = _st(F.interpolate(torch.from_numpy(x), size=(256, 256), mode="bilinear", align_corners=False))
    a3 = None
    for i in range(5):
        w = _st(t[f"conv{i + 1}.w"]).permute(0, 3, 1, 2)
        z = _round_grad(F.conv2d(a, w, None, stride=2, padding=1)) + t[f"conv{i + 1}.b"][None, :, None, None]
        a = _st(torch.relu(z))
        if i == 2:
            a3 = a
    zm = _round_grad(F.conv2d(a3, _st(t["head.w"]).permute(0, 3, 1, 2), None, padding=1))
    smap = zm + t["head.b"][None, :, None, None]
    o = a.mean(dim=(2, 3)) @ t["fc.w"].T + t["fc.b"]
    blk = o.reshape(x.shape[0], 9, 2 * D * R + R)
    return (t, blk[:, :, :D * R].reshape(-1, 9, D, R), blk[:, :, D * R:D * R + R],
            blk[:, :, D * R + R:].reshape(-1, 9, D, R), smap)


def test_generator_mixed_mode_matches_torch_with_bf16_casts():
    """End-to-end pin of the mirror's rounding placement (forward outputs and every parameter
    gradient): both sides take each bf16 decision from float64 values, so they agree to
    float64 rounding; a rounding placed elsewhere, or one missing, moves values by a bf16
    step (about 4e-3 relative) and fails the 1e-9 bar."""
    D, R = 5, 2
    g = np.random.default_rng(18)
    P = _init_params(g, D, R)
    x = g.uniform(size=(2, 3, 300, 280))
    U, s, V, smap, cache = og.forward(P, x, D, R, mixed=True)
    t, tU, ts, tV, tmap = _torch_generator_mixed(P, x, D, R)
    for a, b_ in ((U, tU), (s, ts), (V, tV), (smap, tmap)):
        ref = b_.detach().numpy()
        assert np.abs(a - ref).max() <= 1e-9 * max(1.0, np.abs(ref).max())
    GU, Gs, GV, Gm = (g.normal(size=a.shape) for a in (U, s, V, smap))
    grads = og.backward(P, cache, GU, Gs, GV, Gm, mixed=True)
    L = (tU * torch.from_numpy(GU)).sum() + (ts * torch.from_numpy(Gs)).sum() + \
        (tV * torch.from_numpy(GV)).sum() + (tmap * torch.from_numpy(Gm)).sum()
    L.backward()
    for k in P:
        ref = t[k].grad.numpy()
        assert np.abs(grads[k] - ref).max() <= 1e-9 * max(1.0, np.abs(ref).max()), k
    # and the mirror is not the exact network (the casts are really there)
    U_x = og.forward(P, x, D, R, mixed=False)[0]
    assert np.abs(U - U_x).max() > 1e-6 * np.abs(U_x).max()
