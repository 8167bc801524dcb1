"""GPU parity of the 2D-LUT path (reconstruct, fused apply, backward, uneven-batch plan)
against the fp64 CPU oracle, through the C ABI of libsvdlut.so."""
import numpy as np
import pytest
import torch

import synth
from oracle import lut as ol

pytestmark = pytest.mark.gpu

TOL32 = 1e-5     # max-abs, float32 storage
TOL16 = 2e-3     # max-abs, float16 storage


@pytest.fixture(scope="module")
def svd():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2508_16121_amd as m
    return m


def dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return t.to(dtype) if dtype is not None else t


def host(t):
    torch.cuda.synchronize()
    return t.detach().float().cpu().numpy().astype(np.float64)


def say(msg):
    print(msg, flush=True)


# ------------------------------------------------------------------ reconstruction
@pytest.mark.parametrize("D,R,n", [(33, 8, 36), (17, 4, 9), (2, 1, 3), (40, 64, 9)])
def test_reconstruct_parity(svd, D, R, n):
    say(f"reconstruct D={D} R={R} n={n}")
    g = np.random.default_rng(D * 100 + R)
    U = g.normal(0, 0.1, (n, D, R)).astype(np.float32)
    s = g.uniform(0, 1, (n, R)).astype(np.float32)
    V = g.normal(0, 0.1, (n, D, R)).astype(np.float32)
    T = host(svd.reconstruct(dev(U), dev(s), dev(V)))
    assert np.abs(T - ol.reconstruct(U, s, V)).max() <= TOL32


def test_reconstruct_full_rank_svd(svd):
    D = 17
    A = np.random.default_rng(1).uniform(-1, 1, (D, D))
    u, sig, vt = np.linalg.svd(A)
    T = host(svd.reconstruct(dev(u[None].astype(np.float32)), dev(sig[None].astype(np.float32)),
                             dev(vt.T[None].astype(np.float32).copy())))
    assert np.abs(T[0] - A).max() <= TOL32


# ------------------------------------------------------------------ forward apply
def _check_apply(svd, x, U, s, V, m, bias=None, io=torch.float32, mt=torch.float32, tol=TOL32, label=""):
    say(f"apply {label} x{tuple(x.shape)} D={U.shape[2]} R={U.shape[3]} map{tuple(m.shape)} io={io}")
    xd, md = dev(x, io), dev(m, mt)
    y = svd.apply(xd, dev(U), dev(s), dev(V), md, None if bias is None else dev(bias))
    xq = host(xd)                       # the oracle sees exactly what the GPU read
    mq = host(md)
    ref = ol.apply(xq, U, s, V, mq, bias)
    got = host(y)
    err = np.abs(got - ref).max()
    assert err <= tol, f"max-abs {err}"
    return got, ref


def test_apply_plain_256(svd):
    c = synth.plain_256()
    _check_apply(svd, c.x, c.U, c.s, c.V, c.smap, label="plain 256x256 D17 R4")


def test_apply_identity_returns_input(svd):
    D = 33
    ramp = np.arange(D) / (D - 1)
    U = np.zeros((1, 9, D, 1), np.float32); V = np.zeros_like(U); s = np.zeros((1, 9, 1), np.float32)
    U[0, 0, :, 0], V[0, 0, :, 0], s[0, 0] = ramp, 1, 1           # r from rows of (r, g)
    U[0, 3, :, 0], V[0, 3, :, 0], s[0, 3] = 1, ramp, 1           # g from columns of (r, g)
    U[0, 7, :, 0], V[0, 7, :, 0], s[0, 7] = 1, ramp, 1           # b from columns of (r, b)
    x = np.random.default_rng(3).uniform(-0.3, 1.3, (1, 3, 37, 300)).astype(np.float32)
    x[0, :, 0, :3] = [[0, 1, np.nan]] * 3
    y = svd.apply(dev(x), dev(U), dev(s), dev(V), torch.ones(1, 9, 5, 38, device="cuda"))
    ref = np.fmin(np.fmax(x.astype(np.float64), 0), 1)
    assert np.abs(host(y) - ref).max() <= 1e-6


@pytest.mark.parametrize("shape", [
    (1, 1, 1, 33, 8, 1, 1),       # single pixel, single map cell
    (2, 5, 7, 33, 8, 2, 3),       # W not a multiple of 4
    (1, 3, 300, 17, 4, 1, 40),    # ragged second segment, one map row
    (1, 20, 20, 9, 3, 15, 15),    # map finer than a third of the image (per-pixel map path)
    (3, 64, 80, 2, 1, 8, 10),     # D = 2, batch of three
    (1, 9, 513, 33, 8, 4, 65),    # 513 columns: three segments, last one pixel wide
    (1, 130, 1, 5, 2, 17, 1),     # one column
])
def test_apply_edge_shapes(svd, shape):
    B, H, W, D, R, h, w = shape
    g = np.random.default_rng(sum(shape))
    x = g.uniform(-0.05, 1.05, (B, 3, H, W)).astype(np.float32)
    D1 = D - 1
    x.flat[::7] = (g.integers(0, D1 + 1, x.size)[::7] / D1).astype(np.float32)  # exact knots, 0 and 1
    U, s, V = synth.factors(g, B, D, R)
    m = synth.spatial_map(g, B, h, w)
    bias = g.normal(0, 0.1, (B, 3)).astype(np.float32)
    _check_apply(svd, x, U, s, V, m, bias, label=str(shape))


def test_apply_nan_and_out_of_range(svd):
    g = np.random.default_rng(9)
    x = g.uniform(-2, 3, (1, 3, 16, 64)).astype(np.float32)
    x[0, 1, 3, 5] = np.nan
    x[0, 2, 7, 9] = np.inf
    x[0, 0, 8, 10] = -np.inf
    U, s, V = synth.factors(g, 1, 33, 8)
    m = synth.spatial_map(g, 1, 2, 8)
    _check_apply(svd, x, U, s, V, m, label="nan/inf/out of range")


def test_apply_fp16_storage(svd):
    g = np.random.default_rng(10)
    for (H, W) in [(48, 70), (108, 189), (216, 411)]:
        h, w = synth.map_size(H, W)
        x = synth.image(g, H, W)[None]
        U, s, V = synth.factors(g, 1, 33, 8)
        m = synth.spatial_map(g, 1, h, w)
        _check_apply(svd, x, U, s, V, m, io=torch.float16, mt=torch.float16, tol=TOL16, label="fp16")


def test_apply_fp16_per_pixel_map(svd):
    # map finer than a third of the image: each pixel blends its own pair of map columns
    # (with half-precision I/O, the variant built for 512-thread workgroups)
    g = np.random.default_rng(12)
    for (H, W, h, w) in [(40, 70, 30, 50), (130, 300, 100, 200)]:
        x = synth.image(g, H, W)[None]
        U, s, V = synth.factors(g, 1, 33, 8)
        m = synth.spatial_map(g, 1, h, w)
        _check_apply(svd, x, U, s, V, m, io=torch.float16, mt=torch.float16, tol=TOL16,
                     label="fp16 per-pixel map")


def test_apply_4k_frame_full(svd):
    """Full 3840x2160 frame, D=33 R=8, 270x480 map, float32, in the launch configuration the
    benchmark times: every pixel against the oracle (evaluated in row bands)."""
    c = synth.frame_4k()
    say("apply 4K frame")
    y = host(svd.apply(dev(c.x), dev(c.U), dev(c.s), dev(c.V), dev(c.smap)))[0]
    assert np.isfinite(y).all()
    T = ol.reconstruct(c.U, c.s, c.V)[0]
    H, W = 2160, 3840
    band = 120
    worst = 0.0
    for y0 in range(0, H, band):
        ys = np.repeat(np.arange(y0, y0 + band), W)
        xs = np.tile(np.arange(W), band)
        ref = ol.transform_at(c.x[0], T, c.smap[0], ys, xs).reshape(3, band, W)
        worst = max(worst, float(np.abs(y[:, y0:y0 + band] - ref).max()))
    say(f"  4K max-abs {worst:.2e}")
    assert worst <= TOL32


def test_apply_is_deterministic(svd):
    c = synth.plain_256(5)
    args = [dev(a) for a in (c.x, c.U, c.s, c.V, c.smap)]
    y1 = host(svd.apply(*args))
    y2 = host(svd.apply(*args))
    assert np.array_equal(y1, y2)


def test_apply_rejects_bad_arguments(svd):
    c = synth.plain_256()
    x, U, s, V, m = (dev(a) for a in (c.x, c.U, c.s, c.V, c.smap))
    with pytest.raises(svd.SvdlutError, match="EINVAL"):
        bad = torch.zeros(1, 9, 41, 4, device="cuda")
        svd.apply(x, bad, s[:, :, :4].contiguous(), bad, m)
    with pytest.raises(ValueError):
        svd.apply(x, U, s, V, m[:, :8].contiguous())


@pytest.mark.parametrize("shape", [
    (1, 1, 65535, 40, 64, 1, 65535),    # the longest row, a per-pixel map, the largest D and R
    (1, 65535, 1, 40, 64, 4097, 1),     # the longest column
    (1, 3, 65535, 33, 8, 3, 8192),      # a long row over a map with 8 pixels per column
])
def test_apply_maximum_dimensions(svd, shape):
    """H or W at 65535 (the largest the ABI takes) with D = 40 and R = 64: every pixel against
    the oracle at the fp32 bar."""
    B, H, W, D, R, h, w = shape
    say(f"apply maximum dims {shape}")
    g = np.random.default_rng(sum(shape) % 1000)
    x = g.uniform(-0.05, 1.05, (B, 3, H, W)).astype(np.float32)
    U, s, V = synth.factors(g, B, D, R)
    m = synth.spatial_map(g, B, h, w)
    y = svd.apply(dev(x), dev(U), dev(s), dev(V), dev(m))
    ref = ol.apply(x, U, s, V, m)
    assert np.abs(host(y) - ref).max() <= TOL32
