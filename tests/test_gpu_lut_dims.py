"""GPU parity of the standalone 3D-LUT and 1D-LUT transforms (the other LUT dimensions of the
paper's LUT-dimension analysis) against the fp64 oracle (oracle.lut.trilinear, oracle.lut.lut1d)."""
import numpy as np
import pytest
import torch

from oracle import lut as ol

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def svd():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2508_16121_amd as m
    return m


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def inputs(seed, B, H, W, D):
    g = np.random.default_rng(seed)
    x = g.uniform(-0.05, 1.05, (B, 3, H, W)).astype(np.float32)
    x.flat[::11] = (g.integers(0, D, x.size)[::11] / (D - 1)).astype(np.float32)    # exact knots, 0 and 1
    x.flat[5::97] = np.nan
    return g, x


@pytest.mark.parametrize("B,H,W,D", [(1, 1, 1, 33), (2, 37, 53, 17), (1, 64, 256, 33), (3, 5, 2, 2)])
def test_lut3d_apply_parity(svd, B, H, W, D):
    g, x = inputs(B * 1000 + H + W + D, B, H, W, D)
    T3 = g.normal(0, 0.3, (B, 3, D, D, D)).astype(np.float32)
    y = host(svd.lut3d_apply(torch.from_numpy(x).cuda(), torch.from_numpy(T3).cuda()))
    for b in range(B):
        for c in range(3):
            ref = ol.trilinear(x[b], T3[b, c])
            assert np.abs(y[b, c] - ref).max() <= 1e-5, (b, c)


@pytest.mark.parametrize("B,H,W,D", [(1, 1, 1, 33), (2, 37, 53, 17), (1, 64, 256, 33), (3, 5, 2, 2)])
def test_lut1d_apply_parity(svd, B, H, W, D):
    g, x = inputs(B * 2000 + H + W + D, B, H, W, D)
    T1 = g.normal(0, 1, (B, 3, D)).astype(np.float32)
    y = host(svd.lut1d_apply(torch.from_numpy(x).cuda(), torch.from_numpy(T1).cuda()))
    for b in range(B):
        assert np.abs(y[b] - ol.lut1d(x[b], T1[b])).max() <= 1e-5, b


def test_lut_dims_4k_sampled(svd):
    """Full 4K frame through both transforms; sampled pixels against the oracle."""
    g = np.random.default_rng(71)
    H, W, D = 2160, 3840, 33
    x = g.uniform(0, 1, (1, 3, H, W)).astype(np.float32)
    T3 = g.normal(0, 0.3, (1, 3, D, D, D)).astype(np.float32)
    T1 = g.normal(0, 1, (1, 3, D)).astype(np.float32)
    xt = torch.from_numpy(x).cuda()
    y3 = svd.lut3d_apply(xt, torch.from_numpy(T3).cuda())
    y1 = svd.lut1d_apply(xt, torch.from_numpy(T1).cuda())
    ys = np.concatenate([g.integers(0, H, 2000), [0, H - 1]])
    xs = np.concatenate([g.integers(0, W, 2000), [W - 1, 0]])
    sub = x[0][:, ys, xs][:, None, :]                       # [3][1][n]
    h3 = host(y3)[0][:, ys, xs]
    h1 = host(y1)[0][:, ys, xs]
    for c in range(3):
        assert np.abs(h3[c] - ol.trilinear(sub, T3[0, c])[0]).max() <= 1e-5
    assert np.abs(h1 - ol.lut1d(sub, T1[0])[:, 0]).max() <= 1e-5
