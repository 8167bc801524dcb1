"""Pins of the unfused original-structure oracle (oracle/unfused.py): the 1x1 fusion against
torch conv2d, the identity configuration (fusion passes the image through, identity 3D LUT
returns it), and the 3D lookup of a LUT that is affine in each channel.  CPU only."""
import numpy as np
import torch
import torch.nn.functional as F

from oracle import grid as og
from oracle import unfused as ou


def test_fuse_matches_conv2d_1x1():
    g = np.random.default_rng(51)
    x = g.uniform(0, 1, (3, 7, 9))
    fs = g.normal(size=(6, 7, 9))
    Wf = g.normal(size=(3, 9))
    bf = g.normal(size=3)
    ref = F.conv2d(torch.from_numpy(np.concatenate([x, fs]))[None], torch.from_numpy(Wf)[:, :, None, None],
                   torch.from_numpy(bf))[0].numpy()
    np.testing.assert_allclose(ou.fuse(x, fs, Wf, bf), ref, atol=1e-12)


def test_identity_pipeline_returns_clamped_input():
    g = np.random.default_rng(52)
    x = g.uniform(-0.1, 1.1, (3, 6, 10)).astype(np.float32)
    K, Ds, D = 6, 5, 9
    gr = g.normal(size=(K, 3, Ds, Ds))
    Wf = np.zeros((3, 3 + K))
    Wf[:, :3] = np.eye(3)
    t = np.linspace(0.0, 1.0, D)
    T3 = np.stack([np.broadcast_to(ax, (D, D, D)) for ax in
                   (t[:, None, None], t[None, :, None], t[None, None, :])])
    Y, fs, xbar = ou.original_structure(x, gr, np.ones((K, 3)), np.zeros(K), Wf, np.zeros(3), T3)
    np.testing.assert_allclose(fs, og.slice_grids(x, gr, np.ones((K, 3)), np.zeros(K)), atol=0)
    np.testing.assert_allclose(Y, np.clip(x, 0, 1), atol=1e-6)


def test_channelwise_affine_3d_lut():
    # t^c[i][j][k] = a + b r_i + c g_j + d b_k is reproduced exactly by trilinear lookup
    g = np.random.default_rng(53)
    D = 7
    xbar = g.uniform(0, 1, (3, 5, 6)).astype(np.float32)
    t = np.linspace(0.0, 1.0, D)
    coef = g.normal(size=(3, 4))
    T3 = np.stack([a + b * t[:, None, None] + c * t[None, :, None] + d * t[None, None, :] for a, b, c, d in coef])
    Y = ou.lut3d(xbar, T3)
    q = np.float32(xbar * np.float32(D - 1)).astype(np.float64) / (D - 1)
    for ch, (a, b, c, d) in enumerate(coef):
        np.testing.assert_allclose(Y[ch], a + b * q[0] + c * q[1] + d * q[2], atol=1e-12)
