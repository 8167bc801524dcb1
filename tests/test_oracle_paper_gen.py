"""Pins of the oracle of the paper's own generator (supplementary Tables backbone, gen_lut,
gen_lut_weight, gen_bilateral, gen_bilateral_weight): the parameter counts printed in the
component ablation, torch's convolution / LeakyReLU / instance-norm / pooling / linear
modules with autograd, finite differences and instance-norm invariants.  CPU only."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import paper_generator as pg

D, R, K, Ds = 33, 8, 6, 17


def rand_params(seed, K_=K, D_=D, R_=R, Ds_=Ds):
    g = np.random.default_rng(seed)
    P = {}
    for name, shp in pg.param_shapes(D_, R_, K_, Ds_):
        if name.startswith("conv") and name.endswith(".w"):
            P[name] = g.normal(0, np.sqrt(2.0 / np.prod(shp[1:])), shp)
        elif name.endswith(".g"):
            P[name] = g.uniform(0.5, 1.5, shp)
        elif name.endswith(".w"):
            P[name] = g.normal(0, 0.1, shp)
        else:
            P[name] = g.normal(0, 0.1, shp)
    return P


def test_parameter_counts_match_component_ablation():
    # Table comp_ablation: "Ours" 160.478K, "Only LUT" 109.332K.
    assert pg.param_count(33, 8, 6, 17) == 160_478
    assert pg.param_count(33, 8, 0, 17) == 109_332


def torch_reference(P, x, mask, K_, D_=D, R_=R, Ds_=Ds):
    """The same network from torch.nn.functional modules (float64), returning outputs and
    the leaf tensors so autograd gives the parameter gradients."""
    T = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in P.items()}
    a = F.interpolate(torch.tensor(x, dtype=torch.float64), size=(256, 256), mode="bilinear",
                      align_corners=False, antialias=False)
    for i in range(5):
        a = F.conv2d(a, T[f"conv{i + 1}.w"].permute(0, 3, 1, 2), T[f"conv{i + 1}.b"], stride=2, padding=1)
        a = F.leaky_relu(a, 0.2)
        if i < 4:
            a = F.instance_norm(a, weight=T[f"in{i + 1}.g"], bias=T[f"in{i + 1}.b"], eps=1e-5)
    if mask is not None:
        a = a * torch.tensor(mask, dtype=torch.float64) * 2.0
    f = F.avg_pool2d(a, 4).flatten(1)
    outs = {}
    for h, _ in pg.head_sizes(D_, R_, K_, Ds_):
        outs[h] = F.linear(F.linear(f, T[f"{h}.fc1.w"], T[f"{h}.fc1.b"]), T[f"{h}.fc2.w"], T[f"{h}.fc2.b"])
    B = x.shape[0]
    nU = 9 * D_ * R_
    o = outs["t"]
    res = {"U": o[:, :nU].reshape(B, 9, D_, R_), "s": o[:, nU:nU + 9 * R_].reshape(B, 9, R_),
           "V": o[:, nU + 9 * R_:].reshape(B, 9, D_, R_),
           "lut_w": outs["tw"].reshape(B, 3, 4)[:, :, :3].reshape(B, 9),
           "lut_b": outs["tw"].reshape(B, 3, 4)[:, :, 3]}
    if K_:
        res["grids"] = outs["s"].reshape(B, K_, 3, Ds_, Ds_)
        res["gw"] = outs["sw"].reshape(B, K_, 4)[:, :, :3]
        res["gb"] = outs["sw"].reshape(B, K_, 4)[:, :, 3]
    return res, T


@pytest.mark.parametrize("K_,use_mask", [(6, True), (6, False), (0, True)])
def test_exact_mode_matches_torch_autograd(K_, use_mask):
    P = rand_params(10 + K_, K_)
    g = np.random.default_rng(11)
    x = g.uniform(0, 1, (2, 3, 72, 100))
    mask = (g.uniform(size=(2, 64, 8, 8)) < 0.5).astype(np.float64) if use_mask else None
    out, cache = pg.forward(P, x, D, R, K_, Ds, mask=mask, mixed=False)
    ref, T = torch_reference(P, x, mask, K_)
    assert set(out) == set(ref)
    for k in ref:
        np.testing.assert_allclose(out[k], ref[k].detach().numpy(), rtol=1e-10, atol=1e-12, err_msg=k)
    dout = {k: g.normal(0, 1, v.shape) for k, v in out.items()}
    loss = sum((ref[k] * torch.tensor(dout[k])).sum() for k in ref)
    loss.backward()
    G = pg.backward(P, cache, dout, D, R, K_, Ds, mask=mask, mixed=False)
    assert set(G) == set(P)
    for k in P:
        tg = T[k].grad.numpy()
        np.testing.assert_allclose(G[k], tg, rtol=1e-8, atol=1e-10 * max(1.0, np.abs(tg).max()), err_msg=k)


def test_finite_differences():
    P = rand_params(21)
    g = np.random.default_rng(22)
    x = g.uniform(0, 1, (1, 3, 64, 64))
    mask = (g.uniform(size=(1, 64, 8, 8)) < 0.5).astype(np.float64)
    out, cache = pg.forward(P, x, D, R, K, Ds, mask=mask, mixed=False)
    dout = {k: g.normal(0, 1, v.shape) for k, v in out.items()}
    G = pg.backward(P, cache, dout, D, R, K, Ds, mask=mask, mixed=False)

    def L(PP):
        o, _ = pg.forward(PP, x, D, R, K, Ds, mask=mask, mixed=False)
        return sum((o[k] * dout[k]).sum() for k in o)

    h = 1e-6
    for name in ("conv1.w", "conv3.b", "in1.g", "in4.b", "conv5.w", "t.fc1.w", "tw.fc2.w", "s.fc1.b", "sw.fc2.w"):
        idx = tuple(g.integers(0, n) for n in P[name].shape)
        Pp = {k: v.copy() for k, v in P.items()}
        Pm = {k: v.copy() for k, v in P.items()}
        Pp[name][idx] += h
        Pm[name][idx] -= h
        fd = (L(Pp) - L(Pm)) / (2 * h)
        assert abs(fd - G[name][idx]) <= 1e-5 * max(1.0, abs(fd)), (name, idx, fd, G[name][idx])


def test_instance_norm_output_statistics():
    # exact mode stores the normalised, scaled and shifted activations unrounded: each channel
    # has mean beta and variance gamma^2 var / (var + eps)
    P = rand_params(31)
    x = np.random.default_rng(32).uniform(0, 1, (2, 3, 40, 50))
    _, cache = pg.forward(P, x, D, R, K, Ds, mixed=False)
    for i in range(4):
        a = cache["acts"][i + 1]
        h = cache["hs"][i]
        var = h.var(axis=(1, 2))
        np.testing.assert_allclose(a.mean(axis=(1, 2)), np.broadcast_to(P[f"in{i + 1}.b"], var.shape), atol=1e-10)
        np.testing.assert_allclose(a.var(axis=(1, 2)), P[f"in{i + 1}.g"] ** 2 * var / (var + pg.EPS), rtol=1e-9)


def test_dropout_mask_scaling_and_pool_order():
    # an all-ones keep mask doubles the pooled features; a mask keeping one 4x4 window of one
    # channel leaves only feature 4c + 2py + px
    P = rand_params(41)
    x = np.random.default_rng(42).uniform(0, 1, (1, 3, 32, 32))
    _, c0 = pg.forward(P, x, D, R, K, Ds, mixed=False)
    _, c1 = pg.forward(P, x, D, R, K, Ds, mask=np.ones((1, 64, 8, 8)), mixed=False)
    np.testing.assert_allclose(c1["f"], 2 * c0["f"], rtol=1e-12)
    m = np.zeros((1, 64, 8, 8))
    c, py, px = 5, 1, 0
    m[0, c, 4 * py:4 * py + 4, 4 * px:4 * px + 4] = 1
    _, c2 = pg.forward(P, x, D, R, K, Ds, mask=m, mixed=False)
    nz = np.flatnonzero(c2["f"][0])
    assert list(nz) == [4 * c + 2 * py + px]


def test_mixed_mode_is_bf16_close_to_exact():
    P = rand_params(51)
    x = np.random.default_rng(52).uniform(0, 1, (1, 3, 64, 64))
    a, _ = pg.forward(P, x, D, R, K, Ds, mixed=True)
    b, _ = pg.forward(P, x, D, R, K, Ds, mixed=False)
    for k in a:
        scale = np.abs(b[k]).max()
        assert np.abs(a[k] - b[k]).max() <= 5e-2 * scale, k


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


def torch_reference_mixed(P, x, mask, K_, D_=D, R_=R, Ds_=Ds):
    """torch_reference with bf16 casts where the mirror mode places them: the downsampled
    input, the convolution weights and the normalised activations that feed the next
    convolution are stored as bf16; the gradient of each convolution's output (before its
    bias) is rounded to bf16 before it reaches the convolution's weight and input gradients;
    biases, LeakyReLU, the normalisation, dropout, pooling and the FC generators stay in full
    precision."""
    T = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in P.items()}
    a = _st(F.interpolate(torch.tensor(x, dtype=torch.float64), size=(256, 256), mode="bilinear",
                          align_corners=False, antialias=False))
    for i in range(5):
        z = _round_grad(F.conv2d(a, _st(T[f"conv{i + 1}.w"]).permute(0, 3, 1, 2), None, stride=2, padding=1))
        a = F.leaky_relu(z + T[f"conv{i + 1}.b"][None, :, None, None], 0.2)
        if i < 4:
            a = _st(F.instance_norm(a, weight=T[f"in{i + 1}.g"], bias=T[f"in{i + 1}.b"], eps=1e-5))
    if mask is not None:
        a = a * torch.tensor(mask, dtype=torch.float64) * 2.0
    f = F.avg_pool2d(a, 4).flatten(1)
    outs = {}
    for h, _ in pg.head_sizes(D_, R_, K_, Ds_):
        outs[h] = F.linear(F.linear(f, T[f"{h}.fc1.w"], T[f"{h}.fc1.b"]), T[f"{h}.fc2.w"], T[f"{h}.fc2.b"])
    B = x.shape[0]
    nU = 9 * D_ * R_
    o = outs["t"]
    res = {"U": o[:, :nU].reshape(B, 9, D_, R_), "s": o[:, nU:nU + 9 * R_].reshape(B, 9, R_),
           "V": o[:, nU + 9 * R_:].reshape(B, 9, D_, R_),
           "lut_w": outs["tw"].reshape(B, 3, 4)[:, :, :3].reshape(B, 9),
           "lut_b": outs["tw"].reshape(B, 3, 4)[:, :, 3]}
    if K_:
        res["grids"] = outs["s"].reshape(B, K_, 3, Ds_, Ds_)
        res["gw"] = outs["sw"].reshape(B, K_, 4)[:, :, :3]
        res["gb"] = outs["sw"].reshape(B, K_, 4)[:, :, 3]
    return res, T


@pytest.mark.parametrize("K_,use_mask", [(6, True), (0, False)])
def test_mixed_mode_matches_torch_with_bf16_casts(K_, use_mask):
    """End-to-end pin of the mirror's rounding placement, forward outputs and every parameter
    gradient: both sides take each bf16 decision from float64 values, so they agree to
    float64 rounding; a rounding placed elsewhere, or one missing, moves values by a bf16
    step (about 4e-3 relative) and fails the 1e-9 bar."""
    P = rand_params(60 + K_, K_)
    g = np.random.default_rng(61)
    B = 2
    x = g.uniform(0, 1, (B, 3, 200, 230))
    mask = (g.uniform(size=(B, 64, 8, 8)) < 0.5).astype(np.float64) if use_mask else None
    out, cache = pg.forward(P, x, D, R, K_, Ds, mask=mask, mixed=True)
    ref, T = torch_reference_mixed(P, x, mask, K_)
    for k in out:
        r = ref[k].detach().numpy()
        assert np.abs(out[k] - r).max() <= 1e-9 * max(1.0, np.abs(r).max()), k
    up = {k: g.normal(size=v.shape) for k, v in out.items()}
    grads = pg.backward(P, cache, up, D, R, K_, Ds, mask=mask, mixed=True)
    L = sum((ref[k] * torch.from_numpy(up[k])).sum() for k in out)
    L.backward()
    for k in P:
        r = T[k].grad.numpy()
        assert np.abs(grads[k] - r).max() <= 1e-9 * max(1.0, np.abs(r).max()), k
    exact, _ = pg.forward(P, x, D, R, K_, Ds, mask=mask, mixed=False)
    assert np.abs(out["U"] - exact["U"]).max() > 1e-6 * np.abs(exact["U"]).max()
