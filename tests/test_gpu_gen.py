"""GPU parity of the learned generator (bf16-MFMA convolutions) against the fp64 oracle, Adam
parity, checkpoint/resume, and the gain the trained network brings over the fixed-factor
fallback on held-out synthetic degrade->restore pairs."""
import math
import os
import time

import numpy as np
import pytest
import torch

from oracle import generator as og

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def svd():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2508_16121_amd as m
    return m


@pytest.fixture(scope="module")
def G(svd):
    from paper_2508_16121_amd import generator
    return generator


def say(msg):
    print(msg, flush=True)


def host(t):
    torch.cuda.synchronize()
    return t.detach().float().cpu().numpy().astype(np.float64)


def random_params(D, R, seed):
    """Parameters with every part active (not the identity start), drawn in the test."""
    g = np.random.default_rng(seed)
    out = {}
    for name, shp in og.param_shapes(D, R):
        if name.endswith(".w") and name.startswith("conv"):
            out[name] = g.normal(0, math.sqrt(2.0 / np.prod(shp[1:])), shp)
        elif name.endswith(".w"):
            out[name] = g.normal(0, 0.05, shp)
        else:
            out[name] = g.normal(0, 0.1, shp)
    return out


def rel_close(got, ref, tol, what):
    scale = max(np.abs(ref).max(), 1e-30)
    err = np.abs(got - ref).max()
    assert err <= tol * scale, f"{what}: max-abs {err:.3e} > {tol} x {scale:.3e}"


@pytest.mark.parametrize("hw", [(256, 256), (300, 280)])
def test_generator_forward_parity(svd, G, hw):
    D, R = 33, 8
    P = random_params(D, R, 1)
    g = np.random.default_rng(2)
    x = g.uniform(0, 1, (2, 3) + hw).astype(np.float32)
    gen = G.Generator(D, R, params=og.flatten(P, D, R).astype(np.float32))
    U, s, V, m = gen.forward(torch.from_numpy(x).cuda())
    rU, rs, rV, rm, _ = og.forward(P, x, D, R, mixed=True)
    for a, b, k in ((U, rU, "U"), (s, rs, "s"), (V, rV, "V"), (m, rm, "map")):
        rel_close(host(a), b, 2e-2, k)


def test_generator_forward_parity_4k_frames(svd, G):
    """The inference configuration's frame size (3x2160x3840, two frames of the batch): the
    downsample from 4K is the only size-dependent step."""
    D, R = 33, 8
    P = random_params(D, R, 21)
    g = np.random.default_rng(22)
    x = g.uniform(0, 1, (2, 3, 2160, 3840)).astype(np.float32)
    gen = G.Generator(D, R, params=og.flatten(P, D, R).astype(np.float32))
    U, s, V, m = gen.forward(torch.from_numpy(x).cuda())
    rU, rs, rV, rm, _ = og.forward(P, x, D, R, mixed=True)
    for a, b, k in ((U, rU, "U"), (s, rs, "s"), (V, rV, "V"), (m, rm, "map")):
        rel_close(host(a), b, 2e-2, k)


def test_generator_backward_parity(svd, G):
    D, R = 33, 8
    P = random_params(D, R, 3)
    g = np.random.default_rng(4)
    x = g.uniform(0, 1, (2, 3, 256, 256)).astype(np.float32)
    gen = G.Generator(D, R, params=og.flatten(P, D, R).astype(np.float32))
    U, s, V, m = gen.forward(torch.from_numpy(x).cuda())
    dU, ds, dV, dm = (g.normal(0, 1, t.shape).astype(np.float32) for t in (U, s, V, m))
    grads = gen.backward(*(torch.from_numpy(a).cuda() for a in (dU, ds, dV, dm)))
    _, _, _, _, cache = og.forward(P, x, D, R, mixed=True)
    ref = og.backward(P, cache, dU, ds, dV, dm, mixed=True)
    got = og.unflatten(host(grads), D, R)
    for k in ref:
        rel_close(got[k], ref[k], 3e-2, k)


def test_generator_fp16_input(svd, G):
    g = np.random.default_rng(5)
    x = g.uniform(0, 1, (1, 3, 512, 384)).astype(np.float16)
    gen = G.Generator(33, 8, seed=3)
    a = gen.forward(torch.from_numpy(x).cuda())
    b = gen.forward(torch.from_numpy(x.astype(np.float32)).cuda())
    for u, v in zip(a, b):
        assert torch.equal(u, v)


def test_adam_parity(svd, G):
    g = np.random.default_rng(6)
    th = g.normal(size=1000).astype(np.float32)
    p = torch.from_numpy(th.copy()).cuda()
    opt = G.Adam(p, lr=1e-3)
    m = np.zeros(1000); v = np.zeros(1000); ref = th.astype(np.float64)
    for t in range(1, 8):
        gr = g.normal(size=1000).astype(np.float32)
        opt.step(torch.from_numpy(gr).cuda())
        ref, m, v = og.adam(ref, gr, m, v, t, lr=1e-3)
    assert np.abs(host(p) - ref).max() <= 1e-6


# ------------------------------------------------------------------ training
@pytest.fixture(scope="module")
def data(pair_data):
    return pair_data


def psnr(y, t):
    mse = torch.mean((y.float() - t.float()) ** 2).item()
    return 10 * math.log10(1.0 / mse)


STEPS, BATCH = 2000, 16


def train_generator(svd, G, data, steps=STEPS, seed=0):
    xtr, ttr, _, _ = data
    gen = G.Generator(33, 8, seed=seed)
    tr = G.Trainer(gen, lr=1e-4)
    g = np.random.default_rng(seed)
    for it in range(steps):
        idx = torch.from_numpy(g.integers(0, xtr.shape[0], BATCH)).cuda()
        tr.step(xtr.index_select(0, idx).contiguous(), ttr.index_select(0, idx).contiguous())
    torch.cuda.synchronize()
    return gen, tr


def eval_generator(svd, gen, data):
    _, _, xte, tte = data
    ys = [gen.enhance(xte[i:i + 16].contiguous()) for i in range(0, xte.shape[0], 16)]
    return psnr(torch.cat(ys), tte)


def train_fallback(svd, G, data, steps=STEPS, seed=0):
    """The method without the learned network: one global set of factors and a constant
    spatial map (shared by every image), fitted with the same Adam, loss and pairs."""
    xtr, ttr, _, _ = data
    D, R = 33, 8
    blk = G.identity_factor_block(D, R, np.random.default_rng(seed)).reshape(9, 2 * D * R + R)
    theta = torch.from_numpy(np.concatenate([blk.ravel(), np.ones(9)]).astype(np.float32)).cuda()
    opt = G.Adam(theta, lr=1e-4)
    g = np.random.default_rng(seed)

    def unpack(th, B):
        b = th[:9 * (2 * D * R + R)].view(9, 2 * D * R + R)
        U = b[:, :D * R].reshape(1, 9, D, R).expand(B, -1, -1, -1).contiguous()
        s = b[:, D * R:D * R + R].reshape(1, 9, R).expand(B, -1, -1).contiguous()
        V = b[:, D * R + R:].reshape(1, 9, D, R).expand(B, -1, -1, -1).contiguous()
        m = th[-9:].view(1, 9, 1, 1).expand(B, -1, -1, -1).contiguous()
        return U, s, V, m

    ws = svd.bwd_workspace(BATCH, D, "cuda")
    for it in range(steps):
        idx = torch.from_numpy(g.integers(0, xtr.shape[0], BATCH)).cuda()
        x = xtr.index_select(0, idx).contiguous()
        t = ttr.index_select(0, idx).contiguous()
        U, s, V, m = unpack(theta, BATCH)
        y = svd.apply(x, U, s, V, m)
        _, dy = svd.loss(y, t, "mse")
        r = svd.apply_bwd(x, dy, U, s, V, m, need_dx=False, ws=ws)
        grad = torch.cat([torch.cat([r["dU"].sum(0).reshape(9, -1), r["ds"].sum(0), r["dV"].sum(0).reshape(9, -1)], 1).ravel(),
                          r["dmap"].sum(dim=(0, 2, 3))])
        opt.step(grad.contiguous())
    torch.cuda.synchronize()
    _, _, xte, tte = data
    ys = []
    for i in range(0, xte.shape[0], 16):
        x = xte[i:i + 16].contiguous()
        U, s, V, m = unpack(theta, x.shape[0])
        ys.append(svd.apply(x, U, s, V, m))
    return psnr(torch.cat(ys), tte)


def test_training_gain_over_fixed_factors(svd, G, data):
    """Held-out PSNR: trained generator vs fixed-factor fallback vs doing nothing."""
    _, _, xte, tte = data
    p_id = psnr(xte, tte)
    t0 = time.time()
    gen, _ = train_generator(svd, G, data)
    t1 = time.time()
    p_gen = eval_generator(svd, gen, data)
    p_fb = train_fallback(svd, G, data)
    say(f"held-out PSNR: identity {p_id:.2f} dB, fixed-factor fallback {p_fb:.2f} dB, "
        f"generator {p_gen:.2f} dB ({STEPS} steps x {BATCH}, {t1 - t0:.1f}s)")
    assert p_gen > p_id
    assert p_gen >= p_fb + 1.0


def test_checkpoint_resume(svd, G, data, tmp_path):
    """N steps, save, reload into fresh objects, N more steps vs 2N uninterrupted, in
    deterministic mode: every reduction of the training step has a fixed order, so two
    uninterrupted runs and the resumed run end with bitwise the same parameters, and a run
    that did not load the checkpoint ends far from them."""
    was = svd.deterministic()
    svd.deterministic(True)
    try:
        _checkpoint_resume(svd, G, data, tmp_path)
    finally:
        svd.deterministic(was)


def _checkpoint_resume(svd, G, data, tmp_path):
    n = 20
    gen_a, _ = train_generator(svd, G, data, steps=2 * n, seed=7)
    gen_a2, _ = train_generator(svd, G, data, steps=2 * n, seed=7)
    gen_b, tr_b = train_generator(svd, G, data, steps=n, seed=7)
    path = os.path.join(tmp_path, "ckpt.npz")
    tr_b.save(path)
    gen_c = G.Generator(33, 8, seed=123)
    tr_c = G.Trainer(gen_c, lr=1e-4)
    tr_c.load(path)
    xtr, ttr, _, _ = data
    g = np.random.default_rng(7)
    for it in range(2 * n):
        idx = torch.from_numpy(g.integers(0, xtr.shape[0], BATCH)).cuda()
        if it >= n:
            tr_c.step(xtr.index_select(0, idx).contiguous(), ttr.index_select(0, idx).contiguous())
    torch.cuda.synchronize()
    a, a2, b, c = host(gen_a.params), host(gen_a2.params), host(gen_b.params), host(gen_c.params)
    assert tr_c.opt.t == 2 * n
    assert np.array_equal(a, a2), "two uninterrupted runs differ"
    assert np.array_equal(a, c), f"resumed run differs: max {np.abs(a - c).max():.3e}"
    assert np.abs(a - b).mean() > 1e-6
