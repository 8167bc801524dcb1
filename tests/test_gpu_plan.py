"""GPU parity of the uneven-batch persistent launch (svdlut_plan: HIP graph replay, argument
update, autotuner) against the oracle and against per-image svdlut_apply launches."""
import numpy as np
import pytest
import torch

import synth
from oracle import lut as ol

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def svd():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2508_16121_amd as m
    return m


def say(msg):
    print(msg, flush=True)


def small_batch(n=7, seed0=900, dtype=np.float16):
    bases = ((48, 64), (108, 192), (216, 384))
    images = [synth.uneven_image(i, seed0, 33, 8, bases) for i in range(n)]
    return synth.pack_uneven(images)


def run_plan(svd, packed, io=torch.float16, direct=False, plan=None):
    xf, mf, U, s, V, descs = packed
    x = torch.from_numpy(xf).cuda().to(io)
    m = torch.from_numpy(mf).cuda().to(io)
    y = torch.zeros_like(x)
    Ud, sd, Vd = (torch.from_numpy(a).cuda() for a in (U, s, V))
    plan = plan or svd.Plan(descs, 33, 8, io, io)
    (plan.launch_direct if direct else plan.launch)(x, y, Ud, sd, Vd, m)
    torch.cuda.synchronize()
    return plan, x, m, y, (Ud, sd, Vd)


def oracle_check(packed, x, m, y, tol, npx=None, seed=0):
    xf, mf, U, s, V, descs = packed
    xq = x.float().cpu().numpy().astype(np.float64)
    mq = m.float().cpu().numpy().astype(np.float64)
    yq = y.float().cpu().numpy().astype(np.float64)
    g = np.random.default_rng(seed)
    for b, d in enumerate(descs):
        H, W, h, w = d["H"], d["W"], d["h"], d["w"]
        xi = xq[d["x_off"]:d["x_off"] + 3 * H * W].reshape(3, H, W)
        mi = mq[d["map_off"]:d["map_off"] + 9 * h * w].reshape(9, h, w)
        yi = yq[d["y_off"]:d["y_off"] + 3 * H * W].reshape(3, H, W)
        T = ol.reconstruct(U[b], s[b], V[b])
        if npx is None:
            ref = ol.transform(xi, T, mi)
            err = np.abs(yi - ref).max()
        else:
            ys = np.concatenate([g.integers(0, H, npx), [0, H - 1, H - 1]])
            xs = np.concatenate([g.integers(0, W, npx), [0, W - 1, 0]])
            err = np.abs(yi[:, ys, xs] - ol.transform_at(xi, T, mi, ys, xs)).max()
        assert err <= tol, f"image {b} ({H}x{W}): {err}"


@pytest.mark.parametrize("io,tol", [(torch.float16, 2e-3), (torch.float32, 1e-5)])
def test_plan_small_uneven(svd, io, tol):
    packed = small_batch()
    say(f"plan small {io}")
    plan, x, m, y, f = run_plan(svd, packed, io)
    oracle_check(packed, x, m, y, tol)
    info = plan.info()
    assert info["pixels"] == sum(d["H"] * d["W"] for d in packed[5])
    assert info["graph"] == 1


def test_plan_graph_replay_with_new_buffers(svd):
    packed = small_batch(5, 950)
    plan, x, m, y, (U, s, V) = run_plan(svd, packed)
    # second set of buffers: different content, same shapes -> kernel arguments updated in the graph
    x2 = torch.rand_like(x.float()).to(x.dtype)
    y2 = torch.zeros_like(y)
    U2 = U * 0.5
    plan.launch(x2, y2, U2, s, V, m)
    plan.launch(x2, y2, U2, s, V, m)      # replay with unchanged arguments
    torch.cuda.synchronize()
    xf, mf, Uh, sh, Vh, descs = packed
    oracle_check((xf, mf, Uh * 0.5, sh, Vh, descs), x2, m, y2, 2e-3)
    # the first buffers again, compared bit for bit with the plain launch
    y3 = torch.zeros_like(y)
    plan.launch(x, y3, U, s, V, m)
    y4 = torch.zeros_like(y)
    plan.launch_direct(x, y4, U, s, V, m)
    torch.cuda.synchronize()
    assert torch.equal(y3, y) and torch.equal(y4, y)


def test_plan_autotune(svd, tmp_path, monkeypatch):
    monkeypatch.setenv("SVDLUT_TUNE_CACHE", str(tmp_path / "tune.json"))
    packed = small_batch(6, 970)
    plan, x, m, y, (U, s, V) = run_plan(svd, packed)
    plan.autotune(x, y, U, s, V, m)
    y2 = torch.zeros_like(y)
    plan.launch(x, y2, U, s, V, m)
    torch.cuda.synchronize()
    assert plan.info()["tuned"] == 1
    oracle_check(packed, x, m, y2, 2e-3)


def test_plan_fp16_per_pixel_maps_autotune(svd, tmp_path, monkeypatch):
    # maps finer than a third of their images (per-pixel map columns) with half-precision
    # I/O: default shape and every autotune candidate stay within the variant's 512 threads
    monkeypatch.setenv("SVDLUT_TUNE_CACHE", str(tmp_path / "tune.json"))
    g = synth.rng(990)
    images = []
    for (H, W, h, w) in [(40, 70, 30, 50), (64, 150, 64, 150), (96, 130, 20, 60)]:
        x = synth.image(g, H, W)
        U, s, V = synth.factors(g, 1, 33, 8)
        m = synth.spatial_map(g, 1, h, w)
        images.append((x, U[0], s[0], V[0], m[0]))
    packed = synth.pack_uneven(images)
    say("plan fp16 per-pixel maps")
    plan, x, m, y, (U, s, V) = run_plan(svd, packed)
    assert plan.info()["block"] <= 512
    oracle_check(packed, x, m, y, 2e-3)
    plan.autotune(x, y, U, s, V, m)
    assert plan.info()["tuned"] == 1 and plan.info()["block"] <= 512
    y2 = torch.zeros_like(y)
    plan.launch(x, y2, U, s, V, m)
    torch.cuda.synchronize()
    oracle_check(packed, x, m, y2, 2e-3)


def test_plan_full_uneven_batch_sampled(svd):
    """64 images of uneven size (480x640, 1080x1920, 2160x3840 bases, +-10% width jitter),
    fp16 storage, own D=33 R=8 factors and 1/8-resolution maps: one graph-replayed launch,
    equal bit for bit to 64 separate svdlut_apply launches and within 2e-3 of the oracle on
    sampled pixels of every image."""
    say("c3: generating 64 images")
    images = synth.uneven_batch(64, workers=16)
    packed = synth.pack_uneven(images)
    del images
    plan, x, m, y, (U, s, V) = run_plan(svd, packed)
    descs = packed[5]
    y_loop = torch.zeros_like(y)
    for b, d in enumerate(descs):
        H, W, h, w = d["H"], d["W"], d["h"], d["w"]
        xi = x[d["x_off"]:d["x_off"] + 3 * H * W].view(1, 3, H, W)
        mi = m[d["map_off"]:d["map_off"] + 9 * h * w].view(1, 9, h, w)
        yi = y_loop[d["y_off"]:d["y_off"] + 3 * H * W].view(1, 3, H, W)
        svd.apply(xi, U[b:b + 1], s[b:b + 1], V[b:b + 1], mi, out=yi)
    torch.cuda.synchronize()
    assert torch.equal(y, y_loop)
    oracle_check(packed, x, m, y, 2e-3, npx=300)
