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
    assert (info["tile_px"], info["px_per_lane"]) == (256, 4)
    assert info["tiles"] == sum(d["H"] * -(-d["W"] // 256) for d in packed[5])
    assert 1 <= info["blocks_per_cu"] <= 32


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


_CHILD = r'''
import json, sys
import numpy as np, torch
import synth
import paper_2508_16121_amd as svd
out, autotune = sys.argv[1], sys.argv[2] == "1"
bases = ((48, 64), (108, 192), (216, 384))
images = [synth.uneven_image(i, 960, 33, 8, bases) for i in range(5)]
xf, mf, U, s, V, descs = synth.pack_uneven(images)
x = torch.from_numpy(xf).cuda().half(); m = torch.from_numpy(mf).cuda().half()
Ud, sd, Vd = (torch.from_numpy(a).cuda() for a in (U, s, V))
plan = svd.Plan(descs, 33, 8, torch.float16, torch.float16)
info0 = plan.info()
if autotune:
    plan.autotune(x, torch.zeros_like(x), Ud, sd, Vd, m)
y = torch.zeros_like(x); plan.launch(x, y, Ud, sd, Vd, m)
y2 = torch.zeros_like(x); plan.launch_direct(x, y2, Ud, sd, Vd, m)
torch.cuda.synchronize()
np.save(out + ".npy", y.cpu().numpy())
json.dump({"before": info0, "after": plan.info(), "direct_equal": bool(torch.equal(y, y2))}, open(out + ".json", "w"))
print("child done", flush=True)
'''


def _child(tmp_path, name, env_extra, autotune=False):
    """Run one plan in a fresh process (the library reads SVDLUT_TUNE_CACHE and
    SVDLUT_NO_GRAPH at first use) and return its info and output."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ)
    for k in ("SVDLUT_TUNE_CACHE", "SVDLUT_NO_GRAPH"):
        env.pop(k, None)
    env.update(env_extra)
    out = str(tmp_path / name)
    say(f"plan child {name}: {env_extra} autotune={autotune}")
    r = subprocess.run([sys.executable, "-c", _CHILD, out, "1" if autotune else "0"], cwd=root, env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    return json.load(open(out + ".json")), np.load(out + ".npy")


def test_plan_fallbacks_and_tuning_cache(tmp_path):
    """The plan's fallbacks, each in a fresh process: SVDLUT_NO_GRAPH gives plain launches
    (graph = 0) with the same output bit for bit; a missing cache file leaves the default
    shape and autotune writes a valid one; a later process takes its shape from that file
    without tuning; a corrupt file, or an entry with values out of range, is ignored (the
    default shape, the same output) and autotune replaces it with valid JSON.  The output is
    the same bit for bit in every case with 4 pixels per lane (the workgroup shape changes no
    pixel's arithmetic); a tuned 8-pixel tile agrees to rounding."""
    import json
    base, y_ref = _child(tmp_path, "graph", {})
    assert base["before"]["graph"] == 1 or base["after"]["graph"] == 1
    assert base["direct_equal"]
    # no graph
    nog, y = _child(tmp_path, "nograph", {"SVDLUT_NO_GRAPH": "1"})
    assert nog["after"]["graph"] == 0 and nog["direct_equal"]
    assert np.array_equal(y, y_ref)
    # missing cache file: default shape, autotune creates the file
    cache = tmp_path / "cache.json"
    miss, y = _child(tmp_path, "missing", {"SVDLUT_TUNE_CACHE": str(cache)}, autotune=True)
    assert miss["before"]["tuned"] == 0 and miss["after"]["tuned"] == 1
    assert miss["before"]["block"] == base["before"]["block"]
    assert (base["before"]["px_per_lane"], base["before"]["tile_px"]) == (4, 256)
    entries = json.load(open(cache))
    assert len(entries) == 1
    key, (blk, bpc, px) = next(iter(entries.items()))
    assert blk in (64, 128, 256, 512, 1024) and 1 <= bpc <= 32 and px in (4, 8)
    assert (miss["after"]["block"], miss["after"]["blocks_per_cu"], miss["after"]["px_per_lane"]) == (blk, bpc, px)
    assert miss["after"]["tile_px"] == 64 * px

    def same_output(y):
        # 4 pixels per lane: bit for bit; 8: the map weights come from other staged columns
        if px == 4:
            np.testing.assert_array_equal(y, y_ref)
        else:
            np.testing.assert_allclose(y.astype(np.float32), y_ref.astype(np.float32), rtol=0, atol=2e-3)
    same_output(y)
    # the cached shape is used by the next process without tuning
    hit, y = _child(tmp_path, "hit", {"SVDLUT_TUNE_CACHE": str(cache)})
    assert hit["before"]["tuned"] == 1 and hit["before"]["block"] == blk
    assert hit["before"]["px_per_lane"] == px and hit["before"]["blocks_per_cu"] == bpc
    assert hit["direct_equal"]
    same_output(y)
    # an older two-value entry still reads as 4 pixels per lane
    cache.write_text(json.dumps({key: [blk if blk <= 512 else 512, 1]}))
    old, y = _child(tmp_path, "two_values", {"SVDLUT_TUNE_CACHE": str(cache)})
    assert old["before"]["tuned"] == 1 and old["before"]["px_per_lane"] == 4
    np.testing.assert_array_equal(y, y_ref)
    # corrupt files and out-of-range values are ignored
    for name, text in (("garbage", "\x00\xffnot json{{{["), ("truncated", '{"' + key + '": [51'),
                       ("range", json.dumps({key: [999, 2]})), ("types", json.dumps({key: ["512", "x"]})),
                       ("px", json.dumps({key: [512, 1, 6]})), ("extra", json.dumps({key: [512, 1, 8, 1]}))):
        cache.write_bytes(text.encode("latin-1"))
        bad, y = _child(tmp_path, name, {"SVDLUT_TUNE_CACHE": str(cache)}, autotune=(name == "garbage"))
        assert bad["before"]["tuned"] == 0, name
        assert bad["before"]["block"] == base["before"]["block"], name
        if name == "garbage":
            fixed = json.load(open(cache))          # rewritten as valid JSON
            assert list(fixed) == [key], fixed
        np.testing.assert_array_equal(y, y_ref)


def test_plan_degenerate_images(svd):
    """A batch mixing degenerate images — a single pixel, a single row, a single column, a
    1 x 1 map, a per-pixel map, widths that are not multiples of 4 — in one plan (fp32): every
    pixel against the oracle, and the plain launch bit for bit equal to the graph replay."""
    g = synth.rng(4242)
    specs = [(1, 1, 1, 1), (1, 300, 1, 7), (257, 1, 9, 1), (33, 65, 1, 1), (40, 70, 40, 70), (7, 518, 3, 65),
             (64, 256, 8, 32)]
    images = []
    for (H, W, h, w) in specs:
        x = synth.image(g, H, W)
        U, s, V = synth.factors(g, 1, 33, 8)
        m = synth.spatial_map(g, 1, h, w)
        images.append((x, U[0], s[0], V[0], m[0]))
    packed = synth.pack_uneven(images)
    say("plan degenerate images")
    plan, x, m, y, (U, s, V) = run_plan(svd, packed, io=torch.float32)
    oracle_check(packed, x, m, y, 1e-5)
    y2 = torch.zeros_like(y)
    plan.launch_direct(x, y2, U, s, V, m)
    torch.cuda.synchronize()
    assert torch.equal(y, y2)
    info = plan.info()
    assert info["pixels"] == sum(H * W for (H, W, _, _) in specs)


# (H, W, h, w): rows of 4 and 516 pixels are 4-aligned, but their last 512-pixel segment holds
# fewer than 8 pixels, so they take the element path
WIDE_SPECS = [(1, 4, 1, 1), (3, 5, 2, 1), (9, 7, 3, 1), (16, 8, 2, 2), (5, 9, 2, 2), (17, 13, 3, 2),
              (12, 100, 2, 13), (7, 511, 1, 64), (6, 513, 2, 65), (3, 516, 1, 65), (40, 1000, 5, 125),
              (64, 256, 8, 32), (2, 1024, 1, 128)]


def _images(specs, seed):
    g = synth.rng(seed)
    images = []
    for (H, W, h, w) in specs:
        x = synth.image(g, H, W)
        U, s, V = synth.factors(g, 1, 33, 8)
        m = synth.spatial_map(g, 1, h, w)
        images.append((x, U[0], s[0], V[0], m[0]))
    return synth.pack_uneven(images)


@pytest.mark.parametrize("io,tol,agree", [(torch.float32, 1e-5, 2e-6), (torch.float16, 2e-3, 2e-3)])
def test_plan_wide_tiles(svd, io, tol, agree):
    """8 pixels per lane (512-pixel tiles), set by hand on a batch of ragged and short rows
    (widths 4 to 1024, most not multiples of 8, 4-aligned rows shorter than 8) whose maps
    allow it ((8-1)(w-1) <= W-1): every pixel against the oracle, the 4-pixel tiles to
    rounding, the graph replay equal to the plain launch, and the info fields."""
    packed = _images(WIDE_SPECS, 5150)
    say(f"plan wide tiles {io}")
    descs = packed[5]
    assert all(7 * (d["w"] - 1) <= d["W"] - 1 for d in descs)
    plan4 = svd.Plan(descs, 33, 8, io, io)
    plan4.set_shape(512, 1, 4)
    _, x, m, y4, (U, s, V) = run_plan(svd, packed, io, plan=plan4)
    plan8 = svd.Plan(descs, 33, 8, io, io)
    plan8.set_shape(512, 1, 8)
    info = plan8.info()
    assert (info["px_per_lane"], info["tile_px"], info["block"], info["blocks_per_cu"]) == (8, 512, 512, 1)
    assert info["tiles"] == sum(d["H"] * -(-d["W"] // 512) for d in descs)
    _, _, _, y8, _ = run_plan(svd, packed, io, plan=plan8)
    assert plan8.info()["graph"] == 1
    y8d = torch.zeros_like(y8)
    plan8.launch_direct(x, y8d, U, s, V, m)
    torch.cuda.synchronize()
    assert torch.equal(y8, y8d)
    oracle_check(packed, x, m, y8, tol)
    assert (y8.float() - y4.float()).abs().max().item() <= agree
    # back to 4 pixels per lane on the same plan: the graph is captured again, bit for bit
    # what a 4-pixel plan gives
    plan8.set_shape(512, 1, 4)
    y44 = torch.zeros_like(y8)
    plan8.launch(x, y44, U, s, V, m)
    torch.cuda.synchronize()
    assert torch.equal(y44, y4)


def test_plan_set_shape_refusals(svd):
    """Shapes a batch cannot run are refused and leave the plan as it was: values outside the
    sets (EINVAL), 8 pixels per lane with a map too fine for it or with more than 512 threads,
    and more workgroups per CU than the LDS holds (EUNSUPPORTED)."""
    packed = _images([(20, 40, 20, 40), (8, 64, 1, 8)], 5160)     # the first map is per-pixel
    plan = svd.Plan(packed[5], 33, 8, torch.float32, torch.float32)
    before = plan.info()
    for args, what in (((512, 1, 6), "px_per_lane"), ((500, 1, 4), "block"), ((512, 0, 4), "block"),
                       ((512, 33, 4), "block"), ((256, 1, 8), "not supported"), ((512, 32, 4), "not supported")):
        with pytest.raises(svd.SvdlutError, match=what):
            plan.set_shape(*args)
        assert plan.info() == before, args
    coarse = svd.Plan(_images([(8, 64, 1, 8)], 5161)[5], 33, 8, torch.float32, torch.float32)
    with pytest.raises(svd.SvdlutError, match="not supported"):
        coarse.set_shape(1024, 1, 8)               # 8-pixel variants are built for 512 threads
    coarse.set_shape(256, 2, 8)
    assert coarse.info()["px_per_lane"] == 8
