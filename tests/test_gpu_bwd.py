"""GPU parity of the backward 2D-LUT apply (dU, ds, dV, dmap, dx, dbias), the loss kernel and
the autograd wrapper, against the fp64 oracle and central finite differences."""
import numpy as np
import pytest
import torch

import synth
from oracle import lut as ol
from sum_bounds import order_bars, within

pytestmark = pytest.mark.gpu


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


def close(got, ref, rel=1e-4, what=""):
    """Sums of many float32 atomic contributions: max-abs error within rel of the largest entry."""
    scale = max(np.abs(ref).max(), 1e-30)
    err = np.abs(got - ref).max()
    assert err <= rel * scale, f"{what}: max-abs {err:.3e} vs scale {scale:.3e}"


def dx_bound(G, m, U, s, V, D):
    """Max-abs bound for dx (a per-pixel float32 result with no atomics), derived from its
    arithmetic: dx_a = (D-1) * sum of the six (pair, output channel) terms containing channel
    a, each G_c * S_l * ((1-d)(T10-T00) + d(T11-T01)).  A term takes at most about ten float32
    roundings (the map interpolation, the bracket, the products; relative u = 2^-24 each),
    the six-term sum and the (D-1) factor a few more, so
        |dx_gpu - dx| <= (D-1) * 6 * max|G| * max|S| * max|dT| * 16u
    with |S| <= max|map| and dT the largest difference of neighbouring LUT entries."""
    T = ol.reconstruct(U, s, V)
    dT = max(np.abs(np.diff(T, axis=-1)).max(), np.abs(np.diff(T, axis=-2)).max())
    return (D - 1) * 6 * np.abs(G).max() * np.abs(m).max() * dT * 16 * 2.0 ** -24


def dx_bar(G, m, U, s, V, D):
    """The bound above, asserted to be within 1e-5 (fp32 dx held to 1e-5 max-abs): the small
    cases draw |G| <= 1/4, map values in [0, 1] and factors with |dT| < 0.3."""
    bound = dx_bound(G, m, U, s, V, D)
    assert bound <= 1e-5, bound
    return bound


@pytest.mark.parametrize("shape", [
    (2, 40, 70, 5, 3, 6, 9),       # small LUT, map columns blended piecewise per lane
    (2, 40, 70, 5, 3, 30, 40),     # map finer than a third of the image: per-pixel map columns
    (1, 33, 300, 33, 8, 5, 38),    # two segments, ragged
    (3, 64, 64, 17, 4, 8, 8),      # batch of three
    (1, 1, 1, 9, 2, 1, 1),         # single pixel
    (1, 16, 515, 33, 8, 1, 65),    # one map row
    (2, 48, 530, 33, 8, 1, 1),     # a 1 x 1 map (scalar LUT weights): each wave sums its lanes' terms
    (1, 40, 300, 17, 4, 5, 1),     # one map column over several rows
])
def test_backward_parity_small(svd, shape):
    B, H, W, D, R, h, w = shape
    say(f"bwd {shape}")
    g = np.random.default_rng(sum(shape) + 7)
    x = g.uniform(-0.05, 1.05, (B, 3, H, W)).astype(np.float32)
    U, s, V = synth.factors(g, B, D, R)
    m = synth.spatial_map(g, B, h, w)
    G = g.uniform(-0.25, 0.25, (B, 3, H, W)).astype(np.float32)
    r = svd.apply_bwd(dev(x), dev(G), dev(U), dev(s), dev(V), dev(m), need_bias=True)
    ref = ol.apply_bwd(x, U, s, V, m, G)
    for k in ("dU", "ds", "dV", "dmap", "db"):
        close(host(r[k]), ref[k], 1e-4, k)
    dx = host(r["dx"])
    assert np.abs(dx - ref["dx"]).max() <= dx_bar(G, m, U, s, V, D)
    outside = (x < 0) | (x > 1)
    assert np.all(dx[outside] == 0.0)


@pytest.mark.parametrize("hw", [(2, 2), (1, 1)])
def test_backward_fine_maps_at_d33(svd, hw):
    """Maps at half and at full image resolution with 33x33 LUTs: their per-wave staging
    needs narrow workgroups (the launch picks 128 or 64 threads) but the result is the same
    definition."""
    fh, fw = hw
    B, H, W, D, R = 1, 48, 300, 33, 8
    h, w = H // fh, W // fw
    say(f"bwd fine map {h}x{w}")
    g = np.random.default_rng(77 + fw)
    x = g.uniform(-0.05, 1.05, (B, 3, H, W)).astype(np.float32)
    U, s, V = synth.factors(g, B, D, R)
    m = synth.spatial_map(g, B, h, w)
    G = g.uniform(-0.25, 0.25, (B, 3, H, W)).astype(np.float32)
    r = svd.apply_bwd(dev(x), dev(G), dev(U), dev(s), dev(V), dev(m), need_bias=True)
    ref = ol.apply_bwd(x, U, s, V, m, G)
    for k in ("dU", "ds", "dV", "dmap", "db"):
        close(host(r[k]), ref[k], 1e-4, k)
    assert np.abs(host(r["dx"]) - ref["dx"]).max() <= dx_bar(G, m, U, s, V, D)


def test_backward_map_staging_limit(svd):
    """Per-pixel maps: at D = 36 the 64-thread workgroup still stages a segment's 259 map
    columns next to T and dT (parity as usual); at D = 40 they do not fit the LDS and the call
    is refused with EUNSUPPORTED and a message, not launched."""
    B, H, W, R = 1, 24, 300, 8
    g = np.random.default_rng(1234)
    x = g.uniform(-0.05, 1.05, (B, 3, H, W)).astype(np.float32)
    G = g.uniform(-0.25, 0.25, (B, 3, H, W)).astype(np.float32)
    m = synth.spatial_map(g, B, H, W)
    U, s, V = synth.factors(g, B, 36, R)
    say("bwd per-pixel map at D=36")
    r = svd.apply_bwd(dev(x), dev(G), dev(U), dev(s), dev(V), dev(m), need_bias=True)
    ref = ol.apply_bwd(x, U, s, V, m, G)
    for k in ("dU", "ds", "dV", "dmap", "db"):
        close(host(r[k]), ref[k], 1e-4, k)
    U, s, V = synth.factors(g, B, 40, R)
    say("bwd per-pixel map at D=40: refused")
    with pytest.raises(svd.SvdlutError, match="do not fit the LDS"):
        svd.apply_bwd(dev(x), dev(G), dev(U), dev(s), dev(V), dev(m))


def test_backward_subsets_and_overwrite(svd):
    """Only the requested gradients are produced, and a second call overwrites (no accumulation)."""
    c = synth.single(31, 48, 96, 9, 3, 6, 12)
    G = np.random.default_rng(1).normal(size=c.x.shape).astype(np.float32)
    args = [dev(a) for a in (c.x, G, c.U, c.s, c.V, c.smap)]
    r1 = svd.apply_bwd(*args, need_dx=False, need_factors=True, need_map=False)
    assert set(r1) == {"dU", "ds", "dV"}
    r2 = svd.apply_bwd(*args, need_dx=False, need_factors=True, need_map=False)
    assert np.array_equal(host(r1["ds"]), host(r2["ds"]))
    r3 = svd.apply_bwd(*args, need_dx=True, need_factors=False, need_map=True)
    assert set(r3) == {"dx", "dmap"}
    ref = ol.apply_bwd(c.x, c.U, c.s, c.V, c.smap, G)
    close(host(r3["dmap"]), ref["dmap"], 1e-4, "dmap")
    close(host(r1["dU"]), ref["dU"], 1e-4, "dU")


def test_loss_kernels(svd):
    g = np.random.default_rng(2)
    y = g.normal(size=(2, 3, 37, 41)).astype(np.float32)
    t = g.normal(size=y.shape).astype(np.float32)
    t[0, 0, 0, :5] = y[0, 0, 0, :5]
    for kind, fn in (("l1", ol.l1_loss), ("mse", ol.mse_loss)):
        v, dy = svd.loss(dev(y), dev(t), kind)
        rv, rdy = fn(y, t)
        assert abs(host(v)[0] - rv) <= 1e-5 * max(1.0, abs(rv))
        assert np.abs(host(dy) - rdy).max() <= 1e-6 * np.abs(rdy).max()


def test_loss_kernels_fp16_and_unaligned(svd):
    """fp16 storage (8-byte vector path) and buffers that start off a 16-byte boundary (the
    element path), each with a ragged tail of n mod 4 elements."""
    g = np.random.default_rng(3)
    n = 4 * 1234 + 3
    y = g.uniform(0, 1, n + 1).astype(np.float32)
    t = g.uniform(0, 1, n + 1).astype(np.float32)
    for kind, fn in (("l1", ol.l1_loss), ("mse", ol.mse_loss)):
        yd, td = dev(y)[1:], dev(t)[1:]                      # 4-byte offset: not 16-byte aligned
        v, dy = svd.loss(yd, td, kind)
        rv, rdy = fn(y[1:], t[1:])
        assert abs(host(v)[0] - rv) <= 1e-5 * max(1.0, abs(rv))
        assert np.abs(host(dy) - rdy).max() <= 1e-6 * np.abs(rdy).max()
        yh, th = y[:n].astype(np.float16), t[:n].astype(np.float16)
        v, dy = svd.loss(dev(yh), dev(th), kind)
        rv, rdy = fn(yh.astype(np.float64), th.astype(np.float64))
        assert abs(host(v)[0] - rv) <= 1e-4 * max(1.0, abs(rv))
        assert np.abs(host(dy) - rdy).max() <= 2e-3 * np.abs(rdy).max()


@pytest.mark.parametrize("kind,io,shape,with_bias", [("l1", torch.float32, (2, 37, 70, 17, 4, 6, 9), True),
                                                      ("mse", torch.float32, (3, 64, 300, 33, 8, 8, 38), False),
                                                      ("mse", torch.float32, (1, 21, 513, 33, 8, 3, 65), True),
                                                      ("l1", torch.float16, (2, 40, 128, 33, 8, 5, 16), True)])
def test_fused_loss_backward_matches_separate_passes(svd, kind, io, shape, with_bias):
    """svdlut_apply_loss_bwd against svdlut_apply + svdlut_loss + svdlut_apply_bwd on the same
    inputs: the loss to float rounding, the gradients to the fixed-point bar (fp32) or to the
    fp16 rounding of the separately stored dL/dY (fp16)."""
    B, H, W, D, R, h, w = shape
    c = synth.single(sum(shape), H, W, D, R, h, w)
    g = np.random.default_rng(sum(shape) + 1)
    x = np.concatenate([c.x] * B).astype(np.float32)
    x += g.normal(0, 0.02, x.shape).astype(np.float32) * (np.arange(B)[:, None, None, None] > 0)
    tgt = np.clip(x + g.normal(0, 0.1, x.shape), -0.05, 1.05).astype(np.float32)
    U, s_, V, m = (np.concatenate([a] * B) for a in (c.U, c.s, c.V, c.smap))
    bias = g.normal(0, 0.1, (B, 3)).astype(np.float32) if with_bias else None
    dx_, tg = dev(x, io), dev(tgt, io)
    Ud, sd, Vd, md = dev(U), dev(s_), dev(V), dev(m)
    bd = dev(bias) if with_bias else None
    f = svd.apply_loss_bwd(dx_, tg, Ud, sd, Vd, md, bias=bd, kind=kind, need_bias=True)
    y = svd.apply(dx_, Ud, sd, Vd, md, bias=bd)
    lv, dy = svd.loss(y, tg, kind)
    r = svd.apply_bwd(dx_, dy, Ud, sd, Vd, md, need_bias=True)
    assert abs(host(f["loss"])[0] - host(lv)[0]) <= 2e-6 * abs(host(lv)[0])
    # L1 kinks: where |Y - t| is at rounding level the two paths may take different signs; dx
    # is compared away from them (the accumulated gradients absorb a single pixel)
    yh, th = host(y), host(tg)
    off_kink = np.abs(yh - th) > 1e-5 if kind == "l1" else np.ones(yh.shape, bool)
    tol = 1e-4 if io == torch.float32 else 3e-3
    for k in ("dU", "ds", "dV", "dmap", "db"):
        close(host(f[k]), host(r[k]), tol, k)
    close(host(f["dx"]) * off_kink, host(r["dx"]) * off_kink, tol, "dx")
    # and the loss and gradients against the fp64 oracle (fp32 storage only: dL/dY from the oracle's own Y)
    if io == torch.float32:
        ry = ol.apply(x, U, s_, V, m, bias)
        rl, G = (ol.l1_loss if kind == "l1" else ol.mse_loss)(ry, tgt)
        assert abs(host(f["loss"])[0] - rl) <= 1e-5 * abs(rl)
        ref = ol.apply_bwd(x, U, s_, V, m, G)
        for k in ("dU", "ds", "dV", "dmap"):
            close(host(f[k]), ref[k], 1e-4, k)
        ok = off_kink & ((np.abs(ry - tgt) > 1e-5) if kind == "l1" else True)
        # dx bound of the backward's arithmetic, plus (MSE) what the kernel's own dL/dY adds:
        # it is formed from the kernel's Y, within 1e-5 of the oracle's, so |dG| <= 2e-5 / n
        n = x.size
        dG = 2e-5 / n if kind == "mse" else 0.0
        T = ol.reconstruct(U, s_, V)
        dTm = max(np.abs(np.diff(T, axis=-1)).max(), np.abs(np.diff(T, axis=-2)).max())
        bound = dx_bound(G, m, U, s_, V, D) + (D - 1) * 6 * dG * np.abs(m).max() * dTm
        assert np.abs((host(f["dx"]) - ref["dx"]) * ok).max() <= bound


def test_fused_loss_backward_nonfinite_and_reproducible(svd):
    c = synth.single(77, 32, 96, 17, 4, 4, 12)
    x, U, s_, V, m = (dev(a) for a in (c.x, c.U, c.s, c.V, c.smap))
    t = torch.rand_like(x)
    a = svd.apply_loss_bwd(x, t, U, s_, V, m, kind="mse")
    b = svd.apply_loss_bwd(x, t, U, s_, V, m, kind="mse")
    # the loss, dx and the factor gradients are reproducible bit for bit; dmap is summed
    # across workgroups with float atomics (bitwise only in the deterministic mode)
    for k in ("loss", "dx", "dU", "ds", "dV"):
        assert torch.equal(a[k], b[k]), k
    # dL/dY of the MSE, 2 (Y - t) / n, from the oracle's forward on the same inputs
    Y = ol.apply(c.x, c.U, c.s, c.V, c.smap)
    G = 2.0 * (Y - host(t)) / Y.size
    assert within(host(a["dmap"]), host(b["dmap"]), order_bars(c.x, c.U, c.s, c.V, c.smap, G)["dmap"])
    t[0, 1, 3, 5] = float("nan")
    r = svd.apply_loss_bwd(x, t, U, s_, V, m, kind="mse")
    assert torch.isnan(r["loss"]).all() and torch.isnan(r["dU"]).any()
    r = svd.apply_loss_bwd(x, t, U, s_, V, m, kind="l1")           # sign(NaN) = 0, as in svdlut_loss
    assert torch.isnan(r["loss"]).all() and torch.isfinite(r["dU"]).all()


def test_autograd_matches_apply_bwd(svd):
    c = synth.single(41, 40, 72, 17, 4, 5, 9)
    x, U, s, V, m = (dev(a).requires_grad_() for a in (c.x, c.U, c.s, c.V, c.smap))
    y = svd.apply_autograd(x, U, s, V, m)
    G = torch.randn_like(y)
    (y * G).sum().backward()
    ref = ol.apply_bwd(c.x, c.U, c.s, c.V, c.smap, host(G))
    close(host(U.grad), ref["dU"], 1e-4, "dU")
    close(host(s.grad), ref["ds"], 1e-4, "ds")
    close(host(V.grad), ref["dV"], 1e-4, "dV")
    close(host(m.grad), ref["dmap"], 1e-4, "dmap")
    assert np.abs(host(x.grad) - ref["dx"]).max() <= dx_bound(host(G), c.smap, c.U, c.s, c.V, c.U.shape[2])


# ------------------------------------------------------------------ full-size differentiation batch
@pytest.fixture(scope="module")
def c4(svd):
    """16 x 3 x 512 x 512 fp32, D=33 R=8, 64x64 map, L1 against a seeded target: GPU forward,
    loss and backward in the launch configuration the benchmark times."""
    say("c4: generating inputs")
    c = synth.diff_batch()
    d = {k: dev(getattr(c, k)) for k in ("x", "U", "s", "V", "smap", "target")}
    y = svd.apply(d["x"], d["U"], d["s"], d["V"], d["smap"])
    loss, dy = svd.loss(y, d["target"], "l1")
    r = svd.apply_bwd(d["x"], dy, d["U"], d["s"], d["V"], d["smap"])
    out = {k: host(v) for k, v in r.items()}
    out["y"] = host(y)
    out["loss"] = float(host(loss)[0])
    return c, out


def _oracle_grad_one(c, b, N):
    T = ol.reconstruct(c.U[b], c.s[b], c.V[b])
    Y = ol.transform(c.x[b], T, c.smap[b])
    G = np.sign(Y - c.target[b]) / N
    r = ol.transform_bwd(c.x[b], T, c.smap[b], G)
    dU, ds, dV = ol.factor_grads(r["dT"], c.U[b], c.s[b], c.V[b])
    return Y, dict(dU=dU, ds=ds, dV=dV, dmap=r["dmap"], dx=r["dx"])


def test_c4_forward_and_loss(c4):
    c, out = c4
    N = c.x.size
    g = np.random.default_rng(44)
    tot = 0.0
    for b in range(c.x.shape[0]):
        T = ol.reconstruct(c.U[b], c.s[b], c.V[b])
        ys = g.integers(0, 512, 500); xs = g.integers(0, 512, 500)
        ref = ol.transform_at(c.x[b], T, c.smap[b], ys, xs)
        assert np.abs(out["y"][b][:, ys, xs] - ref).max() <= 1e-5
    Y0 = ol.apply(c.x[:2], c.U[:2], c.s[:2], c.V[:2], c.smap[:2])
    assert np.abs(out["y"][:2] - Y0).max() <= 1e-5
    tot = np.abs(out["y"].astype(np.float64) - c.target).sum() / N
    assert abs(out["loss"] - tot) <= 1e-5 * tot


@pytest.mark.parametrize("b", [0, 15])
def test_c4_gradients_match_oracle(c4, b):
    c, out = c4
    say(f"c4 oracle gradients, image {b}")
    Y, ref = _oracle_grad_one(c, b, c.x.size)
    for k in ("dU", "ds", "dV", "dmap"):
        close(out[k][b], ref[k], 1e-4, k)
    # dx per pixel to the bound of its arithmetic, away from the L1 kinks (|Y - t| at the
    # forward's rounding level, where the two sides may take different signs)
    G = np.sign(Y - c.target[b]) / c.x.size
    ok = np.abs(Y - c.target[b]) > 1e-6
    bound = dx_bound(G, c.smap[b], c.U[b:b + 1], c.s[b:b + 1], c.V[b:b + 1], c.U.shape[2])
    assert np.abs((out["dx"][b] - ref["dx"]) * ok).max() <= bound


def test_c4_finite_differences(c4):
    """Central differences (h = 1e-3) of the fp64 oracle's forward + L1 loss on image 0:
    40 coordinates each of U, s, V, map and x, 200 in all (seed 4).  x coordinates lie more
    than 2h(D-1) from a LUT knot and more than 2h from 0 and 1.  Only the pixels a
    coordinate influences are re-evaluated (the others cancel exactly in the difference).
    Tolerance |g - g_fd| <= 1e-3 max|g_fd| + 1e-2 |g_fd| per kind."""
    c, out = c4
    b, h = 0, 1e-3
    N = c.x.size
    x, U, s, V, m, tgt = c.x[b], c.U[b], c.s[b], c.V[b], c.smap[b], c.target[b]
    D = U.shape[1]
    H, W = x.shape[1:]
    hm, wm = m.shape[1:]
    g = np.random.default_rng(4)
    dec = [ol.decode(x[a], D)[0] for a in range(3)]
    allys, allxs = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")

    def loss_at(T, mm, xx, ys, xs):
        Y = ol.transform_at(xx, T, mm, ys, xs)
        return np.abs(Y - tgt[:, ys, xs]).sum() / N

    def fd_factor(kind, l, i, k):
        cp = {"U": U.copy(), "s": s.copy(), "V": V.copy()}
        if kind == "U":
            a = ol.PAIRS[l % 3][0]; sel = (dec[a] == i) | (dec[a] == i - 1)
        elif kind == "V":
            bb = ol.PAIRS[l % 3][1]; sel = (dec[bb] == i) | (dec[bb] == i - 1)
        else:
            sel = np.ones((H, W), bool)
        ys, xs = allys[sel], allxs[sel]
        vals = []
        for sgn in (1, -1):
            q = {k2: v.copy() for k2, v in cp.items()}
            if kind == "s":
                q["s"][l, k] += sgn * h
            else:
                q[kind][l, i, k] += sgn * h
            vals.append(loss_at(ol.reconstruct(q["U"], q["s"], q["V"]), m, x, ys, xs))
        return (vals[0] - vals[1]) / (2 * h)

    T = ol.reconstruct(U, s, V)
    res = {}
    for kind, n in (("U", 40), ("V", 40), ("s", 40)):
        pairs = []
        for _ in range(n):
            l, i, k = int(g.integers(0, 9)), int(g.integers(0, D)), int(g.integers(0, U.shape[2]))
            gpu = out["d" + kind][b][l, k] if kind == "s" else out["d" + kind][b][l, i, k]
            pairs.append((gpu, fd_factor(kind, l, i, k)))
        res[kind] = pairs
    # map coordinates: pixels within one map cell of the vertex
    pairs = []
    iv_all, _ = ol.axis_coords(H, hm)
    iu_all, _ = ol.axis_coords(W, wm)
    for _ in range(40):
        l, r, cc = int(g.integers(0, 9)), int(g.integers(0, hm)), int(g.integers(0, wm))
        rows = np.nonzero((iv_all == r) | (iv_all == r - 1) | (np.minimum(iv_all + 1, hm - 1) == r))[0]
        cols = np.nonzero((iu_all == cc) | (iu_all == cc - 1) | (np.minimum(iu_all + 1, wm - 1) == cc))[0]
        ys, xs = np.meshgrid(rows, cols, indexing="ij")
        ys, xs = ys.ravel(), xs.ravel()
        vals = []
        for sgn in (1, -1):
            mm = m.astype(np.float64).copy(); mm[l, r, cc] += sgn * h
            vals.append(loss_at(T, mm, x, ys, xs))
        pairs.append((out["dmap"][b][l, r, cc], (vals[0] - vals[1]) / (2 * h)))
    res["map"] = pairs
    # input coordinates away from knots and the clamp
    pairs = []
    while len(pairs) < 40:
        a, yy, xx = int(g.integers(0, 3)), int(g.integers(0, H)), int(g.integers(0, W))
        v = float(x[a, yy, xx])
        q = v * (D - 1)
        if not (2 * h < v < 1 - 2 * h) or abs(q - round(q)) <= 2 * h * (D - 1):
            continue
        vals = []
        for sgn in (1, -1):
            xx2 = x.astype(np.float64).copy(); xx2[a, yy, xx] = v + sgn * h
            vals.append(loss_at(T, m, xx2, np.array([yy]), np.array([xx])))
        pairs.append((out["dx"][b][a, yy, xx], (vals[0] - vals[1]) / (2 * h)))
    res["x"] = pairs
    for kind, pairs in res.items():
        gp = np.array([p[0] for p in pairs]); fd = np.array([p[1] for p in pairs])
        tol = 1e-3 * np.abs(fd).max() + 1e-2 * np.abs(fd)
        bad = np.abs(gp - fd) > tol
        assert not bad.any(), f"{kind}: {np.c_[gp[bad], fd[bad]][:5]}"


@pytest.mark.parametrize("case", ["sparse outliers", "single spike", "map outliers"])
def test_backward_heavy_tailed_inputs(svd, case):
    """Fixed-point accumulation with a heavy-tailed dL/dY (0.1 % of the pixels 1e2-1e4 times
    the rest, or one pixel 1e4 times) or a map with a few large values.  The accumulator grid
    of a workgroup follows the band's sum of |dy| (not pixels x largest |dy|), so the outliers
    must not coarsen the other terms: by linearity the gradient of G + G_out is compared with
    the oracle to 1e-4 of the largest gradient of the ordinary part G alone, plus the float
    rounding of the sums that carry the outliers' own magnitude.  That part: dmap and db leave
    the workgroups as float partials added by atomics (at most 128 per entry here), and dU,
    ds, dV are float sums of 128 workgroup partials of dT followed by products over D = 33, so
    each is within gamma_n (n < 256) of the sum of the absolute values of its terms; those
    sums are the oracle's gradients of |G + G_out| with |U|, |V| (and, for dmap, a LUT of ones
    times max |T|), the maps being nonnegative.  The bar is 1e-4 x scale + 256 u x that
    magnitude, elementwise (u = 2^-24)."""
    B, H, W, D, R, h, w = 2, 128, 256, 33, 8, 16, 32
    say(f"bwd heavy tails: {case}")
    g = np.random.default_rng({"sparse outliers": 91, "single spike": 92, "map outliers": 93}[case])
    x = g.uniform(-0.05, 1.05, (B, 3, H, W)).astype(np.float32)
    U, s, V = synth.factors(g, B, D, R)
    m = synth.spatial_map(g, B, h, w)
    G = g.normal(0, 1, (B, 3, H, W)).astype(np.float32)
    Gall = G.copy()
    if case == "sparse outliers":
        sel = g.uniform(size=G.shape) < 1e-3
        Gall[sel] *= 10.0 ** g.uniform(2, 4, sel.sum()).astype(np.float32)
    elif case == "single spike":
        Gall[0, 1, 77, 130] = 1e4
        Gall[1, 0, 5, 3] = -1e4
    else:
        for _ in range(3):
            m[int(g.integers(0, B)), int(g.integers(0, 9)), int(g.integers(0, h)), int(g.integers(0, w))] = 100.0
    r = svd.apply_bwd(dev(x), dev(Gall), dev(U), dev(s), dev(V), dev(m), need_bias=True)
    ref = ol.apply_bwd(x, U, s, V, m, Gall)
    ref_n = ol.apply_bwd(x, U, s, V, m, G)
    Ga = np.abs(Gall)
    mag = ol.apply_bwd(x, np.abs(U), s, np.abs(V), m, Ga)
    ones = np.zeros_like(U)
    ones[..., 0] = 1.0
    s1 = np.zeros_like(s)
    s1[..., 0] = 1.0
    mag["dmap"] = ol.apply_bwd(x, ones, s1, ones, m, Ga)["dmap"] * np.abs(ol.reconstruct(U, s, V)).max()
    keys = ("dU", "ds", "dV", "dmap", "db") if case != "map outliers" else ("dU", "ds", "dV", "dmap")
    for k in keys:
        err = np.abs(host(r[k]) - ref[k])
        scale = np.abs(ref_n[k] if case != "map outliers" else ref[k]).max()
        bar = 1e-4 * scale + 256 * 2.0 ** -24 * np.abs(mag[k])
        i = np.unravel_index(np.argmax(err / bar), err.shape)
        say(f"  {k}: max-abs {err.max():.3e}, scale {scale:.3e}; worst entry err {err[i]:.3e} "
            f"against bar {bar[i]:.3e}")
        assert (err <= bar).all(), k


@pytest.mark.parametrize("shape", [
    (2, 256, 384, 33, 8, 16, 24),     # 128 workgroups per image, each map row shared by several
    (3, 40, 70, 5, 3, 30, 40),        # per-pixel map columns, ragged
    (1, 33, 300, 17, 4, 1, 1),        # a 1 x 1 map: every workgroup adds to the same entries
])
def test_deterministic_mode_bitwise(svd, shape):
    """Deterministic mode: svdlut_apply_bwd, svdlut_apply_loss_bwd and svdlut_apply_grid_bwd
    give bitwise the same outputs on repeated calls (dmap and dbias included, from
    per-workgroup partials added in workgroup order); dmap and dbias agree with the default
    mode's float atomics to the bound of two orders of the same float sums (sum_bounds), the
    other outputs bitwise; all of them
    match the oracle to 1e-4; a workspace without the mode's share is refused."""
    B, H, W, D, R, h, w = shape
    say(f"deterministic mode {shape}")
    g = np.random.default_rng(sum(shape))
    x = g.uniform(-0.05, 1.05, (B, 3, H, W)).astype(np.float32)
    U, s, V = synth.factors(g, B, D, R)
    m = synth.spatial_map(g, B, h, w)
    G = g.uniform(-0.25, 0.25, (B, 3, H, W)).astype(np.float32)
    tg = g.uniform(0, 1, (B, 3, H, W)).astype(np.float32)
    args = (dev(x), dev(G), dev(U), dev(s), dev(V), dev(m))
    was = svd.deterministic()
    try:
        svd.deterministic(False)
        r0 = svd.apply_bwd(*args, need_bias=True)
        f0 = svd.apply_loss_bwd(dev(x), dev(tg), *args[2:], kind="mse", need_bias=True)
        svd.deterministic(True)
        r1 = svd.apply_bwd(*args, need_bias=True)
        r2 = svd.apply_bwd(*args, need_bias=True,
                           ws=svd.bwd_workspace(B, D, "cuda", (H, W, h, w)))
        f1 = svd.apply_loss_bwd(dev(x), dev(tg), *args[2:], kind="mse", need_bias=True)
        f2 = svd.apply_loss_bwd(dev(x), dev(tg), *args[2:], kind="mse", need_bias=True)
        with pytest.raises(svd.SvdlutError):
            svd.apply_bwd(*args, need_bias=True, ws=svd.bwd_workspace(B, D, "cuda"))
        torch.cuda.synchronize()
    finally:
        svd.deterministic(was)
    bars = order_bars(x, U, s, V, m, G)
    for k in r1:
        assert torch.equal(r1[k], r2[k]), k
        if k in ("dmap", "db"):
            assert within(host(r1[k]), host(r0[k]), bars[k]), k
        else:
            assert torch.equal(r1[k], r0[k]), k
    for k in f1:
        assert torch.equal(f1[k], f2[k]), k
    Y = ol.apply(x, U, s, V, m)
    assert within(host(f1["dmap"]), host(f0["dmap"]), order_bars(x, U, s, V, m, 2.0 * (Y - tg) / Y.size)["dmap"])
    ref = ol.apply_bwd(x, U, s, V, m, G)
    for k in ("dU", "ds", "dV", "dmap", "db"):
        close(host(r1[k]), ref[k], 1e-4, k)


def test_deterministic_mode_grid_backward_bitwise(svd):
    """The bilateral-grid backward in deterministic mode: repeated calls bitwise equal."""
    B, H, W, D, R, h, w, K, Ds = 2, 96, 160, 17, 4, 8, 12, 6, 17
    say("deterministic mode, grid backward")
    g = np.random.default_rng(61)
    x = g.uniform(0, 1, (B, 3, H, W)).astype(np.float32)
    U, s, V = synth.factors(g, B, D, R)
    m = synth.spatial_map(g, B, h, w)
    gr, gw, _ = synth.grids(g, B, K, Ds)
    G = g.normal(0, 1, (B, 3, H, W)).astype(np.float32)
    args = (dev(x), dev(G), dev(U), dev(s), dev(V), dev(m), dev(gr), dev(gw))
    was = svd.deterministic()
    try:
        svd.deterministic(True)
        a = svd.apply_grid_bwd(*args, need_bias=True)
        b = svd.apply_grid_bwd(*args, need_bias=True)
        torch.cuda.synchronize()
    finally:
        svd.deterministic(was)
    for k in a:
        assert torch.equal(a[k], b[k]), k


def test_deterministic_mode_subsets_and_half_storage(svd):
    """Deterministic mode with half-precision storage (x, dL/dY and the map in fp16) and with
    dmap or dbias requested alone: repeated calls bitwise equal, and the same values as the
    default mode to the bound of two orders of the same float sums (sum_bounds)."""
    B, H, W, D, R, h, w = 2, 70, 300, 17, 4, 9, 37
    say("deterministic mode, fp16 storage and subsets")
    g = np.random.default_rng(515)
    x = torch.from_numpy(g.uniform(-0.05, 1.05, (B, 3, H, W)).astype(np.float32)).cuda().half()
    G = torch.from_numpy(g.normal(0, 1, (B, 3, H, W)).astype(np.float32)).cuda().half()
    U, s, V = (dev(a) for a in synth.factors(g, B, D, R))
    m = dev(synth.spatial_map(g, B, h, w)).half()
    was = svd.deterministic()
    try:
        svd.deterministic(False)
        base = svd.apply_bwd(x, G, U, s, V, m, need_dx=False, need_factors=False, need_map=True, need_bias=True)
        svd.deterministic(True)
        runs = [svd.apply_bwd(x, G, U, s, V, m, need_dx=False, need_factors=False, need_map=True, need_bias=True)
                for _ in range(2)]
        only_map = svd.apply_bwd(x, G, U, s, V, m, need_dx=False, need_factors=False, need_map=True)
        only_bias = svd.apply_bwd(x, G, U, s, V, m, need_dx=False, need_factors=False, need_map=False,
                                  need_bias=True)
        torch.cuda.synchronize()
    finally:
        svd.deterministic(was)
    bars = order_bars(host(x), host(U), host(s), host(V), host(m), host(G))
    for k in ("dmap", "db"):
        assert torch.equal(runs[0][k], runs[1][k]), k
        assert within(host(runs[0][k]), host(base[k]), bars[k]), k
    assert torch.equal(only_map["dmap"], runs[0]["dmap"])
    assert torch.equal(only_bias["db"], runs[0]["db"])


@pytest.mark.parametrize("shape", [
    (1, 2, 65535, 40, 64, 2, 512),      # the longest row, the largest D and R
    (1, 65535, 2, 33, 8, 4097, 2),      # the longest column
])
def test_backward_maximum_dimensions(svd, shape):
    """The backward at H or W = 65535 with the largest LUTs: LUT and map gradients against the
    oracle at 1e-4 of their largest value, dx at the bound of its arithmetic."""
    B, H, W, D, R, h, w = shape
    say(f"bwd maximum dims {shape}")
    g = np.random.default_rng(sum(shape) % 997)
    x = g.uniform(-0.05, 1.05, (B, 3, H, W)).astype(np.float32)
    U, s, V = synth.factors(g, B, D, R)
    m = synth.spatial_map(g, B, h, w)
    G = g.uniform(-0.25, 0.25, (B, 3, H, W)).astype(np.float32)
    r = svd.apply_bwd(dev(x), dev(G), dev(U), dev(s), dev(V), dev(m), need_bias=True)
    ref = ol.apply_bwd(x, U, s, V, m, G)
    for k in ("dU", "ds", "dV", "dmap", "db"):
        close(host(r[k]), ref[k], 1e-4, k)
    assert np.abs(host(r["dx"]) - ref["dx"]).max() <= dx_bound(G, m, U, s, V, D)
