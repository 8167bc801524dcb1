"""svdlut_apply_bwd_noalloc (the backward for callers that cannot allocate: its dT partials
live in a library-owned device buffer) against svdlut_apply_bwd with a caller workspace,
both called through the C ABI on the same inputs: two calls in a row, the second on a
smaller batch, so the second also shows that the buffer's previous contents do not leak."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth
from oracle import lut as ol
from sum_bounds import order_bars, within

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2508_16121_amd import _lib
    return _lib.load()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _case(seed, B, H, W, D, R, h, w):
    g = np.random.default_rng(seed)
    x = g.uniform(-0.05, 1.05, (B, 3, H, W)).astype(np.float32)
    U, s, V = synth.factors(g, B, D, R)
    m = synth.spatial_map(g, B, h, w)
    G = g.normal(0, 1, (B, 3, H, W)).astype(np.float32)
    return x, G, U, s, V, m


def _run(lib, noalloc, x, G, U, s, V, m):
    B, _, H, W = x.shape
    D, R = U.shape[2], U.shape[3]
    h, w = m.shape[2], m.shape[3]
    xt, Gt, Ut, st, Vt, mt = (dev(a) for a in (x, G, U, s, V, m))
    out = {"dx": torch.empty_like(xt), "dU": torch.empty_like(Ut), "ds": torch.empty_like(st),
           "dV": torch.empty_like(Vt), "dmap": torch.empty_like(mt),
           "db": torch.empty(B, 3, device="cuda", dtype=torch.float32)}
    for t in out.values():
        t.fill_(float("nan"))             # every output must be written
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    common = [_p(xt), _p(Gt), 0, _p(Ut), _p(st), _p(Vt), _p(mt), 0, _p(out["dx"]), _p(out["dU"]),
              _p(out["ds"]), _p(out["dV"]), _p(out["dmap"]), _p(out["db"]), B, H, W, h, w, D, R]
    if noalloc:
        status = lib.svdlut_apply_bwd_noalloc(*common, stream)
    else:
        n = lib.svdlut_apply_bwd_workspace_size(B, D)
        if lib.svdlut_get_deterministic():
            n = (n + 255) // 256 * 256 + lib.svdlut_deterministic_workspace_size(B, H, W, h, w)
        ws = torch.empty(n // 4 + 64, device="cuda", dtype=torch.float32)
        status = lib.svdlut_apply_bwd(*common, _p(ws), ws.numel() * 4, stream)
    assert status == 0, lib.svdlut_last_error().decode()
    torch.cuda.synchronize()
    return {k: host(v) for k, v in out.items()}


def _same(a, b, ref, what, case):
    # dx and the factor gradients (fixed-point dT summed in a fixed order) are reproducible
    # bit for bit; dmap and db are summed with float atomics in a run-dependent order, so
    # they are held to the bound of two orders of the same float sums
    for k in ("dx", "dU", "ds", "dV"):
        assert np.array_equal(a[k], b[k]), f"{what}: {k} differs from svdlut_apply_bwd"
    x, G, U, s, V, m = case
    bars = order_bars(x, U, s, V, m, G)
    for k in ("dmap", "db"):
        assert within(a[k], b[k], bars[k]), f"{what}: {k}"
    # and both against the fp64 oracle at the backward's parity bar
    for k, rk in (("dU", "dU"), ("ds", "ds"), ("dV", "dV"), ("dmap", "dmap"), ("db", "db"), ("dx", "dx")):
        scale = max(np.abs(ref[rk]).max(), 1e-30)
        assert np.abs(a[k] - ref[rk]).max() <= 1e-4 * scale, f"{what}: {k} vs oracle"


def test_noalloc_matches_workspace_entry_point_twice(lib):
    big = _case(901, 3, 70, 530, 33, 8, 9, 67)      # three images, ragged rows, several segments
    small = _case(902, 1, 21, 100, 17, 4, 3, 13)    # smaller batch and LUT in the same buffer
    for what, case in (("first call", big), ("second call, smaller", small)):
        print(f"noalloc {what}: shape {case[0].shape}", flush=True)
        ref = ol.apply_bwd(*[case[i] for i in (0, 2, 3, 4, 5, 1)])
        a = _run(lib, True, *case)
        b = _run(lib, False, *case)
        _same(a, b, ref, what, case)


def test_noalloc_deterministic_mode_bitwise_twice(lib):
    """In deterministic mode the library buffer also holds the dmap and dbias partials: both
    entry points then agree bit for bit on every output, on two calls in a row."""
    was = lib.svdlut_get_deterministic()
    lib.svdlut_set_deterministic(1)
    try:
        for what, case in (("first call", _case(903, 3, 70, 530, 33, 8, 9, 67)),
                           ("second call, smaller", _case(904, 1, 21, 100, 17, 4, 3, 13))):
            print(f"noalloc deterministic {what}: shape {case[0].shape}", flush=True)
            ref = ol.apply_bwd(*[case[i] for i in (0, 2, 3, 4, 5, 1)])
            a = _run(lib, True, *case)
            b = _run(lib, False, *case)
            for k in a:
                assert np.array_equal(a[k], b[k]), f"{what}: {k}"
            _same(a, b, ref, what, case)
    finally:
        lib.svdlut_set_deterministic(was)


def test_noalloc_rejects_batches_beyond_its_buffer(lib):
    """A batch whose partials exceed the library's buffer is refused before any launch."""
    B, D, R = 600, 33, 8
    need = lib.svdlut_apply_bwd_workspace_size(B, D)
    assert need > 24 * 1024 * 1024
    t = torch.empty(4, device="cuda")
    p = C.c_void_p(t.data_ptr())
    status = lib.svdlut_apply_bwd_noalloc(p, p, 0, p, p, p, p, 0, None, p, p, p, None, None,
                                          B, 4, 4, 1, 1, D, R, None)
    assert status == 1
    assert "scratch" in lib.svdlut_last_error().decode()
