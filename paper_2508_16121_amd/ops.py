"""Torch-facing wrappers of the C ABI: argument checks and marshalling only.

Every computation runs in libsvdlut.so on the caller's current HIP stream; tensors must
be contiguous device tensors.  Shapes follow include/svdlut.h:
    x, y      [B][3][H][W]  float32 or float16
    U, V      [B][9][D][R]  float32;  s [B][9][R] float32
    smap      [B][9][h][w]  float32 or float16
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from ._lib import F16, F32, check

_DT = {torch.float32: F32, torch.float16: F16}


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _need(t, name, dtypes=(torch.float32,), ndim=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor (the library has no CPU path)")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.dtype not in dtypes:
        raise TypeError(f"{name} has dtype {t.dtype}, expected one of {dtypes}")
    if ndim is not None and t.dim() != ndim:
        raise ValueError(f"{name} must have {ndim} dimensions, got {tuple(t.shape)}")


def _factors(U, s, V, B):
    _need(U, "U", ndim=4); _need(s, "s", ndim=3); _need(V, "V", ndim=4)
    if U.shape[0] != B or U.shape[1] != 9 or V.shape != U.shape or s.shape != (B, 9, U.shape[3]):
        raise ValueError(f"factor shapes U{tuple(U.shape)} s{tuple(s.shape)} V{tuple(V.shape)} do not match B={B}")
    return U.shape[2], U.shape[3]


def reconstruct(U, s, V, out=None):
    """T = U diag(s) V^T for every LUT: U, V [..., D, R], s [..., R] -> T [..., D, D]."""
    _need(U, "U"); _need(s, "s"); _need(V, "V")
    D, R = U.shape[-2], U.shape[-1]
    n = U.numel() // (D * R)
    if V.shape != U.shape or s.numel() != n * R:
        raise ValueError("reconstruct: U, V must match and s must be [..., R]")
    if out is None:
        out = torch.empty(*U.shape[:-1], D, device=U.device, dtype=torch.float32)
    _need(out, "out")
    lib = _lib.load()
    check(lib.svdlut_reconstruct(_ptr(U), _ptr(s), _ptr(V), _ptr(out), n, D, R, _stream()), "svdlut_reconstruct")
    return out


def apply(x, U, s, V, smap, bias=None, out=None):
    """Fused reconstruct + spatially weighted 2D-LUT transform of a batch (svdlut_apply)."""
    _need(x, "x", (torch.float32, torch.float16), 4)
    B, C3, H, W = x.shape
    if C3 != 3:
        raise ValueError("x must be [B][3][H][W]")
    D, R = _factors(U, s, V, B)
    _need(smap, "smap", (torch.float32, torch.float16), 4)
    if smap.shape[0] != B or smap.shape[1] != 9:
        raise ValueError("smap must be [B][9][h][w]")
    h, w = smap.shape[2], smap.shape[3]
    if bias is not None:
        _need(bias, "bias")
        if bias.shape != (B, 3):
            raise ValueError("bias must be [B][3]")
    if out is None:
        out = torch.empty_like(x)
    _need(out, "out", (x.dtype,), 4)
    lib = _lib.load()
    check(lib.svdlut_apply(_ptr(x), _ptr(out), _DT[x.dtype], _ptr(U), _ptr(s), _ptr(V), _ptr(smap),
                           _DT[smap.dtype], _ptr(bias), B, H, W, h, w, D, R, _stream()), "svdlut_apply")
    return out



def apply_grid(x, U, s, V, smap, grids, gw, gb, bias=None, out=None):
    """svdlut_apply fused with 2D bilateral-grid slicing (svdlut_apply_grid).

    grids [B][K][3][Ds][Ds] (planes xy, xc, yc), gw [B][K][3], gb [B][K], all float32.
    """
    _need(x, "x", (torch.float32, torch.float16), 4)
    B, C3, H, W = x.shape
    if C3 != 3:
        raise ValueError("x must be [B][3][H][W]")
    D, R = _factors(U, s, V, B)
    _need(smap, "smap", (torch.float32, torch.float16), 4)
    if smap.shape[0] != B or smap.shape[1] != 9:
        raise ValueError("smap must be [B][9][h][w]")
    h, w = smap.shape[2], smap.shape[3]
    _need(grids, "grids", ndim=5)
    _need(gw, "gw", ndim=3)
    _need(gb, "gb", ndim=2)
    K, Ds = grids.shape[1], grids.shape[3]
    if grids.shape != (B, K, 3, Ds, Ds) or gw.shape != (B, K, 3) or gb.shape != (B, K):
        raise ValueError("grids must be [B][K][3][Ds][Ds], gw [B][K][3], gb [B][K]")
    if bias is not None:
        _need(bias, "bias")
        if bias.shape != (B, 3):
            raise ValueError("bias must be [B][3]")
    if out is None:
        out = torch.empty_like(x)
    _need(out, "out", (x.dtype,), 4)
    lib = _lib.load()
    check(lib.svdlut_apply_grid(_ptr(x), _ptr(out), _DT[x.dtype], _ptr(U), _ptr(s), _ptr(V), _ptr(smap),
                                _DT[smap.dtype], _ptr(bias), _ptr(grids), _ptr(gw), _ptr(gb), K, Ds,
                                B, H, W, h, w, D, R, _stream()), "svdlut_apply_grid")
    return out

def deterministic(on=None):
    """The library's deterministic mode (svdlut_set_deterministic / svdlut_get_deterministic):
    with no argument, whether it is on; otherwise switch it and return the new state."""
    lib = _lib.load()
    if on is not None:
        lib.svdlut_set_deterministic(1 if on else 0)
    return bool(lib.svdlut_get_deterministic())


def _workspace(n, dims, device):
    """n bytes of a backward workspace, plus (deterministic mode, dims = (B, H, W, h, w)) the
    dmap/dbias partials after n rounded up to 256 bytes."""
    if dims is not None and deterministic():
        n = (n + 255) // 256 * 256 + _lib.load().svdlut_deterministic_workspace_size(*dims)
    return torch.empty(n // 4 + 64, dtype=torch.float32, device=device)


def bwd_workspace(B, D, device, dims=None):
    """Workspace of svdlut_apply_bwd; dims = (H, W, h, w) adds the deterministic-mode share."""
    n = _lib.load().svdlut_apply_bwd_workspace_size(B, D)
    return _workspace(n, None if dims is None else (B, *dims), device)


def grid_bwd_workspace(B, D, Ds, device, dims=None):
    n = _lib.load().svdlut_apply_grid_bwd_workspace_size(B, D, Ds)
    return _workspace(n, None if dims is None else (B, *dims), device)


def apply_bwd(x, dy, U, s, V, smap, need_dx=True, need_factors=True, need_map=True, need_bias=False,
              ws=None):
    """Gradients through svdlut_apply (svdlut_apply_bwd); returns a dict of the requested ones."""
    _need(x, "x", (torch.float32, torch.float16), 4)
    _need(dy, "dy", (x.dtype,), 4)
    if dy.shape != x.shape:
        raise ValueError("dy must have the shape of x")
    B, _, H, W = x.shape
    D, R = _factors(U, s, V, B)
    _need(smap, "smap", (torch.float32, torch.float16), 4)
    h, w = smap.shape[2], smap.shape[3]
    dev = x.device
    out = {}
    dx = torch.empty_like(x) if need_dx else None
    dU = torch.empty_like(U) if need_factors else None
    ds = torch.empty_like(s) if need_factors else None
    dV = torch.empty_like(V) if need_factors else None
    dmap = torch.empty(B, 9, h, w, device=dev, dtype=torch.float32) if need_map else None
    db = torch.empty(B, 3, device=dev, dtype=torch.float32) if need_bias else None
    if ws is None and (need_factors or ((need_map or need_bias) and deterministic())):
        ws = bwd_workspace(B, D, dev, (H, W, h, w))
    lib = _lib.load()
    wsb = ws.numel() * ws.element_size() if ws is not None else 0
    check(lib.svdlut_apply_bwd(_ptr(x), _ptr(dy), _DT[x.dtype], _ptr(U), _ptr(s), _ptr(V), _ptr(smap),
                               _DT[smap.dtype], _ptr(dx), _ptr(dU), _ptr(ds), _ptr(dV), _ptr(dmap), _ptr(db),
                               B, H, W, h, w, D, R, _ptr(ws), wsb, _stream()), "svdlut_apply_bwd")
    for k, v in (("dx", dx), ("dU", dU), ("ds", ds), ("dV", dV), ("dmap", dmap), ("db", db)):
        if v is not None:
            out[k] = v
    return out


def loss_bwd_workspace(B, D, device, dims=None):
    n = _lib.load().svdlut_apply_loss_bwd_workspace_size(B, D)
    return _workspace(n, None if dims is None else (B, *dims), device)


def apply_loss_bwd(x, target, U, s, V, smap, bias=None, kind="l1", need_dx=True, need_factors=True,
                   need_map=True, need_bias=False, ws=None):
    """Forward, loss and backward in one pass (svdlut_apply_loss_bwd): returns a dict with
    "loss" (float32 [1]) and the requested gradients (dx, dU, ds, dV, dmap, db)."""
    _need(x, "x", (torch.float32, torch.float16), 4)
    _need(target, "target", (x.dtype,), 4)
    if target.shape != x.shape:
        raise ValueError("target must have the shape of x")
    B, _, H, W = x.shape
    D, R = _factors(U, s, V, B)
    _need(smap, "smap", (torch.float32, torch.float16), 4)
    h, w = smap.shape[2], smap.shape[3]
    if bias is not None:
        _need(bias, "bias")
        if bias.shape != (B, 3):
            raise ValueError("bias must be [B][3]")
    dev = x.device
    f32 = dict(device=dev, dtype=torch.float32)
    out = {"loss": torch.empty(1, **f32)}
    if need_dx:
        out["dx"] = torch.empty_like(x)
    if need_factors:
        out["dU"], out["ds"], out["dV"] = torch.empty_like(U), torch.empty_like(s), torch.empty_like(V)
    if need_map:
        out["dmap"] = torch.empty(B, 9, h, w, **f32)
    if need_bias:
        out["db"] = torch.empty(B, 3, **f32)
    if ws is None:
        ws = loss_bwd_workspace(B, D, dev, (H, W, h, w))
    k = {"l1": _lib.LOSS_L1, "mse": _lib.LOSS_MSE}[kind]
    check(_lib.load().svdlut_apply_loss_bwd(
        _ptr(x), _ptr(target), _DT[x.dtype], _ptr(U), _ptr(s), _ptr(V), _ptr(smap), _DT[smap.dtype], _ptr(bias), k,
        _ptr(out["loss"]), _ptr(out.get("dx")), _ptr(out.get("dU")), _ptr(out.get("ds")), _ptr(out.get("dV")),
        _ptr(out.get("dmap")), _ptr(out.get("db")), B, H, W, h, w, D, R, _ptr(ws), ws.numel() * ws.element_size(),
        _stream()), "svdlut_apply_loss_bwd")
    return out


def apply_grid_bwd(x, dy, U, s, V, smap, grids, gw, need_dx=True, need_factors=True, need_map=True,
                   need_bias=False, need_grids=True, ws=None):
    """Gradients through svdlut_apply_grid (svdlut_apply_grid_bwd); returns a dict of the
    requested ones (dx, dU, ds, dV, dmap, db, dgrids, dgw, dgb)."""
    _need(x, "x", (torch.float32, torch.float16), 4)
    _need(dy, "dy", (x.dtype,), 4)
    if dy.shape != x.shape:
        raise ValueError("dy must have the shape of x")
    B, _, H, W = x.shape
    D, R = _factors(U, s, V, B)
    _need(smap, "smap", (torch.float32, torch.float16), 4)
    h, w = smap.shape[2], smap.shape[3]
    _need(grids, "grids", ndim=5)
    _need(gw, "gw", ndim=3)
    K, Ds = grids.shape[1], grids.shape[3]
    if grids.shape != (B, K, 3, Ds, Ds) or gw.shape != (B, K, 3):
        raise ValueError("grids must be [B][K][3][Ds][Ds] and gw [B][K][3]")
    dev = x.device
    f32 = dict(device=dev, dtype=torch.float32)
    dx = torch.empty_like(x) if need_dx else None
    dU = torch.empty_like(U) if need_factors else None
    ds = torch.empty_like(s) if need_factors else None
    dV = torch.empty_like(V) if need_factors else None
    dmap = torch.empty(B, 9, h, w, **f32) if need_map else None
    db = torch.empty(B, 3, **f32) if need_bias else None
    dgr = torch.empty_like(grids) if need_grids else None
    dgw = torch.empty_like(gw) if need_grids else None
    dgb = torch.empty(B, K, **f32) if need_grids else None
    lib = _lib.load()
    if ws is None and (need_factors or need_grids or ((need_map or need_bias) and deterministic())):
        ws = grid_bwd_workspace(B, D, Ds, dev, (H, W, h, w))
    wsb = ws.numel() * ws.element_size() if ws is not None else 0
    check(lib.svdlut_apply_grid_bwd(_ptr(x), _ptr(dy), _DT[x.dtype], _ptr(U), _ptr(s), _ptr(V), _ptr(smap),
                                    _DT[smap.dtype], _ptr(grids), _ptr(gw), K, Ds, _ptr(dx), _ptr(dU), _ptr(ds),
                                    _ptr(dV), _ptr(dmap), _ptr(db), _ptr(dgr), _ptr(dgw), _ptr(dgb),
                                    B, H, W, h, w, D, R, _ptr(ws), wsb, _stream()), "svdlut_apply_grid_bwd")
    out = {}
    for k, v in (("dx", dx), ("dU", dU), ("ds", ds), ("dV", dV), ("dmap", dmap), ("db", db),
                 ("dgrids", dgr), ("dgw", dgw), ("dgb", dgb)):
        if v is not None:
            out[k] = v
    return out


def lut3d_apply(x, T3, out=None, ws=None):
    """Standalone 3D-LUT transform (svdlut_lut3d_apply): x [B][3][H][W] float32, T3
    [B][3][D][D][D] float32 (output channel, then the r, g, b vertex indices)."""
    _need(x, "x", ndim=4)
    _need(T3, "T3", ndim=5)
    B, _, H, W = x.shape
    D = T3.shape[2]
    if T3.shape != (B, 3, D, D, D):
        raise ValueError("T3 must be [B][3][D][D][D]")
    if out is None:
        out = torch.empty_like(x)
    lib = _lib.load()
    if ws is None:
        ws = torch.empty(lib.svdlut_lut3d_workspace_size(B, D) // 4 + 64, device=x.device, dtype=torch.float32)
    check(lib.svdlut_lut3d_apply(_ptr(x), _ptr(out), _ptr(T3), B, H, W, D, _ptr(ws), ws.numel() * 4, _stream()),
          "svdlut_lut3d_apply")
    return out


def lut1d_apply(x, T1, out=None):
    """Per-channel 1D-LUT transform (svdlut_lut1d_apply): x [B][3][H][W], T1 [B][3][D], float32."""
    _need(x, "x", ndim=4)
    _need(T1, "T1", ndim=3)
    B, _, H, W = x.shape
    D = T1.shape[2]
    if T1.shape != (B, 3, D):
        raise ValueError("T1 must be [B][3][D]")
    if out is None:
        out = torch.empty_like(x)
    check(_lib.load().svdlut_lut1d_apply(_ptr(x), _ptr(out), _ptr(T1), B, H, W, D, _stream()),
          "svdlut_lut1d_apply")
    return out


def unfused_apply(x, grids, gw, gb, Wf, bf, T3, out=None, ws=None):
    """The unfused original structure (svdlut_unfused_apply): slicing -> f_s -> 1x1 fusion
    -> 3D LUT, float32.  grids [B][K][3][Ds][Ds], gw [B][K][3], gb [B][K], Wf [B][3][K+3],
    bf [B][3], T3 [B][3][D][D][D]."""
    _need(x, "x", ndim=4)
    B, _, H, W = x.shape
    for t, name, nd in ((grids, "grids", 5), (gw, "gw", 3), (gb, "gb", 2), (Wf, "Wf", 3), (bf, "bf", 2),
                        (T3, "T3", 5)):
        _need(t, name, ndim=nd)
    K, Ds, D = grids.shape[1], grids.shape[3], T3.shape[2]
    if (grids.shape != (B, K, 3, Ds, Ds) or gw.shape != (B, K, 3) or gb.shape != (B, K)
            or Wf.shape != (B, 3, K + 3) or bf.shape != (B, 3) or T3.shape != (B, 3, D, D, D)):
        raise ValueError("unfused_apply: inconsistent shapes")
    lib = _lib.load()
    if ws is None:
        ws = torch.empty(lib.svdlut_unfused_workspace_size(B, H, W, K, D) // 4 + 64, dtype=torch.float32,
                         device=x.device)
    if out is None:
        out = torch.empty_like(x)
    check(lib.svdlut_unfused_apply(_ptr(x), _ptr(out), _ptr(grids), _ptr(gw), _ptr(gb), _ptr(Wf), _ptr(bf),
                                   _ptr(T3), K, Ds, D, B, H, W, _ptr(ws), ws.numel() * 4, _stream()),
          "svdlut_unfused_apply")
    return out


class _ApplyFn(torch.autograd.Function):
    """svdlut_apply forward with svdlut_apply_bwd as its backward."""

    @staticmethod
    def forward(ctx, x, U, s, V, smap, bias):
        ctx.save_for_backward(x, U, s, V, smap)
        ctx.has_bias = bias is not None
        return apply(x, U, s, V, smap, bias)

    @staticmethod
    def backward(ctx, gy):
        x, U, s, V, smap = ctx.saved_tensors
        need = ctx.needs_input_grad
        r = apply_bwd(x, gy.contiguous(), U, s, V, smap, need_dx=need[0],
                      need_factors=need[1] or need[2] or need[3], need_map=need[4],
                      need_bias=ctx.has_bias and need[5])
        dmap = r.get("dmap")
        if dmap is not None and dmap.dtype != smap.dtype:
            dmap = dmap.to(smap.dtype)
        return (r.get("dx"), r.get("dU") if need[1] else None, r.get("ds") if need[2] else None,
                r.get("dV") if need[3] else None, dmap, r.get("db"))


def apply_autograd(x, U, s, V, smap, bias=None):
    """Differentiable svdlut_apply: gradients flow to x, U, s, V, smap (and bias)."""
    return _ApplyFn.apply(x, U, s, V, smap, bias)


def loss(y, target, kind="l1", want_grad=True):
    """Mean L1 or MSE of y against target (svdlut_loss): returns (loss [1] float32, dL/dy or None)."""
    _need(y, "y", (torch.float32, torch.float16))
    _need(target, "target", (y.dtype,))
    if target.shape != y.shape:
        raise ValueError("target must have the shape of y")
    k = {"l1": _lib.LOSS_L1, "mse": _lib.LOSS_MSE}[kind]
    lib = _lib.load()
    n = y.numel()
    wsn = lib.svdlut_loss_workspace_size(n)
    ws = torch.empty(wsn // 4 + 64, dtype=torch.float32, device=y.device)
    out = torch.empty(1, dtype=torch.float32, device=y.device)
    dy = torch.empty_like(y) if want_grad else None
    check(lib.svdlut_loss(_ptr(y), _ptr(target), _DT[y.dtype], n, k, _ptr(out), _ptr(dy), _ptr(ws),
                          ws.numel() * 4, _stream()), "svdlut_loss")
    return out, dy
