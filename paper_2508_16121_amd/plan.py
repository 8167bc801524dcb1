"""Uneven-size batches: packed planar buffers, descriptors and the graph-replayed plan."""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from ._lib import ImageDesc, PlanInfo, check
from .ops import _DT, _need, _ptr, _stream


def pack_offsets(sizes, map_sizes):
    """Element offsets of each image in packed x/y ([3][H][W] each) and map ([9][h][w]) buffers.

    Each image starts on a 64-element boundary so that its rows can use vector accesses.
    Returns (descs list of dicts, total x elements, total map elements).
    """
    descs, xo, mo = [], 0, 0
    for (H, W), (h, w) in zip(sizes, map_sizes):
        descs.append(dict(H=H, W=W, h=h, w=w, x_off=xo, y_off=xo, map_off=mo))
        xo += -(-3 * H * W // 64) * 64
        mo += -(-9 * h * w // 64) * 64
    return descs, xo, mo


class Plan:
    """svdlut_plan: one persistent, HIP-graph-replayed launch over a batch of uneven images."""

    def __init__(self, descs, D, R, io=torch.float16, map_dtype=torch.float16):
        self.B = len(descs)
        arr = (ImageDesc * self.B)(*[ImageDesc(d["H"], d["W"], d["h"], d["w"], d["x_off"], d["y_off"],
                                              d["map_off"]) for d in descs])
        self._descs = arr
        self.D, self.R = D, R
        self.io, self.map_dtype = io, map_dtype
        h = C.c_void_p()
        lib = _lib.load()
        check(lib.svdlut_plan_create(C.cast(arr, C.c_void_p), self.B, D, R, _DT[io], _DT[map_dtype],
                                     C.byref(h)), "svdlut_plan_create")
        self._h = h

    def _args(self, x, y, U, s, V, smap, bias):
        _need(x, "x", (self.io,)); _need(y, "y", (self.io,)); _need(smap, "smap", (self.map_dtype,))
        for t, n in ((U, "U"), (s, "s"), (V, "V")):
            _need(t, n)
        if U.shape != (self.B, 9, self.D, self.R) or V.shape != U.shape or s.shape != (self.B, 9, self.R):
            raise ValueError("factor shapes do not match the plan")
        if bias is not None:
            _need(bias, "bias")
        return (self._h, _ptr(x), _ptr(y), _ptr(U), _ptr(s), _ptr(V), _ptr(smap), _ptr(bias), _stream())

    def launch(self, x, y, U, s, V, smap, bias=None):
        check(_lib.load().svdlut_plan_launch(*self._args(x, y, U, s, V, smap, bias)), "svdlut_plan_launch")
        return y

    def launch_direct(self, x, y, U, s, V, smap, bias=None):
        check(_lib.load().svdlut_plan_launch_direct(*self._args(x, y, U, s, V, smap, bias)),
              "svdlut_plan_launch_direct")
        return y

    def autotune(self, x, y, U, s, V, smap, bias=None):
        check(_lib.load().svdlut_plan_autotune(*self._args(x, y, U, s, V, smap, bias)), "svdlut_plan_autotune")

    def set_shape(self, block, blocks_per_cu, px_per_lane=4):
        """Launch shape by hand: threads per workgroup, workgroups per CU, pixels per lane (4 or 8)."""
        check(_lib.load().svdlut_plan_set_shape(self._h, int(block), int(blocks_per_cu), int(px_per_lane)),
              "svdlut_plan_set_shape")

    def info(self):
        inf = PlanInfo()
        check(_lib.load().svdlut_plan_get_info(self._h, C.byref(inf)), "svdlut_plan_get_info")
        return {k: getattr(inf, k) for k, _ in PlanInfo._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().svdlut_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
