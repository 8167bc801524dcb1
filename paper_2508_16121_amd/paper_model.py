"""The paper's own model: its generator (svdlut_paper_generator_fwd/bwd) feeding the fused
slicing + 2D-LUT transform (svdlut_apply_grid) with scalar LUT weights, and its training step.

All arithmetic runs in libsvdlut.so; this module owns the device buffers and sequences the
calls on the current stream.  The parameter layout is the one documented in include/svdlut.h.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import _lib
from ._lib import check
from .generator import Adam
from .ops import _DT, _need, _ptr, _stream, apply, apply_bwd, apply_grid, apply_grid_bwd, bwd_workspace, \
    deterministic, grid_bwd_workspace, loss

CH = (3, 8, 16, 32, 64, 64)
HID = 8
FEAT = 256


def head_sizes(D=33, R=8, K=6, Ds=17):
    out = [("t", 9 * (2 * D * R + R)), ("tw", 12)]
    if K:
        out += [("s", K * 3 * Ds * Ds), ("sw", 4 * K)]
    return out


def param_shapes(D=33, R=8, K=6, Ds=17):
    """Ordered (name, shape) of the flat parameter vector."""
    out = []
    for i in range(5):
        co, ci = CH[i + 1], CH[i]
        out += [(f"conv{i + 1}.w", (co, 3, 3, ci)), (f"conv{i + 1}.b", (co,))]
        if i < 4:
            out += [(f"norm{i + 1}.scale", (co,)), (f"norm{i + 1}.shift", (co,))]
    for h, n in head_sizes(D, R, K, Ds):
        out += [(f"{h}.fc1.w", (HID, FEAT)), (f"{h}.fc1.b", (HID,)), (f"{h}.fc2.w", (n, HID)), (f"{h}.fc2.b", (n,))]
    return out


def identity_factors(D, R, rng, noise=1e-2):
    """H_t bias in the [U | S | V] order that starts the model at the identity transform:
    rank-one ramps in component 0 of t^r_rg (rows), t^g_rg (columns) and t^b_rb (columns),
    small random components elsewhere so every factor receives a gradient."""
    ramp = np.arange(D) / (D - 1)
    U = rng.normal(0.0, noise, (9, D, R))
    V = rng.normal(0.0, noise, (9, D, R))
    s = np.full((9, R), noise)
    U[:, :, 0] = 0.0; V[:, :, 0] = 0.0; s[:, 0] = 0.0
    for l, (u, v) in {0: (ramp, 1.0), 3: (1.0, ramp), 7: (1.0, ramp)}.items():
        U[l, :, 0] = u
        V[l, :, 0] = v
        s[l, 0] = 1.0
    return np.concatenate([U.ravel(), s.ravel(), V.ravel()])


def init_params(D=33, R=8, K=6, Ds=17, seed=0):
    """He-normal convolutions, unit norm scale, small FC weights; output biases start at the
    identity LUTs with unit LUT weights and zero grids."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shp in param_shapes(D, R, K, Ds):
        if name.startswith("conv") and name.endswith(".w"):
            parts.append(rng.normal(0.0, math.sqrt(2.0 / np.prod(shp[1:])), shp))
        elif name.endswith(".scale"):
            parts.append(np.ones(shp))
        elif name.endswith("fc1.w"):
            parts.append(rng.normal(0.0, 1.0 / math.sqrt(FEAT), shp))
        elif name.endswith("fc2.w"):
            parts.append(rng.normal(0.0, 1e-3, shp))
        elif name == "t.fc2.b":
            parts.append(identity_factors(D, R, rng))
        elif name == "tw.fc2.b":
            parts.append(np.tile([1.0, 1.0, 1.0, 0.0], 3))
        elif name == "sw.fc2.b":
            parts.append(np.tile([1.0, 1.0, 1.0, 0.0], K))
        else:
            parts.append(np.zeros(shp))
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


class PaperGenerator:
    """The paper's generator with device parameters and a per-batch-size workspace."""

    def __init__(self, D=33, R=8, K=6, Ds=17, params=None, seed=0, device="cuda"):
        self.D, self.R, self.K, self.Ds = D, R, K, Ds
        lib = _lib.load()
        self.n = lib.svdlut_paper_generator_param_count(D, R, K, Ds)
        if self.n == 0:
            raise ValueError("D, R, K or Ds out of range")
        if params is None:
            params = init_params(D, R, K, Ds, seed)
        p = torch.as_tensor(params, dtype=torch.float32)
        if p.numel() != self.n:
            raise ValueError(f"expected {self.n} parameters, got {p.numel()}")
        self.params = p.to(device).contiguous()
        self.grads = torch.zeros_like(self.params)
        self._ws = {}

    def workspace(self, B):
        if B not in self._ws:
            n = _lib.load().svdlut_paper_generator_workspace_size(B, self.D, self.R, self.K, self.Ds)
            self._ws[B] = torch.empty(n // 4 + 64, dtype=torch.float32, device=self.params.device)
        return self._ws[B]

    def forward(self, x, keep_mask=None):
        """x [B][3][H][W] (fp32/fp16) -> dict U, s, V, lut_w [B][9][1][1], lut_b [B][3] and, for
        K > 0, grids [B][K][3][Ds][Ds], gw [B][K][3], gb [B][K].  keep_mask: uint8
        [B][64][8][8] dropout keep mask, or None for evaluation."""
        _need(x, "x", (torch.float32, torch.float16), 4)
        B, _, H, W = x.shape
        if keep_mask is not None:
            _need(keep_mask, "keep_mask", (torch.uint8,), 4)
            if keep_mask.shape != (B, 64, 8, 8):
                raise ValueError("keep_mask must be [B][64][8][8] uint8")
        dev = x.device
        D, R, K, Ds = self.D, self.R, self.K, self.Ds
        f32 = dict(device=dev, dtype=torch.float32)
        o = {"U": torch.empty(B, 9, D, R, **f32), "s": torch.empty(B, 9, R, **f32),
             "V": torch.empty(B, 9, D, R, **f32), "lut_w": torch.empty(B, 9, 1, 1, **f32),
             "lut_b": torch.empty(B, 3, **f32)}
        if K:
            o["grids"] = torch.empty(B, K, 3, Ds, Ds, **f32)
            o["gw"] = torch.empty(B, K, 3, **f32)
            o["gb"] = torch.empty(B, K, **f32)
        ws = self.workspace(B)
        check(_lib.load().svdlut_paper_generator_fwd(
            _ptr(self.params), _ptr(x), _DT[x.dtype], B, H, W, D, R, K, Ds, _ptr(keep_mask),
            _ptr(o["U"]), _ptr(o["s"]), _ptr(o["V"]), _ptr(o["lut_w"]), _ptr(o["lut_b"]),
            _ptr(o.get("grids")), _ptr(o.get("gw")), _ptr(o.get("gb")), _ptr(ws), ws.numel() * 4, _stream()),
            "svdlut_paper_generator_fwd")
        return o

    def backward(self, g, keep_mask=None):
        """Parameter gradients (into self.grads) from upstream gradients g (keys of forward's
        output; a missing key counts as zero) and the forward's keep mask."""
        present = [v for v in g.values() if v is not None]
        if not present:
            raise ValueError("backward needs at least one upstream gradient")
        B = present[0].shape[0]
        ws = self.workspace(B)
        for k, v in g.items():
            if v is not None:
                _need(v, k)
        check(_lib.load().svdlut_paper_generator_bwd(
            _ptr(self.params), _ptr(keep_mask), _ptr(g.get("U")), _ptr(g.get("s")), _ptr(g.get("V")),
            _ptr(g.get("lut_w")), _ptr(g.get("lut_b")), _ptr(g.get("grids")), _ptr(g.get("gw")), _ptr(g.get("gb")),
            _ptr(self.grads), B, self.D, self.R, self.K, self.Ds, _ptr(ws), ws.numel() * 4, _stream()),
            "svdlut_paper_generator_bwd")
        return self.grads

    def transform(self, x, o, out=None):
        """The fused slicing + 2D-LUT transform of x with generator outputs o."""
        if self.K:
            return apply_grid(x, o["U"], o["s"], o["V"], o["lut_w"], o["grids"], o["gw"], o["gb"], bias=o["lut_b"],
                              out=out)
        return apply(x, o["U"], o["s"], o["V"], o["lut_w"], bias=o["lut_b"], out=out)

    def enhance(self, x):
        """Inference: generator on x (no dropout), then the fused transform at full resolution."""
        return self.transform(x, self.forward(x))


class PaperEnhancer:
    """Inference of the paper's model for one input shape, captured once into a HIP graph
    (generator + fused transform, about twenty kernels) and replayed per call, so the host
    launch cost is paid once.  Every call copies the input into the graph's own buffer and
    returns the graph's output buffer (overwritten by the next call)."""

    def __init__(self, gen: PaperGenerator, B, H, W, dtype=torch.float32):
        dev = gen.params.device
        self.gen = gen
        self.x = torch.zeros(B, 3, H, W, device=dev, dtype=dtype)
        self.y = torch.empty_like(self.x)
        gen.transform(self.x, gen.forward(self.x), out=self.y)     # workspaces exist before capture
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.o = gen.forward(self.x)
            gen.transform(self.x, self.o, out=self.y)
        torch.cuda.synchronize()

    def __call__(self, x):
        if x.shape != self.x.shape or x.dtype != self.x.dtype:
            raise ValueError(f"this enhancer was captured for {tuple(self.x.shape)} {self.x.dtype}")
        self.x.copy_(x)
        self.graph.replay()
        return self.y


class PaperTrainer:
    """One training step of the paper's model = generator forward (dropout keep mask drawn on
    the device), fused transform, MSE loss, transform backward (factors, LUT weights and bias,
    grids), generator backward and Adam; no host synchronisation."""

    def __init__(self, gen: PaperGenerator, lr=1e-4, dropout=True, seed=0):
        self.gen = gen
        self.opt = Adam(gen.params, lr=lr)
        self.dropout = dropout
        self._rng = torch.Generator(device=gen.params.device)
        self._rng.manual_seed(seed)
        self._bws = {}

    def _mask(self, B, dev):
        if not self.dropout:
            return None
        return (torch.rand(B, 64, 8, 8, device=dev, generator=self._rng) < 0.5).to(torch.uint8)

    def step(self, x, target):
        B = x.shape[0]
        m = self._mask(B, x.device)
        o = self.gen.forward(x, m)
        y = self.gen.transform(x, o)
        lval, dy = loss(y, target, "mse")
        g = self.gen
        H, W = x.shape[2], x.shape[3]
        key = (B, H, W, deterministic())
        if key not in self._bws:
            dims = (H, W, 1, 1)         # the LUT-weight map is 9 x 1 x 1
            self._bws[key] = (grid_bwd_workspace(B, g.D, g.Ds, x.device, dims) if g.K
                              else bwd_workspace(B, g.D, x.device, dims))
        ws = self._bws[key]
        if g.K:
            r = apply_grid_bwd(x, dy, o["U"], o["s"], o["V"], o["lut_w"], o["grids"], o["gw"], need_dx=False,
                               need_bias=True, ws=ws)
            up = {"U": r["dU"], "s": r["ds"], "V": r["dV"], "lut_w": r["dmap"], "lut_b": r["db"],
                  "grids": r["dgrids"], "gw": r["dgw"], "gb": r["dgb"]}
        else:
            r = apply_bwd(x, dy, o["U"], o["s"], o["V"], o["lut_w"], need_dx=False, need_bias=True, ws=ws)
            up = {"U": r["dU"], "s": r["ds"], "V": r["dV"], "lut_w": r["dmap"], "lut_b": r["db"]}
        g.backward(up, m)
        self.opt.step(g.grads)
        return lval

    def state_dict(self):
        return {"params": self.gen.params.detach().cpu().numpy(), "m": self.opt.m.cpu().numpy(),
                "v": self.opt.v.cpu().numpy(), "t": self.opt.t, "rng": self._rng.get_state().cpu().numpy()}

    def load_state_dict(self, st):
        self.gen.params.copy_(torch.as_tensor(st["params"]))
        self.opt.m.copy_(torch.as_tensor(st["m"]))
        self.opt.v.copy_(torch.as_tensor(st["v"]))
        self.opt.t = int(st["t"])
        self._rng.set_state(torch.as_tensor(st["rng"], dtype=torch.uint8))

    def save(self, path):
        np.savez(path, **{k: np.asarray(v) for k, v in self.state_dict().items()})

    def load(self, path):
        with np.load(path, allow_pickle=False) as z:
            self.load_state_dict({k: z[k] for k in z.files})
