"""The learned factor/map generator: parameters, workspace and training step.

All arithmetic runs in libsvdlut.so (svdlut_generator_fwd/bwd, svdlut_apply(_bwd),
svdlut_loss, svdlut_adam_step); this module owns the device buffers and sequences the calls
on the current stream.  Parameter layout is the one documented in include/svdlut.h.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import _lib
from ._lib import check
from .ops import _DT, _need, _ptr, _stream, apply, apply_bwd, apply_loss_bwd, bwd_workspace, deterministic, loss, \
    loss_bwd_workspace

CONV_CH = (3, 16, 32, 64, 128, 128)
HEAD_IN = 64
N_MAP = 9
GAP = 128
MAP_HW = 32


def param_shapes(D=33, R=8):
    """Ordered (name, shape) of the flat parameter vector."""
    out = []
    for i in range(5):
        out.append((f"conv{i + 1}.w", (CONV_CH[i + 1], 3, 3, CONV_CH[i])))
        out.append((f"conv{i + 1}.b", (CONV_CH[i + 1],)))
    out.append(("head.w", (N_MAP, 3, 3, HEAD_IN)))
    out.append(("head.b", (N_MAP,)))
    nfc = 9 * (2 * D * R + R)
    out.append(("fc.w", (nfc, GAP)))
    out.append(("fc.b", (nfc,)))
    return out


def identity_factor_block(D, R, rng, noise=1e-2):
    """FC bias that makes the generator start at the identity transform: rank-one identity
    LUTs (t^r_rg rows = ramp, t^g_rg columns = ramp, t^b_rb columns = ramp) in component 0,
    small random components 1..R-1 so that every factor receives a gradient."""
    ramp = np.arange(D) / (D - 1)
    U = rng.normal(0.0, noise, (9, D, R))
    V = rng.normal(0.0, noise, (9, D, R))
    s = np.full((9, R), noise)
    U[:, :, 0] = 0.0; V[:, :, 0] = 0.0; s[:, 0] = 0.0
    for l, (u, v) in {0: (ramp, 1.0), 3: (1.0, ramp), 7: (1.0, ramp)}.items():
        U[l, :, 0] = u
        V[l, :, 0] = v
        s[l, 0] = 1.0
    return np.concatenate([U.reshape(9, -1), s, V.reshape(9, -1)], axis=1).ravel()


def init_params(D=33, R=8, seed=0):
    """He-normal convolutions, small FC weights, identity FC bias, map head bias 1."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shp in param_shapes(D, R):
        if name.startswith("conv") and name.endswith(".w"):
            fan_in = shp[1] * shp[2] * shp[3]
            parts.append(rng.normal(0.0, math.sqrt(2.0 / fan_in), shp))
        elif name.startswith("conv"):
            parts.append(np.zeros(shp))
        elif name == "head.w":
            parts.append(rng.normal(0.0, 1e-3, shp))
        elif name == "head.b":
            parts.append(np.ones(shp))
        elif name == "fc.w":
            parts.append(rng.normal(0.0, 1e-3, shp))
        else:
            parts.append(identity_factor_block(D, R, rng))
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


class Adam:
    """Standard Adam on a flat float32 parameter tensor (svdlut_adam_step)."""

    def __init__(self, params, lr=1e-4, betas=(0.9, 0.999), eps=1e-8):
        self.p = params
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.lr, self.b1, self.b2, self.eps = lr, betas[0], betas[1], eps
        self.t = 0

    def step(self, grads):
        self.t += 1
        check(_lib.load().svdlut_adam_step(_ptr(self.p), _ptr(grads), _ptr(self.m), _ptr(self.v), self.p.numel(),
                                           self.lr, self.b1, self.b2, self.eps, self.t, _stream()),
              "svdlut_adam_step")

    def state(self):
        return {"m": self.m, "v": self.v, "t": self.t}

    def load_state(self, st):
        self.m.copy_(st["m"]); self.v.copy_(st["v"]); self.t = int(st["t"])


class Generator:
    """Factor/map generator with device parameters and a per-batch-size workspace."""

    def __init__(self, D=33, R=8, params=None, seed=0, device="cuda"):
        self.D, self.R = D, R
        lib = _lib.load()
        self.n = lib.svdlut_generator_param_count(D, R)
        if params is None:
            params = init_params(D, R, seed)
        p = torch.as_tensor(params, dtype=torch.float32)
        if p.numel() != self.n:
            raise ValueError(f"expected {self.n} parameters, got {p.numel()}")
        self.params = p.to(device).contiguous()
        self.grads = torch.zeros_like(self.params)
        self._ws = {}

    def workspace(self, B):
        if B not in self._ws:
            n = _lib.load().svdlut_generator_workspace_size(B, self.D, self.R)
            self._ws[B] = torch.empty(n // 4 + 64, dtype=torch.float32, device=self.params.device)
        return self._ws[B]

    def forward(self, x):
        """x [B][3][H][W] (fp32/fp16, any size) -> U, s, V [B][9][D][R]/[B][9][R], map [B][9][32][32]."""
        _need(x, "x", (torch.float32, torch.float16), 4)
        B, _, H, W = x.shape
        dev = x.device
        U = torch.empty(B, 9, self.D, self.R, device=dev)
        s = torch.empty(B, 9, self.R, device=dev)
        V = torch.empty(B, 9, self.D, self.R, device=dev)
        m = torch.empty(B, 9, MAP_HW, MAP_HW, device=dev)
        ws = self.workspace(B)
        check(_lib.load().svdlut_generator_fwd(_ptr(self.params), _ptr(x), _DT[x.dtype], B, H, W, self.D, self.R,
                                               _ptr(U), _ptr(s), _ptr(V), _ptr(m), _ptr(ws), ws.numel() * 4,
                                               _stream()), "svdlut_generator_fwd")
        self._last_B = B
        return U, s, V, m

    def backward(self, dU, ds, dV, dmap):
        """Gradients of all parameters (into self.grads) from the last forward's activations."""
        B = dU.shape[0]
        ws = self.workspace(B)
        for t, nme in ((dU, "dU"), (ds, "ds"), (dV, "dV"), (dmap, "dmap")):
            _need(t, nme)
        check(_lib.load().svdlut_generator_bwd(_ptr(self.params), _ptr(dU), _ptr(ds), _ptr(dV), _ptr(dmap),
                                               _ptr(self.grads), B, self.D, self.R, _ptr(ws), ws.numel() * 4,
                                               _stream()), "svdlut_generator_bwd")
        return self.grads

    def enhance(self, x):
        """Inference: predict factors and map from x, then apply them to x at full resolution."""
        U, s, V, m = self.forward(x)
        return apply(x, U, s, V, m)


class Trainer:
    """One training step = generator forward, the transform's forward + MSE + backward in one
    fused pass (factors and map gradients), generator backward and Adam, all on the current
    stream with no host sync."""

    def __init__(self, gen: Generator, lr=1e-4):
        self.gen = gen
        self.opt = Adam(gen.params, lr=lr)
        self._bws = {}

    def step(self, x, target):
        U, s, V, m = self.gen.forward(x)
        B, _, H, W = x.shape
        key = (B, H, W, deterministic())
        if key not in self._bws:
            self._bws[key] = loss_bwd_workspace(B, self.gen.D, x.device, (H, W, m.shape[2], m.shape[3]))
        # forward, MSE and backward of the transform in one fused pass
        r = apply_loss_bwd(x, target, U, s, V, m, kind="mse", need_dx=False, need_factors=True, need_map=True,
                           ws=self._bws[key])
        self.gen.backward(r["dU"], r["ds"], r["dV"], r["dmap"])
        self.opt.step(self.gen.grads)
        return r["loss"]

    def state_dict(self):
        return {"params": self.gen.params.detach().cpu().numpy(), "m": self.opt.m.cpu().numpy(),
                "v": self.opt.v.cpu().numpy(), "t": self.opt.t}

    def load_state_dict(self, st):
        self.gen.params.copy_(torch.as_tensor(st["params"]))
        self.opt.m.copy_(torch.as_tensor(st["m"]))
        self.opt.v.copy_(torch.as_tensor(st["v"]))
        self.opt.t = int(st["t"])

    def save(self, path):
        np.savez(path, **{k: np.asarray(v) for k, v in self.state_dict().items()})

    def load(self, path):
        with np.load(path, allow_pickle=False) as z:
            self.load_state_dict({k: z[k] for k in z.files})
