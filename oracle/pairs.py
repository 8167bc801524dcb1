"""Degrade -> restore training pairs for the generator — TEST INFRASTRUCTURE ONLY.

Stands in for the paper's input -> expert-retouched photo pairs (Sec. "Datasets"), which
are not available here.  A base image B is degraded by a random dense 3D colour LUT
(trilinear lookup, Eq. coloren) and a smooth multiplicative gain; the network learns to
map the degraded image back to B.  The random draws come from ``synth``; this module does
the arithmetic.
"""
from __future__ import annotations

import numpy as np

import synth
from . import lut


def degrade(base, lut3d, gain_params):
    """input = clip(gain * I_tri(base; L_c), 0, 1) per channel c; returns float32 [3][H][W]."""
    _, H, W = base.shape
    g = synth.gain_field(gain_params, H, W)
    out = np.stack([lut.trilinear(base, lut3d[c]) for c in range(3)]) * g[None]
    return np.clip(out, 0.0, 1.0).astype(np.float32)


def make_pair(idx: int, H: int = 256, W: int = 256):
    """(input, target) of training pair idx, both float32 [3][H][W]."""
    base, lut3d, gain = synth.pair_draws(idx, H, W)
    return degrade(base, lut3d, gain), base


def make_pairs(first: int, count: int, H: int = 256, W: int = 256):
    xs, ts = zip(*(make_pair(first + i, H, W) for i in range(count)))
    return np.stack(xs), np.stack(ts)
