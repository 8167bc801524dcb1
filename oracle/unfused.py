"""Plain float64 CPU oracle of the unfused "original structure" — TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import this
module; it shares no code with the HIP library.  It follows Sec. "Preliminary" of arXiv
2508.16121 (the spatial-aware 3D-LUT pipeline the paper starts from): slicing of bilateral
grids into spatial features f_s (Eq. slicing, here with the 2D-plane grids of
Eq. Griddecompose), the 1x1-convolution fusion of the image with f_s (Eq. fusion /
spatialfusion) and the 3D-LUT transform by trilinear interpolation (Eq. coloren).  The
cache-effective path replaces all three with one fused pass; this pipeline is the baseline
that shows what writing f_s and the fused image costs.

Readings: f_s has one channel per grid (K channels, grid k queries colour channel k mod 3,
as in oracle/grid.py); the fusion is X_bar_c = sum_j Wf[c][j] * concat(X, f_s)_j + bf[c]
with the K+3 input channels ordered (r, g, b, f_0 .. f_{K-1}); output channel c uses its own
3D LUT t^c indexed [i_r][i_g][i_b] on the fused image's channels.
"""
from __future__ import annotations

import numpy as np

from .grid import slice_grids
from .lut import trilinear


def fuse(x, fs, Wf, bf):
    """1x1 convolution of concat(x, fs): [3][H][W] (Eq. fusion)."""
    inp = np.concatenate([np.asarray(x, dtype=np.float64), np.asarray(fs, dtype=np.float64)])
    return np.einsum("cj,jhw->chw", np.asarray(Wf, dtype=np.float64), inp) + np.asarray(bf, np.float64)[:, None, None]


def lut3d(xbar, T3):
    """Y_c = trilinear lookup of 3D LUT T3[c] at the fused colours (Eq. coloren): [3][H][W].

    The fused image is not clamped before the lookup beyond the LUT decode's own clamp.
    """
    return np.stack([trilinear(xbar, T3[c]) for c in range(3)])


def original_structure(x, g, gw, gb, Wf, bf, T3):
    """Slicing -> f_s -> 1x1 fusion -> 3D LUT for one image; returns (Y, f_s, X_bar)."""
    fs = slice_grids(x, g, gw, gb)
    xbar = fuse(x, fs, Wf, bf)
    return lut3d(xbar.astype(np.float32), T3), fs, xbar
