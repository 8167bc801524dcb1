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


def _fill_shared(args):
    """Worker of make_pairs_parallel: pairs [lo, hi) into the shared arrays."""
    from multiprocessing import shared_memory
    name, count, H, W, first, lo, hi = args
    shm = shared_memory.SharedMemory(name=name)
    try:
        arr = np.ndarray((2, count, 3, H, W), np.float32, buffer=shm.buf)
        for i in range(lo, hi):
            arr[0, i], arr[1, i] = make_pair(first + i, H, W)
        del arr
    finally:
        shm.close()
    return hi - lo


def make_pairs_parallel(first: int, count: int, H: int = 256, W: int = 256, workers: int = 16):
    """make_pairs over `workers` fresh processes (spawned, so a parent that holds a GPU context
    is never forked) writing into shared memory; returns (inputs, targets) float32 arrays."""
    import multiprocessing as mp
    from multiprocessing import shared_memory
    nbytes = 2 * count * 3 * H * W * 4
    shm = shared_memory.SharedMemory(create=True, size=max(nbytes, 1))
    try:
        step = -(-count // max(1, workers * 4))
        jobs = [(shm.name, count, H, W, first, lo, min(count, lo + step)) for lo in range(0, count, step)]
        with mp.get_context("spawn").Pool(max(1, workers)) as pool:
            done = sum(pool.map(_fill_shared, jobs))
        assert done == count
        arr = np.ndarray((2, count, 3, H, W), np.float32, buffer=shm.buf)
        xs, ts = arr[0].copy(), arr[1].copy()
        del arr
    finally:
        shm.close()
        shm.unlink()
    return xs, ts
