"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only draws random numbers and shapes them into arrays; it holds none of
the enhancement method's arithmetic (no LUT reconstruction, lookup, interpolation or
fusion).  Every array is a NumPy array on the host; callers move it where they need it.

Image recipe (stands in for the MIT-Adobe FiveK photos the paper measures on, which are
not available here): per channel c,

    X_c(x, y) = 0.5 + sum_{k<8} a_ck * sin(2*pi*(fx_ck * x / W + fy_ck * y / H) + phi_ck)
                + N(0, 0.02)

with a ~ U(0, 0.25), f ~ U(-4, 4) cycles per image on each axis, phi ~ U(0, 2*pi),
clipped to [0, 1].  The form does not depend on resolution, so a 480x640 frame and a
2160x3840 frame look alike.  Factor draws: U, V ~ N(0, 0.1), s ~ U(0, 1), spatial map
~ U(0, 1), all from the same generator in the order X, U, s, V, map.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

N_LUT = 9          # 3 output channels x 3 colour pairs
N_SINES = 8


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def image(g: np.random.Generator, H: int, W: int) -> np.ndarray:
    """One planar [3][H][W] float32 image in [0, 1] (recipe in the module docstring)."""
    a = g.uniform(0.0, 0.25, size=(3, N_SINES))
    fx = g.uniform(-4.0, 4.0, size=(3, N_SINES))
    fy = g.uniform(-4.0, 4.0, size=(3, N_SINES))
    ph = g.uniform(0.0, 2.0 * math.pi, size=(3, N_SINES))
    xs = np.arange(W, dtype=np.float64) / W
    ys = np.arange(H, dtype=np.float64) / H
    out = np.empty((3, H, W), dtype=np.float32)
    for c in range(3):
        # sum_k a_k sin(A_k(x) + B_k(y)) = [cos B | sin B] @ [a sin A ; a cos A]
        A = 2.0 * math.pi * fx[c][:, None] * xs[None, :] + ph[c][:, None]      # [8][W]
        B = 2.0 * math.pi * fy[c][:, None] * ys[None, :]                       # [8][H]
        left = np.concatenate([np.cos(B), np.sin(B)], axis=0).T                # [H][16]
        right = np.concatenate([a[c][:, None] * np.sin(A), a[c][:, None] * np.cos(A)], axis=0)
        out[c] = (0.5 + left @ right).astype(np.float32)
    out += np.float32(0.02) * g.standard_normal(size=out.shape, dtype=np.float32)
    np.clip(out, 0.0, 1.0, out=out)
    return out


def factors(g: np.random.Generator, n_img: int, D: int, R: int):
    """Per-image rank-R factors: U, V [n][9][D][R] ~ N(0, 0.1); s [n][9][R] ~ U(0, 1)."""
    U = g.normal(0.0, 0.1, size=(n_img, N_LUT, D, R)).astype(np.float32)
    s = g.uniform(0.0, 1.0, size=(n_img, N_LUT, R)).astype(np.float32)
    V = g.normal(0.0, 0.1, size=(n_img, N_LUT, D, R)).astype(np.float32)
    return U, s, V


def spatial_map(g: np.random.Generator, n_img: int, h: int, w: int) -> np.ndarray:
    """Low-resolution spatial weight map [n][9][h][w] ~ U(0, 1), float32."""
    return g.uniform(0.0, 1.0, size=(n_img, N_LUT, h, w)).astype(np.float32)


def grids(g: np.random.Generator, n_img: int, K: int = 6, Ds: int = 17):
    """Bilateral grids [n][K][3][Ds][Ds] ~ N(0, 0.1), plane weights [n][K][3] ~ U(0, 1) and
    biases [n][K] ~ N(0, 0.01), float32, drawn in that order."""
    gr = g.normal(0.0, 0.1, size=(n_img, K, 3, Ds, Ds)).astype(np.float32)
    gw = g.uniform(0.0, 1.0, size=(n_img, K, 3)).astype(np.float32)
    gb = g.normal(0.0, 0.01, size=(n_img, K)).astype(np.float32)
    return gr, gw, gb


def grid_case(seed: int, H: int, W: int, D: int, R: int, h: int, w: int, K: int = 6, Ds: int = 17):
    """One image with factors, map and grids: X, U, s, V, map, grids, weights, biases from
    default_rng(seed) in that order."""
    g = rng(seed)
    x = image(g, H, W)[None]
    U, s, V = factors(g, 1, D, R)
    m = spatial_map(g, 1, h, w)
    gr, gw, gb = grids(g, 1, K, Ds)
    return Case(x, U, s, V, m), gr, gw, gb


def map_size(H: int, W: int, div: int = 8):
    """Map resolution at 1/div of the image: (ceil(H/div), ceil(W/div))."""
    return -(-H // div), -(-W // div)


@dataclass
class Case:
    """One batch of same-size images with their factors and maps (all host float32)."""
    x: np.ndarray        # [B][3][H][W]
    U: np.ndarray        # [B][9][D][R]
    s: np.ndarray        # [B][9][R]
    V: np.ndarray        # [B][9][D][R]
    smap: np.ndarray     # [B][9][h][w]
    target: np.ndarray | None = None   # [B][3][H][W] when the case has a loss target

    @property
    def shape(self):
        B, _, H, W = self.x.shape
        return B, H, W, self.U.shape[2], self.U.shape[3], self.smap.shape[2], self.smap.shape[3]


def single(seed: int, H: int, W: int, D: int, R: int, h: int, w: int) -> Case:
    """One image drawn in the order X, U, s, V, map from default_rng(seed)."""
    g = rng(seed)
    x = image(g, H, W)[None]
    U, s, V = factors(g, 1, D, R)
    m = spatial_map(g, 1, h, w)
    return Case(x, U, s, V, m)


def plain_256(seed: int = 1) -> Case:
    """Plain path: one 256x256 image, 17x17 LUTs at rank 4, 32x32 map."""
    return single(seed, 256, 256, 17, 4, 32, 32)


def frame_4k(seed: int = 2) -> Case:
    """One 2160x3840 frame, 33x33 LUTs at rank 8, 270x480 map (1/8 resolution)."""
    return single(seed, 2160, 3840, 33, 8, 270, 480)


def diff_batch(n: int = 16, H: int = 512, W: int = 512, D: int = 33, R: int = 8,
               h: int = 64, w: int = 64, seed0: int = 4000, tseed0: int = 4500) -> Case:
    """Differentiation batch: image b from seed seed0+b (X, U, s, V, map), target image from tseed0+b."""
    xs, Us, ss, Vs, ms, ts = [], [], [], [], [], []
    for b in range(n):
        c = single(seed0 + b, H, W, D, R, h, w)
        xs.append(c.x); Us.append(c.U); ss.append(c.s); Vs.append(c.V); ms.append(c.smap)
        ts.append(image(rng(tseed0 + b), H, W)[None])
    cat = lambda a: np.concatenate(a, axis=0)
    return Case(cat(xs), cat(Us), cat(ss), cat(Vs), cat(ms), cat(ts))


BASE_SIZES = ((480, 640), (1080, 1920), (2160, 3840))


def uneven_sizes(n: int = 64, seed0: int = 3000, bases=BASE_SIZES, jitter: float = 0.1):
    """(H, W) per image: base size drawn uniformly, then W = round(W0 * (1 + j)), j ~ U(-jitter, jitter)."""
    out = []
    for i in range(n):
        g = rng(seed0 + i)
        H0, W0 = bases[int(g.integers(0, len(bases)))]
        j = g.uniform(-jitter, jitter)
        out.append((H0, max(1, int(round(W0 * (1.0 + j))))))
    return out


def uneven_image(i: int, seed0: int = 3000, D: int = 33, R: int = 8, bases=BASE_SIZES,
                 jitter: float = 0.1):
    """Image i of the uneven batch: size draw, then X, U, s, V, map from default_rng(seed0+i)."""
    g = rng(seed0 + i)
    H0, W0 = bases[int(g.integers(0, len(bases)))]
    j = g.uniform(-jitter, jitter)
    H, W = H0, max(1, int(round(W0 * (1.0 + j))))
    h, w = map_size(H, W)
    x = image(g, H, W)
    U, s, V = factors(g, 1, D, R)
    m = spatial_map(g, 1, h, w)
    return x, U[0], s[0], V[0], m[0]


# ---------------------------------------------------------------- training pairs (learned generator)
PAIR_SEED0 = 5_000_000


def degradation(g: np.random.Generator, D: int = 33, sigma: float = 3.0, std: float = 0.05,
                gain_amp: float = 0.2):
    """Random draws for one degrade->restore training pair.

    Returns (lut3d [3][D][D][D], gain parameters (fx, fy, phase)).  The 3D LUT is the
    identity plus N(0, std) vertex noise, Gaussian-smoothed over the lattice (sigma in
    vertices) and rescaled back to the given std; the gain is
    1 + gain_amp * sin(2*pi*(fx*x' + fy*y') + phase) with |f| <= 1 cycle per image.
    """
    from scipy.ndimage import gaussian_filter

    ramp = np.arange(D, dtype=np.float64) / (D - 1)
    ident = np.stack(np.meshgrid(ramp, ramp, ramp, indexing="ij"))   # [3][D][D][D]: channel c = axis c
    noise = g.normal(0.0, std, size=(3, D, D, D))
    for c in range(3):
        sm = gaussian_filter(noise[c], sigma=sigma, mode="nearest")
        noise[c] = sm * (std / max(sm.std(), 1e-12))
    fx, fy = g.uniform(-1.0, 1.0, size=2)
    ph = g.uniform(0.0, 2.0 * math.pi)
    return ident + noise, (float(fx), float(fy), float(ph), gain_amp)


def gain_field(params, H: int, W: int) -> np.ndarray:
    """Smooth multiplicative gain [H][W] for the parameters returned by degradation()."""
    fx, fy, ph, amp = params
    xs = np.arange(W, dtype=np.float64) / max(W - 1, 1)
    ys = np.arange(H, dtype=np.float64) / max(H - 1, 1)
    return 1.0 + amp * np.sin(2.0 * math.pi * (fx * xs[None, :] + fy * ys[:, None]) + ph)


def pair_draws(idx: int, H: int = 256, W: int = 256, D: int = 33):
    """Base image, 3D LUT and gain parameters of training pair idx (seed PAIR_SEED0 + idx)."""
    g = rng(PAIR_SEED0 + idx)
    base = image(g, H, W)
    lut3d, gain = degradation(g, D)
    return base, lut3d, gain


def uneven_batch(n: int = 64, seed0: int = 3000, D: int = 33, R: int = 8, workers: int = 8, bases=BASE_SIZES):
    """All images of the uneven batch (list of (x, U, s, V, map)), drawn on a thread pool."""
    from concurrent.futures import ThreadPoolExecutor

    with ThreadPoolExecutor(max(1, workers)) as ex:
        return list(ex.map(lambda i: uneven_image(i, seed0, D, R, bases), range(n)))


def pack_uneven(images, align: int = 64):
    """Pack per-image arrays [(x [3][H][W], U, s, V, map [9][h][w]), ...] into flat planar
    buffers.  Each image starts on an `align`-element boundary.  Returns
    (x_flat float32, map_flat float32, U [B][9][D][R], s [B][9][R], V [B][9][D][R], descs)
    where descs[b] = dict(H, W, h, w, x_off, y_off, map_off) in elements."""
    descs, xo, mo = [], 0, 0
    for x, U, s, V, m in images:
        _, H, W = x.shape
        _, h, w = m.shape
        descs.append(dict(H=H, W=W, h=h, w=w, x_off=xo, y_off=xo, map_off=mo))
        xo += -(-x.size // align) * align
        mo += -(-m.size // align) * align
    xf = np.zeros(xo, np.float32)
    mf = np.zeros(mo, np.float32)
    for d, (x, U, s, V, m) in zip(descs, images):
        xf[d["x_off"]:d["x_off"] + x.size] = x.ravel()
        mf[d["map_off"]:d["map_off"] + m.size] = m.ravel()
    U = np.stack([im[1] for im in images])
    s = np.stack([im[2] for im in images])
    V = np.stack([im[3] for im in images])
    return xf, mf, U, s, V, descs
