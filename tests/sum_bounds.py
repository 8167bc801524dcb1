"""Elementwise bounds for comparing two backward results whose dmap and dbias are float sums
taken in different orders (float atomics across workgroups in the default mode, a fixed order in
the deterministic mode).  Each result is within gamma_n = n u / (1 - n u) of the sum of the
absolute values of the entry's terms, where n bounds the additions on any entry's path: the
conversion of a workgroup's fixed-point sum, at most 256 workgroup partials, and for dbias the
wave and workgroup reductions (under 300 in all).  The absolute-value sums come from the oracle:
dbias's is sum |dL/dY| over the image, dmap's is the map gradient of |dL/dY| through a LUT of ones
(the maps are nonnegative) times max |T|.  Two results then differ by at most twice that bound."""
import numpy as np

from oracle import lut as ol

U32 = 2.0 ** -24
N_ADD = 300


def order_bars(x, U, s, V, m, G):
    """{"dmap": [B][9][h][w], "db": [B][3]} bounds of |run1 - run2| for those two outputs."""
    Ga = np.abs(np.asarray(G, np.float64))
    ones = np.zeros_like(np.asarray(U, np.float64))
    ones[..., 0] = 1.0
    s1 = np.zeros_like(np.asarray(s, np.float64))
    s1[..., 0] = 1.0
    mag_map = ol.apply_bwd(x, ones, s1, ones, m, Ga)["dmap"] * np.abs(ol.reconstruct(U, s, V)).max()
    mag_db = Ga.sum(axis=(2, 3))
    gamma = N_ADD * U32 / (1 - N_ADD * U32)
    return {"dmap": 2 * gamma * mag_map, "db": 2 * gamma * mag_db}


def within(a, b, bar):
    """True when |a - b| <= bar elementwise (a, b numpy arrays)."""
    return bool((np.abs(np.asarray(a, np.float64) - np.asarray(b, np.float64)) <= bar).all())
