"""Comparison helpers for GPU-vs-oracle parity (test infrastructure)."""
import numpy as np

# Positions: FP32 GPU against the FP64 oracle, normwise per level:
#   max |P_gpu - P_ref| / max |P_ref| <= 1e-5.
# Every rule is a convex combination of at most ~30 terms, so one level adds
# O(30) FP32 roundings of magnitude <= max|P| * 2^-24 ~ 6e-8 relative, i.e.
# <~2e-6 per level and <~1e-5 after six levels in the worst case.
POS_TOL = 1e-5


def normwise_err(got, ref):
    ref = np.asarray(ref, np.float64)
    got = np.asarray(got, np.float64)
    scale = np.abs(ref).max()
    return float(np.abs(got - ref).max() / (scale if scale > 0 else 1.0))


def edge_keys(lohi):
    lohi = np.asarray(lohi, np.int64)
    return lohi[:, 1] * (1 << 32) + lohi[:, 0]


def level_edges(verts, order):
    """(lo, hi) of the edges of a uniform face table, in (hi, lo) order."""
    f = np.asarray(verts, np.int64).reshape(-1, order)
    a = f.reshape(-1)
    b = np.roll(f, -1, axis=1).reshape(-1)
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    k = np.unique(hi * (1 << 32) + lo)
    return np.stack([k & 0xffffffff, k >> 32], 1)


def crease_table(oracle_level, edges):
    """Oracle crease list (lo, hi, sigma) placed onto edge ids -> dense sigma."""
    sig = np.zeros(edges.shape[0], np.float64)
    if oracle_level.crease_sharp.size:
        keys = edge_keys(edges)
        ck = edge_keys(oracle_level.crease_verts)
        idx = np.searchsorted(keys, ck)
        assert np.all(keys[idx] == ck)
        sig[idx] = oracle_level.crease_sharp
    return sig
