"""Uniform sampling of K cells of an m x n grid without replacement.

The paper only says that entries are sampled at random (Sec. V.B, Sec. V.C).
The sampler is fixed here so that it is reproducible and parallel: every cell
id e = i*n + j gets the key  key(e) = SplitMix64 output number e  of a stream
seeded with `seed`, i.e. mix64(seed + (e+1) * 0x9E3779B97F4A7C15) with
Stafford's "Mix13" finaliser (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014).  Phi is the set of the K
smallest (key, e) pairs, returned sorted by e, which is row-major (CSR) order.

Everything is 64-bit integer arithmetic, so any implementation of this rule
gives the same set bit for bit.
"""

import numpy as np

GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix64(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def splitmix64_output(seed, e):
    """Output number e (0-based) of the SplitMix64 stream seeded with `seed`."""
    e = np.asarray(e, dtype=np.uint64)
    with np.errstate(over="ignore"):
        x = np.uint64(seed) + (e + np.uint64(1)) * GOLDEN_GAMMA
    return _mix64(x)


def sample_cells(m, n, K, seed):
    """Return the K sampled cell ids (int64, ascending) of an m x n grid."""
    total = int(m) * int(n)
    if not (0 <= K <= total):
        raise ValueError(f"K={K} outside [0, {total}]")
    if K == 0:
        return np.zeros(0, dtype=np.int64)
    if K == total:
        return np.arange(total, dtype=np.int64)
    keys = splitmix64_output(seed, np.arange(total, dtype=np.uint64))
    kth = np.partition(keys, K - 1)[K - 1]
    below = np.flatnonzero(keys < kth)
    ties = np.flatnonzero(keys == kth)          # ascending e breaks ties
    cells = np.concatenate([below, ties[: K - below.size]])
    cells.sort()
    return cells.astype(np.int64)


def cells_to_coo(cells, n):
    cells = np.asarray(cells, dtype=np.int64)
    return cells // n, (cells % n).astype(np.int64)
