"""Synthetic completion problems (inputs only).

Recipes
-------
planted      M = U V^T with U (m x r), V (n x r) i.i.d. N(0, 1); Phi uniform
             without replacement (``sampler``), K = floor(ratio*m*n + 0.5).
image_like   A = U diag(255 * i^-1.5) V^T with Haar-random orthogonal U, V
             (QR of a Gaussian matrix with the sign of diag(R) folded in,
             Mezzadri 2007), clipped to [0, 255]; Phi uniform.  Stand-in for
             the paper's colour image (Sec. V.B).
ratings      Zipf(s) row degrees water-filled under the cap n and summing to
             nnz exactly, placed on rows in a seeded random order; each row's
             columns drawn without replacement with probability proportional
             to a (permuted) Zipf(s) column weight; values
             round(3.5 + (U_i . V_j) / sqrt(r)) clipped to 1..5 with
             U, V ~ N(0, 1).  Stand-in for the MovieLens sets (Sec. V.C).
serving_trace  Poisson arrivals and per-request planted problems.
sparse_square  the ratings recipe on a square n x n matrix with a given mean
             number of entries per row, and sparser copies made by keeping a
             seeded uniform subset of its entries.  Stand-in for the
             45,115 x 45,115 rating matrix and its two thinned versions that
             the randomized-SVD comparison of Sec. V.A uses (97, 24 and 9
             entries per row).
"""

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from .sampler import sample_cells, cells_to_coo


@dataclass
class Problem:
    m: int
    n: int
    rows: np.ndarray            # int64, COO row ids (row-major order)
    cols: np.ndarray            # int64, COO column ids
    vals: np.ndarray            # float64, M at Phi
    name: str = ""
    U: Optional[np.ndarray] = None      # planted factors, when known
    V: Optional[np.ndarray] = None
    dense: Optional[np.ndarray] = None  # full ground truth, when small
    meta: dict = field(default_factory=dict)
    offset: float = 0.0         # truth = offset + scale * U V^T (before any
    scale: float = 1.0          # rounding or clipping of the observed values)

    @property
    def nnz(self):
        return int(self.vals.size)

    def truth_dense(self, max_cells=1 << 25):
        """The full ground truth, or None when unknown or above max_cells."""
        if self.dense is not None:
            return self.dense
        if self.U is not None and self.m * self.n <= max_cells:
            return self.offset + self.scale * (self.U @ self.V.T)
        return None

    def truth_at(self, rows, cols):
        """Ground truth at the given cells, or None when unknown."""
        if self.dense is not None:
            return self.dense[rows, cols]
        if self.U is None:
            return None
        return self.offset + self.scale * np.einsum(
            "ij,ij->i", self.U[rows], self.V[cols])


def planted(m, n, rank, ratio, seed_data, seed_phi, name="planted"):
    rng = np.random.default_rng(seed_data)
    U = rng.standard_normal((m, rank))
    V = rng.standard_normal((n, rank))
    K = int(np.floor(ratio * m * n + 0.5))
    rows, cols = cells_to_coo(sample_cells(m, n, K, seed_phi), n)
    vals = np.empty(K)
    for a in range(0, K, 1 << 18):            # chunks keep the gathers small
        b = min(K, a + (1 << 18))
        vals[a:b] = np.einsum("ij,ij->i", U[rows[a:b]], V[cols[a:b]])
    return Problem(m, n, rows, cols, vals, name=name, U=U, V=V,
                   meta=dict(rank=rank, ratio=ratio, seed_data=seed_data,
                             seed_phi=seed_phi))


def _haar(n, rng):
    z = rng.standard_normal((n, n))
    q, r = np.linalg.qr(z)
    return q * np.sign(np.diag(r))


def image_like(n=1024, ratio=0.5, seed_data=2, seed_phi=102, name="image"):
    rng = np.random.default_rng(seed_data)
    U = _haar(n, rng)
    V = _haar(n, rng)
    s = 255.0 * np.arange(1, n + 1, dtype=np.float64) ** -1.5
    A = np.clip((U * s) @ V.T, 0.0, 255.0)
    K = int(np.floor(ratio * n * n + 0.5))
    rows, cols = cells_to_coo(sample_cells(n, n, K, seed_phi), n)
    vals = A[rows, cols].copy()
    return Problem(n, n, rows, cols, vals, name=name, dense=A,
                   meta=dict(ratio=ratio, seed_data=seed_data,
                             seed_phi=seed_phi))


def zipf_degrees(count, total, cap, s):
    """Integer degrees d_r ~ r^-s (r = 1..count), each <= cap, sum == total."""
    if total > count * cap:
        raise ValueError("total exceeds count*cap")
    w = np.arange(1, count + 1, dtype=np.float64) ** -s
    capped = np.zeros(count, dtype=bool)
    d = np.zeros(count)
    for _ in range(count + 1):             # water-filling
        free = ~capped
        rest = total - cap * capped.sum()
        d[free] = rest * w[free] / w[free].sum()
        d[capped] = cap
        over = free & (d > cap)
        if not over.any():
            break
        capped |= over
    base = np.floor(d).astype(np.int64)
    short = int(total - base.sum())
    frac = d - base
    frac[base >= cap] = -1.0
    order = np.lexsort((np.arange(count), -frac))   # largest remainder first
    base[order[:short]] += 1
    assert base.sum() == total and base.max() <= cap
    return base


def ratings(m, n, nnz, rank, s=1.1, seed_data=3, name="ratings"):
    rng = np.random.default_rng(seed_data)
    deg = zipf_degrees(m, nnz, n, s)[rng.permutation(m)]
    colw = (np.arange(1, n + 1, dtype=np.float64) ** -s)[rng.permutation(n)]
    colp = colw / colw.sum()
    cdf = np.cumsum(colp)
    cdf[-1] = 1.0
    rows_out = np.empty(nnz, dtype=np.int64)
    cols_out = np.empty(nnz, dtype=np.int64)
    pos = 0
    for i in range(m):
        d = int(deg[i])
        if d == 0:
            continue
        if d >= n:
            c = np.arange(n, dtype=np.int64)
        elif d > 256:
            # Efraimidis-Spirakis keys u^(1/w): top-d keys = weighted sample
            # without replacement.
            key = np.log(rng.random(n)) / colw
            c = np.sort(np.argpartition(-key, d - 1)[:d]).astype(np.int64)
        else:
            # successive sampling: draw with replacement, keep first arrivals
            got = np.zeros(0, dtype=np.int64)
            while got.size < d:
                draw = np.searchsorted(cdf, rng.random(4 * d + 16), side="right")
                draw = np.minimum(draw, n - 1)
                allc = np.concatenate([got, draw])
                _, first = np.unique(allc, return_index=True)
                got = allc[np.sort(first)][:d]
            c = np.sort(got)
        rows_out[pos:pos + d] = i
        cols_out[pos:pos + d] = c
        pos += d
    assert pos == nnz
    U = rng.standard_normal((m, rank))
    V = rng.standard_normal((n, rank))
    raw = np.einsum("ij,ij->i", U[rows_out], V[cols_out]) / np.sqrt(rank)
    vals = np.clip(np.rint(3.5 + raw), 1.0, 5.0)
    return Problem(m, n, rows_out, cols_out, vals, name=name, U=U, V=V,
                   offset=3.5, scale=1.0 / np.sqrt(rank),
                   meta=dict(rank=rank, s=s, seed_data=seed_data,
                             integer_values=True))


def serving_trace(num=256, mean_gap_s=0.05, seed=4, mn_range=(200, 4000),
                  rank_range=(5, 50), ratio_range=(0.1, 0.4), base_seed=4000):
    """Request descriptors (no matrices): arrival time, shape, rank, ratio."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(mean_gap_s, size=num)
    t = np.cumsum(gaps) - gaps[0]
    reqs = []
    for j in range(num):
        m = int(rng.integers(mn_range[0], mn_range[1] + 1))
        n = int(rng.integers(mn_range[0], mn_range[1] + 1))
        r = int(rng.integers(rank_range[0], rank_range[1] + 1))
        ratio = float(rng.uniform(*ratio_range))
        reqs.append(dict(id=j, t_arrival=float(t[j]), m=m, n=n, rank=r,
                         ratio=ratio, seed_data=base_seed + j,
                         seed_phi=base_seed + 100000 + j))
    return reqs


def request_problem(req):
    return planted(req["m"], req["n"], req["rank"], req["ratio"],
                   req["seed_data"], req["seed_phi"],
                   name=f"req{req['id']}")


def sparse_square(n=45115, per_row=(97, 24, 9), rank=20, seed_data=6, seed_thin=7,
                  name="sparse45k"):
    """Problems of mean row density per_row[0], per_row[1], ...: the first is
    generated by ``ratings``, each later one keeps a uniform random subset of
    the first one's entries (sorted, so still in row-major order)."""
    full = ratings(n, n, int(per_row[0]) * n, rank, seed_data=seed_data,
                   name=f"{name}_{per_row[0]}")
    out = [full]
    rng = np.random.default_rng(seed_thin)
    for d in per_row[1:]:
        keep = np.sort(rng.choice(full.nnz, size=int(d) * n, replace=False))
        out.append(Problem(n, n, full.rows[keep], full.cols[keep], full.vals[keep],
                           name=f"{name}_{d}", U=full.U, V=full.V,
                           offset=full.offset, scale=full.scale,
                           meta=dict(full.meta, thinned_from=per_row[0])))
    return out
