"""Singular value thresholding with an exact SVD (Eq. (6), Alg. 2).

This is the definition the fast method approximates: Alg. 6 replaces the
truncated SVD of Alg. 2 by rSVD-BKI with subspace recycling and claims the
same recovered matrix and iteration count (Sec. IV.C, Sec. V).

Iteration (Eq. (6)):
    X^i = shrink(Y^{i-1}, tau)
    Y^i = Y^{i-1} + delta P_Phi(M - X^i)
with Y^0 = c delta P_Phi(M), c = ceil(tau / (delta ||P_Phi(M)||_2)), and the
stop test ||P_Phi(X^i - M)||_F / ||P_Phi(M)||_F < eps checked before the
update (Alg. 2).  shrink applies the soft threshold
max(sigma - tau, 0) to every singular value.  Alg. 2's incremental rank
search only serves to find every singular value above tau; a full
SVD finds them directly.  An optional rank cap keeps the largest k_max.

Defaults (Sec. II.C): tau = 5 n, l = 5.  The step size delta is not fixed by
the paper; the default is 1.2 m n / |Phi|.
"""

import math
from dataclasses import dataclass, field, asdict
from typing import List

import numpy as np


@dataclass
class SVTParams:
    tau: float = 0.0          # 0 -> 5 n
    delta: float = 0.0        # 0 -> 1.2 m n / |Phi|
    eps: float = 1e-4
    i_max: int = 200
    l: int = 5
    s: int = 10
    p_init: int = 3
    p_min: int = 1
    p_max: int = 8
    adaptive_p: int = 1
    i_reuse: int = 0
    q_reuse: int = 10
    recycle: int = 0          # 0 off, 1 reuse Q, 2 reuse U
    ritz_tol: float = 1e-4    # 0 -> the paper's gate alone
    k_max: int = 0            # rank cap, 0 -> none
    seed: int = 12345
    c: float = 0.0            # 0 -> ceil(tau / (delta ||P_Phi(M)||_2))

    @classmethod
    def from_dict(cls, d):
        names = set(cls.__dataclass_fields__)
        return cls(**{k: v for k, v in d.items() if k in names})

    def resolved(self, m, n, nnz):
        p = SVTParams(**asdict(self))
        if p.tau <= 0:
            p.tau = 5.0 * n
        if p.delta <= 0:
            p.delta = 1.2 * m * n / nnz
        return p


def shrink_factors(Y, tau, k_max=0):
    """shrink(Y, tau) of a dense Y as factors (U_r, S_r - tau, V_r)."""
    U, S, Vt = np.linalg.svd(Y, full_matrices=False)
    r = int(np.count_nonzero(S > tau))
    if k_max:
        r = min(r, k_max)
    return U[:, :r], S[:r] - tau, Vt[:r].T, S


def shrink(Y, tau, k_max=0):
    """Soft-threshold the singular values of a dense Y at level tau."""
    U, sig, V, _ = shrink_factors(Y, tau, k_max)
    return (U * sig) @ V.T


def spectral_norm(m, n, rows, cols, vals):
    """||P_Phi(M)||_2, the largest singular value of the sampled matrix."""
    if m * n <= 6_000_000:
        P = np.zeros((m, n))
        P[rows, cols] = vals
        return float(np.linalg.svd(P, compute_uv=False)[0])
    import scipy.sparse
    import scipy.sparse.linalg
    A = scipy.sparse.csr_matrix((vals, (rows, cols)), shape=(m, n))
    # PROPACK's Lanczos bidiagonalisation with a seeded start and room for
    # up to 400 Lanczos vectors: SciPy's default (10 for k = 1) gives up
    # before convergence when the top singular values are clustered
    s = scipy.sparse.linalg.svds(A, k=1, tol=1e-14, return_singular_vectors=False,
                                 solver="propack", maxiter=min(m, n, 400),
                                 rng=np.random.default_rng(0))
    return float(s[0])


def initial_c(tau, delta, norm2):
    return float(math.ceil(tau / (delta * norm2)))


@dataclass
class SVTResult:
    U: np.ndarray             # m x r
    sig: np.ndarray           # S - tau, descending (r)
    V: np.ndarray             # n x r
    iters: int
    res: float
    rank: int
    converged: bool
    x_phi: np.ndarray         # P_Phi(X) in the input (COO) order
    c: float
    res_hist: List[float] = field(default_factory=list)
    rank_hist: List[int] = field(default_factory=list)
    extra: dict = field(default_factory=dict)

    def dense(self):
        return (self.U * self.sig) @ self.V.T


def svt_exact(m, n, rows, cols, vals, params, callback=None):
    """Plain SVT with a dense FP64 SVD per step (Alg. 2)."""
    prm = SVTParams.from_dict(params) if isinstance(params, dict) else params
    prm = prm.resolved(m, n, len(vals))
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64)
    mnorm = float(np.linalg.norm(vals))
    c = prm.c if prm.c > 0 else initial_c(prm.tau, prm.delta,
                                          spectral_norm(m, n, rows, cols, vals))
    Y = np.zeros((m, n))
    Y[rows, cols] = c * prm.delta * vals                  # Y^0
    res_hist, rank_hist = [], []
    U = np.zeros((m, 0)); sig = np.zeros(0); V = np.zeros((n, 0))
    x_phi, r, res, conv, i = np.zeros_like(vals), 0, 1.0, False, 0
    for i in range(1, prm.i_max + 1):
        U, sig, V, _ = shrink_factors(Y, prm.tau, prm.k_max)   # X^i
        r = sig.size
        x_phi = np.einsum("ij,ij->i", U[rows] * sig, V[cols])
        res = float(np.linalg.norm(x_phi - vals)) / mnorm
        res_hist.append(res)
        rank_hist.append(r)
        if callback is not None:
            callback(i, U, sig, V, Y, res)
        if res < prm.eps:
            conv = True
            break
        Y[rows, cols] += prm.delta * (vals - x_phi)          # Y^i
    return SVTResult(U=U, sig=sig, V=V, iters=i, res=res, rank=r,
                     converged=conv, x_phi=x_phi, c=c,
                     res_hist=res_hist, rank_hist=rank_hist)
