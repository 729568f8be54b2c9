"""Randomized truncated SVD of a (sparse) matrix A (Sec. II.B, Sec. III).

Each routine is written from what it computes, not from a printed listing:

basic_rsvd  the randomized SVD of Sec. II.B (Alg. 1): an orthonormal basis
            of the range of (A A^T)^p A Omega, kept orthonormal after every
            product, then the exact SVD of the projection Q^T A.
rsvd_pi     rSVD-PI (Sec. III.A, Alg. 4).  Theorem 1: it gives the same
            subspace as basic_rsvd -- range((A A^T)^p A Omega) -- with the
            cheaper LU normalisation between the power iterations (Lemma 3:
            the P^T L factor spans the same range), and it finishes with
            eigSVD (Alg. 3) instead of a QR + SVD.
rsvd_bki    rSVD-BKI (Sec. III.B, Alg. 5).  Theorem 2: its basis spans the
            block Krylov space [A Omega, (A A^T) A Omega, ...,
            (A A^T)^p A Omega] of Musco & Musco; every block is
            LU-normalised before it feeds the next product (Lemma 3), and
            the top k singular triplets come from eigSVD of B^T = A^T Q.

Both finish with the Rayleigh-Ritz step of Sec. II.B: for an orthonormal Q
the SVD of B = Q^T A gives U = Q W; only the projector Q Q^T matters there
(Lemma 2), so any orthonormalisation of the basis gives the same result.

All three take the Gaussian test matrix Omega (n x b, b = k + s) as an
input so that another implementation can be fed the same Omega.  Outputs
keep the paper's convention: singular values ascending, U (m x k), V (n x k)
(the listings' "V in R^{k x n}" is read as n x k).
"""

import numpy as np
import scipy.linalg

from .eigsvd import eigsvd_top


def lu_factor(X):
    """First output of Matlab-style lu(X): the row-permuted unit lower
    trapezoidal factor P^T L with X = (P^T L) U (Eq. (9), Lemma 3)."""
    PL, _ = scipy.linalg.lu(np.asarray(X, dtype=np.float64), permute_l=True)
    return PL


def orth(X):
    """Orthonormal basis of range(X) by a reduced QR factorisation."""
    q, _ = np.linalg.qr(np.asarray(X, dtype=np.float64), mode="reduced")
    return q


def _times_aat(A, H):
    """A (A^T H): one power-iteration product, two sparse products."""
    return np.asarray(A @ np.asarray(A.T @ H))


def _top_k_of_projection(A, Q, k):
    """Rayleigh-Ritz step (Sec. II.B) with eigSVD (Alg. 3): the k largest
    singular triplets of B = Q^T A, lifted back to U = Q W.  eigSVD runs on
    the tall B^T = A^T Q (n x L), whose left singular vectors are V."""
    Bt = np.asarray(A.T @ Q)
    V, S, W = eigsvd_top(Bt, k)                 # ascending, top k of L
    return Q @ W, S, V


def basic_rsvd(A, k, p, Omega):
    """Alg. 1 with a QR after every product (the textbook form)."""
    Q = orth(A @ Omega)
    for _ in range(p):
        Q = orth(A @ orth(A.T @ Q))
    B = np.asarray((A.T @ Q).T)
    U, S, Vt = np.linalg.svd(B, full_matrices=False)
    return (Q @ U)[:, :k], S[:k], Vt[:k].T


def rsvd_pi(A, k, p, Omega):
    """rSVD-PI: basis of range((A A^T)^p A Omega), LU-normalised between
    the power iterations and orthonormalised once at the end, then the top
    k triplets of the projection (Theorem 1)."""
    H = lu_factor(A @ Omega) if p > 0 else np.asarray(A @ Omega)
    for it in range(p):
        H = _times_aat(A, H)
        if it < p - 1:
            H = lu_factor(H)
    return _top_k_of_projection(A, orth(H), k)


def rsvd_bki(A, k, p, Omega, return_q=False):
    """rSVD-BKI: orthonormal basis of the (p + 1)-block Krylov space built
    from LU-normalised blocks, then the top k triplets of the projection
    (Theorem 2).  With return_q the basis Q (m x (p + 1) b) is returned too,
    for recycling (Sec. IV.B)."""
    block = lu_factor(A @ Omega)
    blocks = [block]
    for _ in range(p):
        block = lu_factor(_times_aat(A, block))
        blocks.append(block)
    Q = orth(np.hstack(blocks))
    if Q.shape[1] != (p + 1) * Omega.shape[1]:
        raise ValueError("Krylov basis narrower than (p + 1) b")
    U, S, V = _top_k_of_projection(A, Q, k)
    if return_q:
        return U, S, V, Q
    return U, S, V
