"""Randomized truncated SVD of a (sparse) matrix A (Sec. II.B, Sec. III).

All three take the Gaussian test matrix Omega (n x (k+s)) as an input, so a
caller can feed the same Omega to another implementation.

basic_rsvd  Alg. 1: Q = orth(A Omega); p power iterations with orth after
            every product; B = Q^T A; svd(B); U = Q U; keep the first k.
rsvd_pi     Alg. 4: LU (its P^T L factor) between the A(A^T .) pairs,
            eigSVD for the last Q and for B^T, keep ind = s+1 : k+s.
rsvd_bki    Alg. 5: H_0 = lu(A Omega); H_i = lu(A (A^T H_{i-1})) for
            i = 1..p; Q = orth([H_0 .. H_p]); B = Q^T A; [V, S, U] =
            eigSVD(B^T); keep ind = (k+s)(p+1)-k+1 : (k+s)(p+1).
            The listing guards step 4 with "if i < p" although step 6 stacks
            H_p and `ind` counts (p+1)(k+s) columns; H_p is read as formed
            for every i, with the LU skipped for i = p because orth follows.

Outputs keep the paper's convention: singular values ascending, U (m x k),
V (n x k) (the listings' "V in R^{k x n}" is read as n x k).
"""

import numpy as np
import scipy.linalg

from .eigsvd import eigsvd, eigsvd_top


def lu_factor(X):
    """First output of Matlab-style lu(X): the row-permuted unit lower
    trapezoidal factor P^T L with X = (P^T L) U (Eq. (9), Lemma 3)."""
    PL, _ = scipy.linalg.lu(np.asarray(X, dtype=np.float64), permute_l=True)
    return PL


def orth(X):
    """Orthonormal basis of range(X) by a reduced QR factorisation."""
    q, _ = np.linalg.qr(np.asarray(X, dtype=np.float64), mode="reduced")
    return q


def basic_rsvd(A, k, p, Omega):
    Q = orth(A @ Omega)
    for _ in range(p):
        G = orth(A.T @ Q)
        Q = orth(A @ G)
    B = np.asarray((A.T @ Q).T)
    U, S, Vt = np.linalg.svd(B, full_matrices=False)
    U = Q @ U
    return U[:, :k], S[:k], Vt[:k].T


def rsvd_pi(A, k, p, Omega):
    b = Omega.shape[1]
    s = b - k
    Q = np.asarray(A @ Omega)
    for i in range(p + 1):
        if i < p:
            Q = lu_factor(Q)
        else:
            Q, _, _ = eigsvd(Q)
            break
        Q = np.asarray(A @ (A.T @ Q))
    Bt = np.asarray(A.T @ Q)                    # B^T = A^T Q  (n x b)
    V, S, U = eigsvd(Bt)
    ind = slice(s, s + k)
    return Q @ U[:, ind], S[ind], V[:, ind]


def rsvd_bki(A, k, p, Omega, return_q=False):
    b = Omega.shape[1]
    H = [lu_factor(A @ Omega)]
    for i in range(1, p + 1):
        Hi = np.asarray(A @ (A.T @ H[i - 1]))
        H.append(lu_factor(Hi) if i < p else Hi)
    Q = orth(np.hstack(H))                      # m x (p+1) b
    L = Q.shape[1]
    assert L == (p + 1) * b
    Bt = np.asarray(A.T @ Q)                    # B^T = (Q^T A)^T, n x L
    V, S, W = eigsvd_top(Bt, k)                 # ind = last k of L
    U = Q @ W
    if return_q:
        return U, S, V, Q
    return U, S, V
