"""eigSVD (Alg. 3, Lemma 1): the economic SVD of a tall matrix via eig(A^T A).

Steps, for A (m x n, m >= n):
  1. B = A^T A
  2. [V, D] = eig(B)            (symmetric; eigenvalues ascending)
  3. S = sqrt(D)
  4. U = A V S^-1
The singular values come out in ascending order (remark after Lemma 1).
Round-off can leave tiny negative entries in D, and a rank-deficient A makes
S^-1 undefined (same remark); S is therefore taken as sqrt(max(D, 0)), and
``eigsvd_top`` forms U only for the kept (largest) columns, and refuses a
kept value at the round-off floor of D (S_j <= sqrt(n u) S_max, u the unit
round-off), where A V S^-1 would carry no accurate digits.
"""

import numpy as np


def eigsvd(A):
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if m < n:
        raise ValueError("eigSVD needs m >= n")
    B = A.T @ A
    D, V = np.linalg.eigh(B)
    S = np.sqrt(np.maximum(D, 0.0))
    with np.errstate(divide="ignore", invalid="ignore"):
        U = (A @ V) / S
    return U, S, V


def eigsvd_top(A, k):
    """eigSVD restricted to the k largest values (still ascending)."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if m < n:
        raise ValueError("eigSVD needs m >= n")
    if not 0 < k <= n:
        raise ValueError("k out of range")
    B = A.T @ A
    D, V = np.linalg.eigh(B)
    D, V = D[n - k:], V[:, n - k:]
    S = np.sqrt(np.maximum(D, 0.0))
    if S[0] <= np.sqrt(n * np.finfo(np.float64).eps) * S[-1]:
        raise np.linalg.LinAlgError("eigSVD: kept singular value at round-off")
    U = (A @ V) / S
    return U, S, V
