"""eigSVD (Sec. III.A, Alg. 3): the economic SVD of a tall matrix A (m x n,
m >= n) read off the symmetric eigendecomposition of its Gram matrix A^T A
(Lemma 1: the eigenvectors are the right singular vectors, the square roots
of the eigenvalues the singular values, and A V S^-1 the left singular
vectors).

The values come out ascending, as the eigensolver returns them (the remark
after Lemma 1).  Round-off can leave tiny negative eigenvalues, and a
rank-deficient A makes S^-1 undefined (same remark): S is taken as
sqrt(max(D, 0)), and ``eigsvd_top`` forms the left vectors only for the kept
(largest) values and refuses a kept value at the round-off floor of D
(S_j <= sqrt(n u) S_max, u the unit round-off), where A V S^-1 would carry no
accurate digits.
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
