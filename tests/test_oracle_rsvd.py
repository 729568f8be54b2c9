"""Pins of the randomized SVDs (Alg. 1, 4, 5) against Lemmas 2-3, Theorems
1-2, exact special cases and the Eq. (4) error bound."""

import numpy as np
import pytest
import scipy.sparse

from oracle import basic_rsvd, gaussian_block, lu_factor, rsvd_bki, rsvd_pi
from oracle.rsvd import orth


def _decaying(m, n, seed, decay=0.9, noise=0.0):
    rng = np.random.default_rng(seed)
    r = min(m, n)
    U, _ = np.linalg.qr(rng.standard_normal((m, r)))
    V, _ = np.linalg.qr(rng.standard_normal((n, r)))
    s = decay ** np.arange(r) * 100.0
    return (U * s) @ V.T + noise * rng.standard_normal((m, n))


def _proj(X):
    q = orth(X)
    return q @ q.T


def test_lu_factor_lemma3_range_and_structure():
    rng = np.random.default_rng(0)
    K = rng.standard_normal((50, 8))
    PL = lu_factor(K)
    # same column space (Lemma 3)
    assert np.linalg.norm(_proj(PL) - _proj(K)) < 1e-12
    # P^T L is a row permutation of a unit lower trapezoidal matrix, with
    # entries bounded by 1 (partial pivoting)
    assert np.max(np.abs(PL)) <= 1.0 + 1e-15
    ones = np.isclose(PL, 1.0)
    assert ones.sum(axis=0).min() >= 1
    # K = (P^T L) U for an upper-triangular U
    U = np.linalg.lstsq(PL, K, rcond=None)[0]
    assert np.allclose(np.tril(U, -1), 0.0, atol=1e-12)
    assert np.allclose(PL @ U, K, atol=1e-12)


@pytest.mark.parametrize("p", [0, 1, 4])
def test_theorem1_rsvd_pi_equals_basic(p):
    A = _decaying(400, 300, 1, decay=0.97)
    k, s = 20, 10
    om = gaussian_block(300, k + s, 5, 1, 0)
    U1, S1, V1 = basic_rsvd(A, k, p, om)
    U4, S4, V4 = rsvd_pi(A, k, p, om)
    assert np.allclose(S4[::-1], S1, rtol=1e-9)
    X1 = (U1 * S1) @ V1.T
    X4 = (U4 * S4) @ V4.T
    assert np.linalg.norm(X1 - X4) / np.linalg.norm(X1) < 1e-9


def test_theorem2_rsvd_bki_equals_plain_block_krylov():
    A = _decaying(300, 200, 2, decay=0.95)
    k, s, p = 15, 5, 2
    om = gaussian_block(200, k + s, 6, 1, 0)
    U, S, V = rsvd_bki(A, k, p, om)
    # original block Krylov: Q = orth([A om, (A A^T) A om, (A A^T)^2 A om]),
    # then the exact SVD of Q^T A (Musco & Musco), no LU in between
    K0 = A @ om
    K1 = A @ (A.T @ K0)
    K2 = A @ (A.T @ K1)
    Q = orth(np.hstack([K0, K1, K2]))
    Sd = np.linalg.svd(Q.T @ A, compute_uv=False)[:k]
    assert np.allclose(S[::-1], Sd, rtol=1e-9)


@pytest.mark.parametrize("which", ["low_rank", "full_krylov"])
def test_rsvd_bki_exact_cases(which):
    rng = np.random.default_rng(3)
    if which == "low_rank":          # rank(A) <= k + s
        A = rng.standard_normal((120, 12)) @ rng.standard_normal((12, 90))
        k, s, p = 8, 6, 1
    else:                            # (p+1)(k+s) >= min(m, n)
        A = rng.standard_normal((80, 40))
        k, s, p = 10, 10, 1
    om = gaussian_block(A.shape[1], k + s, 1, 1, 0)
    U, S, V = rsvd_bki(A, k, p, om)
    Ud, Sd, Vtd = np.linalg.svd(A, full_matrices=False)
    assert np.allclose(S[::-1], Sd[:k], rtol=1e-11)
    Xk = (Ud[:, :k] * Sd[:k]) @ Vtd[:k]
    assert np.linalg.norm((U * S) @ V.T - Xk) / np.linalg.norm(Xk) < 1e-10
    assert np.linalg.norm(U.T @ U - np.eye(k)) < 1e-12


def test_rsvd_bki_eq4_bound_and_p_monotone():
    A = scipy.sparse.random(600, 400, density=0.05, random_state=4,
                            data_rvs=np.random.default_rng(4).standard_normal)
    A = scipy.sparse.csr_matrix(A)
    Ad = A.toarray()
    Sd = np.linalg.svd(Ad, compute_uv=False)
    k, s = 20, 10
    best = np.sqrt(np.sum(Sd[k:] ** 2))
    errs = []
    for p in (0, 1, 3):
        om = gaussian_block(400, k + s, 7, 1, 0)
        U, S, V = rsvd_bki(A, k, p, om)
        errs.append(np.linalg.norm(Ad - (U * S) @ V.T))
    assert errs[2] <= 1.05 * best                 # Eq. (4), eps = 0.05
    assert errs[0] >= errs[1] >= errs[2] * (1 - 1e-12)
    # the kept values are the largest ones, and never exceed the true ones
    assert np.all(S[::-1] <= Sd[:k] * (1 + 1e-12))
    assert np.allclose(S[::-1], Sd[:k], rtol=3e-2)      # flat spectrum


def test_lemma2_projector_independent_of_basis():
    A = _decaying(200, 150, 5, decay=0.96, noise=1e-3)
    om = gaussian_block(150, 25, 2, 1, 0)
    H = A @ om
    P1 = _proj(H)
    P2 = _proj(lu_factor(H))
    # eigSVD's U as the basis (the "replace Q by U" idea)
    from oracle import eigsvd
    U, _, _ = eigsvd(H)
    P3 = U @ U.T
    assert np.linalg.norm(P1 - P2) < 1e-10
    assert np.linalg.norm(P1 - P3) < 1e-10
