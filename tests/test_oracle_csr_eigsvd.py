"""Pins of the CSR/CSC layout and of eigSVD (Alg. 3, Lemma 1)."""

import numpy as np
import pytest
import scipy.sparse

from oracle import canonical_csr, eigsvd, eigsvd_top
from oracle.csr import CSRError


def _random_coo(m, n, K, seed):
    rng = np.random.default_rng(seed)
    cells = rng.choice(m * n, size=K, replace=False)
    return cells // n, cells % n


@pytest.mark.parametrize("m,n,K", [(40, 30, 200), (1, 50, 20), (60, 1, 10),
                                   (25, 25, 625), (100, 80, 1)])
def test_csr_matches_scipy(m, n, K):
    rows, cols = _random_coo(m, n, K, m + n)
    lay = canonical_csr(m, n, rows, cols)
    vals = np.arange(K, dtype=np.float64) + 1.0
    A = scipy.sparse.csr_matrix((vals, (rows, cols)), shape=(m, n))
    A.sort_indices()
    assert np.array_equal(lay["row_ptr"], A.indptr)
    assert np.array_equal(lay["col_idx"], A.indices)
    assert np.array_equal(vals[lay["order"]], A.data)
    C = A.tocsc()
    C.sort_indices()
    assert np.array_equal(lay["col_ptr"], C.indptr)
    assert np.array_equal(lay["row_idx"], C.indices)
    assert np.array_equal(A.data[lay["perm"]], C.data)


def test_csr_rejects_bad_input():
    with pytest.raises(CSRError):
        canonical_csr(3, 3, [0, 1, 1], [0, 2, 2])
    with pytest.raises(CSRError):
        canonical_csr(3, 3, [0, 3], [0, 0])
    with pytest.raises(CSRError):
        canonical_csr(3, 3, [0, 1], [0, -1])


def _matrix_with_spectrum(m, n, s, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, len(s))))
    V, _ = np.linalg.qr(rng.standard_normal((n, len(s))))
    return (U * s) @ V.T


def test_eigsvd_closed_form():
    A = np.array([[3.0, 0.0], [0.0, 4.0], [0.0, 0.0]])
    U, S, V = eigsvd(A)
    assert np.allclose(S, [3.0, 4.0], rtol=0, atol=1e-15)     # ascending
    assert np.allclose(np.abs(V), np.eye(2))
    assert np.allclose(np.abs(U), np.eye(3)[:, :2])


@pytest.mark.parametrize("kappa", [1e1, 1e3, 1e4])
def test_eigsvd_lemma1_matches_svd(kappa):
    m, n = 300, 40
    s = np.logspace(0, np.log10(kappa), n)[::-1]
    A = _matrix_with_spectrum(m, n, s, 5)
    U, S, V = eigsvd(A)
    Ud, Sd, Vtd = np.linalg.svd(A, full_matrices=False)
    assert np.all(np.diff(S) >= 0)
    rel = np.abs(S[::-1] - Sd) / Sd
    bound = 1e-13 * (Sd[0] / Sd) ** 2 + 1e-14
    assert np.all(rel <= bound)
    assert np.linalg.norm(U.T @ U - np.eye(n)) < 1e-15 * kappa ** 2 * 10
    assert np.linalg.norm((U * S) @ V.T - A) / np.linalg.norm(A) < 1e-12 * kappa
    # singular subspaces agree (vectors are unique up to sign)
    assert np.allclose(np.abs(np.sum(V[:, ::-1] * Vtd.T, axis=0)), 1.0,
                       atol=1e-8 * kappa)


def test_eigsvd_top_subset_and_rank_deficiency():
    A = _matrix_with_spectrum(200, 30, np.linspace(5, 1, 30), 1)
    U, S, V = eigsvd(A)
    Ut, St, Vt = eigsvd_top(A, 7)
    assert np.allclose(St, S[-7:], rtol=1e-14)
    assert np.allclose(np.abs(np.sum(Ut * U[:, -7:], axis=0)), 1.0, atol=1e-12)
    B = _matrix_with_spectrum(100, 10, np.array([3.0, 2.0, 1.0]), 2)
    with pytest.raises(np.linalg.LinAlgError):
        eigsvd_top(B, 5)
    Ub, Sb, Vb = eigsvd_top(B, 3)
    assert np.allclose(Sb, [1.0, 2.0, 3.0], rtol=1e-10)
