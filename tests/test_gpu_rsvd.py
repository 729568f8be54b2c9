"""GPU parity of the standalone randomized SVDs against the oracle on the same
test matrix: rSVD-PI (Alg. 4) and rSVD-BKI (Alg. 5), one-shot and on a
resident matrix, from small ragged shapes up to the 45,115 x 45,115 sparse
matrix of the randomized-SVD comparison (Sec. V.A) at k = 100."""

import numpy as np
import pytest
import scipy.sparse

import synth
from oracle import gaussian_block, rsvd_bki, rsvd_pi

pytestmark = pytest.mark.gpu


def _sparse(p):
    return scipy.sparse.csr_matrix((p.vals, (p.rows, p.cols)), shape=(p.m, p.n))


def _desc(U, S, V):
    """The oracle returns the top k in ascending order (Alg. 3): flip."""
    return U[:, ::-1], S[::-1], V[:, ::-1]


def _proj_dist(Ua, Ub):
    """||Ua Ua^T - Ub Ub^T||_F for matrices with orthonormal columns."""
    k = Ua.shape[1]
    return np.sqrt(max(0.0, 2.0 * k - 2.0 * np.linalg.norm(Ua.T @ Ub) ** 2))


# block widths b = k + s from 7 to 80: every register tiling of the fused
# Gram's Cholesky (b <= 8, 16, 24, 32, 64) and the Cholesky kernel beyond
@pytest.mark.parametrize("m,n,k,s,p", [(500, 500, 11, 10, 3), (700, 300, 5, 10, 0),
                                       (300, 700, 20, 10, 1), (400, 400, 1, 10, 8),
                                       (257, 1031, 7, 3, 5), (130, 90, 30, 40, 2),
                                       (200, 150, 3, 4, 2), (700, 400, 40, 10, 1),
                                       (600, 500, 70, 10, 1)])
def test_rsvd_pi_matches_oracle_same_omega(m, n, k, s, p):
    from paper_1810_06860_amd import rsvd_pi as gpu_pi
    prob = synth.planted(m, n, 8, 0.3, seed_data=m + k, seed_phi=n + p)
    A = _sparse(prob)
    om = gaussian_block(n, k + s, 78, 4, 1)
    Uo, So, Vo = _desc(*rsvd_pi(A, k, p, om))
    Ug, Sg, Vg = gpu_pi(m, n, prob.rows, prob.cols, prob.vals, k, s, p, seed=78,
                        step=4, attempt=1)
    np.testing.assert_allclose(Sg, So, rtol=1e-8)
    Xo = (Uo * So) @ Vo.T
    Xg = (Ug * Sg) @ Vg.T
    assert np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo) < 1e-8
    assert np.linalg.norm(Ug.T @ Ug - np.eye(k)) < 1e-10
    assert np.all(np.diff(Sg) <= 0)


def test_rsvd_pi_exact_low_rank():
    """rank(A) = k + s (every cell observed, planted rank 10): the range of
    A Omega is the range of A, so every power iteration count returns the
    exact top-k SVD."""
    from paper_1810_06860_amd import rsvd_pi as gpu_pi
    prob = synth.planted(300, 200, 10, 1.0, seed_data=1, seed_phi=2)
    A = _sparse(prob).toarray()
    Sd = np.linalg.svd(A, compute_uv=False)[:4]
    for p in (0, 3):
        U, S, V = gpu_pi(300, 200, prob.rows, prob.cols, prob.vals, 4, 6, p, seed=3)
        np.testing.assert_allclose(S, Sd, rtol=1e-9)


def test_rsvd_pi_rejects_a_basis_wider_than_the_matrix():
    from paper_1810_06860_amd import MCError, rsvd_pi as gpu_pi
    prob = synth.planted(40, 30, 2, 0.5, seed_data=1, seed_phi=2)
    with pytest.raises(MCError):
        gpu_pi(40, 30, prob.rows, prob.cols, prob.vals, 25, 10, 1, seed=1)
    # a basis of exactly min(m, n) columns is allowed (PI keeps one block)
    U, S, V = gpu_pi(40, 30, prob.rows, prob.cols, prob.vals, 20, 10, 2, seed=1)
    Sd = np.linalg.svd(_sparse(prob).toarray(), compute_uv=False)[:20]
    np.testing.assert_allclose(S, Sd, rtol=1e-9)


def test_resident_matrix_matches_one_shot_calls():
    """mc_rsvd_init/run: repeated calls (graph replays after the first) give
    what the one-shot entry points give for the same (seed, step, attempt)."""
    from paper_1810_06860_amd import RSVD, rsvd_bki as gpu_bki, rsvd_pi as gpu_pi
    prob = synth.planted(600, 450, 6, 0.25, seed_data=9, seed_phi=19)
    h = RSVD(prob.m, prob.n, prob.rows, prob.cols, prob.vals, s=10, seed=5)
    try:
        for method, fn, p in (("pi", gpu_pi, 2), ("bki", gpu_bki, 2), ("pi", gpu_pi, 2),
                              ("pi", gpu_pi, 0), ("bki", gpu_bki, 1)):
            for step in (1, 2):
                U, S, V = h.run(method, 9, p, step=step)
                U1, S1, V1 = fn(prob.m, prob.n, prob.rows, prob.cols, prob.vals, 9, 10,
                                p, seed=5, step=step)
                np.testing.assert_allclose(S, S1, rtol=1e-13)
                assert np.linalg.norm((U * S) @ V.T - (U1 * S1) @ V1.T) <= \
                    1e-12 * np.linalg.norm(S1)
                _, S2, _ = h.run(method, 9, p, step=step, factors=False)
                np.testing.assert_allclose(S2, S, rtol=1e-13)
    finally:
        h.close()


@pytest.fixture(scope="module")
def sparse45k():
    return synth.sparse_square()


@pytest.mark.parametrize("method,p", [("pi", 0), ("pi", 4), ("bki", 4)])
def test_full_size_45k_matches_oracle(sparse45k, method, p):
    """The 45,115 x 45,115 matrix with 9 entries per row at k = 100, s = 10
    (the launch shapes that the benchmark times), against the oracle on the
    same test matrix: singular values, the top-k projector, orthonormality,
    and the approximation error from both sides."""
    from paper_1810_06860_amd import RSVD
    prob = sparse45k[2]
    A = _sparse(prob)
    k, s = 100, 10
    om = gaussian_block(prob.n, k + s, 31, 1, 0)
    ref = rsvd_pi if method == "pi" else rsvd_bki
    Uo, So, Vo = _desc(*ref(A, k, p, om))
    h = RSVD(prob.m, prob.n, prob.rows, prob.cols, prob.vals, s=s, seed=31)
    try:
        Ug, Sg, Vg = h.run(method, k, p, step=1)
    finally:
        h.close()
    np.testing.assert_allclose(Sg, So, rtol=1e-8)
    assert _proj_dist(Ug, Uo) < 1e-6
    assert _proj_dist(Vg, Vo) < 1e-6
    assert np.linalg.norm(Ug.T @ Ug - np.eye(k)) < 1e-9
    assert np.linalg.norm(Vg.T @ Vg - np.eye(k)) < 1e-9
    # A^T U = V S for the computed triplets (Rayleigh-Ritz: V = A^T U S^-1)
    np.testing.assert_allclose(A.T @ Ug, Vg * Sg, rtol=0, atol=1e-9 * Sg[0])
