"""Pins of the oracle's recycled SVD (Sec. IV.B), its Ritz residual and the
large-shape branch of its spectral norm.

Recycling replaces rSVD-BKI by the Rayleigh-Ritz step on a saved basis: the
singular triplets of basis^T Y, lifted back by the basis (Lemma 2).  The
oracle computes them with eigSVD (Alg. 3) of Y^T basis; the pins below take
the same triplets from LAPACK's SVD of the dense projection instead, and the
Ritz residual from a constructed case whose value is known in closed form.
"""

import numpy as np
import pytest
import scipy.sparse

import synth
from oracle import FastSVT, spectral_norm
from oracle.svt import SVTParams


def _proj(X):
    q, _ = np.linalg.qr(X)
    return q @ q.T


def _small_solver(strategy, seed=11, **kw):
    p = synth.planted(120, 100, 4, 0.35, seed_data=seed, seed_phi=seed + 100)
    prm = dict(tau=500.0, delta=1.2 / 0.35, eps=1e-3, i_max=250, recycle=strategy,
               **kw)
    return p, FastSVT(p.m, p.n, p.rows, p.cols, p.vals, prm)


@pytest.mark.parametrize("strategy", [1, 2])
def test_recycled_equals_dense_svd_of_projection(strategy):
    # _recycled on a given Y and basis: the top k of svd(basis^T Y)
    rng = np.random.default_rng(20 + strategy)
    m, n, w, k = 90, 70, 24 if strategy == 1 else 9, 6
    dense = rng.standard_normal((m, 5)) @ rng.standard_normal((5, n)) * 3.0
    dense += 0.05 * rng.standard_normal((m, n))
    mask = rng.random((m, n)) < 0.6
    Y = scipy.sparse.csr_matrix(np.where(mask, dense, 0.0))
    Yd = Y.toarray()
    basis, _ = np.linalg.qr(Yd @ rng.standard_normal((n, w)))
    _, f = _small_solver(strategy)
    f.saved = basis
    U, S, V = f._recycled(Y, k)
    W, Sd, Zt = np.linalg.svd(basis.T @ Yd, full_matrices=False)
    assert np.all(np.diff(S) <= 0)
    assert np.allclose(S, Sd[:k], rtol=1e-12, atol=0)
    assert np.linalg.norm(_proj(U) - _proj(basis @ W[:, :k])) < 1e-10
    assert np.linalg.norm(_proj(V) - _proj(Zt[:k].T)) < 1e-10
    # the left Ritz condition holds exactly: Y^T U = V diag(S)
    assert np.allclose(Yd.T @ U, V * S, rtol=0, atol=1e-10 * S[0])


@pytest.mark.parametrize("strategy", [1, 2])
def test_recycled_steps_equal_dense_projection(strategy):
    # through FastSVT.step: every step served by recycled calls alone returns
    # the top k of svd(saved^T Y^{i-1}) and X from its top r
    p, f = _small_solver(strategy, i_reuse=20, q_reuse=3, ritz_tol=0.0)
    checked = 0
    for _ in range(60):
        basis = None if f.saved is None else f.saved.copy()
        Yd = f.Y().toarray()
        info = f.step()
        if info.fresh == 0 and info.recycled > 0:
            W, Sd, Zt = np.linalg.svd(basis.T @ Yd, full_matrices=False)
            assert np.allclose(info.S, Sd[:info.k], rtol=1e-12, atol=0)
            r = info.r
            Xd = (basis @ W[:, :r] * (Sd[:r] - f.prm.tau)) @ Zt[:r]
            X = (f.U * f.sig) @ f.V.T
            assert np.linalg.norm(X - Xd) <= 1e-11 * np.linalg.norm(Xd)
            checked += 1
        if info.converged:
            break
    assert checked >= 10


def test_ritz_residual_closed_form():
    # exact singular triplets give a zero residual; turning v_0 by theta
    # towards v_5 gives ||Y v - s_0 u_0|| = sqrt(((1 - cos t) s_0)^2 +
    # (sin t s_5)^2), divided by s_0
    rng = np.random.default_rng(5)
    Yd = rng.standard_normal((40, 30))
    Ud, Sd, Vtd = np.linalg.svd(Yd, full_matrices=False)
    Y = scipy.sparse.csr_matrix(Yd)
    _, f = _small_solver(1)
    k = 3
    U, S, V = Ud[:, :k], Sd[:k], Vtd[:k].T.copy()
    assert f._ritz(Y, U, S, V) < 1e-13
    t = 0.3
    V[:, 0] = np.cos(t) * Vtd[0] + np.sin(t) * Vtd[5]
    want = np.hypot((1 - np.cos(t)) * Sd[0], np.sin(t) * Sd[5]) / Sd[0]
    assert f._ritz(Y, U, S, V) == pytest.approx(want, rel=1e-12)
    # the worst column decides: turning v_2 further gives its own ratio
    t2 = 0.5
    V[:, 2] = np.cos(t2) * Vtd[2] + np.sin(t2) * Vtd[7]
    want2 = np.hypot((1 - np.cos(t2)) * Sd[2], np.sin(t2) * Sd[7]) / Sd[2]
    assert f._ritz(Y, U, S, V) == pytest.approx(max(want, want2), rel=1e-12)


@pytest.mark.parametrize("strategy", [1, 2])
def test_guarded_solve_accepts_recycles(strategy):
    # the Ritz guard at 1e-3 keeps some recycled results on this problem
    _, f = _small_solver(strategy, i_reuse=20, q_reuse=3, ritz_tol=1e-3)
    for _ in range(250):
        if f.step().converged:
            break
    assert f.converged
    assert f.recycled_total - f.rejected_total > 0


def test_spectral_norm_large_shape_branch():
    # m n = 6.3e6 > 6e6 takes the sparse (PROPACK) route
    m, n = 3000, 2100
    rng = np.random.default_rng(8)
    A = scipy.sparse.random(m, n, density=0.003, random_state=9, format="coo",
                            data_rvs=rng.standard_normal)
    got = spectral_norm(m, n, A.row.astype(np.int64), A.col.astype(np.int64), A.data)
    want = np.linalg.svd(A.toarray(), compute_uv=False)[0]
    assert got == pytest.approx(want, rel=1e-10)
    # closed form: a diagonal of distinct values has norm max |d_i|
    d = np.linspace(-7.5, 3.0, 2100)
    idx = np.arange(2100, dtype=np.int64)
    got = spectral_norm(m, n, idx * 1, idx, d)
    assert got == pytest.approx(7.5, rel=1e-12)


def test_params_resolved_defaults():
    prm = SVTParams().resolved(30, 20, 150)
    assert prm.tau == 100.0 and prm.delta == pytest.approx(1.2 * 600 / 150)
