"""Pins of the SVT oracles: closed form on a fully observed matrix, the
proximal characterisation of shrink, planted recovery, the adaptive-p rule,
and fast SVT (Alg. 6) against plain SVT (Alg. 2)."""

import math

import numpy as np
import pytest

import synth
from oracle import (FastSVT, SVTParams, adapt_p, fast_svt, initial_c, shrink,
                    shrink_factors, svt_exact)


def _spectral(m, n, s, seed):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.standard_normal((m, len(s))))
    V, _ = np.linalg.qr(rng.standard_normal((n, len(s))))
    return U, np.asarray(s, dtype=np.float64), V


def test_shrink_is_prox_of_nuclear_norm():
    rng = np.random.default_rng(1)
    Y = rng.standard_normal((9, 7)) * 3
    tau = 2.5
    U, sig, V, S = shrink_factors(Y, tau)
    X = (U * sig) @ V.T
    r = sig.size
    assert 0 < r < 7
    G = (Y - X) / tau                          # must lie in d||X||_*
    assert np.allclose(U.T @ G @ V, np.eye(r), atol=1e-12)
    Pu = np.eye(9) - U @ U.T
    Pv = np.eye(7) - V @ V.T
    assert np.linalg.norm(Pu @ G @ Pv, 2) <= 1 + 1e-12
    # independent route: X = Y V diag(max(0, 1 - tau/s)) V^T from eig(Y^T Y)
    lam, W = np.linalg.eigh(Y.T @ Y)
    s = np.sqrt(np.maximum(lam, 0))
    f = np.where(s > tau, 1 - tau / np.where(s > 0, s, 1), 0.0)
    assert np.allclose(Y @ (W * f) @ W.T, X, atol=1e-12)


@pytest.mark.parametrize("delta,tau", [(1.0, 30.0), (1.7, 55.0)])
def test_svt_closed_form_fully_observed(delta, tau):
    m, n = 12, 9
    U, s, V = _spectral(m, n, [40.0, 25.0, 11.0, 3.0], 2)
    M = (U * s) @ V.T
    rows, cols = np.divmod(np.arange(m * n), n)
    vals = M[rows, cols]
    prm = dict(tau=tau, delta=delta, eps=1e-14, i_max=40)
    got = []
    svt_exact(m, n, rows, cols, vals, prm,
              callback=lambda i, Ur, sg, Vr, Y, res: got.append(
                  ((Ur * sg) @ Vr.T, res)))
    c = math.ceil(tau / (delta * s[0]))
    y = c * delta * s
    for X, res in got:
        x = np.maximum(y - tau, 0.0)
        want = (U * x) @ V.T
        assert np.linalg.norm(X - want) <= 1e-12 * max(1.0, np.linalg.norm(want))
        assert res == pytest.approx(np.linalg.norm(x - s) / np.linalg.norm(s),
                                    rel=1e-9, abs=1e-14)
        y = y + delta * (s - x)


def test_initial_c():
    assert initial_c(2500.0, 6.0, 125.5) == math.ceil(2500 / (6 * 125.5))
    assert initial_c(10.0, 1.0, 10.0) == 1.0


def test_sddmm_formula_brute_force():
    rng = np.random.default_rng(4)
    m, n, r = 11, 8, 3
    U, sig, V = rng.standard_normal((m, r)), rng.random(r), rng.standard_normal((n, r))
    rows = np.array([0, 0, 3, 5, 10, 10, 7])
    cols = np.array([1, 7, 0, 4, 2, 3, 7])
    X = (U * sig) @ V.T
    x = np.einsum("ij,ij->i", U[rows] * sig, V[cols])
    assert np.allclose(x, X[rows, cols], rtol=1e-14, atol=1e-14)


def test_adapt_p_rule():
    prm = SVTParams(p_min=1, p_max=5, adaptive_p=1)
    p, st = adapt_p(3, 0, [0.5], prm)
    assert (p, st) == (3, 0)                       # no history yet
    p, st = adapt_p(3, 4, [0.5, 0.6], prm)
    assert (p, st) == (4, 0)                       # error rose
    p, st = adapt_p(5, 0, [0.5, 0.6], prm)
    assert (p, st) == (5, 0)                       # clamped at p_max
    p, st = 3, 0
    errs = [1.0]
    for j in range(10):
        errs.append(errs[-1] * 0.9)
        p, st = adapt_p(p, st, errs, prm)
    assert (p, st) == (2, 0)                       # ten decreases in a row
    p, st = adapt_p(3, 2, [0.5, 0.5], prm)
    assert (p, st) == (3, 3)                       # tie counts as no rise
    prm0 = SVTParams(adaptive_p=0)
    assert adapt_p(3, 0, [0.5, 0.9], prm0) == (3, 0)


def test_planted500_exact_and_fast():
    prob, prm = synth.make_problem("planted500")
    M = prob.truth_dense()
    ex = svt_exact(prob.m, prob.n, prob.rows, prob.cols, prob.vals, prm)
    assert ex.converged and ex.rank == 10
    assert 100 <= ex.iters <= 160
    assert np.linalg.norm(ex.dense() - M) / np.linalg.norm(M) < 1e-3
    fs = fast_svt(prob.m, prob.n, prob.rows, prob.cols, prob.vals, prm)
    assert fs.converged and fs.rank == 10
    assert abs(fs.iters - ex.iters) <= 3
    assert fs.c == ex.c
    rel = np.linalg.norm(fs.dense() - ex.dense()) / np.linalg.norm(ex.dense())
    assert rel < 1e-3


def _small_planted(m=90, n=70, rank=3, ratio=0.45, seed=7):
    p = synth.planted(m, n, rank, ratio, seed_data=seed, seed_phi=seed + 100)
    return p


def test_fast_svt_exact_krylov_equals_exact_svt():
    # b = min(k + s, n) = n makes Q span all of range(Y): rSVD-BKI is exact
    p = _small_planted(m=60, n=30, rank=3, ratio=0.6, seed=3)
    prm = dict(tau=150.0, delta=1.5, eps=1e-6, i_max=25, s=30)
    steps = []
    svt_exact(p.m, p.n, p.rows, p.cols, p.vals, prm,
              callback=lambda i, U, sg, V, Y, res: steps.append((sg.copy(), res)))
    f = FastSVT(p.m, p.n, p.rows, p.cols, p.vals, prm)
    for sg, res in steps:
        info = f.step()
        assert info.r == sg.size
        assert np.allclose(f.sig, sg, rtol=1e-10, atol=1e-10)
        assert info.res == pytest.approx(res, rel=1e-9)


@pytest.mark.parametrize("strategy", [1, 2])
def test_guarded_recycling_matches_plain(strategy):
    p = _small_planted(m=120, n=100, rank=4, ratio=0.35, seed=11)
    base = dict(tau=500.0, delta=1.2 / 0.35, eps=1e-3, i_max=250)
    plain = fast_svt(p.m, p.n, p.rows, p.cols, p.vals, base)
    rec = fast_svt(p.m, p.n, p.rows, p.cols, p.vals,
                   dict(base, recycle=strategy, i_reuse=20, q_reuse=3,
                        ritz_tol=1e-3))
    assert plain.converged and rec.converged
    # recycled counts every attempt, rejected ones included
    assert rec.extra["recycled"] - rec.extra["rejected"] > 0
    rel = np.linalg.norm(rec.dense() - plain.dense()) / np.linalg.norm(plain.dense())
    assert rel < 1e-3


@pytest.mark.parametrize("strategy", [1, 2])
def test_rejected_recycles_leave_no_trace(strategy):
    # A guard that rejects every recycled result must reproduce the solve
    # without recycling exactly: a discarded call changes no state, and the
    # rSVD-BKI calls draw the same test matrices.  The s-th rejection in a
    # row (step i) suspends recycling for the rest of step i and steps
    # i+1 .. i+q_reuse*2^(s-1); the step after that tries again.
    p = _small_planted(m=120, n=100, rank=4, ratio=0.35, seed=11)
    base = dict(tau=500.0, delta=1.2 / 0.35, eps=1e-3, i_max=80)
    plain = FastSVT(p.m, p.n, p.rows, p.cols, p.vals, base)
    q_reuse = 3
    rej = FastSVT(p.m, p.n, p.rows, p.cols, p.vals,
                  dict(base, recycle=strategy, i_reuse=20, q_reuse=q_reuse,
                       ritz_tol=1e-300))
    last_rej, run, tried = None, 0, []
    for _ in range(80):
        a, b = plain.step(), rej.step()
        assert (a.res, a.r, a.k, a.p, a.fresh) == (b.res, b.r, b.k, b.p, b.fresh)
        assert np.array_equal(a.S, b.S)
        assert b.recycled == b.rejected <= 1
        if last_rej is not None:
            pause = q_reuse * 2 ** (run - 1)
            if b.i <= last_rej + pause:
                assert b.recycled == 0, b.i
            if b.i == last_rej + pause + 1:
                assert b.recycled > 0, b.i
        if b.rejected:
            last_rej, run = b.i, run + 1
            tried.append(b.i)
        if a.converged:
            break
    # attempts at steps 20, 24, 31, 44 (pauses of 3, 6, 12 steps), ...
    assert tried[:3] == [20, 24, 31], tried
    assert rej.rejected_total == len(tried)
    assert np.array_equal(plain.U, rej.U) and np.array_equal(plain.V, rej.V)


def test_accepted_recycle_resets_the_pause():
    # a guard that accepts resets the run of rejections: the pause after the
    # next rejection is q_reuse again
    p = _small_planted(m=120, n=100, rank=4, ratio=0.35, seed=11)
    base = dict(tau=500.0, delta=1.2 / 0.35, eps=1e-12, i_max=60, recycle=1,
                i_reuse=10, q_reuse=2)
    f = FastSVT(p.m, p.n, p.rows, p.cols, p.vals, dict(base, ritz_tol=1e-300))
    while f.rej_run < 2:                 # attempts at steps 10 and 13
        f.step()
    assert f.i == 13
    # from here the guard accepts every recycled result
    f.prm.ritz_tol = 1e300
    acc = None
    for _ in range(30):
        b = f.step()
        if b.recycled > b.rejected:
            acc = b.i
            break
    assert acc is not None and f.rej_run == 0
    f.prm.ritz_tol = 1e-300
    while True:
        b = f.step()
        if b.rejected:
            break
    i_rej = b.i
    assert f.rej_run == 1
    seen = [f.step() for _ in range(3)]
    assert [x.recycled for x in seen[:2]] == [0, 0]      # pause of q_reuse = 2
    assert seen[2].recycled > 0 and seen[2].i == i_rej + 3


def test_rank_cap():
    p = _small_planted(m=80, n=60, rank=6, ratio=0.5, seed=5)
    prm = dict(tau=300.0, delta=2.4, eps=1e-5, i_max=40, k_max=3)
    ex = svt_exact(p.m, p.n, p.rows, p.cols, p.vals, prm)
    fs = fast_svt(p.m, p.n, p.rows, p.cols, p.vals, prm)
    assert max(ex.rank_hist) <= 3 and fs.rank <= 3
