"""Fast SVT (Sec. IV, Alg. 6): the SVT iteration of Eq. (6) whose truncated
SVD is rSVD-BKI (Sec. III.B), with subspace recycling (Sec. IV.B) and the
adaptive power parameter (Sec. IV.C).

Each step finds every singular value of Y^{i-1} above tau by the rank
search of Alg. 2 (k starts one above the previous rank and grows by l while
the smallest computed value still exceeds tau), shrinks them by tau, and
takes the residual and the update of Y on Phi (Eq. (6)).  The SVD of each
rank-search call is a fresh rSVD-BKI call, or -- once recycling is allowed
(step index >= i_reuse, fewer than q_reuse recycled calls since the last
fresh one) -- the Rayleigh-Ritz step on the basis the last fresh call left:
its Q (strategy 1) or its U (strategy 2).

Readings of points the paper leaves open:
* The update of Alg. 6 is written with P_Omega; Omega is the random test
  matrix, so it is read as P_Phi, on which Y lives anyway.
* Singular values are used in descending order (eigSVD returns them
  ascending).
* q counts SVD calls: +1 per recycled call, reset by every rSVD-BKI call.
  The recycled basis is the one saved by the last rSVD-BKI call.  A recycle
  that would need more columns than that basis holds runs rSVD-BKI instead.
* Guarded recycling (ritz_tol > 0) is an addition, not in the paper: a
  recycled result whose Ritz residual max_j ||Y v_j - s_j u_j|| / s_j
  exceeds ritz_tol is discarded and rSVD-BKI runs instead.  A rejection in
  step i also suspends recycling for the rest of step i and for the next
  q_reuse * 2^(s - 1) steps, s being the number of rejections since the
  last accepted recycled result (exponent capped at 20): every call of
  those steps is rSVD-BKI, so an operator whose recycled results keep
  failing the guard pays for fewer and fewer discarded calls.  With
  ritz_tol = 0 nothing is rejected and the paper's rule applies unchanged.
* Block width b = min(k + s, min(m, n)) and the power parameter is clamped so
  that (p + 1) b <= min(m, n) (eigSVD of B^T needs n >= (p + 1) b, Alg. 3).
* The rank search stops at the cap min(m, n, k_max).
* Omega of rSVD-BKI call number `attempt` within step i is
  ``gaussian_block(n, b, seed, i, attempt)``.
* The stop test comes before the update (Alg. 2 and Alg. 6 leave the loop
  on convergence), so Y is not updated on the converging step.
"""

from dataclasses import dataclass

import numpy as np
import scipy.sparse

from .csr import canonical_csr
from .eigsvd import eigsvd_top
from .philox import gaussian_block
from .rsvd import rsvd_bki
from .svt import SVTParams, SVTResult, initial_c, spectral_norm


def adapt_p(p, streak, err_hist, prm):
    """Adaptive power parameter (Sec. IV.C).  Returns (p, streak)."""
    if not prm.adaptive_p or len(err_hist) < 2:
        return p, streak
    if err_hist[-1] > err_hist[-2]:
        p, streak = p + 1, 0
    else:
        streak += 1
        if streak == 10:
            p, streak = p - 1, 0
    return min(max(p, prm.p_min), prm.p_max), streak


@dataclass
class StepInfo:
    i: int
    res: float
    r: int
    k: int
    p: int
    fresh: int
    recycled: int
    rejected: int
    converged: bool
    S: np.ndarray


class FastSVT:
    """Alg. 6 with the state kept between steps, for step-wise comparison."""

    def __init__(self, m, n, rows, cols, vals, params):
        prm = SVTParams.from_dict(params) if isinstance(params, dict) else params
        self.prm = prm.resolved(m, n, len(vals))
        self.m, self.n = int(m), int(n)
        lay = canonical_csr(m, n, rows, cols)
        self.lay = lay
        self.order = lay["order"]
        self.rows = np.asarray(rows, dtype=np.int64)[self.order]
        self.cols = lay["col_idx"]
        self.mvals = np.asarray(vals, dtype=np.float64)[self.order]
        self.mnorm = float(np.linalg.norm(self.mvals))
        nu = spectral_norm(m, n, self.rows, self.cols, self.mvals)
        self.norm2 = nu
        self.c = (self.prm.c if self.prm.c > 0
                  else initial_c(self.prm.tau, self.prm.delta, nu))
        self.y = self.c * self.prm.delta * self.mvals        # Y^0 on Phi
        self.i = 0
        self.r = 0
        self.q = 0
        self.p = self.prm.p_init
        self.streak = 0
        self.rej_i = 0          # last step with a rejected recycled call
        self.rej_run = 0        # rejections since the last accepted recycle
        self.err_hist = []
        self.saved = None
        self.kcap = min(self.m, self.n)
        if self.prm.k_max > 0:
            self.kcap = min(self.kcap, self.prm.k_max)
        self.U = np.zeros((m, 0)); self.sig = np.zeros(0)
        self.V = np.zeros((n, 0))
        self.x_phi = np.zeros_like(self.mvals)
        self.converged = False
        self.fresh_total = 0
        self.recycled_total = 0
        self.rejected_total = 0

    # -- Y as a sparse operator with the fixed structure of Phi ------------
    def Y(self):
        return scipy.sparse.csr_matrix(
            (self.y, self.cols, self.lay["row_ptr"]), shape=(self.m, self.n))

    def widths(self, k, p):
        mn = min(self.m, self.n)
        b = min(k + self.prm.s, mn)
        return b, max(0, min(p, mn // b - 1))

    def _fresh(self, Y, k, attempt):
        b, p_eff = self.widths(k, self.p)
        omega = gaussian_block(self.n, b, self.prm.seed, self.i, attempt)
        U, S, V, Q = rsvd_bki(Y, k, p_eff, omega, return_q=True)
        U, S, V = U[:, ::-1], S[::-1], V[:, ::-1]             # descending
        self.saved = Q if self.prm.recycle == 1 else U
        self.q = 0
        return U, S, V

    def _recycled(self, Y, k):
        basis = self.saved
        Bt = np.asarray(Y.T @ basis)                         # (basis^T Y)^T
        V, S, W = eigsvd_top(Bt, k)
        U = basis @ W
        return U[:, ::-1], S[::-1], V[:, ::-1]

    def _ritz(self, Y, U, S, V):
        R = np.asarray(Y @ V) - U * S
        return float(np.max(np.linalg.norm(R, axis=0) / S))

    def step(self):
        if self.converged:
            raise RuntimeError("solve already converged")
        prm = self.prm
        self.i += 1
        Y = self.Y()
        k = min(self.r + 1, self.kcap)
        self.p, self.streak = adapt_p(self.p, self.streak, self.err_hist, prm)
        attempt = fresh = recycled = rejected = 0
        while True:
            pause = prm.q_reuse * 2 ** min(self.rej_run - 1, 20) if self.rej_run else 0
            suspended = 0 < self.rej_i <= self.i <= self.rej_i + pause
            use_fresh = (prm.recycle == 0 or self.i < prm.i_reuse
                         or self.q == prm.q_reuse or self.saved is None
                         or k > self.saved.shape[1] or suspended)
            if not use_fresh:
                U, S, V = self._recycled(Y, k)
                self.q += 1
                recycled += 1
                if prm.ritz_tol > 0 and self._ritz(Y, U, S, V) > prm.ritz_tol:
                    use_fresh = True
                    rejected += 1
                    self.rej_i = self.i
                    self.rej_run += 1
                else:
                    self.rej_run = 0
            if use_fresh:
                U, S, V = self._fresh(Y, k, attempt)
                attempt += 1
                fresh += 1
            if S[-1] <= prm.tau or k >= self.kcap:
                break
            k = min(k + prm.l, self.kcap)
        r = int(np.count_nonzero(S > prm.tau))
        self.r = r
        self.U, self.sig, self.V = U[:, :r], S[:r] - prm.tau, V[:, :r]
        self.x_phi = np.einsum("ij,ij->i", self.U[self.rows] * self.sig,
                               self.V[self.cols])
        res = float(np.linalg.norm(self.x_phi - self.mvals)) / self.mnorm
        self.err_hist.append(res)
        self.fresh_total += fresh
        self.recycled_total += recycled
        self.rejected_total += rejected
        if res < prm.eps:
            self.converged = True
        else:
            self.y = self.y + prm.delta * (self.mvals - self.x_phi)
        return StepInfo(self.i, res, r, k, self.p, fresh, recycled, rejected,
                        self.converged, S.copy())

    def x_phi_input_order(self):
        out = np.empty_like(self.x_phi)
        out[self.order] = self.x_phi
        return out

    def result(self):
        return SVTResult(U=self.U, sig=self.sig, V=self.V, iters=self.i,
                         res=self.err_hist[-1] if self.err_hist else 1.0,
                         rank=self.r, converged=self.converged,
                         x_phi=self.x_phi_input_order(), c=self.c,
                         res_hist=list(self.err_hist),
                         extra=dict(fresh=self.fresh_total,
                                    recycled=self.recycled_total,
                                    rejected=self.rejected_total))


def fast_svt(m, n, rows, cols, vals, params, callback=None):
    solver = FastSVT(m, n, rows, cols, vals, params)
    for _ in range(solver.prm.i_max):
        info = solver.step()
        if callback is not None:
            callback(solver, info)
        if info.converged:
            break
    return solver.result()
