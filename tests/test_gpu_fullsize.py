"""GPU parity at the sizes that are measured: the two rating workloads at full
size for their first steps, and the image workload through a whole 300-step
solve (fresh and recycled phases), each against the oracle's fast SVT
(Alg. 6) drawing the same test matrices, compared at equal step index."""

import numpy as np
import pytest

import synth
from oracle import FastSVT

pytestmark = pytest.mark.gpu


def factored_rel_diff(f1, f2):
    """||U1 S1 V1^T - U2 S2 V2^T||_F / ||U2 S2 V2^T||_F without forming the
    matrices (they can be 140,000 x 27,000).  The difference is A B^T with
    A = [U1 S1, -U2 S2], B = [V1, V2]; with B = Q R (reduced QR) its norm is
    ||A R^T||_F, which subtracts the two factorisations entry by entry.  The
    trace form ||X1||^2 + ||X2||^2 - 2<X1, X2> would cancel in the squares and
    resolve no relative difference below about 1e-8."""
    import numpy as np
    U1, s1, V1 = f1
    U2, s2, V2 = f2
    A2 = U2 * s2
    den = np.linalg.norm(A2 @ np.linalg.qr(V2, mode="r").T) if V2.shape[1] else 0.0
    if V1.shape[1] + V2.shape[1] == 0:
        return 0.0
    A = np.hstack([U1 * s1, -A2])
    R = np.linalg.qr(np.hstack([V1, V2]), mode="r")
    num = np.linalg.norm(A @ R.T)
    return num / den if den > 0 else float(num)


@pytest.mark.parametrize("name,steps", [("ratings70k", 3), ("ratings140k", 3)])
def test_ratings_full_size_first_steps_match_oracle(name, steps):
    from paper_1810_06860_amd import SVT
    prob, prm = synth.make_problem(name)
    print(f"{name}: {prob.m} x {prob.n}, nnz {prob.nnz}", flush=True)
    orc = FastSVT(prob.m, prob.n, prob.rows, prob.cols, prob.vals, prm)
    g = SVT(prob.m, prob.n, prob.rows, prob.cols, prob.vals, prm)
    res = g.result()
    assert res["c"] == orc.c
    assert res["norm2"] == pytest.approx(orc.norm2, rel=1e-10)
    for i in range(steps):
        oi = orc.step()
        gi = g.step()
        assert (gi["r"], gi["k"], gi["p"], gi["fresh"]) == (oi.r, oi.k, oi.p, oi.fresh), i
        assert gi["res"] == pytest.approx(oi.res, rel=1e-8)
        np.testing.assert_allclose(g.sigma(), oi.S, rtol=1e-8)
    rel = factored_rel_diff(g.factors(), (orc.U, orc.sig, orc.V))
    print(f"{name}: step {steps}, rank {gi['r']}, res {gi['res']:.6f}, X vs oracle {rel:.1e}")
    assert rel < 1e-8
    np.testing.assert_allclose(g.observed(), orc.x_phi_input_order(), rtol=1e-8,
                               atol=1e-10 * np.abs(orc.x_phi).max())


def test_image1024_whole_solve_matches_oracle():
    # strategy-2 recycling by the paper's rule from step 100 (q_reuse 10),
    # p = 2 fixed: every step of the 300 against the oracle
    from paper_1810_06860_amd import SVT
    prob, prm = synth.make_problem("image1024")
    orc = FastSVT(prob.m, prob.n, prob.rows, prob.cols, prob.vals, prm)
    g = SVT(prob.m, prob.n, prob.rows, prob.cols, prob.vals, prm)
    assert g.result()["c"] == orc.c
    worst, recycled = 0.0, 0
    for i in range(prm["i_max"]):
        oi = orc.step()
        gi = g.step()
        assert (gi["r"], gi["k"], gi["fresh"], gi["recycled"], gi["rejected"]) == \
            (oi.r, oi.k, oi.fresh, oi.recycled, oi.rejected), i
        worst = max(worst, abs(gi["res"] - oi.res) / oi.res)
        recycled += gi["recycled"]
        if oi.converged:
            assert gi["converged"]
            break
    U, sig, V = g.factors()
    Xg = (U * sig) @ V.T
    Xo = (orc.U * orc.sig) @ orc.V.T
    rel = np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo)
    print(f"image1024: {i + 1} steps, {recycled} recycled calls, rank {gi['r']}, "
          f"res {gi['res']:.5f}, max res rel diff {worst:.1e}, X vs oracle {rel:.1e}")
    assert recycled > 100
    assert worst < 1e-8
    assert rel < 1e-8
