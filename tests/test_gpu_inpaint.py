"""GPU parity of the image-inpainting form (Sec. V.B, Eq. (10)): the stacked
three-channel stand-in, strategy-2 recycling with the Ritz guard, compared
with the oracle's fast SVT (Alg. 6) at equal step index over whole solves of
the 1/4-scaled instances, and over the first steps at full size
(6144 x 2048)."""

import numpy as np
import pytest

import synth
from oracle import FastSVT

pytestmark = pytest.mark.gpu


def _run_pair(name, steps=None):
    from paper_1810_06860_amd import SVT
    from threadpoolctl import threadpool_limits
    prob, prm = synth.make_problem(name)
    print(f"{name}: {prob.m} x {prob.n}, nnz {prob.nnz}", flush=True)
    g = SVT(prob.m, prob.n, prob.rows, prob.cols, prob.vals, prm)
    with threadpool_limits(limits=4):
        orc = FastSVT(prob.m, prob.n, prob.rows, prob.cols, prob.vals, prm)
        assert g.result()["c"] == orc.c
        worst = 0.0
        for i in range(steps or prm["i_max"]):
            oi = orc.step()
            gi = g.step()
            assert (gi["r"], gi["k"], gi["p"], gi["fresh"], gi["recycled"],
                    gi["rejected"]) == (oi.r, oi.k, oi.p, oi.fresh, oi.recycled,
                                        oi.rejected), i
            worst = max(worst, abs(gi["res"] - oi.res) / oi.res)
            np.testing.assert_allclose(g.sigma(), oi.S, rtol=1e-8)
            if oi.converged:
                assert gi["converged"]
                break
    U, sig, V = g.factors()
    Xg = (U * sig) @ V.T
    Xo = (orc.U * orc.sig) @ orc.V.T
    rel = np.linalg.norm(Xg - Xo) / np.linalg.norm(Xo)
    mae_g, mae_o = synth.mae_all_pixels(Xg, prob), synth.mae_all_pixels(Xo, prob)
    g.close()
    print(f"{name}: {i + 1} steps, rank {gi['r']}, res {gi['res']:.5f}, converged "
          f"{gi['converged']}, recycled {orc.recycled_total} (rejected "
          f"{orc.rejected_total}), max res rel diff {worst:.1e}, X vs oracle "
          f"{rel:.1e}, MAE {mae_g:.4f} (oracle {mae_o:.4f})")
    assert worst < 1e-8
    assert rel < 1e-8
    assert mae_g == pytest.approx(mae_o, rel=1e-8)
    return gi, mae_g


@pytest.mark.parametrize("name", ["inpaint10_s4", "inpaint20_s4"])
def test_inpaint_scaled_whole_solve_matches_oracle(name):
    gi, mae = _run_pair(name)
    assert gi["converged"]
    assert mae < 15.0


def test_inpaint_full_size_first_steps_match_oracle():
    _run_pair("inpaint10", steps=4)
