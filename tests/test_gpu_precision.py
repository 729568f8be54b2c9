"""Reduced-precision modes (FP32 / BF16 SpMM, SDDMM and Gram with FP32
accumulation; FP64 eigensolve, Cholesky factors and master iterate) against
the FP64 GPU solve and the FP64 oracle."""

import numpy as np
import pytest

import synth
from oracle import svt_exact

pytestmark = pytest.mark.gpu


def _solve(prob, prm, precision):
    from paper_1810_06860_amd import SVT
    s = SVT(prob.m, prob.n, prob.rows, prob.cols, prob.vals, dict(prm, precision=precision))
    out = s.solve()
    U, sig, V = s.factors()
    return out, (U * sig) @ V.T


@pytest.fixture(scope="module")
def planted():
    prob, prm = synth.make_problem("planted500")
    ex = svt_exact(prob.m, prob.n, prob.rows, prob.cols, prob.vals, prm)
    out64, X64 = _solve(prob, prm, "fp64")
    return prob, prm, ex.dense(), X64, out64


@pytest.mark.parametrize("precision,tol_oracle", [("fp32", 1e-3), ("bf16", 1e-3)])
def test_reduced_precision_planted500(planted, precision, tol_oracle):
    prob, prm, Xo, X64, out64 = planted
    out, X = _solve(prob, prm, precision)
    rel_oracle = np.linalg.norm(X - Xo) / np.linalg.norm(Xo)
    rel_fp64 = np.linalg.norm(X - X64) / np.linalg.norm(X64)
    M = prob.truth_dense()
    rel_truth = np.linalg.norm(X - M) / np.linalg.norm(M)
    print(f"{precision}: iters {out['iters']} (fp64 {out64['iters']}), "
          f"rank {out['rank']}, X vs oracle {rel_oracle:.2e}, vs fp64 GPU "
          f"{rel_fp64:.2e}, vs truth {rel_truth:.2e}")
    assert out["rank"] == 10
    assert rel_oracle < tol_oracle


def test_bf16_operator_halves_value_traffic():
    from paper_1810_06860_amd import SVT
    prob, prm = synth.make_problem("planted500")
    per = {}
    for prec in ("fp64", "fp32", "bf16"):
        s = SVT(prob.m, prob.n, prob.rows, prob.cols, prob.vals,
                dict(prm, precision=prec, use_graphs=0))
        s.step()
        s.profile(True)
        s.step()
        p = s.get_profile()
        per[prec] = p["spmm_fwd"]["bytes"] / max(p["spmm_fwd"]["launches"], 1)
    assert per["fp32"] < per["fp64"] and per["bf16"] < per["fp32"]


def test_bf16_and_fp32_on_scaled_ratings_against_fp64():
    # power-law sampled ratings at 1/10 scale: reduced-precision forms against
    # the FP64 GPU form after the same number of steps
    from paper_1810_06860_amd import SVT
    prob, prm = synth.make_problem("ratings70k_s10")
    X = {}
    for prec in ("fp64", "fp32", "bf16"):
        s = SVT(prob.m, prob.n, prob.rows, prob.cols, prob.vals, dict(prm, precision=prec))
        for _ in range(40):
            info = s.step()
        U, sig, V = s.factors()
        X[prec] = (U * sig) @ V.T
        print(f"{prec}: rank {info['r']} res {info['res']:.5f}")
    for prec, tol in (("fp32", 1e-5), ("bf16", 1e-3)):
        rel = np.linalg.norm(X[prec] - X["fp64"]) / np.linalg.norm(X["fp64"])
        print(f"{prec} vs fp64: {rel:.2e}")
        assert rel < tol
