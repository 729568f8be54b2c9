"""bench.py contract checks that need no GPU."""

import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_arguments_and_defaults():
    b = _bench()
    old = sys.argv
    try:
        sys.argv = ["bench.py"]
        a = b.parse()
    finally:
        sys.argv = old
    assert (a.gpus, a.workload, a.precision) == (1, "ratings140k", "fp64")
    assert a.steps > 0 and a.warmup >= 0


def test_roofline_picks_the_dominant_family():
    b = _bench()
    prof = {"spmm_fwd": dict(launches=10, ms=1.0, bytes=8e9, flops=1e9),
            "eigensolve": dict(launches=2, ms=3.0, bytes=0.0, flops=6e9),
            "rng": dict(launches=0, ms=0.0, bytes=0.0, flops=0.0)}
    # the eigensolve (latency-bound) never takes the roofline while another
    # family has time, even a larger share
    dom, roof = b.roofline(prof, "fp64", "no-such-workload")
    assert dom == "spmm_fwd" and roof["bound"] == "hbm" and roof["unit"] == "GB/s"
    assert abs(roof["frac"] - roof["achieved"] / 8000.0) < 1e-4
    prof["gram"] = dict(launches=5, ms=2.0, bytes=1e8, flops=4e9)
    dom, roof = b.roofline(prof, "fp64", "no-such-workload")
    # 40 FLOP/B is past the FP64 ridge (9.8): the matrix-core peak bounds it
    assert dom == "gram" and roof["bound"] == "mfma" and roof["unit"] == "TFLOP/s"
    assert abs(roof["achieved"] - 4e9 / 5 / 0.4e-3 / 1e12) < 1e-3
    # a sparse product past the ridge is bound by the vector ALUs
    dom, roof = b.roofline({"spmm_bwd": dict(launches=1, ms=1.0, bytes=1e8, flops=2e9)},
                           "fp64", "no-such-workload", copy_gbps=6000.0)
    assert roof["bound"] == "alu" and "copy_roof_GBps" not in roof
    dom, roof = b.roofline({"spmm_bwd": dict(launches=1, ms=1.0, bytes=1e9, flops=2e9)},
                           "fp64", "no-such-workload", copy_gbps=6000.0)
    assert roof["bound"] == "hbm" and roof["copy_roof_GBps"] == 6000.0
    assert abs(roof["frac_of_copy_roof"] - 1000.0 / 6000.0) < 1e-4
    # alone, it reports its flop rate against the FP64 vector peak
    dom, roof = b.roofline({"eigensolve": prof["eigensolve"]}, "fp64", "no-such-workload")
    assert dom == "eigensolve" and roof["bound"] == "alu" and roof["traffic"] is None
    assert abs(roof["achieved"] - 6e9 / 2 / 1.5e-3 / 1e12) < 1e-3


def test_measured_traffic_is_tied_to_sources():
    b = _bench()
    v = b.measured_traffic("image1024", "gram", "fp64")
    assert v is None or v > 0
    assert b.measured_traffic("image1024", "gram", "bf16") is None


def test_sparse_families_report_their_gathers():
    b = _bench()
    prof = {"spmm_bwd": dict(launches=4, ms=2.0, bytes=1e9, flops=8e9),
            "gram": dict(launches=4, ms=1.0, bytes=1e8, flops=1e9)}
    t = b.family_table(prof, 3e-3, "fp64")
    # nnz b = flops / 2 rows of 8 bytes in 2 ms
    assert t["spmm_bwd"]["gather_GBps"] == round(4e9 * 8 / 2e-3 / 1e9, 1)
    assert "gather_GBps" not in t["gram"]
    t32 = b.family_table(prof, 3e-3, "bf16")
    assert t32["spmm_bwd"]["gather_GBps"] == round(4e9 * 4 / 2e-3 / 1e9, 1)
    dom, roof = b.roofline(prof, "fp64", "no-such-workload")
    assert dom == "spmm_bwd" and roof["gather_GBps"] == t["spmm_bwd"]["gather_GBps"]
