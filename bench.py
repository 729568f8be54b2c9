#!/usr/bin/env python3
"""Fast-SVT benchmark on one MI355X: SVT steps/s plus the roofline of the
dominant kernel and the CPU oracle timed beside it.

    python bench.py [--steps K] [--warmup W] [--workload ratings140k]
                    [--precision fp64] [--cpu-seconds 30]

A "step" is one iteration of the fast SVT algorithm (Alg. 6): the rank
search with rSVD-BKI (or a recycled basis), shrinkage, the residual on Phi
and the update of Y.  The default workload is the largest rating shape
(140,000 x 27,000, 2.0e7 observed integer ratings, rank cap 100) in FP64.
The solve starts untimed (problem set-up, then its first steps up to the
middle of the step budget -- `--start-step`, half of i_max by default -- and W
warm-up steps), then K consecutive steps are timed with the stream
synchronised on both sides, so the window sees the ranks, block widths and
recycled calls of the solve's middle rather than its first, rank-1 steps.  All
inputs and solver state are resident in HBM for the whole timed region.
Beside that window the line reports the same solve run whole (steps/s from
the first step to i_max or convergence), the BF16 form against it, per-kernel
times of the window, the CPU oracle on the host cores and its step-by-step
agreement with a fresh GPU solve.

Prints one JSON line.
"""

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("SVT steps/sec + SpMM HBM GB/s at rel.err\u22641e-3; "
          "p50/p99 solve latency")
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6          # MI355X FP64 (vector and matrix)
FP32_PEAK_TFLOPS = 157.3

# families whose algorithmic intensity is below the FP64 ridge (78.6 TFLOP/s
# / 8 TB/s): the sparse products, the fused SDDMM, and the Gram / panel
# products of the tall-skinny blocks (2 N b^2 flops on 8 N b bytes, b <= 40)
HBM_FAMILIES = ("spmm_fwd", "spmm_bwd", "sddmm", "gram", "panel_gemm")


def source_sha(files):
    """Digest of kernel source files: committed HBM counters are valid only
    for the kernels they were taken on."""
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_1810_06860_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload, family, precision):
    """HBM bytes per launch of `family` from the committed PMC runs
    (FETCH_SIZE + WRITE_SIZE, calibrated), or None when absent or when the
    family's kernel source changed since."""
    try:
        with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
            tj = json.load(fh)
        ent = tj[workload]
        if ent.get("precision") != precision:
            return None
        fam = ent["families"][family]
        if fam["sha256"] != source_sha(fam["sources"]):
            return None
        return fam["bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--start-step", type=int, default=-1,
                    help="untimed solve steps run before the warm-up, so that the "
                         "timed window sits inside the solve (-1: half of i_max; "
                         "0: the window starts at the solve's first step)")
    ap.add_argument("--workload", default="ratings140k")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "bf16"])
    ap.add_argument("--cpu-seconds", type=float, default=30.0)
    ap.add_argument("--prof-steps", type=int, default=0,
                    help="steps of the event-profiled pass (per-kernel times); "
                         "0: the same steps as the timed region")
    ap.add_argument("--ritz-tol", type=float, default=None,
                    help="override the workload's Ritz guard (0: the paper's "
                         "recycling rule alone)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--eager", action="store_true",
                    help="launch kernel by kernel in the timed region too "
                         "(no HIP graphs), e.g. under a counter profiler")
    ap.add_argument("--serve", type=int, default=32,
                    help="requests of the serving trace to run (0: skip)")
    ap.add_argument("--serve-budget-gib", type=float, default=32.0)
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--serve-streams", type=int, default=16,
                    help="streams the served solves are dealt to (one per slot by default)")
    ap.add_argument("--serve-graphs", type=int, default=1,
                    help="1: served solves replay captured graphs")
    ap.add_argument("--serve-grouped", type=int, default=1,
                    help="1: also serve the same requests in batched rounds "
                         "(mc_svt_step_group, shared sparse-product launches)")
    ap.add_argument("--calls", type=int, default=10,
                    help="sparse45k: timed calls per case")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="also run a plain device copy of this size (for "
                         "calibrating HBM counters under a profiler)")
    ap.add_argument("--whole", type=int, default=1,
                    help="1: also run the workload's whole solve (and its BF16 "
                         "form) and report steps/s over it")
    ap.add_argument("--modes", default="bf16",
                    help="reduced-precision forms run whole beside the FP64 "
                         "one (comma list of fp32, bf16; empty: none)")
    return ap.parse_args()


def roofline(prof, prec, workload, copy_gbps=None):
    fams = {k: v for k, v in prof.items() if v["launches"] > 0 and v["ms"] > 0}
    if not fams:
        return None, None
    # the small dense eigensolve is a chain of dependent steps on one
    # workgroup (latency-bound, no roofline); its time share is in the
    # kernel table, and the roofline goes to the largest of the others
    cand = [k for k in fams if k != "eigensolve"] or list(fams)
    dom = max(cand, key=lambda k: fams[k]["ms"])
    v = fams[dom]
    per_launch_ms = v["ms"] / v["launches"]
    # FP64 arithmetic in the FP64 form, FP32 accumulation in the others
    peak = FP64_PEAK_TFLOPS if prec == "fp64" else FP32_PEAK_TFLOPS
    ridge = peak * 1e12 / (HBM_PEAK_GBS * 1e9)            # FLOP per byte
    intensity = v["flops"] / v["bytes"] if v["bytes"] else float("inf")
    if dom in HBM_FAMILIES and intensity < ridge:
        achieved = v["bytes"] / v["launches"] / (per_launch_ms * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=round(achieved, 2), peak=HBM_PEAK_GBS,
                    unit="GB/s")
    else:
        achieved = v["flops"] / v["launches"] / (per_launch_ms * 1e-3) / 1e12
        bound = "mfma" if dom in ("gram", "panel_gemm") else "alu"
        roof = dict(bound=bound, achieved=round(achieved, 4), peak=peak,
                    unit="TFLOP/s")
    roof["frac"] = round(roof["achieved"] / roof["peak"], 5)
    roof["intensity_flop_per_byte"] = round(intensity, 3)
    if roof["bound"] == "hbm" and copy_gbps:
        roof["copy_roof_GBps"] = round(copy_gbps, 1)
        roof["frac_of_copy_roof"] = round(roof["achieved"] / copy_gbps, 5)
    g = gather_bytes(dom, v["flops"], prec)
    if g:
        # what the product actually moves from L2 / MALL / HBM per second
        roof["gather_GBps"] = round(g / v["launches"] / (per_launch_ms * 1e-3) / 1e9, 1)
    roof["traffic"] = measured_traffic(workload, dom, prec)
    roof["kernel"] = dom
    roof["launches"] = v["launches"]
    roof["avg_launch_us"] = round(per_launch_ms * 1e3, 3)
    return dom, roof


def copy_roof(torch, mib=2048, reps=5):
    """Measured device-to-device copy rate (bytes read + written per second):
    the HBM roof the box actually gives, beside the 8 TB/s datasheet figure."""
    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del src, dst
    return 2.0 * n * 8 / (best * 1e-3) / 1e9


def gather_bytes(family, flops, prec):
    """Panel bytes a sparse product gathers: one b-wide row of X per nonzero
    (nnz b = flops / 2), in the panel type (FP64, else FP32).  Not counted in
    the algorithmic bytes, which read X once."""
    if not family.startswith("spmm"):
        return None
    return flops / 2.0 * (8 if prec == "fp64" else 4)


def family_table(prof, total_s, prec="fp64"):
    out = {}
    for k, v in prof.items():
        if v["launches"] == 0:
            continue
        ms = v["ms"]
        ent = dict(launches=v["launches"], ms=round(ms, 3),
                   share=round(ms * 1e-3 / total_s, 4) if total_s > 0 else None)
        if v["bytes"] and ms > 0:
            ent["GBps"] = round(v["bytes"] / (ms * 1e-3) / 1e9, 1)
        if v["flops"] and ms > 0:
            ent["TFLOPs"] = round(v["flops"] / (ms * 1e-3) / 1e12, 4)
        g = gather_bytes(k, v["flops"], prec)
        if g and ms > 0:
            ent["gather_GBps"] = round(g / (ms * 1e-3) / 1e9, 1)
        out[k] = ent
    return out


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


def cpu_baseline(prob, prm, budget_s, max_steps):
    import numpy as np
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = len(os.sched_getaffinity(0))
    try:
        import numpy as np
        blas = ",".join(sorted({i.get("internal_api", "?") for i in threadpool_info()
                                if i.get("user_api") == "blas"})) or "unknown"
    except Exception:
        blas = "unknown"
    t0 = time.perf_counter()
    orc = oracle.FastSVT(prob.m, prob.n, prob.rows, prob.cols, prob.vals, prm)
    t_init = time.perf_counter() - t0
    steps = 0
    infos = []
    t0 = time.perf_counter()
    while steps < max_steps and time.perf_counter() - t0 < budget_s:
        info = orc.step()
        infos.append(info)
        steps += 1
        if info.converged:
            break
    dt = time.perf_counter() - t0
    return orc, infos, dict(value=round(steps / dt, 4), unit="steps/s", cores=int(threads),
                            kind="oracle", blas=blas,
                            sample=(f"first {steps} fast-SVT steps of the same workload "
                                    f"(NumPy/SciPy FP64, {dt:.1f} s wall after a "
                                    f"{t_init:.1f} s set-up)"))


def serving_leg(a):
    """Continuous batching over the first a.serve requests of the trace:
    Poisson arrivals (mean gap 50 ms), planted problems of uneven shape, FP32
    kernels with FP64 eigensolves, admission by device footprint."""
    import concurrent.futures as cf
    import torch
    import synth
    from paper_1810_06860_amd import serving
    trace = synth.serving_trace()
    desc = trace[: a.serve]
    t0 = time.perf_counter()
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with cf.ThreadPoolExecutor(workers) as ex:
        problems = list(ex.map(synth.request_problem, desc))
    gen_s = time.perf_counter() - t0
    log(f"serving: {len(problems)} requests generated in {gen_s:.1f} s")
    reqs = []
    for d, p in zip(desc, problems):
        prm = dict(synth.serving_params(p.m, p.n, p.nnz), precision="fp32")
        reqs.append(serving.Request(d["id"], d["t_arrival"], p, prm))
    streams = [torch.cuda.Stream() for _ in range(a.serve_streams)]
    torch.cuda.synchronize()
    served = serving.serve(reqs, budget_bytes=int(a.serve_budget_gib * (1 << 30)),
                           max_active=a.serve_slots, stream_pool=streams,
                           graphs=bool(a.serve_graphs),
                           on_done=lambda s, n: log(f"serving: {n}/{len(reqs)} done "
                                                    f"(req {s.id}, {s.steps} steps, "
                                                    f"{s.latency:.2f} s{', ' + s.error if s.error else ''})"))
    torch.cuda.synchronize()
    out = serving.summarize(served)
    if a.serve_grouped:
        # the same arrivals served in batched rounds (one driver thread, the
        # sparse products of each stage launched together for all solves)
        g0 = time.perf_counter()
        grouped = serving.serve_grouped(
            reqs, budget_bytes=int(a.serve_budget_gib * (1 << 30)),
            max_active=a.serve_slots, stream_pool=streams,
            on_done=lambda s, n: log(f"serving grouped: {n}/{len(reqs)} done "
                                     f"(req {s.id}, {s.steps} steps, {s.latency:.2f} s)"))
        torch.cuda.synchronize()
        gsum = serving.summarize(grouped)
        same = {s.id: (s.steps, s.rank, s.res) for s in served}
        gsum["same_steps_rank_residual_as_streams"] = all(
            same.get(s.id) == (s.steps, s.rank, s.res) for s in grouped)
        gsum["wall_s"] = round(time.perf_counter() - g0, 2)
        for key in ("p50_s", "p99_s", "mean_s", "max_s", "makespan_s", "steps_per_s"):
            if gsum.get(key) is not None:
                gsum[key] = round(gsum[key], 4)
        out["grouped_rounds"] = gsum
    errs = [f"req {s.id}: {s.error}" for s in served if s.error]
    if errs:
        out["errors"] = errs
    out.update(precision="fp32 kernels, fp64 eig", budget_gib=a.serve_budget_gib,
               graphs=bool(a.serve_graphs),
               slots=a.serve_slots, streams=a.serve_streams,
               nnz_total=int(sum(p.nnz for p in problems)),
               arrivals="Poisson, mean gap 50 ms", generation_s=round(gen_s, 1),
               subset=f"the first {len(desc)} of the {len(trace)}-request trace")
    for key in ("p50_s", "p99_s", "mean_s", "max_s", "makespan_s", "steps_per_s"):
        if out.get(key) is not None:
            out[key] = round(out[key], 4)
    return out


RSVD_METRIC = "rSVD calls/sec (k=100, s=10) at the oracle's singular values to 1e-8"
RSVD_CASES = (("pi", 0), ("pi", 4), ("bki", 4))   # Table I rows (p = 0, 4) + BKI


def rsvd_main(a):
    """Truncated SVDs of the 45,115 x 45,115 sparse matrices (97, 24 and 9
    entries per row) at k = 100: rSVD-PI at p = 0 and 4, rSVD-BKI at p = 4,
    on a matrix kept resident in HBM (mc_rsvd_init / mc_rsvd_run).  A call
    is timed from its launch to its k singular values on the host.  The
    headline is rSVD-PI at p = 4 on the densest matrix."""
    import numpy as np
    import scipy.sparse
    import torch
    import synth
    from paper_1810_06860_amd import RSVD

    torch.cuda.set_device(0)
    k, s, seed = 100, 10, 11
    t0 = time.perf_counter()
    probs = synth.sparse_square()
    log(f"sparse45k: matrices generated in {time.perf_counter() - t0:.1f} s")
    cases = []
    head = None
    for prob in probs:
        fro2 = float(np.sum(prob.vals ** 2))
        h = RSVD(prob.m, prob.n, prob.rows, prob.cols, prob.vals, s=s,
                 precision=a.precision, seed=seed)
        for method, p in RSVD_CASES:
            for w in range(max(1, a.warmup)):
                h.run(method, k, p, step=1000 + w, factors=False)
            torch.cuda.synchronize()
            c0 = time.perf_counter()
            for c in range(a.calls):
                _, S, _ = h.run(method, k, p, step=1 + c, factors=False)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - c0) / a.calls
            err = float(np.sqrt(max(0.0, 1.0 - np.sum(S ** 2) / fro2)))
            row = dict(matrix=prob.name, nnz=prob.nnz, method=method, p=p,
                       ms_per_call=round(dt * 1e3, 3), error=round(err, 5))
            log(f"sparse45k: {row}")
            cases.append(row)
            if head is None and method == "pi" and p == 4:
                head = (prob, row, S, a.calls)
        if prob is probs[0]:
            # per-family kernel times of the headline case, kernel by kernel
            h.profile(True)
            for c in range(3):
                h.run("pi", k, 4, step=1 + c, factors=False)
            prof = h.get_profile()
            h.profile(False)
        h.close()
    prob, row, S_last, ncalls = head
    _, roof = roofline(prof, a.precision, "sparse45k")
    acc = {}
    cpu = None
    if not a.no_cpu_baseline:
        # the oracle's rSVD-PI on the same matrix and test matrix as the last
        # timed headline call
        import oracle
        try:
            from threadpoolctl import threadpool_info
            threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
        except Exception:
            threads = len(os.sched_getaffinity(0))
        A = scipy.sparse.csr_matrix((prob.vals, (prob.rows, prob.cols)),
                                    shape=(prob.m, prob.n))
        om = oracle.gaussian_block(prob.n, k + s, seed, ncalls, 0)
        c0 = time.perf_counter()
        _, So, _ = oracle.rsvd_pi(A, k, 4, om)
        dt = time.perf_counter() - c0
        So = So[::-1]
        cpu = dict(value=round(1.0 / dt, 4), unit="calls/s", cores=int(threads),
                   kind="oracle",
                   sample=f"one rSVD-PI call (p=4, k=100) on {prob.name} "
                          f"(NumPy/SciPy FP64, {dt:.1f} s wall)")
        if a.precision == "fp64":
            acc["sigma_max_rel_diff_vs_oracle"] = float(np.max(np.abs(S_last - So) / So))
    line = {
        "metric": RSVD_METRIC,
        "value": round(1e3 / row["ms_per_call"], 4),
        "unit": "calls/s",
        "n_gpus": 1,
        "steps": ncalls,
        "warmup": max(1, a.warmup),
        "ms_per_step": row["ms_per_call"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}[a.precision],
        "data": "synthetic",
        "config": {"workload": "sparse45k", "m": prob.m, "n": prob.n, "nnz": prob.nnz,
                   "k": k, "s": s, "method": "rsvd_pi", "p": 4,
                   "precision": a.precision},
        "roofline": roof,
        "cpu_baseline": cpu,
        "accuracy": acc,
        "cases": cases,
        "kernels": family_table(prof, sum(v["ms"] for v in prof.values()) * 1e-3,
                                a.precision),
    }
    print(json.dumps(line))


def per_kp_times(infos, step_ms):
    """Mean step time per (k, p) of the steps in a window."""
    acc = {}
    for inf, ms in zip(infos, step_ms):
        key = f"k={inf['k']},p={inf['p']}"
        n, t = acc.get(key, (0, 0.0))
        acc[key] = (n + 1, t + ms)
    return {key: dict(steps=n, ms=round(t / n, 3)) for key, (n, t) in acc.items()}


def run_whole(SVT, prob, prm, log_name):
    """One solve from its first step to i_max or convergence, timed whole."""
    import torch
    s = SVT(prob.m, prob.n, prob.rows, prob.cols, prob.vals, prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = s.solve()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    f = s.factors()
    s.close()
    rec = dict(steps=out["iters"], steps_per_s=round(out["iters"] / dt, 4),
               s=round(dt, 3), converged=bool(out["converged"]), res_last=out["res"],
               rank=out["rank"], fresh=out["fresh"], recycled=out["recycled"],
               rejected=out["rejected"])
    if prob.meta.get("value_scale"):
        # image inpainting: Eq. (10) over every pixel of the stacked channels
        import synth
        U, sig, V = f
        rec["mae_all_pixels"] = round(synth.mae_all_pixels((U * sig) @ V.T, prob), 4)
    log(f"{log_name}: {rec}")
    return rec, f


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if a.workload == "sparse45k":
        return rsvd_main(a)
    import numpy as np
    import torch

    import synth
    from paper_1810_06860_amd import SVT

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    log(f"workload {a.workload}")
    g0 = time.perf_counter()
    prob, prm = synth.make_problem(a.workload)
    log(f"generated in {time.perf_counter() - g0:.1f} s: {prob.m} x {prob.n}, "
        f"nnz {prob.nnz}")
    prm = dict(prm)
    prm["precision"] = a.precision
    start = prm["i_max"] // 2 if a.start_step < 0 else a.start_step
    prm["i_max"] = max(prm["i_max"], start + a.warmup + a.steps)
    if a.ritz_tol is not None:
        prm["ritz_tol"] = a.ritz_tol
    if a.eager:
        prm["use_graphs"] = 0
    copy_gbps = copy_roof(torch)
    log(f"device copy roof: {copy_gbps:.0f} GB/s")
    solver = SVT(prob.m, prob.n, prob.rows, prob.cols, prob.vals, prm)
    warm = []
    for _ in range(start + a.warmup):
        info = solver.step()
        warm.append(info)
        if info["converged"]:
            raise SystemExit("workload converged before the timed window; lower "
                             "--start-step or --warmup")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos, step_ms = [], []
    for _ in range(a.steps):
        s0 = time.perf_counter()
        info = solver.step()
        step_ms.append((time.perf_counter() - s0) * 1e3)
        infos.append(info)
        if info["converged"]:
            break
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    done = len(infos)
    dt = t1 - t0
    value = done / dt
    log(f"timed: {done} steps in {dt:.3f} s")
    window = dict(first_step=start + a.warmup + 1, last_step=start + a.warmup + done,
                  untimed_before=dict(solve_steps=start, warmup=a.warmup),
                  rank=[min(i["r"] for i in infos), max(i["r"] for i in infos)],
                  k=[min(i["k"] for i in infos), max(i["k"] for i in infos)],
                  p=sorted({i["p"] for i in infos}),
                  fresh=sum(i["fresh"] for i in infos),
                  recycled=sum(i["recycled"] for i in infos),
                  rejected=sum(i["rejected"] for i in infos),
                  per_kp=per_kp_times(infos, step_ms))
    # Per-kernel durations: the same window re-run with kernel-by-kernel
    # launches and HIP events around each launch on the solve's stream.
    prof_solver = SVT(prob.m, prob.n, prob.rows, prob.cols, prob.vals,
                      dict(prm, use_graphs=0))
    for _ in range(start + a.warmup):
        prof_solver.step()
    prof_solver.profile(True)
    torch.cuda.synchronize()
    tp0 = time.perf_counter()
    pdone = 0
    for _ in range(min(a.prof_steps, a.steps) if a.prof_steps > 0 else a.steps):
        pinfo = prof_solver.step()
        pdone += 1
        if pinfo["converged"]:
            break
    torch.cuda.synchronize()
    tp1 = time.perf_counter()
    prof = prof_solver.get_profile()
    prof_solver.profile(False)
    prof_solver.close()
    prof_ms = (tp1 - tp0) * 1e3 / pdone if pdone else None
    log(f"profiled pass: {pdone} steps")
    dom, roof = roofline(prof, a.precision, a.workload, copy_gbps)
    U, sig, V = solver.factors()
    solver.close()
    acc = dict(res_last=infos[-1]["res"], rank=infos[-1]["r"],
               steps_total=start + a.warmup + done,
               converged=bool(infos[-1]["converged"]))
    # the solve run whole, and its reduced-precision forms against it
    whole, modes, whole_f = None, {}, None
    if a.whole:
        whole, whole_f = run_whole(SVT, prob, prm, "whole solve")
        for mode in [x for x in a.modes.split(",") if x and x != a.precision]:
            rec, f = run_whole(SVT, prob, dict(prm, precision=mode), f"whole {mode}")
            rec["rel_err_vs_" + a.precision] = float(factored_rel_diff(f, whole_f))
            modes[mode] = rec
    if a.precision != "fp64":
        # the plain FP64 form on the same GPU, same steps: speed and distance
        ref = SVT(prob.m, prob.n, prob.rows, prob.cols, prob.vals,
                  dict(prm, precision="fp64"))
        for _ in range(start + a.warmup):
            ref.step()
        torch.cuda.synchronize()
        r0 = time.perf_counter()
        for _ in range(done):
            rinfo = ref.step()
        torch.cuda.synchronize()
        r1 = time.perf_counter()
        U64, s64, V64 = ref.factors()
        ref.close()
        acc["fp64_steps_per_s"] = round(done / (r1 - r0), 4)
        acc["fp64_res_last"] = rinfo["res"]
        acc["rel_err_vs_fp64"] = float(factored_rel_diff((U, sig, V), (U64, s64, V64)))
        log(f"fp64 form: {acc['fp64_steps_per_s']} steps/s, X rel diff "
            f"{acc['rel_err_vs_fp64']:.3e}")
    truth = prob.truth_dense()
    if truth is not None:
        X = (U * sig) @ V.T
        acc["rel_err_vs_truth"] = float(np.linalg.norm(X - truth) /
                                        np.linalg.norm(truth))
        if prob.meta.get("value_scale"):
            acc["mae_all_pixels"] = synth.mae_all_pixels(X, prob)
    else:
        # large shapes: on 2^20 cells drawn uniformly (seeded), on and off Phi
        g = np.random.default_rng(7)
        ri = g.integers(0, prob.m, 1 << 20)
        ci = g.integers(0, prob.n, 1 << 20)
        t = prob.truth_at(ri, ci)
        if t is not None:
            x = np.einsum("ij,ij->i", U[ri] * sig, V[ci])
            acc["rel_err_vs_truth_sampled"] = float(np.linalg.norm(x - t) /
                                                    np.linalg.norm(t))
    cpu = None
    if not a.no_cpu_baseline:
        orc, oinfos, cpu = cpu_baseline(prob, prm, a.cpu_seconds,
                                          start + a.warmup + done)
        log(f"cpu baseline: {cpu['value']} steps/s over {len(oinfos)} steps")
        # a fresh GPU solve against the oracle, step by step from step 1
        gpu_hist = warm + infos
        j = len(oinfos)
        same = all((g["r"], g["k"], g["p"], g["fresh"], g["recycled"], g["rejected"]) ==
                   (o.r, o.k, o.p, o.fresh, o.recycled, o.rejected)
                   for g, o in zip(gpu_hist, oinfos))
        acc["oracle_steps_compared"] = j
        acc["oracle_same_control"] = bool(same)
        acc["res_hist_max_rel_diff"] = float(max(
            abs(g["res"] - o.res) / max(abs(o.res), 1e-300)
            for g, o in zip(gpu_hist, oinfos)))
        chk = SVT(prob.m, prob.n, prob.rows, prob.cols, prob.vals, prm)
        for _ in range(j):
            chk.step()
        acc["rel_err_vs_oracle"] = float(factored_rel_diff(chk.factors(),
                                                           (orc.U, orc.sig, orc.V)))
        acc["sigma_max_rel_diff_vs_oracle"] = float(np.max(
            np.abs(chk.sigma() - oinfos[-1].S) / np.abs(oinfos[-1].S)))
        chk.close()
        log(f"oracle agreement over {j} steps: X {acc['rel_err_vs_oracle']:.2e}, "
            f"residuals {acc['res_hist_max_rel_diff']:.2e}")
    serve = serving_leg(a) if a.serve > 0 else None
    if a.copy_calib_mib:
        n = a.copy_calib_mib * (1 << 20) // 4
        src = torch.empty(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    line = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": done,
        "warmup": a.warmup,
        "ms_per_step": round(dt * 1e3 / done, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}[a.precision],
        "data": "synthetic",
        "config": {"workload": a.workload, "m": prob.m, "n": prob.n,
                   "nnz": prob.nnz, "precision": a.precision,
                   "recycle": prm["recycle"], "ritz_tol": prm["ritz_tol"],
                   "p_init": prm["p_init"], "k_max": prm["k_max"],
                   "adaptive_p": prm["adaptive_p"], "tau": prm["tau"],
                   "delta": prm["delta"], "eps": prm["eps"], "i_max": prm["i_max"]},
        "window": window,
        "roofline": roof,
        "cpu_baseline": cpu,
        "accuracy": acc,
        "whole_solve": whole,
        "modes": modes or None,
        "serving": serve,
        "kernels": family_table(prof, tp1 - tp0, a.precision),
        "profiled_pass": {"steps": pdone,
                          "ms_per_step": round(prof_ms, 4) if prof_ms else None,
                          "launch": "kernel by kernel, HIP events per launch"},
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
