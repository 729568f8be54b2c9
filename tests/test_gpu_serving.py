"""Served solves (continuous batching, overlapping streams) against the same
requests solved alone, and against the FP64 form."""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _X(f):
    U, s, V = f
    return (U * s) @ V.T


@pytest.mark.parametrize("graphs", [False, True])
def test_served_results_equal_alone_and_close_to_fp64(graphs):
    # the bench serves with captured graphs (relaxed capture from several host
    # threads over shared streams): both forms must give each request the
    # bits of its solve alone
    import torch
    from paper_1810_06860_amd import SVT, serving
    desc = synth.serving_trace(num=8, mean_gap_s=0.003, mn_range=(200, 500),
                               rank_range=(5, 20), ratio_range=(0.2, 0.4))
    problems = [synth.request_problem(r) for r in desc]
    params = [dict(synth.serving_params(p.m, p.n, p.nnz), precision="fp32")
              for p in problems]
    alone, fp64 = {}, {}
    for j, (p, prm) in enumerate(zip(problems, params)):
        with SVT(p.m, p.n, p.rows, p.cols, p.vals, prm) as s:
            out = s.solve()
            alone[j] = (out, s.factors())
        with SVT(p.m, p.n, p.rows, p.cols, p.vals, dict(prm, precision="fp64")) as s:
            s.solve()
            fp64[j] = s.factors()
    streams = [torch.cuda.Stream() for _ in range(4)]
    reqs = [serving.Request(j, d["t_arrival"], p, prm)
            for j, (d, p, prm) in enumerate(zip(desc, problems, params))]
    served = serving.serve(reqs, budget_bytes=1 << 34, max_active=8, keep_factors=True,
                           stream_pool=streams, graphs=graphs)
    torch.cuda.synchronize()
    assert sorted(s.id for s in served) == list(range(len(desc)))
    for s in served:
        out, f = alone[s.id]
        assert s.status == 0
        assert s.steps == out["iters"]
        assert s.rank == out["rank"]
        Xa, Xs = _X(f), _X(s.factors)
        # identical kernels on identical inputs: the mix changes nothing
        assert np.array_equal(Xa, Xs), np.abs(Xa - Xs).max()
        X64 = _X(fp64[s.id])
        rel = np.linalg.norm(Xs - X64) / np.linalg.norm(X64)
        print(f"req {s.id}: {problems[s.id].m}x{problems[s.id].n} steps {s.steps} "
              f"rank {s.rank} conv {s.converged} latency {s.latency * 1e3:.1f} ms "
              f"vs fp64 {rel:.2e}")
        assert rel < 1e-3
    summ = serving.summarize(served)
    print(summ)


def test_step_many_equals_single_steps():
    # several handles advanced together by mc_svt_step_many (host worker
    # threads, direct launches) against the same problems stepped one by one
    from paper_1810_06860_amd import SVT, step_many
    probs = [synth.planted(260 + 40 * j, 220 + 30 * j, 4 + j, 0.35, seed_data=70 + j,
                           seed_phi=170 + j) for j in range(4)]
    prm = dict(eps=1e-6, i_max=40, use_graphs=0)
    many = [SVT(p.m, p.n, p.rows, p.cols, p.vals, prm) for p in probs]
    one = [SVT(p.m, p.n, p.rows, p.cols, p.vals, prm) for p in probs]
    for _ in range(25):
        infos, status = step_many(many)
        for j, s in enumerate(one):
            if status[j] == 0:
                assert s.step() == infos[j]
            else:
                assert status[j] == 7          # MC_EDONE: converged earlier
    for a, b in zip(many, one):
        Ua, sa, Va = a.factors()
        Ub, sb, Vb = b.factors()
        assert np.array_equal(sa, sb) and np.array_equal(Ua, Ub) and np.array_equal(Va, Vb)


def test_step_group_equals_single_steps():
    # handles of every kind advanced by mc_svt_step_group (FP64 and FP32
    # products batched per kind, BF16 and recycled calls launched alone)
    # against the same problems stepped one by one with graphs off: the same
    # per-segment kernels run in either form, so every result is bit-identical
    from paper_1810_06860_amd import SVT, step_group
    probs = [synth.planted(260 + 40 * j, 220 + 30 * j, 4 + j, 0.35, seed_data=80 + j,
                           seed_phi=180 + j) for j in range(6)]
    prms = [dict(eps=1e-6, i_max=40, use_graphs=0, precision=prec)
            for prec in ("fp64", "fp32", "fp64", "fp32", "bf16", "fp64")]
    # one recycling solve (strategy 1 from step 10, Ritz guard on)
    prms[5].update(recycle=1, i_reuse=10, q_reuse=3, ritz_tol=1e-3)
    grp = [SVT(p.m, p.n, p.rows, p.cols, p.vals, q) for p, q in zip(probs, prms)]
    one = [SVT(p.m, p.n, p.rows, p.cols, p.vals, q) for p, q in zip(probs, prms)]
    for it in range(25):
        infos, status = step_group(grp)
        for j, s in enumerate(one):
            if status[j] == 0:
                assert s.step() == infos[j], (it, j)
            else:
                assert status[j] == 7          # MC_EDONE: converged earlier
    assert sum(s.result()["recycled"] for s in grp) > 0
    for a, b in zip(grp, one):
        Ua, sa, Va = a.factors()
        Ub, sb, Vb = b.factors()
        assert np.array_equal(sa, sb) and np.array_equal(Ua, Ub) and np.array_equal(Va, Vb)
        a.close()
        b.close()


def test_grouped_serving_equals_alone_at_trace_shapes():
    # the first requests of the 256-request serving trace (m, n up to 4000,
    # 10-40 % observed), served in batched rounds, against each solved alone
    # (graphs on, the bench's form): bit-identical, and within 1e-3 of FP64
    import torch
    from paper_1810_06860_amd import SVT, serving
    desc = synth.serving_trace()[:6]
    problems = [synth.request_problem(r) for r in desc]
    params = [dict(synth.serving_params(p.m, p.n, p.nnz), precision="fp32", i_max=60)
              for p in problems]
    alone, fp64 = {}, {}
    for j, (p, prm) in enumerate(zip(problems, params)):
        with SVT(p.m, p.n, p.rows, p.cols, p.vals, prm) as s:
            for _ in range(prm["i_max"]):
                if s.step()["converged"]:
                    break
            alone[j] = (s.result(), s.factors())
        with SVT(p.m, p.n, p.rows, p.cols, p.vals, dict(prm, precision="fp64")) as s:
            for _ in range(prm["i_max"]):
                if s.step()["converged"]:
                    break
            fp64[j] = s.factors()
    streams = [torch.cuda.Stream() for _ in range(4)]
    reqs = [serving.Request(j, 0.0, p, prm) for j, (p, prm) in enumerate(zip(problems, params))]
    served = serving.serve_grouped(reqs, budget_bytes=1 << 36, max_active=6,
                                   keep_factors=True, stream_pool=streams)
    torch.cuda.synchronize()
    assert sorted(s.id for s in served) == list(range(len(desc)))
    for s in served:
        res, f = alone[s.id]
        assert s.status == 0 and s.steps == res["iters"] and s.rank == res["rank"]
        Xa, Xs = _X(f), _X(s.factors)
        assert np.array_equal(Xa, Xs), np.abs(Xa - Xs).max()
        X64 = _X(fp64[s.id])
        rel = np.linalg.norm(Xs - X64) / np.linalg.norm(X64)
        print(f"req {s.id}: {problems[s.id].m}x{problems[s.id].n} nnz {problems[s.id].nnz} "
              f"steps {s.steps} rank {s.rank} vs fp64 {rel:.2e}")
        assert rel < 1e-3
