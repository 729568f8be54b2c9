"""Request-loop bookkeeping of the serving path (no device: fake solves)."""

import types

import numpy as np
import pytest

from paper_1810_06860_amd import serving


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeSolve:
    def __init__(self, req, log):
        self.req, self.i, self.log, self.closed = req, 0, log, False
        log.append(("admit", req.id))

    def close(self):
        self.closed = True
        self.log.append(("done", self.req.id))


def _setup(need, fps, arrivals, clock, step_cost=1e-3):
    log, live = [], []

    def factory(req):
        s = FakeSolve(req, log)
        live.append(s)
        return s

    def stepper(solves):
        clock.t += step_cost
        infos = []
        for s in solves:
            assert not s.closed
            s.i += 1
            infos.append(dict(i=s.i, r=1, res=1.0 / s.i,
                              converged=int(s.i >= need[s.req.id])))
        return infos, [0] * len(solves)

    reqs = [serving.Request(j, arrivals[j], types.SimpleNamespace(), dict(i_max=50))
            for j in range(len(need))]
    return reqs, factory, stepper, (lambda r: fps[r.id]), log, live


def test_budget_and_fifo_admission():
    clock = FakeClock()
    need = [5, 3, 8, 2, 4, 6]
    fps = [40, 30, 50, 10, 20, 30]
    arrivals = [0.0, 0.0, 0.001, 0.001, 0.002, 0.010]
    reqs, factory, stepper, fp, log, live = _setup(need, fps, arrivals, clock)
    used, peak = [0], [0]

    def fp_tracked(r):
        return fp(r)

    out = serving.serve(reqs, budget_bytes=100, max_active=8, solver_factory=factory,
                        stepper=stepper, footprint_fn=fp_tracked, clock=clock,
                        sleep=clock.sleep)
    # memory in use never exceeds the budget
    for ev, rid in log:
        used[0] += fps[rid] if ev == "admit" else -fps[rid]
        peak[0] = max(peak[0], used[0])
    assert peak[0] <= 100
    # admission is in arrival order
    admits = [rid for ev, rid in log if ev == "admit"]
    assert admits == sorted(admits, key=lambda j: (arrivals[j], j))
    assert sorted(s.id for s in out) == list(range(len(need)))
    for s in out:
        assert s.steps == need[s.id]
        assert s.converged
        assert s.latency >= need[s.id] * 1e-3 - 1e-12
        assert s.t_admit >= s.t_arrival
    assert all(s.closed for s in live)
    summ = serving.summarize(out)
    assert summ["requests"] == 6 and summ["converged"] == 6
    assert summ["p50_s"] <= summ["p99_s"] <= summ["max_s"]


def test_oversize_request_runs_alone_and_max_active():
    clock = FakeClock()
    need = [3, 3, 3, 3]
    fps = [500, 10, 10, 10]            # the first is larger than the budget
    arrivals = [0.0, 0.0, 0.0, 0.0]
    reqs, factory, stepper, fp, log, live = _setup(need, fps, arrivals, clock)
    active, peak_active = [0], [0]

    def stepper_count(solves):
        peak_active[0] = max(peak_active[0], len(solves))
        if any(s.req.id == 0 for s in solves):
            assert len(solves) == 1
        return stepper(solves)

    out = serving.serve(reqs, budget_bytes=100, max_active=2, solver_factory=factory,
                        stepper=stepper_count, footprint_fn=fp, clock=clock,
                        sleep=clock.sleep)
    assert peak_active[0] <= 2
    assert len(out) == 4


def test_i_max_retires_unconverged():
    clock = FakeClock()
    reqs, factory, stepper, fp, log, live = _setup([1000], [1], [0.0], clock)
    reqs[0].params["i_max"] = 7
    out = serving.serve(reqs, budget_bytes=10, solver_factory=factory, stepper=stepper,
                        footprint_fn=fp, clock=clock, sleep=clock.sleep)
    assert out[0].steps == 7 and not out[0].converged


def test_idle_until_next_arrival():
    clock = FakeClock()
    reqs, factory, stepper, fp, log, live = _setup([2, 2], [1, 1], [0.0, 5.0], clock)
    out = serving.serve(reqs, budget_bytes=10, solver_factory=factory, stepper=stepper,
                        footprint_fn=fp, clock=clock, sleep=clock.sleep)
    second = [s for s in out if s.id == 1][0]
    assert second.t_admit >= 5.0
    assert second.latency == pytest.approx(2e-3, abs=1e-9)
