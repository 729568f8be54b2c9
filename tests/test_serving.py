"""Request-loop bookkeeping of the serving path (no device: fake solves that
take a fixed time per step)."""

import threading
import time
import types

import pytest

from paper_1810_06860_amd import serving

STEP_S = 0.002


class Ledger:
    """Memory and slot use seen by the fake solves, checked against limits."""

    def __init__(self, fps):
        self.fps, self.used, self.peak, self.active, self.peak_active = fps, 0, 0, 0, 0
        self.order, self.lock = [], threading.Lock()

    def admit(self, rid):
        with self.lock:
            self.used += self.fps[rid]
            self.active += 1
            self.peak = max(self.peak, self.used)
            self.peak_active = max(self.peak_active, self.active)
            self.order.append(rid)

    def leave(self, rid):
        with self.lock:
            self.used -= self.fps[rid]
            self.active -= 1


class FakeSolve:
    def __init__(self, req, need, ledger):
        self.req, self.need, self.i, self.ledger = req, need, 0, ledger
        ledger.admit(req.id)

    def step(self):
        time.sleep(STEP_S)
        self.i += 1
        return dict(i=self.i, r=1, res=1.0 / self.i, converged=int(self.i >= self.need))

    def factors(self):
        return None

    def close(self):
        self.ledger.leave(self.req.id)


def _run(need, fps, arrivals, budget, max_active=8, i_max=50):
    ledger = Ledger(fps)
    reqs = [serving.Request(j, arrivals[j], types.SimpleNamespace(), dict(i_max=i_max))
            for j in range(len(need))]
    out = serving.serve(reqs, budget_bytes=budget, max_active=max_active,
                        solver_factory=lambda r: FakeSolve(r, need[r.id], ledger),
                        footprint_fn=lambda r: fps[r.id])
    return out, ledger


def test_budget_fifo_and_latency():
    need = [5, 3, 8, 2, 4, 6]
    fps = [40, 30, 50, 10, 20, 30]
    arrivals = [0.0, 0.0, 0.01, 0.01, 0.02, 0.05]
    out, ledger = _run(need, fps, arrivals, budget=100)
    assert ledger.peak <= 100
    # admission follows arrival order
    assert ledger.order == sorted(ledger.order, key=lambda j: (arrivals[j], j))
    assert sorted(s.id for s in out) == list(range(len(need)))
    for s in out:
        assert s.steps == need[s.id] and s.converged
        assert s.t_admit >= s.t_arrival - 1e-9
        assert s.latency >= need[s.id] * STEP_S * 0.9
    summ = serving.summarize(out)
    assert summ["requests"] == 6 and summ["converged"] == 6
    assert summ["p50_s"] <= summ["p99_s"] <= summ["max_s"]


def test_short_requests_do_not_wait_for_long_ones():
    # one long solve and several short ones admitted together: the short ones
    # finish long before the long one (no lock-step rounds)
    need = [200, 3, 3, 3]
    out, ledger = _run(need, [1, 1, 1, 1], [0.0] * 4, budget=10)
    lat = {s.id: s.latency for s in out}
    assert max(lat[1], lat[2], lat[3]) < 0.5 * lat[0]


def test_oversize_alone_and_slot_limit():
    need = [3, 3, 3, 3, 3]
    fps = [500, 10, 10, 10, 10]          # the first is larger than the budget
    out, ledger = _run(need, fps, [0.0] * 5, budget=100, max_active=2)
    assert ledger.peak_active <= 2
    assert len(out) == 5
    first = [s for s in out if s.id == 0][0]
    others = [s for s in out if s.id != 0]
    assert all(o.t_admit >= first.t_done - 1e-3 for o in others)


def test_i_max_retires_unconverged_and_idle_wait():
    out, _ = _run([1000, 2], [1, 1], [0.0, 0.2], budget=10, i_max=7)
    a = [s for s in out if s.id == 0][0]
    b = [s for s in out if s.id == 1][0]
    assert a.steps == 7 and not a.converged
    assert b.t_admit >= 0.2 - 1e-9


class _Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class _RoundSolve:
    """A solve that never converges; closes into a ledger of retirements."""

    def __init__(self, req, closed):
        self.req, self.i, self.closed = req, 0, closed

    def step(self):
        self.i += 1
        return dict(i=self.i, r=1, res=1.0, converged=0)

    def factors(self):
        return None

    def close(self):
        self.closed.append(self.req.id)


def test_grouped_rounds_admission_and_retirement():
    # batched rounds: every admitted solve takes one step per round; arrivals
    # join between rounds while slots and memory allow; a solve retires in
    # the round it reaches i_max
    clock = _Clock()
    rounds, closed = [], []

    def step_group(solves):
        rounds.append(sorted(s.req.id for s in solves))
        clock.t += 0.01
        return [s.step() for s in solves], [0] * len(solves)

    reqs = [serving.Request(0, 0.0, None, dict(i_max=3)),
            serving.Request(1, 0.0, None, dict(i_max=1)),
            serving.Request(2, 0.0, None, dict(i_max=2)),
            serving.Request(3, 0.015, None, dict(i_max=2))]
    fp = {0: 40, 1: 40, 2: 40, 3: 10}
    done = serving.serve_grouped(reqs, budget_bytes=100, max_active=4,
                                 solver_factory=lambda r: _RoundSolve(r, closed),
                                 footprint_fn=lambda r: fp[r.id], clock=clock,
                                 step_group=step_group)
    assert sorted(s.id for s in done) == [0, 1, 2, 3]
    # request 2 waits for memory until request 1 retires; request 3 arrives
    # at 15 ms and joins the round after that
    assert rounds[0] == [0, 1]
    assert rounds[1] == [0, 2]
    assert rounds[2] == [0, 2, 3]
    assert {s.id: s.steps for s in done} == {0: 3, 1: 1, 2: 2, 3: 2}
    assert closed == [1, 0, 2, 3]
    assert all(not s.converged for s in done)
