"""Continuous-batching request loop for completion solves.

Requests arrive over time.  Each admitted request becomes one SVT handle
whose iterate, factors and workspaces stay resident on the device until it
finishes.  The loop

* admits the waiting requests whose arrival time has passed, in arrival
  order, while a slot is free and the sum of the admitted solves' device
  footprints (``mc_svt_footprint``) stays within the memory budget (a request
  larger than the whole budget is admitted only when nothing else runs);
* runs every admitted solve on a worker thread of its own, step after step
  (``mc_svt_step``), on a stream of its own, so the device work of all
  admitted solves overlaps and a short request never waits for the steps of
  a long one;
* retires each solve when it converges or reaches i_max, which frees its slot
  and memory for the next arrivals.

Latency is completion time minus arrival time.  The solver factory and the
footprint are parameters, so the loop can be exercised without a device.

With ``grouped=True`` one driver thread advances all admitted solves
together, one SVT step each per round (``mc_svt_step_group``): their fresh
rSVD-BKI calls run in lock-step stages and the sparse products of a stage go
out in shared launches, so the device sees one launch per stage and lane form
for the whole batch instead of one per solve.  Admission and retirement
happen between rounds; results are the same as each request solved alone.
"""

import collections
import ctypes as C
import threading
import time
from dataclasses import dataclass

import numpy as np

MC_OK = 0
MC_ENOTCONV = 8


@dataclass
class Request:
    id: int
    t_arrival: float
    problem: object            # synth.Problem-like: m, n, rows, cols, vals
    params: dict


@dataclass
class Served:
    id: int
    t_arrival: float
    t_admit: float
    t_done: float
    steps: int
    status: int
    converged: bool
    rank: int
    res: float
    footprint: int
    factors: tuple = None
    error: str = ""

    @property
    def latency(self):
        return self.t_done - self.t_arrival


def _default_factory(stream_pool, graphs):
    from .svt import SVT
    counter = [0]
    lock = threading.Lock()

    def make(req):
        st = None
        if stream_pool:
            with lock:
                s = stream_pool[counter[0] % len(stream_pool)]
                counter[0] += 1
            st = C.c_void_p(s.cuda_stream)
        p = req.problem
        prm = dict(req.params, use_graphs=int(bool(graphs)))
        return SVT(p.m, p.n, p.rows, p.cols, p.vals, prm, stream=st)
    return make


def _run_to_end(solver, i_max):
    """Step one solve until it converges or reaches i_max."""
    from .svt import MCError
    steps, last, status, err = 0, {}, MC_OK, ""
    try:
        while steps < i_max:
            last = solver.step()
            steps += 1
            if last.get("converged"):
                break
    except MCError as e:
        status, err = e.status, str(e)
    return steps, last, status, err


def serve(requests, budget_bytes, max_active=16, solver_factory=None,
          footprint_fn=None, clock=time.perf_counter, keep_factors=False,
          stream_pool=None, on_done=None, device=None, graphs=False):
    """Run the request loop until every request is served.

    Returns a list of `Served` records in completion order; `on_done(record,
    count)` is called as each request completes.  With `graphs`, each solve
    replays captured graphs of its SVD calls (a capture the runtime drops
    falls back to direct launches for that solve).
    """
    if solver_factory is None:
        solver_factory = _default_factory(stream_pool, graphs)
    if footprint_fn is None:
        from .svt import footprint

        def footprint_fn(req):
            p = req.problem
            return footprint(p.m, p.n, p.rows.size, req.params)

    pending = collections.deque(sorted(requests, key=lambda r: (r.t_arrival, r.id)))
    cv = threading.Condition()
    state = dict(used=0, active=0)
    done, threads, errors = [], [], []
    t0 = clock()

    def worker(req, fp, t_admit):
        try:
            if device is not None:
                device()
            solver = solver_factory(req)
            steps, last, status, err = _run_to_end(solver, req.params.get("i_max", 200))
            facs = solver.factors() if keep_factors and status == MC_OK else None
            solver.close()
            rec = Served(id=req.id, t_arrival=req.t_arrival, t_admit=t_admit,
                         t_done=clock() - t0, steps=steps, status=int(status),
                         converged=bool(last.get("converged", 0)),
                         rank=int(last.get("r", 0)),
                         res=float(last.get("res", float("nan"))), footprint=fp,
                         factors=facs, error=err)
        except Exception as e:                       # reported after the loop
            errors.append(e)
            rec = None
        with cv:
            state["used"] -= fp
            state["active"] -= 1
            if rec is not None:
                done.append(rec)
                if on_done is not None:
                    on_done(rec, len(done))
            cv.notify_all()

    with cv:
        while pending or state["active"]:
            now = clock() - t0
            admitted = False
            while pending and pending[0].t_arrival <= now and state["active"] < max_active:
                req = pending[0]
                fp = int(footprint_fn(req))
                if state["active"] and state["used"] + fp > budget_bytes:
                    break                                  # wait for memory
                pending.popleft()
                state["used"] += fp
                state["active"] += 1
                th = threading.Thread(target=worker, args=(req, fp, now), daemon=True)
                threads.append(th)
                th.start()
                admitted = True
            if admitted:
                continue
            # sleep until the next arrival or a completion
            timeout = None
            if pending and pending[0].t_arrival > now:
                timeout = pending[0].t_arrival - now
            if timeout is None and not state["active"]:
                continue
            cv.wait(timeout=timeout if timeout is not None else 1.0)
    for th in threads:
        th.join()
    if errors:
        raise errors[0]
    return done


def serve_grouped(requests, budget_bytes, max_active=16, solver_factory=None,
                  footprint_fn=None, clock=time.perf_counter, keep_factors=False,
                  stream_pool=None, on_done=None, step_group=None):
    """The request loop with batched rounds: between rounds, arrivals are
    admitted (arrival order, free slot, footprint within the budget) and
    finished solves retired; each round advances every admitted solve by one
    step with `step_group` (``mc_svt_step_group`` by default).  Returns the
    `Served` records in completion order."""
    if solver_factory is None:
        solver_factory = _default_factory(stream_pool, False)
    if footprint_fn is None:
        from .svt import footprint

        def footprint_fn(req):
            p = req.problem
            return footprint(p.m, p.n, p.rows.size, req.params)
    if step_group is None:
        from .svt import step_group
    pending = collections.deque(sorted(requests, key=lambda r: (r.t_arrival, r.id)))
    active = []             # [req, solver, footprint, t_admit, steps, last]
    used = 0
    done = []
    t0 = clock()

    def retire(entry, status, err=""):
        nonlocal used
        req, solver, fp, t_admit, steps, last = entry
        facs = solver.factors() if keep_factors and status == MC_OK else None
        solver.close()
        rec = Served(id=req.id, t_arrival=req.t_arrival, t_admit=t_admit,
                     t_done=clock() - t0, steps=steps, status=int(status),
                     converged=bool(last.get("converged", 0)),
                     rank=int(last.get("r", 0)),
                     res=float(last.get("res", float("nan"))), footprint=fp,
                     factors=facs, error=err)
        used -= fp
        done.append(rec)
        if on_done is not None:
            on_done(rec, len(done))

    while pending or active:
        now = clock() - t0
        while pending and pending[0].t_arrival <= now and len(active) < max_active:
            req = pending[0]
            fp = int(footprint_fn(req))
            if active and used + fp > budget_bytes:
                break                                      # wait for memory
            pending.popleft()
            used += fp
            active.append([req, solver_factory(req), fp, now, 0, {}])
        if not active:
            time.sleep(max(0.0, pending[0].t_arrival - (clock() - t0)))
            continue
        infos, status = step_group([e[1] for e in active])
        still = []
        for e, info, st in zip(active, infos, status):
            if st == MC_OK:
                e[4] += 1
                e[5] = info
            i_max = e[0].params.get("i_max", 200)
            if st != MC_OK or info.get("converged") or e[4] >= i_max:
                err = "" if st == MC_OK else f"status {st}"
                retire(e, st, err)
            else:
                still.append(e)
        active = still
    return done


def summarize(served):
    lat = np.array([s.latency for s in served])
    steps = sum(s.steps for s in served)
    span = max(s.t_done for s in served) - min(s.t_arrival for s in served)
    return dict(requests=len(served),
                p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                mean_s=float(lat.mean()), max_s=float(lat.max()),
                makespan_s=float(span), steps_total=int(steps),
                steps_per_s=float(steps / span) if span > 0 else None,
                converged=int(sum(s.converged for s in served)),
                failed=int(sum(s.status != MC_OK for s in served)))
