"""Continuous-batching request loop for completion solves.

Requests arrive over time.  Each admitted request becomes one SVT handle
whose iterate, factors and workspaces stay resident on the device between
steps.  One round of the loop:

* admits the waiting requests whose arrival time has passed, in arrival
  order, while a slot is free and the sum of the admitted solves' device
  footprints (``mc_svt_footprint``) stays within the memory budget (a request
  larger than the whole budget is admitted only when nothing else runs);
* advances every admitted solve by one fast-SVT step with
  ``mc_svt_step_many``: their device work overlaps on separate streams while
  the host serves their read-backs in turn;
* retires the solves that converged or reached i_max, freeing their memory.

Latency is completion time minus arrival time.  The solver, the stepping
call, the footprint and the clock are parameters, so the loop's bookkeeping
can be exercised without a device.
"""

import collections
import time
from dataclasses import dataclass, field

import numpy as np

MC_OK = 0


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

    @property
    def latency(self):
        return self.t_done - self.t_arrival


@dataclass
class _Slot:
    req: Request
    solver: object
    fp: int
    t_admit: float
    steps: int = 0
    last: dict = field(default_factory=dict)


def _default_factory(stream_pool):
    from .svt import SVT
    import ctypes as C
    counter = [0]

    def make(req):
        st = None
        if stream_pool:
            s = stream_pool[counter[0] % len(stream_pool)]
            counter[0] += 1
            st = C.c_void_p(s.cuda_stream)
        p = req.problem
        return SVT(p.m, p.n, p.rows, p.cols, p.vals, req.params, stream=st)
    return make


def serve(requests, budget_bytes, max_active=16, solver_factory=None, stepper=None,
          footprint_fn=None, clock=time.perf_counter, sleep=time.sleep,
          keep_factors=False, stream_pool=None):
    """Run the request loop until every request is served.

    Returns a list of `Served` records in completion order.
    """
    if solver_factory is None:
        solver_factory = _default_factory(stream_pool)
    if stepper is None:
        from .svt import step_many
        stepper = step_many
    if footprint_fn is None:
        from .svt import footprint

        def footprint_fn(req):
            p = req.problem
            return footprint(p.m, p.n, p.rows.size, req.params)

    pending = collections.deque(sorted(requests, key=lambda r: (r.t_arrival, r.id)))
    active, done = [], []
    used = 0
    t0 = clock()
    while pending or active:
        now = clock() - t0
        while pending and pending[0].t_arrival <= now and len(active) < max_active:
            req = pending[0]
            fp = int(footprint_fn(req))
            if active and used + fp > budget_bytes:
                break                                  # wait for memory
            pending.popleft()
            active.append(_Slot(req, solver_factory(req), fp, clock() - t0))
            used += fp
        if not active:
            sleep(max(0.0, pending[0].t_arrival - (clock() - t0)))
            continue
        infos, statuses = stepper([s.solver for s in active])
        now = clock() - t0
        keep = []
        for s, info, st in zip(active, infos, statuses):
            if st == MC_OK:
                s.steps += 1
                s.last = info
            finished = (st != MC_OK or info.get("converged", 0) or
                        s.steps >= s.req.params.get("i_max", 200))
            if not finished:
                keep.append(s)
                continue
            facs = s.solver.factors() if keep_factors and st == MC_OK else None
            done.append(Served(id=s.req.id, t_arrival=s.req.t_arrival, t_admit=s.t_admit,
                               t_done=now, steps=s.steps, status=int(st),
                               converged=bool(s.last.get("converged", 0)),
                               rank=int(s.last.get("r", 0)),
                               res=float(s.last.get("res", float("nan"))),
                               footprint=s.fp, factors=facs))
            s.solver.close()
            used -= s.fp
        active = keep
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
