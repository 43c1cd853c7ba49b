"""Continuous-batching serving loop over the PASD C ABI.

Requests (one TRPCA solve each) arrive over time.  The loop admits arrived
requests while a slot is free and their device footprint (pasd_footprint)
fits the HBM budget, keeps every admitted solve resident on the GPU, and
advances all of them together: each step is `step_iters` iterations of every
resident solve as grouped kernel launches, followed by one batched status
read (pasd_query_batch).  The grouped step is launched directly
(pasd_step_batch) while the resident set changes; once the same set has been
stepped `graph_after` times in a row it is captured as a HIP graph
(pasd_batch_create) and replayed (pasd_batch_step) until a solve is admitted
or retired (graphs=False: always direct).  Solves that converged or hit their
iteration cap are retired (results copied out, device memory released) and
their slots go to waiting requests.  A request's latency is its completion
time minus its arrival time, queueing included.

The numerical work of a solve is the same alone and in the mix: the batched
kernels compute every problem with its own data and the same arithmetic (up
to the grouping of GEMM-M's partial sums, which differs for a solve launched
alone with I_n > 176, where results agree to rounding).
"""

from __future__ import annotations

import collections
import dataclasses
import time
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import pasd as P


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the run
    T: object               # torch CUDA tensor (state dtype) or numpy array
    ranks: Sequence[int]
    tol: float = 1e-6
    max_iter: int = 1000


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    completed: float
    iterations: int
    converged: bool
    done: int = 0
    X: object = None
    E: object = None

    @property
    def latency(self) -> float:
        return self.completed - self.arrival


class Server:
    def __init__(self, precision: str = "fp32", max_slots: int = 64,
                 hbm_budget: Optional[int] = None, step_iters: int = 4, device: int = 0,
                 keep_results: bool = True, graphs: bool = True, graph_after: int = 2):
        import torch
        self.precision = precision
        self.graphs = bool(graphs)
        self.graph_after = int(graph_after)
        self.max_slots = int(max_slots)
        self.step_iters = int(step_iters)
        self.device = device
        self.keep_results = keep_results
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info(device)
            hbm_budget = int(free * 0.8)
        self.hbm_budget = int(hbm_budget)
        self.stats: Dict[str, float] = {}

    def _footprint(self, req: Request) -> int:
        dims = tuple(int(d) for d in req.T.shape)
        cfg = P.make_config(dims, req.ranks, tol=req.tol, max_iter=req.max_iter,
                            precision=self.precision, device=self.device)
        return P.footprint(cfg)

    def run(self, requests: List[Request], realtime: bool = True) -> List[Result]:
        """Serve `requests` (sorted by arrival); with realtime=False every request
        is treated as arrived at time 0 (saturation throughput)."""
        import torch
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        active: List[tuple] = []  # (request, solver, footprint, admitted)
        results: List[Result] = []
        used = 0
        steps = 0
        captures = 0
        graph = None  # BatchGraph of the current resident set
        graph_set: tuple = ()
        stable = 0  # consecutive steps of the current set
        t0 = time.perf_counter()
        while pending or active:
            now = time.perf_counter() - t0
            while pending and len(active) < self.max_slots:
                req = pending[0]
                if realtime and req.arrival > now:
                    break
                fp = self._footprint(req)
                if used + fp > self.hbm_budget and active:
                    break
                pending.popleft()
                s = P.Solver(req.T, req.ranks, tol=req.tol, max_iter=req.max_iter,
                             precision=self.precision, device=self.device)
                used += fp
                active.append((req, s, fp, time.perf_counter() - t0))
            if not active:
                if pending and realtime:
                    wait = pending[0].arrival - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.01))
                continue
            solvers = [a[1] for a in active]
            key = tuple(id(x) for x in solvers)
            if key != graph_set:
                if graph is not None:
                    graph.close()
                    graph = None
                graph_set = key
                stable = 0
            stable += 1
            if graph is None and self.graphs and stable > self.graph_after:
                graph = P.BatchGraph(solvers, self.step_iters)
                captures += 1
            if graph is not None:
                graph.step()
            else:
                P.step_batch(solvers, self.step_iters)
            infos = P.query_batch(solvers)
            steps += 1
            keep = []
            for (req, s, fp, adm), info in zip(active, infos):
                if info.done:
                    X = E = None
                    if self.keep_results:
                        X, E = s.result()
                    done_t = time.perf_counter() - t0
                    results.append(Result(req.rid, req.arrival if realtime else 0.0, adm, done_t,
                                          info.iterations, bool(info.converged), info.done, X, E))
                    if graph is not None:  # the graph holds this solve's state
                        graph.close()
                        graph = None
                    graph_set = ()
                    s.close()
                    used -= fp
                else:
                    keep.append((req, s, fp, adm))
            active = keep
        if graph is not None:
            graph.close()
        torch.cuda.synchronize()
        self.stats = {"steps": steps, "captures": captures, "wall_s": time.perf_counter() - t0}
        return sorted(results, key=lambda r: r.rid)


def latency_summary(results: List[Result]) -> dict:
    lat = np.array([r.latency for r in results])
    wall = max(r.completed for r in results) - min(r.arrival for r in results)
    return {"count": len(results), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "solves_per_s": len(results) / wall if wall > 0 else float("inf"),
            "converged": int(sum(r.converged for r in results)),
            "floor": int(sum(r.done == 4 for r in results))}


def service_times(requests: List[Request], precision: str = "fp32", device: int = 0) -> Dict[int, float]:
    """Seconds each request takes when served alone by plain calls: context
    creation (allocation and the copy of T), pasd_solve, the copy-out of X and
    E, and release."""
    import torch
    out = {}
    for req in requests:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = P.Solver(req.T, req.ranks, tol=req.tol, max_iter=req.max_iter, precision=precision,
                     device=device)
        s.solve()
        s.result()
        s.close()
        torch.cuda.synchronize()
        out[req.rid] = time.perf_counter() - t0
    return out


def sequential_replay(requests: List[Request], service: Dict[int, float]) -> List[Result]:
    """The trace served one request at a time, service starting at
    max(arrival, previous completion), with measured service times."""
    results = []
    clock = 0.0
    for req in sorted(requests, key=lambda r: r.arrival):
        start = max(clock, req.arrival)
        clock = start + service[req.rid]
        results.append(Result(req.rid, req.arrival, start, clock, 0, True))
    return results


def sequential(requests: List[Request], precision: str = "fp32", device: int = 0) -> List[Result]:
    """The same trace served one solve at a time with plain pasd_solve (no
    batching); service starts at max(arrival, previous completion)."""
    import torch
    results = []
    clock = 0.0
    for req in sorted(requests, key=lambda r: r.arrival):
        s = P.Solver(req.T, req.ranks, tol=req.tol, max_iter=req.max_iter, precision=precision,
                     device=device)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info = s.solve()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        s.close()
        start = max(clock, req.arrival)
        clock = start + dt
        results.append(Result(req.rid, req.arrival, start, clock, info.iterations,
                              bool(info.converged)))
    return results
