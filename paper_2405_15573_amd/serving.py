"""Serving loop: many resident operators, GMRES solve requests arriving over time.

* Operators stay resident in HBM in two forms: complex128 in the many-RHS layout (true
  residuals) and a low-precision form (complex64 or bf16 pairs) for the inner products
  of mixed-precision GMRES with iterative refinement.
* Requests (operator, right-hand sides, tolerance, arrival time) are admitted in arrival
  order when their solve workspace fits the HBM budget (``Admission``); otherwise they
  wait in the queue and are admitted as finished solves free their memory.
* Continuous batching: every step gives each admitted solve one product; the products of
  all solves are grouped per (operator, precision) into multi-column products inside the
  library (``uhm_krylov_step``), so solves on the same operator share one pass over it and
  the device work of different solves overlaps within a step.  Solves that arrive while
  others run join at the next step; finished solves leave and free their slot.
* Each solve's columns are products of its own Krylov vectors only, with per-column
  reductions that do not depend on the other columns, so its result is the same alone or
  in any mix.

Latency = completion - arrival; throughput = completed solves / span of the run.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field

import numpy as np


def solve_footprint(n: int, nrhs: int, restart: int) -> int:
    """Device bytes a GMRES-IR solve holds: the (m+1) Krylov vectors and the dozen
    n x nrhs complex128 work vectors, plus product staging (bounded by the same size), and
    the least-squares state of a cycle (Hessenberg columns, rotations, g; complex128)."""
    return 16 * n * nrhs * (restart + 1 + 12) + 16 * nrhs * (restart + 1) * (restart + 4)


class Admission:
    """Arrival-order admission against a memory budget (pure host logic).

    ``offer`` queues a request; ``admit`` returns the requests that now fit, in arrival
    order, stopping at the first that does not (no overtaking, so no starvation);
    ``release`` returns a finished request's bytes.  A request larger than the whole budget
    is rejected at ``offer``."""

    def __init__(self, budget_bytes: int, max_active: int = 1 << 30):
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.used = 0
        self.active = 0
        self.queue = collections.deque()
        self.rejected = []

    def offer(self, req, nbytes: int) -> bool:
        if nbytes > self.budget:
            self.rejected.append(req)
            return False
        self.queue.append((req, int(nbytes)))
        return True

    def admit(self):
        out = []
        while self.queue and self.active < self.max_active and self.used + self.queue[0][1] <= self.budget:
            req, nb = self.queue.popleft()
            self.used += nb
            self.active += 1
            out.append((req, nb))
        return out

    def release(self, nbytes: int):
        self.used -= int(nbytes)
        self.active -= 1
        if self.used < 0 or self.active < 0:
            raise RuntimeError("admission accounting went negative")


@dataclass
class Request:
    rid: int
    op: int
    b: object            # torch complex128 tensor (n, r) on the device
    tol: float
    arrival: float       # seconds after the start of the run
    start: float = math.nan
    finish: float = math.nan
    info: dict = field(default_factory=dict)
    code: int = 0
    x: object = None


class Server:
    def __init__(self, host_ops, low_storage: str = "c64", restart: int = 50, inner_tol: float = 1e-4,
                 max_iterations: int = 1000, max_refinements: int = 30, hbm_budget: int | None = None,
                 max_active: int = 256, stream=None, keep_solutions: bool = False, inner_cycles: int = 1):
        import torch

        from . import binding
        self.binding = binding
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.high = [binding.upload(op, storage="c128multi", stream=self.stream) for op in host_ops]
        self.low = [binding.upload(op, storage=low_storage, stream=self.stream) for op in host_ops]
        self.n = [int(op.n) for op in host_ops]
        self.restart = restart
        self.inner_tol = inner_tol
        self.max_iterations = max_iterations
        self.max_refinements = max_refinements
        self.inner_cycles = inner_cycles
        if inner_cycles > 0:   # every inner_cycles cycles is one refinement step
            self.max_refinements = max(max_refinements, max_iterations // (restart * inner_cycles) + 2)
        # time inside the batched steps, their count and the solves they served
        self.step_s = 0.0
        self.steps = 0
        self.step_solves = 0
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = int(0.6 * free)
        self.admission = Admission(hbm_budget, max_active)
        self.keep_solutions = keep_solutions

    def footprint(self, req: Request) -> int:
        return solve_footprint(self.n[req.op], int(req.b.shape[1]), self.restart)

    def serve(self, requests, clock=time.perf_counter, log=None):
        """Run the requests (sorted by arrival) to completion; returns them with times filled."""
        reqs = sorted(requests, key=lambda q: q.arrival)
        adm = self.admission
        active = []      # (request, solve, bytes)
        t0 = clock()
        i = 0
        done = 0
        steps = 0
        while i < len(reqs) or adm.queue or active:
            now = clock() - t0
            while i < len(reqs) and reqs[i].arrival <= now:
                adm.offer(reqs[i], self.footprint(reqs[i]))
                i += 1
            for req, nb in adm.admit():
                req.start = clock() - t0
                k = self.binding.Krylov(req.b, req.tol, mixed=True, restart=self.restart,
                                        max_iterations=self.max_iterations, max_refinements=self.max_refinements,
                                        inner_tol=self.inner_tol, stream=self.stream,
                                        inner_cycles=self.inner_cycles)
                active.append((req, k, nb))
            if not active:
                if i < len(reqs):
                    time.sleep(max(0.0, reqs[i].arrival - (clock() - t0)))
                continue
            ts = clock()
            self.binding.krylov_step([a[1] for a in active], [self.high[a[0].op] for a in active],
                                     [self.low[a[0].op] for a in active], stream=self.stream)
            self.step_s += clock() - ts
            self.steps += 1
            self.step_solves += len(active)
            steps += 1
            still = []
            for req, k, nb in active:
                if k.pending() == self.binding.KRYLOV_DONE:
                    x, info, rc = k.result()
                    req.finish = clock() - t0
                    req.info, req.code = info, rc
                    if self.keep_solutions:
                        req.x = x
                    k.free()
                    adm.release(nb)
                    done += 1
                else:
                    still.append((req, k, nb))
            active = still
            if log is not None and steps % 200 == 0:
                log(f"  serving: t={clock() - t0:.1f}s step {steps} active {len(active)} queued {len(adm.queue)} "
                    f"done {done}/{len(reqs)}")
        return reqs

    @staticmethod
    def report(reqs) -> dict:
        fin = [q for q in reqs if not math.isnan(q.finish)]
        lat = np.array([q.finish - q.arrival for q in fin])
        if not len(fin):
            return {"completed": 0}
        span = max(q.finish for q in fin) - min(q.arrival for q in reqs)
        conv = np.array([q.finish - q.arrival for q in fin if q.code == 0])
        return {
            "completed": len(fin),
            "converged": int(sum(1 for q in fin if q.code == 0)),
            "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()),
            "solves_per_s": len(fin) / span if span > 0 else float("inf"),
            "mean_wait_s": float(np.mean([q.start - q.arrival for q in fin])),
            "mean_iterations": float(np.mean([q.info.get("iterations", 0) for q in fin])),
            "max_rel_residual": float(max(q.info.get("rel_residual", 0.0) for q in fin)),
            # the same latencies over the solves that reached their tolerance
            "p50_converged_s": float(np.percentile(conv, 50)) if conv.size else None,
            "p99_converged_s": float(np.percentile(conv, 99)) if conv.size else None,
        }

    def free(self):
        for o in self.high + self.low:
            o.free()
