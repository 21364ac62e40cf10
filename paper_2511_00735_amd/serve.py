"""Serving loop: continuous batching of Helmholtz solves on one GPU.

Requests (workloads.Problem with an arrival time) arrive over time.  A feeder
thread releases them at their arrival times; worker threads, each with its own
HIP stream and library context, repeatedly take the next batch and run it end
to end (leaf build, merges, right-hand side, preconditioned FGMRES) through
the library's group calls, so that every step of a batch runs in shared
launches.  Batching and admission are decided here, on the host:

* a batch holds requests of one shape (n, N): the oldest pending request fixes
  the shape, and younger requests of the same shape join it in arrival order,
  up to ``max_batch``;
* a batch is admitted only when its exact device footprint (the group
  workspace plus its input and output vectors) fits in what is left of the
  memory budget; otherwise it shrinks, and if even the oldest request alone
  does not fit, the worker waits until running batches release memory;
* requests that arrive while other batches run are admitted as workers and
  memory free up, so builds and solves of different batches overlap on the
  device (one stream per worker).

Latency of a request = completion - arrival.  The V-cycle inside each batch is
replayed from a captured HIP graph (the library's default).
"""
import threading
import time
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np


@dataclass
class Record:
    name: str
    n: int
    N: int
    arrival: float
    start: float = 0.0
    finish: float = 0.0
    batch: int = 0
    iterations: int = 0
    relres: float = float("nan")
    status: int = -1
    dof: int = 0

    @property
    def latency(self):
        return self.finish - self.arrival


class Planner:
    """Host-side batching and admission (no GPU): picks the next batch from the
    pending requests given the free memory.  ``footprint(shape, count)`` is the
    device bytes a batch of ``count`` requests of ``shape`` needs."""

    def __init__(self, footprint: Callable[[tuple, int], int], budget: int, max_batch: int = 32,
                 batch_budget: Optional[int] = None):
        self.footprint = footprint
        self.budget = int(budget)
        self.max_batch = int(max_batch)
        # bytes one batch may take (a lone request may exceed it while it
        # fits the free budget)
        self.batch_budget = int(batch_budget) if batch_budget is not None else self.budget
        self.pending: List = []     # (arrival order) requests waiting
        self.in_use = 0
        self.hold = False           # no admissions (a batch waits for the others to drain)

    @staticmethod
    def shape(req):
        return (req.n, req.N)

    def add(self, req):
        self.pending.append(req)

    def take(self):
        """Next batch (list of requests and its footprint), or None when the
        oldest request cannot be admitted yet (or nothing is pending)."""
        if not self.pending or self.hold:
            return None
        key = self.shape(self.pending[0])
        same = [r for r in self.pending if self.shape(r) == key][: self.max_batch]
        free = self.budget - self.in_use
        cap = min(free, self.batch_budget)
        count = len(same)
        while count > 0 and self.footprint(key, count) > cap:
            count -= 1
        if count == 0 and self.footprint(key, 1) <= free:
            count = 1
        if count == 0:
            if self.in_use == 0:
                raise ValueError(f"a single {key} request needs {self.footprint(key, 1)} bytes, "
                                 f"more than the memory budget {self.budget}")
            return None
        batch = same[:count]
        taken = set(id(r) for r in batch)
        self.pending = [r for r in self.pending if id(r) not in taken]
        need = self.footprint(key, count)
        self.in_use += need
        return batch, need

    def release(self, nbytes):
        self.in_use -= int(nbytes)

    def requeue(self, batch):
        """Puts the requests of a batch that could not run back among the
        pending ones, in arrival order."""
        self.pending = sorted(self.pending + list(batch), key=lambda r: r.arrival)


class Server:
    """Runs a request trace through the library in real time.

    precision: "mixed" or "fp64"; workers: concurrent batches (streams);
    memory_budget: device bytes the admitted batches may hold together, one
    batch at most memory_budget / workers (a lone request may take more);
    graphs: each worker replays its V-cycles from HIP graphs (several host
    threads launching at once).  A batch whose allocation fails (the caching
    allocator's free memory split by other batches) goes back to the pending
    requests; nothing is admitted until the running batches have finished and
    the cache has been released, then batching resumes."""

    def __init__(self, precision="mixed", workers=3, max_batch=32, memory_budget=200 << 30, tol=1e-8,
                 coarse_iters=5, restart=60, maxit=600, keep_solutions=False, graphs=True):
        import torch
        from . import hps
        self.torch = torch
        self.hps = hps
        self.prec = hps.HPS_MIXED if precision == "mixed" else hps.HPS_FP64
        self.precision = precision
        self.workers = int(workers)
        self.max_batch = int(max_batch)
        self.budget = int(memory_budget)
        self.tol = tol
        self.coarse_iters = coarse_iters
        self.restart = restart
        self.maxit = maxit
        self.keep = keep_solutions
        self.graphs = bool(graphs)
        self.solutions = {}
        self._coords = {}
        self._coord_lock = threading.Lock()

    # ---- shapes and footprints -------------------------------------------
    def desc(self, n, N, kappa=1.0):
        return self.hps.make_desc(n, N, kappa, levels=0, coarse_iters=self.coarse_iters, restart=self.restart,
                                  precision=self.prec)

    def footprint(self, shape, count):
        n, N = shape
        ws = self.hps.group_workspace_bytes(self.desc(n, N), count)
        E, p = n * n, N - 1
        vec = 16 * E * 4 * p                      # one canonical complex vector
        inputs = 8 * E * (N + 1) ** 2 + 3 * vec   # b at the nodes, t, rhs, g
        return ws + 256 + count * inputs

    def _node_data(self, n, N):
        """Device node and slot coordinates of a shape (cached)."""
        key = (n, N)
        with self._coord_lock:
            if key not in self._coords:
                torch = self.torch
                d = self.desc(n, N)
                x, y = self.hps.node_coords(d)
                sx, sy, nx, ny = self.hps.slot_coords(d)
                dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
                self._coords[key] = (dev(x), dev(y), dev(sx), dev(sy), dev(nx), dev(ny))
                torch.cuda.synchronize()
            return self._coords[key]

    # ---- synthetic inputs, evaluated on the device ------------------------
    def _inputs(self, req, coords):
        torch = self.torch
        x, y, sx, sy, nx, ny = coords
        b = torch.zeros_like(x)
        bm = req.b
        for a, cx, cy, w in zip(bm.a, bm.cx, bm.cy, bm.w):
            b += float(a) * torch.exp(-((x - float(cx)) ** 2 + (y - float(cy)) ** 2) / float(w))
        wv = req.wave
        u = torch.exp(1j * wv.kappa * (wv.d[0] * sx + wv.d[1] * sy))
        t = 1j * (wv.kappa * (wv.d[0] * nx + wv.d[1] * ny) + wv.eta) * u
        return b.contiguous(), t.to(torch.complex128).contiguous()

    # ---- one batch on one worker's stream ---------------------------------
    def _run_batch(self, ctx, batch, records):
        torch, hps = self.torch, self.hps
        n, N = batch[0].n, batch[0].N
        coords = self._node_data(n, N)
        t0 = time.perf_counter() - self._t0
        for r in batch:
            records[r.name].start = t0
            records[r.name].batch = len(batch)
        desc = self.desc(n, N, batch[0].kappa)
        group = hps.Group(ctx, desc, [r.kappa for r in batch], [r.eta for r in batch])
        ins = [self._inputs(r, coords) for r in batch]
        group.build_leaves([i[0] for i in ins])
        group.merge_all()
        rhs = group.set_rhs([i[1] for i in ins])
        gs, infos = group.gmres_solve(rhs, tol=self.tol, maxit=self.maxit)
        t1 = time.perf_counter() - self._t0
        for r, info, g in zip(batch, infos, gs):
            rec = records[r.name]
            rec.finish = t1
            rec.iterations = info["iterations"]
            rec.relres = info["relres_true"]
            rec.status = info["status"]
            if self.keep:
                self.solutions[r.name] = g.clone()
        del group, ins, rhs, gs

    def run(self, trace):
        """Serve `trace` (requests with .arrival in seconds, ascending);
        returns (records by name, summary dict)."""
        torch, hps = self.torch, self.hps
        planner = Planner(self.footprint, self.budget, self.max_batch,
                          batch_budget=self.budget // max(1, self.workers))
        records = {r.name: Record(r.name, r.n, r.N, r.arrival, dof=r.skeleton_dof) for r in trace}
        cond = threading.Condition()
        state = {"fed": 0, "done": False, "error": None}
        retried = set()   # ids of requests whose batch ran out of memory once
        # cached blocks of earlier work go back to the device: the workers'
        # new streams and their kernels' scratch are allocated by the runtime
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        for shape in sorted(set((r.n, r.N) for r in trace)):
            self._node_data(*shape)
        self._t0 = time.perf_counter()

        def feeder():
            i = 0
            while i < len(trace):
                wait = trace[i].arrival - (time.perf_counter() - self._t0)
                if wait > 0:
                    time.sleep(wait)
                    continue
                with cond:  # everything that has arrived by now, in one step
                    now = time.perf_counter() - self._t0
                    while i < len(trace) and trace[i].arrival <= now:
                        planner.add(trace[i])
                        i += 1
                    state["fed"] = i
                    cond.notify_all()
            with cond:
                state["done"] = True
                cond.notify_all()

        def worker():
            stream = torch.cuda.Stream()
            ctx = hps.Context(stream)
            ctx.set_graphs(self.graphs)
            try:
                while True:
                    with cond:
                        while True:
                            if state["error"] is not None:
                                return
                            got = planner.take()
                            if got is not None:
                                break
                            if state["done"] and not planner.pending:
                                return
                            cond.wait(timeout=0.05)
                    batch, need = got
                    oom = False
                    try:
                        with torch.cuda.stream(stream):
                            self._run_batch(ctx, batch, records)
                    except torch.OutOfMemoryError:
                        if any(id(r) in retried for r in batch):
                            raise
                        oom = True
                    if oom:
                        # the device memory is there but split across other
                        # batches' cached blocks: hand the batch back, admit
                        # nothing until the running batches have finished,
                        # release the cache; a batch that fails twice is an error
                        retried.update(id(r) for r in batch)
                        with cond:
                            planner.release(need)
                            planner.requeue(batch)
                            planner.hold = True
                            cond.notify_all()
                            while planner.in_use > 0 and state["error"] is None:
                                cond.wait(timeout=0.05)
                        torch.cuda.synchronize()
                        torch.cuda.empty_cache()
                        with cond:
                            planner.hold = False
                            cond.notify_all()
                        continue
                    with cond:
                        planner.release(need)
                        cond.notify_all()
            except BaseException as exc:  # surface the first failure to the caller
                with cond:
                    state["error"] = exc
                    cond.notify_all()

        threads = [threading.Thread(target=feeder, daemon=True)]
        threads += [threading.Thread(target=worker, daemon=True) for _ in range(self.workers)]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        torch.cuda.synchronize()
        if state["error"] is not None:
            raise state["error"]
        return records, summarize(records.values())


def summarize(records):
    recs = list(records)
    done = [r for r in recs if r.finish > 0]
    if not done:
        return {"requests": len(recs), "completed": 0}
    lat = np.array([r.latency for r in done])
    t_first = min(r.arrival for r in recs)
    makespan = max(r.finish for r in done) - t_first
    dof = sum(r.dof for r in done)
    batches = [r.batch for r in done]
    return {
        "requests": len(recs),
        "completed": len(done),
        "converged": int(sum(1 for r in done if r.status == 0)),
        "makespan_s": round(makespan, 3),
        "solves_per_s": round(len(done) / makespan, 2),
        "dof_per_s": round(dof / makespan, 1),
        "latency_p50_ms": round(1e3 * float(np.percentile(lat, 50)), 2),
        "latency_p99_ms": round(1e3 * float(np.percentile(lat, 99)), 2),
        "latency_max_ms": round(1e3 * float(lat.max()), 2),
        "mean_batch": round(float(np.mean(batches)), 2),
        "max_relres": float(max(r.relres for r in done)),
    }
