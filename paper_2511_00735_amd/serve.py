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
  workspace plus its input and output vectors) fits in a worker's arena (a
  fixed share of the memory budget, allocated once per worker); otherwise it
  shrinks;
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

    @staticmethod
    def shape(req):
        return (req.n, req.N)

    def add(self, req):
        self.pending.append(req)

    def take(self):
        """Next batch (list of requests and its footprint), or None when the
        oldest request cannot be admitted yet (or nothing is pending)."""
        if not self.pending:
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


class Server:
    """Runs a request trace through the library in real time.

    precision: "mixed" or "fp64"; workers: concurrent batches (streams);
    memory_budget: device bytes for all workers together.  Each worker holds
    one arena of memory_budget / workers bytes, allocated once when it starts;
    every batch it runs is carved out of that arena (the group workspace of
    the library's exact footprint, each request's coefficient, boundary data,
    right-hand side and solution, and the temporaries that evaluate the
    inputs), so serving makes no device allocation per batch and the caching
    allocator cannot fragment.  A batch never exceeds an arena; a request
    that alone exceeds it is refused when the run starts.  graphs: each worker
    replays its V-cycles from HIP graphs (several host threads launching at
    once)."""

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
        self.arena_bytes = (self.budget // max(1, self.workers)) & ~255
        self.tol = tol
        self.coarse_iters = coarse_iters
        self.restart = restart
        self.maxit = maxit
        self.keep = keep_solutions
        self.graphs = bool(graphs)
        self.solutions = {}
        self._coords = {}
        self._coord_lock = threading.Lock()

    # ---- shapes, footprints and the arena layout ---------------------------
    def desc(self, n, N, kappa=1.0):
        return self.hps.make_desc(n, N, kappa, levels=0, coarse_iters=self.coarse_iters, restart=self.restart,
                                  precision=self.prec)

    @staticmethod
    def _up(nbytes):
        return (int(nbytes) + 255) & ~255

    def layout(self, shape, count):
        """Byte offsets of a batch inside an arena: the group workspace, then
        per request b [E][(N+1)^2] (FP64) and the complex canonical vectors t,
        rhs, g, then three FP64 temporaries for evaluating the inputs.
        Returns (offsets dict, total bytes)."""
        n, N = shape
        E, p = n * n, N - 1
        nodes = 8 * E * (N + 1) ** 2
        vec = 16 * E * 4 * p
        off = {"ws": 0}
        cur = self._up(self.hps.group_workspace_bytes(self.desc(n, N), count))
        off["req"] = []
        for _ in range(count):
            r = {}
            for key, nb in (("b", nodes), ("t", vec), ("rhs", vec), ("g", vec)):
                r[key] = cur
                cur += self._up(nb)
            off["req"].append(r)
        for key in ("tmpa", "tmpb", "tmpc"):
            off[key] = cur
            cur += self._up(nodes)
        return off, cur

    def footprint(self, shape, count):
        return self.layout(shape, count)[1]

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

    # ---- synthetic inputs, evaluated on the device into arena views --------
    def _inputs_into(self, req, coords, b, t, tmpa, tmpb, tmpc):
        torch = self.torch
        x, y, sx, sy, nx, ny = coords
        b.zero_()
        bm = req.b
        for a, cx, cy, w in zip(bm.a, bm.cx, bm.cy, bm.w):
            torch.sub(x, float(cx), out=tmpa)
            tmpa.square_()
            torch.sub(y, float(cy), out=tmpb)
            tmpb.square_()
            tmpa.add_(tmpb).div_(-float(w)).exp_()
            b.add_(tmpa, alpha=float(a))
        # t = i (kappa d.n + eta) exp(i kappa d.x) at the slots
        wv = req.wave
        ns = sx.numel()
        ph, cf, tv = tmpa.view(-1)[:ns], tmpb.view(-1)[:ns], tmpc.view(-1)[:ns]
        torch.mul(sx, wv.kappa * wv.d[0], out=ph)
        ph.add_(sy, alpha=wv.kappa * wv.d[1])
        torch.mul(nx, wv.kappa * wv.d[0], out=cf)
        cf.add_(ny, alpha=wv.kappa * wv.d[1]).add_(wv.eta)
        tr = torch.view_as_real(t)
        torch.sin(ph, out=tv)
        tv.mul_(cf).neg_()
        tr[:, 0].copy_(tv)
        torch.cos(ph, out=tv)
        tv.mul_(cf)
        tr[:, 1].copy_(tv)

    def _views(self, arena, shape, count):
        """Typed views of one batch's buffers inside `arena` (uint8)."""
        torch = self.torch
        n, N = shape
        E, p = n * n, N - 1
        off, total = self.layout(shape, count)
        ws_bytes = self.hps.group_workspace_bytes(self.desc(n, N), count)
        nodes, ns = E * (N + 1) ** 2, E * 4 * p

        def f64(o, cnt):
            return arena[o:o + 8 * cnt].view(torch.float64)

        def c128(o, cnt):
            return arena[o:o + 16 * cnt].view(torch.complex128)

        reqs = [dict(b=f64(r["b"], nodes).view(E, (N + 1) ** 2), t=c128(r["t"], ns), rhs=c128(r["rhs"], ns),
                     g=c128(r["g"], ns)) for r in off["req"]]
        tmp = [f64(off[k], nodes).view(E, (N + 1) ** 2) for k in ("tmpa", "tmpb", "tmpc")]
        return arena[0:ws_bytes], reqs, tmp

    # ---- one batch on one worker's stream ---------------------------------
    def _run_batch(self, ctx, arena, batch, records):
        hps = self.hps
        n, N = batch[0].n, batch[0].N
        coords = self._node_data(n, N)
        t0 = time.perf_counter() - self._t0
        for r in batch:
            records[r.name].start = t0
            records[r.name].batch = len(batch)
        ws, bufs, (tmpa, tmpb, tmpc) = self._views(arena, (n, N), len(batch))
        group = hps.Group(ctx, self.desc(n, N, batch[0].kappa), [r.kappa for r in batch],
                          [r.eta for r in batch], workspace=ws)
        for r, v in zip(batch, bufs):
            self._inputs_into(r, coords, v["b"], v["t"], tmpa, tmpb, tmpc)
        group.build_leaves([v["b"] for v in bufs])
        group.merge_all()
        hps.set_rhs([group], [v["t"] for v in bufs], [v["rhs"] for v in bufs])
        infos = hps.gmres_solve([group], [v["rhs"] for v in bufs], [v["g"] for v in bufs],
                                self.tol, self.maxit)
        t1 = time.perf_counter() - self._t0
        for r, info, v in zip(batch, infos, bufs):
            rec = records[r.name]
            rec.finish = t1
            rec.iterations = info["iterations"]
            rec.relres = info["relres_true"]
            rec.status = info["status"]
            if self.keep:
                self.solutions[r.name] = v["g"].clone()
        del group

    def run(self, trace):
        """Serve `trace` (requests with .arrival in seconds, ascending);
        returns (records by name, summary dict)."""
        torch, hps = self.torch, self.hps
        for shape in sorted(set((r.n, r.N) for r in trace)):
            need = self.footprint(shape, 1)
            if need > self.arena_bytes:
                raise ValueError(f"a single {shape} request needs {need} bytes, more than a worker's "
                                 f"arena ({self.arena_bytes} bytes of the {self.budget}-byte budget)")
        planner = Planner(self.footprint, self.arena_bytes * self.workers, self.max_batch,
                          batch_budget=self.arena_bytes)
        records = {r.name: Record(r.name, r.n, r.N, r.arrival, dof=r.skeleton_dof) for r in trace}
        cond = threading.Condition()
        state = {"fed": 0, "done": False, "error": None}
        # cached blocks of earlier work go back to the device before the
        # arenas are taken
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        for shape in sorted(set((r.n, r.N) for r in trace)):
            self._node_data(*shape)
        arenas = [torch.empty(self.arena_bytes, dtype=torch.uint8, device="cuda") for _ in range(self.workers)]
        torch.cuda.synchronize()
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

        def worker(arena):
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
                    with torch.cuda.stream(stream):
                        self._run_batch(ctx, arena, batch, records)
                    with cond:
                        planner.release(need)
                        cond.notify_all()
            except BaseException as exc:  # surface the first failure to the caller
                with cond:
                    state["error"] = exc
                    cond.notify_all()

        threads = [threading.Thread(target=feeder, daemon=True)]
        threads += [threading.Thread(target=worker, args=(arenas[i],), daemon=True) for i in range(self.workers)]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        torch.cuda.synchronize()
        del arenas
        if state["error"] is not None:
            raise state["error"]
        summary = summarize(records.values())
        summary["arena_gib_per_worker"] = round(self.arena_bytes / 2 ** 30, 2)
        return records, summary


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
