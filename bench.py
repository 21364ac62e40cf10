"""Benchmark: one step = the whole hot path on one problem.

Workload (default): 64x64 elements, GLL order 16, kappa = eta = 200, coefficient
b = sum of 8 seeded Gaussian bumps (seed 3), plane-wave impedance data,
coarse level L = 12 (the top interface), 5 coarse GMRES iterations, flexible
GMRES(60) to a relative residual of 1e-8.  One step = leaf ItI build + all 11
merge levels + right-hand side + preconditioned FGMRES solve.  The coefficient
and boundary data are on the device before the timed region starts.

Metric: skeleton DOF per second = 4 (N-1) n (n-1) / (build + solve time).
The headline run is the mixed-precision path; the plain FP64 path runs on the
same inputs beside it.

Roofline: the dominant kernel is the leaf kernel (one launch per up to 4096
elements: the whole 64x64 leaf level).  Its launches inside the timed steps are
bracketed by HIP events on the library's stream (library option
HPS_OPT_TIMING); achieved = the flops the kernel executes for the elements a
launch builds / the mean launch duration, against the FP64 peak.  The dense
complex LU count of the method as stated (the n_loc x n_loc element solve) is
reported beside it under its own key.  The HBM traffic per launch comes from
the rocprofv3 counter summary under profiles/ (FETCH_SIZE and WRITE_SIZE,
scaled by a plain copy kernel's readings), and is reported only while the leaf
kernel source and the elements per launch still match the ones measured; it is
set beside the algorithmic bytes (coefficient in, T and H out).

Accuracy: every GPU solution is compared (outside the timed region) with the
oracle's direct HPS solution of the same inputs, computed on the host; the
oracle's run is also the CPU baseline.

Prints ONE JSON line (see the repository documentation for the fields).
--traffic-probe instead runs one 1 GiB device copy (the counter calibration)
and one leaf build of the workload, for rocprofv3 --pmc runs.
"""
import hashlib
import argparse
import json
import math
import os
import sys
import time

# Blocks above 1 GiB are never split by PyTorch's caching allocator: a freed
# workspace stays whole, so it is reused or released in one piece when a later
# allocation (a larger serving batch) needs the memory.  Set before torch loads.
os.environ.setdefault("PYTORCH_ALLOC_CONF", "max_split_size_mb:1024")

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "skeleton DOF/s to rel.res 1e-8, mixed vs FP64; served solves/s + p99 latency"
UNIT = "skeleton DOF/s"
MI355X_HBM_GBS = 8000.0
MI355X_FP64_TFLOPS = 78.6   # FP64 vector FMA: 256 CU x 4 SIMD x 16 lanes x 2 flops x 2.4 GHz
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "leaf_kernel_64x64_N16_traffic.md")
LEAF_SOURCE = os.path.join(ROOT, "paper_2511_00735_amd", "csrc", "leaf.hip")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=64)
    ap.add_argument("--order", type=int, default=16)
    ap.add_argument("--kappa", type=float, default=200.0)
    ap.add_argument("--levels", type=int, default=12)
    ap.add_argument("--coarse-iters", type=int, default=5)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--precision", choices=["mixed", "fp64"], default="mixed")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the plain FP64 run of the same workload")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="one 1 GiB device copy, then one leaf build (for rocprofv3 --pmc runs)")
    ap.add_argument("--solve-probe", action="store_true",
                    help="one 1 GiB device copy, then a built workload and 4 V-cycles and 4 M_1 "
                         "products (for rocprofv3 --pmc runs)")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of the request trace served beside the headline (0: skip)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-problem batch")
    ap.add_argument("--no-sweep", action="store_true", help="skip the Table 1 sweep on the paper's workload")
    return ap.parse_args()


def leaf_flops_algorithmic(N):
    """Flops of the leaf ItI map of one element as the method states it: dense
    LU of the n_loc x n_loc complex element matrix, the solves for the 4(N-1)
    boundary columns and the load column, and the product with the outgoing
    impedance operator (8 real flops per complex multiply-add)."""
    nloc = (N + 1) ** 2 - 4
    return 8.0 / 3.0 * nloc ** 3 + 32.0 * (N - 1) * nloc ** 2 + 128.0 * (N - 1) ** 2 * (N + 2)


def leaf_bytes_algorithmic(N):
    """HBM bytes a leaf build must move per element: the coefficient at the
    (N+1)^2 nodes in (FP64), the 4(N-1) x 4(N-1) complex FP64 map T and the
    complex load H out."""
    m = 4 * (N - 1)
    return 8 * (N + 1) ** 2 + 16 * m * m + 16 * m


def progress(msg):
    """Progress line on stderr (stdout carries the one JSON result line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def leaf_traffic_record():
    """(bytes per launch, source hash, elements per launch) from the committed
    counter summary, or None."""
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    rec = {}
    for ln in lines:
        if ln.startswith("- ") and ": " in ln:
            k, v = ln[2:].split(": ", 1)
            rec[k.strip()] = v.strip().strip("`")
    try:
        return (float(rec["traffic_bytes_per_launch"]), rec["leaf_source_sha256"],
                float(rec["elements_per_launch"]))
    except KeyError:
        return None


def leaf_flops_executed(N):
    """Real flops of the leaf kernel per element: partial LU of the bordered
    real matrix over p^2 pivots, then complex Gauss-Jordan of R + i eta I."""
    p = N - 1
    nloc = p * p + 4 * p
    ncol = nloc + 2
    f = 0
    for k in range(p * p):
        r, c = nloc - k - 1, ncol - k - 1
        f += r + 2 * r * c            # scale column + rank-1 update
    m = 4 * p
    f += 8 * m ** 3                   # complex Gauss-Jordan inverse (m^3 complex MACs)
    return f


def merge_flops_executed(n, N, L):
    """Complex-counted (8 flops / MAC) flops of all merges 1..L-1."""
    p = N - 1
    tot = 0
    per_level = []
    for level in range(1, L):
        wx, wy = 2 ** (level // 2), 2 ** ((level - 1) // 2)
        b = 2 * (wx + wy) * p
        m = (wy if level % 2 else wx) * p
        e = b - m
        pairs = (n // wx) * (n // wy) // 2
        macs = m ** 3 + m ** 3 + m * m * e + 2 * m * m * e + 2 * m * m * e + 4 * m * e * e
        per_level.append(8 * macs * pairs)
        tot += 8 * macs * pairs
    return tot, per_level


def oracle_job(pr):
    """The oracle's whole job on the host at all of its cores (NumPy/LAPACK's
    default threading): leaf maps of every element, the merge hierarchy and the
    direct HPS solve with the exact top-level solve (build + solve).  Returns
    (g, seconds, phase seconds); g is the reference the GPU solutions are
    compared with (outside any timed region)."""
    from oracle import gll, leaf, merge, mesh, direct
    n, N, p = pr.n, pr.N, pr.N - 1
    t0 = time.perf_counter()
    xi = gll.gll_nodes(N)
    c = leaf.nodal_coefficient(N, n, pr.kappa, pr.b, xi)
    T, H = leaf.leaves(N, 1.0 / n, pr.kappa, pr.eta, c)
    t1 = time.perf_counter()
    hier = merge.build_hierarchy(n, p, T, H, top=mesh.lmax(n))
    t2 = time.perf_counter()
    xs, ys, nx, ny = mesh.canonical_slot_coords(n, N, xi)
    g = direct.solve(n, p, T, H, pr.wave.t(xs, ys, nx, ny), hierarchy=hier)
    t3 = time.perf_counter()
    return g, t3 - t0, {"leaves": t1 - t0, "merges": t2 - t1, "downward_solve": t3 - t2}


def oracle_thread_ratio(pr, levels=9):
    """Time of the oracle at 1 thread over its time at all cores, on a bounded
    sample of the same workload: the leaf maps of 64 elements and one pair
    merge at each of levels 1..`levels`."""
    from threadpoolctl import threadpool_limits
    from oracle import gll, leaf, merge
    n, N, p = pr.n, pr.N, pr.N - 1
    xi = gll.gll_nodes(N)
    c = leaf.nodal_coefficient(N, n, pr.kappa, pr.b, xi)[:64]

    def sample():
        t0 = time.perf_counter()
        T, _ = leaf.leaves(N, 1.0 / n, pr.kappa, pr.eta, c)
        cur = [T[0], T[1]]
        for level in range(1, levels + 1):
            Tm, _, _ = merge.merge_pair(level, p, cur[0], cur[1])
            cur = [Tm, Tm]
        return time.perf_counter() - t0

    t_all = min(sample() for _ in range(2))
    with threadpool_limits(1):
        t_one = min(sample() for _ in range(2))
    return t_one / t_all, t_one, t_all


def cpu_baseline(pr):
    """cpu_baseline: the oracle's whole job timed once at all host cores (its
    solution is the reference of err_vs_oracle), and the same job at one
    thread estimated with the 1-thread / all-core time ratio of a sample."""
    g, secs, parts = oracle_job(pr)
    ratio, t_one, t_all = oracle_thread_ratio(pr)
    cores = len(os.sched_getaffinity(0))
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    out = {
        "value": round(pr.skeleton_dof / secs, 1),
        "unit": UNIT,
        "cores": min(cores, threads),
        "kind": "oracle",
        "sample": (f"the whole job once (not a sample): oracle leaf maps of all {pr.n * pr.n} elements, "
                   f"merge hierarchy and direct HPS solve with the exact top solve, FP64, "
                   f"{secs:.1f} s at {min(cores, threads)} threads "
                   f"(leaves {parts['leaves']:.1f} s, merges {parts['merges']:.1f} s, "
                   f"downward solve {parts['downward_solve']:.1f} s)"),
        "one_thread": {
            "value": round(pr.skeleton_dof / (secs * ratio), 1),
            "estimate": (f"whole-job time x {ratio:.2f}, the 1-thread / all-core time ratio of a sample "
                         f"(leaf maps of 64 elements and one pair merge at levels 1-9: "
                         f"{t_one:.2f} s vs {t_all:.2f} s, best of 2)"),
        },
    }
    return out, g


def run_precision(args, pr, precision, hps, torch):
    """Build + solve the workload `steps` times (after `warmup` untimed steps)
    in one precision; returns timings, the mean per-phase event times of the
    timed steps and the solution."""
    ctx = hps.Context()
    stream = ctx.stream
    prec = hps.HPS_MIXED if precision == "mixed" else hps.HPS_FP64
    desc = hps.make_desc(pr.n, pr.N, pr.kappa, pr.eta, levels=pr.levels,
                         coarse_iters=pr.coarse_iters, precision=prec)
    prob = hps.Problem(ctx, desc)
    b_nodes = prob.coefficient_nodes(pr.b)
    t_data = prob.boundary_data(pr.wave.t)
    rhs = torch.empty(prob.nslots, dtype=torch.complex128, device="cuda")
    g = torch.empty_like(rhs)

    def step(ev=None):
        # ev: four events recorded on the library's stream around the phases
        if ev is not None:
            ev[0].record(stream)
        prob.build_leaves(b_nodes)
        if ev is not None:
            ev[1].record(stream)
        prob.merge_all()
        if ev is not None:
            ev[2].record(stream)
        hps.set_rhs([prob], [t_data], [rhs])
        info = prob.gmres_solve(rhs, tol=pr.tol, maxit=600, out=g)[1]
        if ev is not None:
            ev[3].record(stream)
        return info

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    ctx.set_timing(True)
    t0 = time.perf_counter()
    infos = [step(evs[i]) for i in range(args.steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    leaf_launches, leaf_ms, leaf_units = ctx.kernel_time(hps.HPS_KERNEL_LEAF)
    ctx.set_timing(False)
    phases = np.array([[e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2]), e[2].elapsed_time(e[3])]
                       for e in evs])
    return {
        "ms": 1e3 * dt / args.steps,
        "value": pr.skeleton_dof * args.steps / dt,
        "info": infos[-1],
        "iterations_per_step": [i["iterations"] for i in infos],
        "phase_ms": list(phases.mean(axis=0)),
        "g": g.clone(),
        "leaf": (leaf_launches, leaf_ms, leaf_units),
    }


def run_batch_c4(hps, torch):
    """The 256 seeded problems of mixed shapes as one batch (all arriving at
    t = 0): grouped by shape through the serving loop, against the same
    problems solved one at a time (after one untimed batched pass)."""
    from paper_2511_00735_amd import workloads
    from paper_2511_00735_amd.serve import Server
    probs = workloads.c4(256, seed=4)
    out = {"problems": len(probs), "shapes": len(set((p.n, p.N) for p in probs)),
           "skeleton_dof": int(sum(p.skeleton_dof for p in probs))}
    # one untimed pass first (first-call set-up of every group shape)
    Server(precision="mixed", memory_budget=200 << 30, workers=3, max_batch=64).run(probs)
    for label, kw in (("batched", dict(workers=3, max_batch=64)), ("one_by_one", dict(workers=1, max_batch=1))):
        srv = Server(precision="mixed", memory_budget=200 << 30, **kw)
        _, summ = srv.run(probs)
        out[label] = {k: summ[k] for k in ("makespan_s", "solves_per_s", "dof_per_s", "mean_batch",
                                           "converged", "max_relres")}
    out["batched_over_one_by_one"] = round(out["batched"]["dof_per_s"] / out["one_by_one"]["dof_per_s"], 3)
    return out


def run_table1_sweep(hps, torch, precision="fp64"):
    """The paper's Table 1 on its own experiment (X1: Gaussian bump, scattering
    source, t = 0, 64x64, N = 16, kappa = 670): every (#levels L, gamma,
    coarse iterations k) cell of the table -- gamma = 1 with k in {4, 5, 6}
    for L = 2..12, gamma = 2 with k in {2, 3, 4} for L = 2..7 -- plus the
    exact coarse space (direct HPS), each built and solved once to a relative
    residual of 1e-8 (FGMRES(60), x0 = 0).  Per cell: PMem = the problem's
    device workspace in MB (the library's exact footprint), It, Bt = leaf
    build + merges, St = right-hand side + solve (device times from the
    library's events).  One workspace, sized for the largest cell, serves
    every cell."""
    from paper_2511_00735_amd import workloads
    pr = workloads.x1(64)
    prec = hps.HPS_MIXED if precision == "mixed" else hps.HPS_FP64
    cells = [(L, 1, k) for L in range(2, 13) for k in (4, 5, 6)]
    cells += [(L, 2, k) for L in range(2, 8) for k in (2, 3, 4)]
    cells += [(12, 1, -1)]
    descs = {c: hps.make_desc(pr.n, pr.N, pr.kappa, pr.eta, levels=c[0], coarse_iters=c[2], gamma=c[1],
                              precision=prec) for c in cells}
    nbytes = max(hps.workspace_bytes(d) for d in descs.values())
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    ctx = hps.Context()
    rows = []
    b_nodes = s_nodes = t_data = None
    for c in cells:
        d = descs[c]
        prob = hps.Problem(ctx, d, workspace=ws)
        if b_nodes is None:
            b_nodes, s_nodes = prob.coefficient_nodes(pr.b), prob.source_nodes(pr.s)
            t_data = prob.boundary_data(pr.wave.t)
        prob.build_leaves(b_nodes, s_nodes)
        prob.merge_all()
        rhs = prob.set_rhs(t_data)
        _, info = prob.gmres_solve(rhs, tol=1e-8, maxit=600)
        L, gamma, k = c
        rows.append({"levels": L, "gamma": gamma, "coarse_iters": "exact" if k < 0 else k,
                     "pmem_mb": round(hps.workspace_bytes(d) / 1e6, 1), "iterations": info["iterations"],
                     "build_ms": round(1e3 * info["t_build_s"], 2), "solve_ms": round(1e3 * info["t_solve_s"], 2),
                     "relres": info["relres_true"], "converged": info["status"] == 0})
        del prob
    best = min((r for r in rows if r["converged"]), key=lambda r: r["build_ms"] + r["solve_ms"])
    return {"workload": (f"the paper's experiment: 64x64 elements, N=16, kappa=eta={pr.kappa:.1f} (9.6 points per "
                         "wavelength), b = 1.5 exp(-160 r^2), s = -kappa^2 b exp(i kappa x), t = 0, "
                         f"FGMRES(60) to 1e-8, {precision}"),
            "columns": "levels, gamma, coarse_iters, pmem_mb, iterations, build_ms, solve_ms, relres",
            "rows": [[r["levels"], r["gamma"], r["coarse_iters"], r["pmem_mb"], r["iterations"], r["build_ms"],
                      r["solve_ms"], r["relres"]] for r in rows],
            "best": {**best, "dof_per_s": round(pr.skeleton_dof / (1e-3 * (best["build_ms"] + best["solve_ms"])), 1)}}


def run_repeated_solves(hps, torch, pr, precision="mixed", nrhs=16):
    """Many solves with one built operator (the paper notes that the best
    setting depends on how many solves share a build): the workload's
    operator is built once, then `nrhs` right-hand sides (plane waves of
    different directions) are solved to 1e-8.  Reports the build time, the
    mean solve time and the skeleton DOF/s amortised over all solves."""
    ctx = hps.Context()
    prec = hps.HPS_MIXED if precision == "mixed" else hps.HPS_FP64
    desc = hps.make_desc(pr.n, pr.N, pr.kappa, pr.eta, levels=pr.levels, coarse_iters=pr.coarse_iters,
                         precision=prec)
    prob = hps.Problem(ctx, desc)
    b_nodes = prob.coefficient_nodes(pr.b)
    ts = [prob.boundary_data(workloads_plane(pr, 2 * math.pi * k / nrhs).t) for k in range(nrhs)]
    rhs = torch.empty(prob.nslots, dtype=torch.complex128, device="cuda")
    g = torch.empty_like(rhs)
    for _ in range(2):        # warm-up of both phases
        prob.build_leaves(b_nodes)
        prob.merge_all()
        hps.set_rhs([prob], [ts[0]], [rhs])
        prob.gmres_solve(rhs, tol=pr.tol, maxit=600, out=g)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    prob.build_leaves(b_nodes)
    prob.merge_all()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    its = []
    for t in ts:
        hps.set_rhs([prob], [t], [rhs])
        its.append(prob.gmres_solve(rhs, tol=pr.tol, maxit=600, out=g)[1]["iterations"])
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    build, solve = t1 - t0, (t2 - t1) / nrhs
    return {"precision": precision, "solves": nrhs, "build_ms": round(1e3 * build, 3),
            "mean_solve_ms": round(1e3 * solve, 3), "iterations": its,
            "amortised_dof_per_s": round(pr.skeleton_dof * nrhs / (t2 - t0), 1),
            "single_solve_dof_per_s": round(pr.skeleton_dof / (build + solve), 1)}


def run_rectangles(hps, torch, pr, precision="mixed", steps=3):
    """The workload's 4096 elements, N and kappa on rectangular meshes
    (128 x 32 and 32 x 128 elements of side 1/128, all 12 merge levels, the
    same coarse solve and tolerance): build + solve per step, DOF/s and
    iterations, beside the square 64 x 64 mesh of the headline."""
    out = {}
    prec = hps.HPS_MIXED if precision == "mixed" else hps.HPS_FP64
    for nx, ny in ((128, 32), (32, 128)):
        ctx = hps.Context()
        desc = hps.make_desc(nx, pr.N, pr.kappa, pr.eta, coarse_iters=pr.coarse_iters, precision=prec, ny=ny)
        prob = hps.Problem(ctx, desc)
        b_nodes = prob.coefficient_nodes(pr.b)
        t = prob.boundary_data(pr.wave.t)
        rhs = torch.empty(prob.nslots, dtype=torch.complex128, device="cuda")
        g = torch.empty_like(rhs)
        dof = 4 * (pr.N - 1) * nx * ny - 2 * (pr.N - 1) * (nx + ny)

        def step():
            prob.build_leaves(b_nodes)
            prob.merge_all()
            hps.set_rhs([prob], [t], [rhs])
            return prob.gmres_solve(rhs, tol=pr.tol, maxit=600, out=g)[1]

        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            info = step()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / steps * 1e3
        out[f"{nx}x{ny}"] = {"skeleton_dof": dof, "ms_per_step": round(ms, 3),
                             "dof_per_s": round(dof / ms * 1e3, 1), "iterations": info["iterations"],
                             "relres_true": info["relres_true"]}
        del prob, ctx
    return {"precision": precision, "levels": 12, "meshes": out}


def workloads_plane(pr, theta):
    from paper_2511_00735_amd import workloads
    return workloads.PlaneWave(pr.kappa, pr.eta, (math.cos(theta), math.sin(theta)))


def run_serving(hps, torch, seconds):
    """The first `seconds` of the seeded Poisson request trace (50 req/s, 10%
    128x128 N=16 kappa=400), served in real time, mixed vs FP64."""
    from paper_2511_00735_amd import workloads
    from paper_2511_00735_amd.serve import Server
    trace = workloads.c5(duration=seconds)
    out = {"trace": (f"{seconds:g} s of the seeded Poisson trace (50 req/s): {len(trace)} requests, "
                     f"{sum(1 for r in trace if r.n == 128)} at 128x128 N=16 kappa=400"),
           "workers": 3, "memory_budget_gib": 200}
    for prec in ("mixed", "fp64"):
        progress(f"serving {len(trace)} requests over {seconds:g} s, {prec}")
        srv = Server(precision=prec, workers=3, max_batch=32, memory_budget=200 << 30)
        _, summ = srv.run(trace)
        out[prec] = summ
        progress(f"serving {prec}: {summ.get('solves_per_s')} solves/s, p99 {summ.get('latency_p99_ms')} ms")
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2511_00735_amd import hps, workloads
    # the caching allocator stays under 90% of the device, so that the HIP
    # runtime's own allocations (queues, kernel scratch) always find memory
    torch.cuda.set_per_process_memory_fraction(0.9)

    pr = workloads.c3()
    pr.n, pr.N, pr.kappa, pr.eta = args.n, args.order, args.kappa, args.kappa
    pr.levels, pr.coarse_iters, pr.tol = args.levels, args.coarse_iters, args.tol
    pr.wave = workloads.PlaneWave(pr.kappa, pr.eta)
    dof = pr.skeleton_dof

    if args.solve_probe:
        nbytes = 1 << 30
        a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        ctx = hps.Context()
        prec = hps.HPS_MIXED if args.precision == "mixed" else hps.HPS_FP64
        prob = hps.Problem(ctx, hps.make_desc(pr.n, pr.N, pr.kappa, pr.eta, levels=pr.levels,
                                              coarse_iters=pr.coarse_iters, precision=prec))
        prob.build_leaves(prob.coefficient_nodes(pr.b))
        prob.merge_all()
        rhs = prob.set_rhs(prob.boundary_data(pr.wave.t))
        z = torch.empty_like(rhs)
        w = torch.empty_like(rhs)
        ctx.sync()
        for _ in range(4):
            prob.precond_apply(rhs, out=z)
        for _ in range(4):
            prob.skeleton_apply(z, out=w)
        ctx.sync()
        print(json.dumps({"probe": "solve", "copy_bytes_read": nbytes, "copy_bytes_written": nbytes,
                          "vcycles": 4, "m1_products": 4}), flush=True)
        return

    if args.traffic_probe:
        nbytes = 1 << 30
        a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        ctx = hps.Context()
        prec = hps.HPS_MIXED if args.precision == "mixed" else hps.HPS_FP64
        prob = hps.Problem(ctx, hps.make_desc(pr.n, pr.N, pr.kappa, pr.eta, levels=pr.levels,
                                              coarse_iters=pr.coarse_iters, precision=prec))
        b_nodes = prob.coefficient_nodes(pr.b)
        torch.cuda.synchronize()
        prob.build_leaves(b_nodes)
        ctx.sync()
        print(json.dumps({"probe": "traffic", "copy_bytes_read": nbytes, "copy_bytes_written": nbytes,
                          "leaf_elements": pr.n * pr.n}), flush=True)
        return

    main_run = run_precision(args, pr, args.precision, hps, torch)
    ref = None
    if args.precision == "mixed" and not args.no_compare:
        ref = run_precision(args, pr, "fp64", hps, torch)
    t_leaf, t_merge, t_solve = main_run["phase_ms"]
    leaf_f = leaf_flops_executed(pr.N) * pr.n * pr.n
    merge_f, _ = merge_flops_executed(pr.n, pr.N, pr.levels)
    leaf_tf = leaf_f / (t_leaf * 1e-3) / 1e12
    merge_tf = merge_f / (t_merge * 1e-3) / 1e12
    # dominant kernel: the leaf kernel, timed per launch with HIP events
    nl, lms, lunits = main_run["leaf"]
    per_launch_ms = lms / max(nl, 1)
    per_launch_units = lunits / max(nl, 1)
    per_launch_s = per_launch_ms * 1e-3
    executed = leaf_flops_executed(pr.N) * per_launch_units
    dense = leaf_flops_algorithmic(pr.N) * per_launch_units
    ach = executed / per_launch_s / 1e12
    alg_bytes = leaf_bytes_algorithmic(pr.N) * per_launch_units
    traffic = None
    rec = leaf_traffic_record()
    if rec is not None:
        src_hash = hashlib.sha256(open(LEAF_SOURCE, "rb").read()).hexdigest()
        if src_hash == rec[1] and per_launch_units == rec[2]:
            traffic = rec[0]
    roof = {"bound": "alu", "achieved": round(ach, 3), "peak": MI355X_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": round(ach / MI355X_FP64_TFLOPS, 4), "traffic": traffic,
            "kernel": "leaf_kernel (hps_build_leaves; FP64)",
            "launches": nl, "units_per_launch": per_launch_units, "avg_launch_ms": round(per_launch_ms, 4),
            "executed_flops_per_launch": executed,
            "algorithmic_bytes_per_launch": alg_bytes,
            "traffic_over_algorithmic_bytes": None if traffic is None else round(traffic / alg_bytes, 1),
            "hbm_gbs": None if traffic is None else round(traffic / per_launch_s / 1e9, 1),
            "hbm_frac": None if traffic is None else round(traffic / per_launch_s / 1e9 / MI355X_HBM_GBS, 4),
            "dense_lu_equivalent": {"flops_per_launch": dense, "tflops": round(dense / per_launch_s / 1e12, 3)}}
    info = main_run["info"]
    cfg = {"workload": (f"{pr.n}x{pr.n} elements, N={pr.N}, kappa=eta={pr.kappa:g}, "
                        f"8 seeded bumps (seed 3), plane-wave t, L={pr.levels}, "
                        f"{pr.coarse_iters} coarse GMRES its, FGMRES(60) to {pr.tol:g}"),
           "precision": args.precision, "skeleton_dof": dof,
           "iterations": info["iterations"], "relres_true": info["relres_true"],
           "phase_ms": {"leaves": round(t_leaf, 3), "merges": round(t_merge, 3),
                        "rhs+solve": round(t_solve, 3),
                        "note": f"mean over the {args.steps} timed steps (HIP events on the library's stream)"},
           "phase_tflops": {"leaves": round(leaf_tf, 3), "merges": round(merge_tf, 3)}}
    if ref is not None:
        gm, gf = main_run["g"], ref["g"]
        cfg["fp64_same_gpu"] = {
            "value": round(ref["value"], 1), "ms_per_step": round(ref["ms"], 3),
            "iterations": ref["info"]["iterations"], "relres_true": ref["info"]["relres_true"],
            "phase_ms": {"leaves": round(ref["phase_ms"][0], 3), "merges": round(ref["phase_ms"][1], 3),
                         "rhs+solve": round(ref["phase_ms"][2], 3)}}
        cfg["mixed_over_fp64"] = round(main_run["value"] / ref["value"], 3)
        cfg["rel_diff_mixed_vs_fp64_solution"] = float(torch.linalg.norm(gm - gf) / torch.linalg.norm(gf))
    out = {
        "metric": METRIC, "value": round(main_run["value"], 1), "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(main_run["ms"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64+c128" if args.precision == "mixed" else "c128",
        "data": "synthetic", "config": cfg, "roofline": roof,
    }
    progress("headline done: %.1f DOF/s" % main_run["value"])
    if not args.no_sweep:
        cfg["table1_sweep"] = run_table1_sweep(hps, torch)
        progress("Table 1 sweep done")
        cfg["repeated_solves"] = {"mixed": run_repeated_solves(hps, torch, pr, "mixed"),
                                  "fp64": run_repeated_solves(hps, torch, pr, "fp64")}
        progress("repeated solves done")
        cfg["rectangular_meshes"] = run_rectangles(hps, torch, pr)
        progress("rectangular meshes done")
    if not args.no_batch:
        cfg["batch_256_problems"] = run_batch_c4(hps, torch)
        progress("256-problem batch done")
    if args.serve_seconds > 0:
        cfg["serving"] = run_serving(hps, torch, args.serve_seconds)
    if not args.no_cpu_baseline:
        progress("oracle on the host (whole job, then a 1-thread sample)")
        out["cpu_baseline"], g_ref = cpu_baseline(pr)
        g_ref = torch.from_numpy(g_ref)
        err = {args.precision: float(torch.linalg.norm(main_run["g"].cpu() - g_ref) / torch.linalg.norm(g_ref))}
        if ref is not None:
            err["fp64"] = float(torch.linalg.norm(ref["g"].cpu() - g_ref) / torch.linalg.norm(g_ref))
        err["reference"] = ("the oracle's direct HPS solution (exact discrete skeleton solution, FP64, host); "
                            f"GPU solutions stop at relative residual {pr.tol:g}")
        cfg["err_vs_oracle"] = err
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
