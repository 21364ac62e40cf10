"""The serving loop: requests that arrive together are batched and overlap on
the device; each result is the same as the request solved alone, and a sample
of them matches the oracle."""
import math

import numpy as np
import pytest

from paper_2511_00735_amd import workloads
from tests.gpu_cases import rel

pytestmark = pytest.mark.gpu


def _trace(seed=7):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(15):
        t = 0.05 * (i // 5)               # three bursts of five requests
        n = int(rng.choice([4, 8]))
        N = int(rng.choice([4, 6]))
        k = float(rng.uniform(6.0, 16.0))
        th = float(rng.uniform(0, 2 * math.pi))
        pr = workloads.Problem(n, N, k, k, workloads.draw_bumps(rng, int(rng.integers(1, 4))),
                               workloads.PlaneWave(k, k, (math.cos(th), math.sin(th))), levels=0,
                               coarse_iters=3, tol=1e-12)
        pr.name = f"s{i}"
        pr.arrival = t
        out.append(pr)
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_served_results_equal_alone(hps, ctx, precision):
    from paper_2511_00735_amd.serve import Server
    print(f"[serve] {precision}", flush=True)
    trace = _trace()
    srv = Server(precision=precision, workers=2, max_batch=8, tol=1e-12, coarse_iters=3,
                 memory_budget=8 << 30, keep_solutions=True)
    records, summary = srv.run(trace)
    assert summary["completed"] == len(trace) and summary["converged"] == len(trace), summary
    assert summary["mean_batch"] > 1.0, summary              # requests did share launches
    prec = hps.HPS_MIXED if precision == "mixed" else hps.HPS_FP64
    for pr in trace:
        desc = hps.make_desc(pr.n, pr.N, pr.kappa, levels=0, coarse_iters=3, precision=prec)
        prob = hps.Problem(ctx, desc)
        b, t = prob.coefficient_nodes(pr.b), prob.boundary_data(pr.wave.t)
        prob.build_leaves(b)
        prob.merge_all()
        g, info = prob.gmres_solve(prob.set_rhs(t), tol=1e-12, maxit=600)
        assert info["relres_true"] <= 1e-12
        assert rel(srv.solutions[pr.name].cpu().numpy(), g.cpu().numpy()) < 1e-10, pr.name
    # and a sample of the served results against the oracle's direct solution
    from tests.gpu_cases import oracle_case
    for pr in trace[:5]:
        oc = oracle_case(pr.n, pr.N, pr.kappa, pr.b, pr.wave.t)
        assert rel(srv.solutions[pr.name].cpu().numpy(), oc["g"]) < 1e-10, pr.name
