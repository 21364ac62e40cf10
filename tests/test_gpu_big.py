"""The 128x128-element class of the serving trace (N = 16, kappa = 400, 16384
elements, 975,360 skeleton unknowns, 14 merge levels), the largest problem the
benchmarks run.  The oracle cannot solve it in a test's time, so the parity is
sampled and the rest is checked through properties that hold at any size:

* 48 leaf ItI maps (corners, edges and seeded interior elements) against the
  oracle's leaf maps of the same elements: per map <= 1e-11 relative, per
  entry <= 1e-11 max|T|;
* the FP64 and mixed solves converge to their tolerance (true residual with
  the FP64 operator M_1 built from those leaf maps);
* the two solutions agree within what their tolerances allow.
"""
import numpy as np
import pytest

from tests.gpu_cases import rel
from paper_2511_00735_amd import workloads

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]


def _big_request():
    return next(pr for pr in workloads.c5(duration=60.0) if pr.n == 128)


def test_big_sampled_leaf_maps_and_solves(hps, ctx):
    import torch
    from oracle import gll, leaf
    pr = _big_request()
    n, N = pr.n, pr.N
    print(f"[big] {pr.name}: {n}x{n}, N={N}, kappa={pr.kappa:g}", flush=True)
    rng = np.random.default_rng(12)
    sel = sorted({0, n - 1, n * (n - 1), n * n - 1, n // 2, n * (n // 2)}
                 | set(int(e) for e in rng.choice(n * n, 42, replace=False)))
    xi = gll.gll_nodes(N)
    c = leaf.nodal_coefficient(N, n, pr.kappa, pr.b, xi)[sel]
    To, _ = leaf.leaves(N, 1.0 / n, pr.kappa, pr.eta, c)
    sols = {}
    for precision, tol in (("fp64", 1e-10), ("mixed", 1e-8)):
        prec = hps.HPS_MIXED if precision == "mixed" else hps.HPS_FP64
        prob = hps.Problem(ctx, hps.make_desc(n, N, pr.kappa, pr.eta, coarse_iters=pr.coarse_iters,
                                              precision=prec))
        prob.build_leaves(prob.coefficient_nodes(pr.b))
        if precision == "fp64":
            T1 = prob.level_T(1)
            where = {hps.tree_box_xy(1, j, n, n): j for j in range(n * n)}   # element -> map slot
            pos = torch.tensor([where[(e % n, e // n)] for e in sel], device=T1.device)
            Tg = T1[pos].cpu().numpy()
            scale = np.abs(To).max()
            for i, e in enumerate(sel):
                assert rel(Tg[i], To[i]) <= 1e-11, (e, rel(Tg[i], To[i]))
                assert np.abs(Tg[i] - To[i]).max() <= 1e-11 * scale, e
        prob.merge_all()
        rhs = prob.set_rhs(prob.boundary_data(pr.wave.t))
        g, info = prob.gmres_solve(rhs, tol=tol, maxit=600)
        print(f"[big] {precision}: {info['iterations']} iterations, relres {info['relres_true']:.2e}",
              flush=True)
        assert info["status"] == 0 and info["relres_true"] <= tol, info
        sols[precision] = g.cpu().numpy()
        del prob
    assert rel(sols["mixed"], sols["fp64"]) <= 1e-6
