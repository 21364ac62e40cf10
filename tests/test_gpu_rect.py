"""Rectangular meshes of nx x ny elements (powers of two) through the C ABI,
against the oracle on the same mesh: leaf maps and RHS (tree-order placement),
every merged box map, the V-cycle, and FGMRES solutions (FP64 and mixed), on
wide and tall meshes whose merges end with runs along one direction, including
level-1 pair counts that take the two-workgroups-per-pair kernels."""
import numpy as np
import pytest

from paper_2511_00735_amd import workloads
from tests.gpu_cases import oracle_case, gpu_problem, rel, box_maps_by_xy, oracle_hierarchy

pytestmark = pytest.mark.gpu


def _bump(x, y):
    return 0.6 * np.exp(-((x - 0.4) ** 2 + (y - 0.2) ** 2) / 0.05) - 0.3 * np.sin(3 * x * y)


def _src(x, y):
    return np.exp(1j * (2 * x - y)) * (1 + x * y)


@pytest.mark.parametrize("n,N", [((8, 2), 5), ((2, 8), 6), ((16, 1), 4)])
def test_rect_leaf_maps_rhs_and_matvec(hps, ctx, n, N):
    import torch
    from oracle import mesh, skeleton
    print(f"[rect leaf] {n} N={N}", flush=True)
    kappa = 11.0
    wave = workloads.PlaneWave(kappa, kappa, (0.6, 0.8))
    oc = oracle_case(n, N, kappa, _bump, wave.t, _src, with_direct=False)
    prob = gpu_problem(hps, ctx, n, N, kappa, _bump, _src, merge=False)
    nx, ny = n
    assert (prob.nx, prob.ny, prob.E, prob.lmax) == (nx, ny, nx * ny, mesh.lmax(n))
    Tg = box_maps_by_xy(hps, prob, 1)
    for e in range(nx * ny):
        assert rel(Tg[(e % nx, e // nx)], oc["T"][e]) < 1e-11, e
    rhs = prob.set_rhs(prob.boundary_data(wave.t)).cpu().numpy()
    assert rel(rhs, oc["rhs"]) < 1e-11
    rng = np.random.default_rng(1)
    g = rng.standard_normal(prob.nslots) + 1j * rng.standard_normal(prob.nslots)
    g[mesh.physical_slot_mask(n, N - 1)] = 0
    out = prob.skeleton_apply(torch.from_numpy(g).cuda()).cpu().numpy()
    ref = skeleton.apply(n, N - 1, 1, skeleton.leaf_boxT(n, oc["T"]), g)
    assert rel(out, ref) < 1e-12


@pytest.mark.parametrize("n,N", [((8, 2), 5), ((2, 8), 5), ((16, 4), 6), ((4, 32), 4)])
def test_rect_merge_levels(hps, ctx, n, N):
    from oracle import mesh
    print(f"[rect merge] {n} N={N}", flush=True)
    kappa = 14.0
    wave = workloads.PlaneWave(kappa, kappa)
    oc = oracle_case(n, N, kappa, _bump, wave.t, None, with_direct=False)
    prob = gpu_problem(hps, ctx, n, N, kappa, _bump, coarse_iters=-1)
    L = prob.lmax
    To = oracle_hierarchy(oc, L)
    for level in range(1, L + 1):
        Tg = box_maps_by_xy(hps, prob, level)
        assert len(Tg) == len(To[level - 1]), level
        for key, Tref in To[level - 1].items():
            keep = np.arange(Tref.shape[0])
            if level > 1:
                keep = np.nonzero(~mesh.box_local_physical_mask(n, N - 1, level, *key))[0]
            assert rel(Tg[key][np.ix_(keep, keep)], Tref[np.ix_(keep, keep)]) < 1e-10, (level, key)


@pytest.mark.parametrize("n,N,levels,k", [((8, 2), 5, 4, -1), ((8, 2), 5, 3, 3), ((2, 8), 5, 4, 2),
                                          ((16, 4), 4, 6, 3), ((4, 16), 4, 5, 2)])
def test_rect_precond_apply(hps, ctx, n, N, levels, k):
    import torch
    from oracle import mesh, multigrid
    print(f"[rect precond] {n} N={N} L={levels} k={k}", flush=True)
    kappa = 8.0
    wave = workloads.PlaneWave(kappa, kappa)
    oc = oracle_case(n, N, kappa, _bump, wave.t, None, with_direct=False)
    prob = gpu_problem(hps, ctx, n, N, kappa, _bump, levels=levels, coarse_iters=k)
    hier = multigrid.Hierarchy(n, N - 1, oc["T"], levels=levels)
    rng = np.random.default_rng(levels * 10 + k)
    r = rng.standard_normal(prob.nslots) + 1j * rng.standard_normal(prob.nslots)
    r[mesh.physical_slot_mask(n, N - 1)] = 0
    z = prob.precond_apply(torch.from_numpy(r).cuda()).cpu().numpy()
    zr = hier.apply(r, None if k < 0 else k)
    assert rel(z, zr) < 1e-10


@pytest.mark.parametrize("n,N,k,precision", [((8, 2), 6, 3, "fp64"), ((2, 8), 6, -1, "fp64"),
                                             ((32, 8), 6, 4, "fp64"), ((32, 8), 6, 4, "mixed"),
                                             ((8, 32), 8, 5, "mixed")])
def test_rect_solve_matches_oracle(hps, ctx, n, N, k, precision):
    print(f"[rect solve] {n} N={N} k={k} {precision}", flush=True)
    kappa = 20.0
    wave = workloads.PlaneWave(kappa, kappa, (0.8, 0.6))
    oc = oracle_case(n, N, kappa, _bump, wave.t, _src)
    nx, ny = n
    prec = hps.HPS_MIXED if precision == "mixed" else hps.HPS_FP64
    desc = hps.make_desc(nx, N, kappa, coarse_iters=k, precision=prec, ny=ny)
    prob = hps.Problem(ctx, desc)
    prob.build_leaves(prob.coefficient_nodes(_bump), prob.source_nodes(_src))
    prob.merge_all()
    rhs = prob.set_rhs(prob.boundary_data(wave.t))
    g, info = prob.gmres_solve(rhs, tol=1e-12, maxit=600)
    assert info["status"] == 0 and info["relres_true"] <= 1e-12, info
    assert rel(g.cpu().numpy(), oc["g"]) < 1e-10
    if k == -1:
        assert info["iterations"] == 1

