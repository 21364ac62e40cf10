"""Cross-problem batching: a group of problems of one shape (different
wavenumbers, coefficients and boundary data) runs every hot-path step in the
same launches.  Each member must give what the same problem gives alone (up to
the summation order of split reductions) and, through that, what the oracle
gives."""
import math

import numpy as np
import pytest

from paper_2511_00735_amd import workloads
from tests.gpu_cases import oracle_case, rel

pytestmark = pytest.mark.gpu


def _members(count, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        kappa = float(rng.uniform(8.0, 20.0))
        bumps = workloads.draw_bumps(rng, int(rng.integers(1, 4)))
        th = float(rng.uniform(0, 2 * math.pi))
        out.append((kappa, bumps, workloads.PlaneWave(kappa, kappa, (math.cos(th), math.sin(th)))))
    return out


def _group(hps, ctx, n, N, members, levels=0, coarse_iters=3, precision=None):
    precision = hps.HPS_FP64 if precision is None else precision
    desc = hps.make_desc(n, N, members[0][0], levels=levels, coarse_iters=coarse_iters, precision=precision)
    grp = hps.Group(ctx, desc, [m[0] for m in members])
    # inputs evaluated at the library's nodes (the same for every member)
    probe = hps.Problem(ctx, desc)
    b_nodes = [probe.coefficient_nodes(m[1]) for m in members]
    ts = [probe.boundary_data(m[2].t) for m in members]
    grp.build_leaves(b_nodes)
    grp.merge_all()
    return grp, b_nodes, ts


def _alone(hps, ctx, n, N, member, b_nodes, levels=0, coarse_iters=3, precision=None):
    precision = hps.HPS_FP64 if precision is None else precision
    desc = hps.make_desc(n, N, member[0], levels=levels, coarse_iters=coarse_iters, precision=precision)
    prob = hps.Problem(ctx, desc)
    prob.build_leaves(b_nodes)
    prob.merge_all()
    return prob


GROUP_CASES = [
    # name, n, N, levels, coarse iterations, members
    ("k3_top", 8, 6, 0, 3, 3),
    ("direct", 8, 5, 0, -1, 2),
    ("coarse_below_top", 16, 4, 6, 2, 3),
]


@pytest.mark.parametrize("name,n,N,levels,k,count", GROUP_CASES, ids=[c[0] for c in GROUP_CASES])
def test_group_members_match_alone_and_oracle(hps, ctx, name, n, N, levels, k, count):
    print(f"[group] {name}", flush=True)
    members = _members(count, seed=11 + n + N)
    grp, b_nodes, ts = _group(hps, ctx, n, N, members, levels=levels, coarse_iters=k)
    rhs = grp.set_rhs(ts)
    gs, infos = grp.gmres_solve(rhs, tol=1e-12, maxit=400)
    for q, m in enumerate(members):
        prob = _alone(hps, ctx, n, N, m, b_nodes[q], levels=levels, coarse_iters=k)
        r1 = prob.set_rhs(ts[q])
        g1, info1 = prob.gmres_solve(r1, tol=1e-12, maxit=400)
        assert infos[q]["status"] == 0 and infos[q]["relres_true"] <= 1e-12, infos[q]
        assert rel(rhs[q].cpu().numpy(), r1.cpu().numpy()) == 0.0
        assert rel(gs[q].cpu().numpy(), g1.cpu().numpy()) < 1e-10, q
        if k == -1:
            assert infos[q]["iterations"] == 1
    # member 0 against the oracle's direct solve
    oc = oracle_case(n, N, members[0][0], members[0][1], members[0][2].t)
    assert rel(gs[0].cpu().numpy(), oc["g"]) < 1e-10


def test_group_precond_and_maps_match_alone(hps, ctx):
    import torch
    from oracle import mesh
    n, N, k = 8, 6, 3
    members = _members(3, seed=5)
    grp, b_nodes, ts = _group(hps, ctx, n, N, members, coarse_iters=k)
    rng = np.random.default_rng(3)
    rs = []
    for _ in members:
        r = rng.standard_normal(grp.nslots) + 1j * rng.standard_normal(grp.nslots)
        r[mesh.physical_slot_mask(n, N - 1)] = 0
        rs.append(torch.from_numpy(r).cuda())
    zs = grp.precond_apply(rs)
    for q, m in enumerate(members):
        prob = _alone(hps, ctx, n, N, m, b_nodes[q], coarse_iters=k)
        z1 = prob.precond_apply(rs[q])
        assert rel(zs[q].cpu().numpy(), z1.cpu().numpy()) < 1e-12, q
        for level in (1, 3, prob.levels):
            Tg = grp.level_T(q, level).cpu().numpy()
            T1 = prob.level_T(level).cpu().numpy()
            assert rel(Tg, T1) < 1e-12, (q, level)


def test_group_leaf_launches_span_problems(hps, ctx):
    """40 problems of 16 elements: leaf launches cover at most 32 problems, so
    the group needs two; every member's leaf maps equal its own build."""
    n, N = 4, 4
    members = _members(40, seed=9)
    desc = hps.make_desc(n, N, members[0][0], coarse_iters=2)
    grp = hps.Group(ctx, desc, [m[0] for m in members])
    probe = hps.Problem(ctx, desc)
    b_nodes = [probe.coefficient_nodes(m[1]) for m in members]
    grp.build_leaves(b_nodes)
    for q in (0, 31, 32, 39):
        prob = _alone(hps, ctx, n, N, members[q], b_nodes[q], coarse_iters=2)
        assert np.array_equal(grp.level_T(q, 1).cpu().numpy(), prob.level_T(1).cpu().numpy()), q


def test_group_mixed_precision(hps, ctx):
    n, N = 16, 6
    members = _members(2, seed=21)
    grp, b_nodes, ts = _group(hps, ctx, n, N, members, coarse_iters=4, precision=hps.HPS_MIXED)
    rhs = grp.set_rhs(ts)
    gs, infos = grp.gmres_solve(rhs, tol=1e-12, maxit=400)
    for q, m in enumerate(members):
        prob = _alone(hps, ctx, n, N, m, b_nodes[q], coarse_iters=4, precision=hps.HPS_MIXED)
        g1, info1 = prob.gmres_solve(prob.set_rhs(ts[q]), tol=1e-12, maxit=400)
        assert infos[q]["relres_true"] <= 1e-12
        assert rel(gs[q].cpu().numpy(), g1.cpu().numpy()) < 1e-10, q
    oc = oracle_case(n, N, members[1][0], members[1][1], members[1][2].t)
    assert rel(gs[1].cpu().numpy(), oc["g"]) < 1e-10


def test_group_argument_checks(hps, ctx):
    desc = hps.make_desc(4, 4, 5.0, coarse_iters=2)
    with pytest.raises(hps.HPSError):
        hps.Group(ctx, desc, [5.0, -1.0])
    grp = hps.Group(ctx, desc, [5.0, 6.0])
    probe = hps.Problem(ctx, desc)
    b = probe.coefficient_nodes(workloads.zero_field)
    with pytest.raises(ValueError):
        grp.build_leaves([b])            # two problems need two arrays


def test_group_iteration_graph_matches_eager(hps, ctx):
    """A group's FGMRES iterations replayed from the captured iteration graph give
    bitwise the eager group solve for every member."""
    import torch
    members = _members(3, 11)
    grp, _, ts = _group(hps, ctx, 8, 6, members, coarse_iters=3)
    rhs = grp.set_rhs(ts)
    ctx.set_graphs(False)
    ge, ie = grp.gmres_solve(rhs, tol=1e-10)
    ge = [g.clone() for g in ge]
    ctx.set_graphs(True)
    try:
        for rep in range(2):
            gg, ig = grp.gmres_solve(rhs, tol=1e-10)
            ctx.sync()
            for q in range(len(members)):
                assert ig[q]["iterations"] == ie[q]["iterations"], (rep, q)
                assert torch.equal(gg[q], ge[q]), (rep, q)
    finally:
        ctx.set_graphs(False)
