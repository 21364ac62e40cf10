"""Shared builders for the GPU parity tests: the same seeded problem, solved by
the oracle (CPU, FP64) and by the HIP library through its C ABI."""
import numpy as np

from oracle import gll, leaf, mesh, skeleton, direct, merge


def oracle_case(n, N, kappa, b_fn, t_fn, s_fn=None, eta=None, with_direct=True):
    """n: elements per side, or the pair (nx, ny) of a rectangular mesh."""
    eta = kappa if eta is None else eta
    p = N - 1
    xi = gll.gll_nodes(N)
    c = leaf.nodal_coefficient(N, n, kappa, b_fn, xi)
    s = None
    if s_fn is not None:
        X, Y = mesh.element_node_coords(n, N, xi)
        s = s_fn(X, Y).reshape(mesh.num_elements(n), -1)
    T, H = leaf.leaves(N, mesh.element_size(n), kappa, eta, c, s)
    xs, ys, nx, ny = mesh.canonical_slot_coords(n, N, xi)
    t = t_fn(xs, ys, nx, ny)
    rhs = skeleton.rhs(n, p, T, H, t)
    out = dict(n=n, N=N, p=p, T=T, H=H, t=t, rhs=rhs)
    if with_direct:
        out["g"] = direct.solve(n, p, T, H, t)
    return out


def gpu_problem(hps, ctx, n, N, kappa, b_fn, s_fn=None, eta=None, levels=0, coarse_iters=5,
                restart=60, merge=True):
    nx, ny = mesh.dims(n)
    desc = hps.make_desc(nx, N, kappa, eta, levels=levels, coarse_iters=coarse_iters,
                         restart=restart, ny=ny)
    prob = hps.Problem(ctx, desc)
    b_nodes = prob.coefficient_nodes(b_fn)
    s_nodes = prob.source_nodes(s_fn) if s_fn is not None else None
    prob.build_leaves(b_nodes, s_nodes)
    if merge:
        prob.merge_all()
    return prob


def rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def box_maps_by_xy(hps, prob, level):
    """GPU machine maps of a level keyed by box coordinates (bx, by)."""
    T = prob.level_T(level).cpu().numpy()
    return {hps.tree_box_xy(level, j, prob.nx, prob.ny): T[j] for j in range(T.shape[0])}


def oracle_hierarchy(case, top):
    T, _ = merge.build_hierarchy(case["n"], case["p"], case["T"], None, top=top)
    return T
