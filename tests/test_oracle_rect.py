"""Pins of the oracle on rectangular meshes of nx x ny elements (powers of two):
square elements of side 1/max(nx, ny), merges alternating x, y while both
directions have merges left and then along the longer direction.

* the level geometry (merge axes, box sizes, pair counts, the root box);
* every box map at every level reproduces a polynomial solution exactly (pins
  the merge tree on both kinds of tail: all-x and all-y);
* the skeleton solution and direct HPS equal the polynomial exactly, and agree
  with the element-DOF brute force for generic data;
* MG with an exact coarse solve equals M_1^-1;
* spectral convergence in N to a plane wave on a 4:1 rectangle.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import brute, direct, gll, leaf, merge, mesh, multigrid, skeleton
from paper_2511_00735_amd import workloads
from tests.manufactured import PolySolution


def setup(n, N, kappa, bfn, t_fn, s_fn=None):
    p = N - 1
    xi = gll.gll_nodes(N)
    c = leaf.nodal_coefficient(N, n, kappa, bfn, xi)
    s = None
    if s_fn is not None:
        X, Y = mesh.element_node_coords(n, N, xi)
        s = s_fn(X, Y).reshape(mesh.num_elements(n), -1)
    T, H = leaf.leaves(N, mesh.element_size(n), kappa, kappa, c, s)
    xs, ys, nx, ny = mesh.canonical_slot_coords(n, N, xi)
    t = t_fn(xs, ys, nx, ny)
    rhs = skeleton.rhs(n, p, T, H, t)
    M1, unk = skeleton.assemble(n, p, 1, skeleton.leaf_boxT(n, T))
    g = np.zeros_like(rhs)
    g[unk] = spla.spsolve(M1.tocsc(), rhs[unk])
    return dict(p=p, xi=xi, c=c, s=s, T=T, H=H, t=t, rhs=rhs, M1=M1, unk=unk, g=g,
                coords=(xs, ys, nx, ny))


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_rect_level_geometry():
    # 8 x 2: x, y, then x, x
    n = (8, 2)
    assert mesh.lmax(n) == 4
    assert [mesh.merge_axis(l, n) for l in range(1, 5)] == ["x", "y", "x", "x"]
    assert [mesh.box_dims(l, n) for l in range(1, 6)] == [(1, 1), (2, 1), (2, 2), (4, 2), (8, 2)]
    assert [len(mesh.pairs(n, l)) for l in range(1, 5)] == [8, 4, 2, 1]
    # 2 x 8: x, y, then y, y
    n = (2, 8)
    assert [mesh.merge_axis(l, n) for l in range(1, 5)] == ["x", "y", "y", "y"]
    assert [mesh.box_dims(l, n) for l in range(1, 6)] == [(1, 1), (2, 1), (2, 2), (2, 4), (2, 8)]
    # a single row or column: every merge along it
    assert [mesh.merge_axis(l, (4, 1)) for l in (1, 2)] == ["x", "x"]
    assert [mesh.merge_axis(l, (1, 4)) for l in (1, 2)] == ["y", "y"]
    # square meshes keep the alternating rule
    assert [mesh.merge_axis(l, 4) for l in range(1, 5)] == ["x", "y", "x", "y"]
    for n in [(8, 2), (2, 8), (4, 1), (1, 4), (16, 4), (4, 16)]:
        nx, ny = n
        L = mesh.lmax(n)
        assert mesh.box_dims(L + 1, n) == (nx, ny) and mesh.box_grid(n, L + 1) == (1, 1)
        assert mesh.element_size(n) == 1.0 / max(nx, ny)
        # every slot is a boundary slot of exactly one box at every level
        p = 2
        for level in range(1, L + 2):
            nbx, nby = mesh.box_grid(n, level)
            sl = np.concatenate([mesh.box_slots(n, p, level, bx, by)
                                 for by in range(nby) for bx in range(nbx)])
            assert len(np.unique(sl)) == len(sl)


@pytest.mark.parametrize("n,N", [((8, 2), 4), ((2, 4), 5), ((4, 1), 4), ((1, 8), 3)])
def test_rect_every_box_reproduces_polynomial(n, N):
    kappa = 6.0
    u = PolySolution(N, seed=5, x0=0.35, y0=0.2)
    bfn = lambda x, y: 0.3 * np.sin(4 * x) * np.cos(3 * y)
    cfn = lambda x, y: kappa ** 2 * (1 - bfn(x, y))
    xi = gll.gll_nodes(N)
    c = leaf.nodal_coefficient(N, n, kappa, bfn, xi)
    X, Y = mesh.element_node_coords(n, N, xi)
    s = u.source(cfn)(X, Y).reshape(mesh.num_elements(n), -1)
    T, H = leaf.leaves(N, mesh.element_size(n), kappa, kappa, c, s)
    p = N - 1
    Tl, Hl = merge.build_hierarchy(n, p, T, H)
    xs, ys, nx, ny = mesh.canonical_slot_coords(n, N, xi)
    gx, gy = u.grad(xs, ys)
    dn = gx * nx + gy * ny
    f = dn + 1j * kappa * u.u(xs, ys)
    o = -(dn - 1j * kappa * u.u(xs, ys))
    for level in range(1, mesh.lmax(n) + 1):
        assert len(Tl[level - 1]) == np.prod(mesh.box_grid(n, level))
        for (bx, by), Tb in Tl[level - 1].items():
            sl = mesh.box_slots(n, p, level, bx, by)
            lhs = Tb @ f[sl] + Hl[level - 1][(bx, by)]
            np.testing.assert_allclose(lhs, o[sl], atol=1e-9 * np.abs(o).max(),
                                       err_msg=f"level {level} box {(bx, by)}")


@pytest.mark.parametrize("n,N", [((4, 2), 5), ((2, 8), 4), ((8, 1), 4)])
def test_rect_polynomial_is_exact_discrete_solution(n, N):
    kappa = 7.0
    u = PolySolution(N, seed=2)
    bfn = lambda x, y: 0.25 * np.cos(2 * x - y)
    cfn = lambda x, y: kappa ** 2 * (1 - bfn(x, y))
    d = setup(n, N, kappa, bfn, u.t(kappa), u.source(cfn))
    exact = np.where(mesh.physical_slot_mask(n, d["p"]), 0, u.t(kappa)(*d["coords"]))
    assert rel(d["g"], exact) < 1e-11
    assert rel(direct.solve(n, d["p"], d["T"], d["H"], d["t"]), exact) < 1e-11


def test_rect_brute_force_agrees():
    n, N, kappa = (4, 2), 4, 6.0
    bfn = lambda x, y: 0.3 * np.sin(3 * x) + 0.1 * y
    pw = workloads.PlaneWave(kappa, kappa, (0.6, 0.8))
    d = setup(n, N, kappa, bfn, pw.t, lambda x, y: np.exp(1j * x) * (1 + y))
    gb, _ = brute.solve(n, N, kappa, kappa, d["c"], d["s"], d["t"])
    assert rel(gb, d["g"]) < 1e-11
    assert rel(direct.solve(n, d["p"], d["T"], d["H"], d["t"]), d["g"]) < 1e-11


@pytest.mark.parametrize("n,levels", [((8, 2), 2), ((8, 2), 3), ((8, 2), 4), ((2, 8), 3)])
def test_rect_mg_with_exact_coarse_is_inverse(n, levels):
    N, kappa = 4, 8.0
    pw = workloads.PlaneWave(kappa, kappa)
    d = setup(n, N, kappa, lambda x, y: 0.4 * np.exp(-((x - .5) ** 2 + (y - .2) ** 2) / .1), pw.t)
    hier = multigrid.Hierarchy(n, d["p"], d["T"], levels=levels)
    rng = np.random.default_rng(levels)
    r = np.zeros(len(d["rhs"]), dtype=complex)
    r[d["unk"]] = rng.standard_normal(len(d["unk"])) + 1j * rng.standard_normal(len(d["unk"]))
    z = hier.apply(r, k=None)
    ref = np.zeros_like(r)
    ref[d["unk"]] = spla.spsolve(d["M1"].tocsc(), r[d["unk"]])
    assert rel(z, ref) < 1e-12


def test_rect_plane_wave_spectral_convergence():
    n, kappa = (8, 2), 12.0
    pw = workloads.PlaneWave(kappa, kappa, (0.8, 0.6))
    errs = []
    for N in (4, 6, 8, 10):
        d = setup(n, N, kappa, lambda x, y: 0.0 * x, pw.t)
        xs, ys, nx, ny = d["coords"]
        exact = np.where(mesh.physical_slot_mask(n, N - 1), 0, pw.t(xs, ys, nx, ny))
        errs.append(rel(d["g"], exact))
    assert errs[3] < 1e-7
    assert all(b < 0.1 * a for a, b in zip(errs, errs[1:]))
