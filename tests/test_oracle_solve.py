"""Pins of the oracle's skeleton system and solvers (Sec. 3.2, 4.2, 4.3, Table 1).

* exact discrete solution for a global polynomial (sparse LU and direct HPS);
* agreement with the element-DOF brute force (no ItI map involved);
* spectral convergence in N to the exact plane-wave impedance data;
* MG with an exact coarse solve equals M_1^-1 (block-inverse identity);
* FGMRES preconditioned by direct HPS converges in one iteration (Table 1);
* k-step GMRES equals brute-force Krylov least squares; k = dim is exact;
* FGMRES with the identity preconditioner matches scipy's GMRES.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import gll, leaf, mesh, skeleton, direct, multigrid, krylov, brute
from paper_2511_00735_amd import workloads
from tests.manufactured import PolySolution


def setup(n, N, kappa, bfn, t_fn, s_fn=None):
    p = N - 1
    xi = gll.gll_nodes(N)
    c = leaf.nodal_coefficient(N, n, kappa, bfn, xi)
    s = None
    if s_fn is not None:
        X, Y = mesh.element_node_coords(n, N, xi)
        s = s_fn(X, Y).reshape(n * n, -1)
    T, H = leaf.leaves(N, 1.0 / n, kappa, kappa, c, s)
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


@pytest.mark.parametrize("n,N", [(4, 5), (2, 8), (8, 3)])
def test_polynomial_is_exact_discrete_solution(n, N):
    kappa = 7.0
    u = PolySolution(N, seed=n + N)
    bfn = lambda x, y: 0.25 * np.cos(2 * x - y)
    cfn = lambda x, y: kappa ** 2 * (1 - bfn(x, y))
    d = setup(n, N, kappa, bfn, u.t(kappa), u.source(cfn))
    exact = np.where(mesh.physical_slot_mask(n, d["p"]), 0, u.t(kappa)(*d["coords"]))
    assert rel(d["g"], exact) < 1e-11
    assert rel(direct.solve(n, d["p"], d["T"], d["H"], d["t"]), exact) < 1e-11


def test_brute_force_agrees():
    n, N, kappa = 2, 5, 6.0
    u = PolySolution(3, seed=1)
    bfn = lambda x, y: 0.3 * np.sin(3 * x) + 0.1 * y
    cfn = lambda x, y: kappa ** 2 * (1 - bfn(x, y))
    pw = workloads.PlaneWave(kappa, kappa)
    # a source that is not a polynomial solution: generic data
    d = setup(n, N, kappa, bfn, pw.t, lambda x, y: np.exp(1j * x) * (1 + y))
    gb, _ = brute.solve(n, N, kappa, kappa, d["c"], d["s"], d["t"])
    assert rel(gb, d["g"]) < 1e-11


def test_c1_plane_wave_spectral_convergence():
    pr = workloads.c1()
    errs = []
    for N in (4, 6, 8, 10):
        d = setup(pr.n, N, pr.kappa, pr.b, pr.wave.t)
        xs, ys, nx, ny = d["coords"]
        exact = np.where(mesh.physical_slot_mask(pr.n, N - 1), 0, pr.wave.t(xs, ys, nx, ny))
        errs.append(rel(d["g"], exact))
    assert errs[2] < 1e-5 and errs[3] < 1e-7
    assert all(b < 0.1 * a for a, b in zip(errs, errs[1:]))


@pytest.mark.parametrize("levels", [2, 3, 4])
def test_mg_with_exact_coarse_is_inverse(levels):
    n, N, kappa = 4, 4, 8.0
    pr = workloads.c1()
    d = setup(n, N, kappa, lambda x, y: 0.4 * np.exp(-((x - .5) ** 2 + (y - .5) ** 2) / .1), pr.wave.t)
    hier = multigrid.Hierarchy(n, d["p"], d["T"], levels=levels)
    rng = np.random.default_rng(levels)
    r = np.zeros(len(d["rhs"]), dtype=complex)
    r[d["unk"]] = rng.standard_normal(len(d["unk"])) + 1j * rng.standard_normal(len(d["unk"]))
    z = hier.apply(r, k=None)
    ref = np.zeros_like(r)
    ref[d["unk"]] = spla.spsolve(d["M1"].tocsc(), r[d["unk"]])
    assert rel(z, ref) < 1e-12


def test_c1_direct_and_fgmres():
    pr = workloads.c1()
    d = setup(pr.n, pr.N, pr.kappa, pr.b, pr.wave.t)
    g_direct = direct.solve(pr.n, d["p"], d["T"], d["H"], d["t"])
    assert rel(g_direct, d["g"]) < 1e-12
    hier = multigrid.Hierarchy(pr.n, d["p"], d["T"], levels=pr.levels)
    Mv = lambda v: skeleton.apply(pr.n, d["p"], 1, skeleton.leaf_boxT(pr.n, d["T"]), v)
    x, it, _, rr = krylov.fgmres(Mv, d["rhs"], lambda v: hier.apply(v, None), tol=1e-10)
    assert it == 1 and rel(x, d["g"]) < 1e-12          # exact coarse space: It = 1
    x, it, hist, rr = krylov.fgmres(Mv, d["rhs"], lambda v: hier.apply(v, pr.coarse_iters),
                                    tol=pr.tol)
    assert rr <= pr.tol and rel(x, d["g"]) < 1e-9
    assert all(b <= a * (1 + 1e-12) for a, b in zip(hist, hist[1:]))   # monotone
    _, it0, _, _ = krylov.fgmres(Mv, d["rhs"], None, tol=pr.tol)
    assert it < it0                                      # the preconditioner helps


def test_gmres_ksteps_is_krylov_least_squares():
    rng = np.random.default_rng(11)
    n = 12
    A = np.eye(n) + 0.4 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    r = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    for k in (1, 3, 6):
        x = krylov.gmres_ksteps(lambda v: A @ v, r, k)
        K = np.stack([np.linalg.matrix_power(A, j) @ r for j in range(k)], 1)
        Q, _ = np.linalg.qr(K)
        y, *_ = np.linalg.lstsq(A @ Q, r, rcond=None)
        np.testing.assert_allclose(x, Q @ y, atol=1e-10)
    x = krylov.gmres_ksteps(lambda v: A @ v, r, n)
    np.testing.assert_allclose(A @ x, r, atol=1e-10)


def test_fgmres_identity_matches_scipy():
    rng = np.random.default_rng(5)
    n = 150
    A = np.eye(n) * 3 + (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, it, hist, rr = krylov.fgmres(lambda v: A @ v, b, None, tol=1e-12, restart=60)
    assert rr <= 1e-12
    xs, info = spla.gmres(A, b, rtol=1e-13, restart=60, maxiter=50)
    np.testing.assert_allclose(x, xs, atol=1e-10)
    # restarts: a short restart length still converges and counts all iterations
    x2, it2, _, rr2 = krylov.fgmres(lambda v: A @ v, b, None, tol=1e-12, restart=5)
    assert rr2 <= 1e-12 and it2 > it
