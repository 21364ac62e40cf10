"""Pins of the oracle's leaf operators (Sec. 3.1, eq. ItIOperator).

* exact identity: interior rows of Lt reproduce (M (x) M)(-Lap u - c u) for u in
  Q_N (GLL summation by parts) -- pins the "- diag(c)" reading and the scaling;
* exact polynomial reproduction: T I_i u + H = I_o u for u in Q_N;
* closed form: plane waves satisfy T I_i u = I_o u with spectral accuracy in N;
* energy balance for real c (near-unitarity on resolved data);
* rotation symmetry of T for a constant coefficient.
"""
import numpy as np
import pytest

from oracle import gll, leaf, mesh
from tests.manufactured import PolySolution, PlaneWaves


def element_grid(N, h, x0=0.0, y0=0.0):
    xi = gll.gll_nodes(N)
    xs = x0 + (1 + xi) * h / 2
    ys = y0 + (1 + xi) * h / 2
    X, Y = np.meshgrid(xs, ys, indexing="ij")   # [i, j]
    return X, Y


def side_data(N, h, fn, x0=0.0, y0=0.0):
    """Evaluate fn(x, y, nx, ny) on the element's [l; r; b; t] non-corner nodes."""
    X, Y = element_grid(N, h, x0, y0)
    normals = {mesh.L_: (-1, 0), mesh.R_: (1, 0), mesh.B_: (0, -1), mesh.T_: (0, 1)}
    out = []
    for s in range(4):
        i, j = mesh.side_nodes_ij(N, s)
        out.append(fn(X[i, j], Y[i, j], *normals[s]))
    return np.concatenate(out)


@pytest.mark.parametrize("N", [3, 6, 9])
def test_interior_rows_exact_on_QN(N):
    h, kappa = 0.3, 7.0
    u = PolySolution(N, seed=N, x0=0.1, y0=0.2)
    b = lambda x, y: 0.4 * np.sin(2 * x + y)
    X, Y = element_grid(N, h)
    c = (kappa ** 2 * (1 - b(X, Y))).ravel()
    Lt = leaf.local_operator(N, h, c)
    _, w, _, _, _ = leaf.element_1d(N, h)
    lhs = (Lt @ u.u(X, Y).ravel()).reshape(N + 1, N + 1)
    rhs = (h / 2) ** 2 * np.outer(w, w) * (-u.lap(X, Y) - c.reshape(N + 1, N + 1) * u.u(X, Y))
    np.testing.assert_allclose(lhs[1:N, 1:N], rhs[1:N, 1:N], atol=1e-9 * np.abs(rhs).max())
    # the "+ diag(c)" sign as printed would fail this identity by O(c u)
    Lplus = Lt + 2 * np.diag(c) @ np.kron(np.diag((h / 2) * w), np.diag((h / 2) * w))
    bad = (Lplus @ u.u(X, Y).ravel()).reshape(N + 1, N + 1)
    assert np.abs(bad - rhs)[1:N, 1:N].max() > 1e-3 * np.abs(rhs).max()


@pytest.mark.parametrize("N", [4, 8, 12])
def test_leaf_polynomial_reproduction(N):
    h, kappa = 0.25, 9.0
    u = PolySolution(N, seed=10 + N, x0=0.3, y0=0.1)
    bfn = lambda x, y: 0.5 * np.cos(3 * x) * np.exp(-y)
    cfn = lambda x, y: kappa ** 2 * (1 - bfn(x, y))
    X, Y = element_grid(N, h)
    c = cfn(X, Y).ravel()
    s = u.source(cfn)(X, Y).ravel()
    T, H = leaf.leaf_itI(N, h, kappa, kappa, c, s)
    f = side_data(N, h, u.t(kappa))                                  # I_i u
    o = side_data(N, h, lambda x, y, nx, ny: -(u.grad(x, y)[0] * nx + u.grad(x, y)[1] * ny
                                               - 1j * kappa * u.u(x, y)))   # I_o u
    np.testing.assert_allclose(T @ f + H, o, atol=1e-10 * np.abs(o).max())


def test_leaf_batched_equals_single():
    N, n, kappa = 6, 2, 5.0
    h = 1.0 / n
    rng = np.random.default_rng(1)
    c = kappa ** 2 * (1 - 0.3 * rng.standard_normal((n * n, (N + 1) ** 2)))
    s = rng.standard_normal((n * n, (N + 1) ** 2)) + 1j * rng.standard_normal((n * n, (N + 1) ** 2))
    T, H = leaf.leaves(N, h, kappa, kappa, c, s, chunk=3)
    for e in range(n * n):
        Te, He = leaf.leaf_itI(N, h, kappa, kappa, c[e], s[e])
        np.testing.assert_allclose(T[e], Te, atol=1e-13)
        np.testing.assert_allclose(H[e], He, atol=1e-13)


def test_plane_wave_spectral_convergence():
    h, kappa = 0.25, 10.0
    pw = PlaneWaves(kappa, count=1, seed=3)
    errs = []
    for N in (4, 8, 12, 16):
        T, _ = leaf.leaf_itI(N, h, kappa, kappa, kappa ** 2 * np.ones((N + 1) ** 2))
        f = side_data(N, h, lambda x, y, nx, ny: pw.dn(x, y, nx, ny) + 1j * kappa * pw.u(x, y))
        o = side_data(N, h, lambda x, y, nx, ny: -(pw.dn(x, y, nx, ny) - 1j * kappa * pw.u(x, y)))
        errs.append(np.linalg.norm(T @ f - o) / np.linalg.norm(o))
    assert errs[-1] < 1e-11
    assert all(b < a * 1e-2 for a, b in zip(errs[:-2], errs[1:-1]))


def test_energy_balance_real_c():
    """For real c, |I_o u| = |I_i u| in L2(boundary) for every solution u
    (Green's identity); the discrete T keeps this on resolved data."""
    h, kappa = 0.25, 10.0
    pw = PlaneWaves(kappa, count=4, seed=7)
    gaps = []
    for N in (6, 10, 16):
        xi, w, _ = gll.gll(N)
        wb = np.tile((h / 2) * w[1:N], 4)
        T, _ = leaf.leaf_itI(N, h, kappa, kappa, kappa ** 2 * np.ones((N + 1) ** 2))
        f = side_data(N, h, lambda x, y, nx, ny: pw.dn(x, y, nx, ny) + 1j * kappa * pw.u(x, y))
        o = T @ f
        gaps.append(abs(np.sqrt(wb @ np.abs(o) ** 2) / np.sqrt(wb @ np.abs(f) ** 2) - 1))
    # corner nodes carry no unknowns, so the weighted balance converges but is not exact
    assert gaps[-1] < 2e-2 and gaps[-1] < gaps[0]


def test_rotation_symmetry_constant_c():
    """Rotating the element by 90 degrees maps side l->b->r->t->l; for a constant
    coefficient T must be invariant under the induced permutation."""
    N, h, kappa = 7, 0.2, 6.0
    T, _ = leaf.leaf_itI(N, h, kappa, kappa, kappa ** 2 * np.ones((N + 1) ** 2))
    p = N - 1
    k = np.arange(p)
    # rotation (x, y) -> (1 - y, x) about the element centre: node (i, j) -> (N - j, i)
    # l(j) -> b(i = N - j), b(i) -> r(j = i), r(j) -> t(i = N - j), t(i) -> l(j = i)
    perm = np.empty(4 * p, dtype=int)
    perm[0 * p + k] = 2 * p + (p - 1 - k)     # l -> b reversed
    perm[2 * p + k] = 1 * p + k               # b -> r
    perm[1 * p + k] = 3 * p + (p - 1 - k)     # r -> t reversed
    perm[3 * p + k] = 0 * p + k               # t -> l
    Pm = np.zeros((4 * p, 4 * p))
    Pm[perm, np.arange(4 * p)] = 1
    np.testing.assert_allclose(Pm @ T @ Pm.T, T, atol=1e-11)
