"""Pins of the oracle's field recovery (Sec. 3.1 local problem; corner values
by the extrapolation reading):

* a global u in Q_N with matching source and boundary data is recovered
  exactly at every non-corner node (the discrete system reproduces Q_N), and
  at the corners too when its degree is <= N-2;
* a resolved plane wave (b = 0, s = 0) is recovered with an error that falls
  spectrally in N (closed-form exact solution);
* the two elements sharing an edge give the same field on it.
"""
import numpy as np
import pytest

from oracle import direct, field, gll, leaf, mesh
from tests.manufactured import PolySolution
from paper_2511_00735_amd import workloads


def _bump(x, y):
    return 0.5 * np.exp(-((x - 0.3) ** 2 + (y - 0.6) ** 2) / 0.1)


def _solve_fields(n, N, kappa, b_fn, t_fn, s_fn=None):
    xi = gll.gll_nodes(N)
    c = leaf.nodal_coefficient(N, n, kappa, b_fn, xi)
    X, Y = mesh.element_node_coords(n, N, xi)
    s = None if s_fn is None else s_fn(X, Y).reshape(n * n, -1)
    T, H = leaf.leaves(N, 1.0 / n, kappa, kappa, c, s)
    xs, ys, nx, ny = mesh.canonical_slot_coords(n, N, xi)
    t = t_fn(xs, ys, nx, ny)
    g = direct.solve(n, N - 1, T, H, t)
    u = field.fields(n, N, kappa, c, s, g, t)
    return u, X.reshape(n * n, -1), Y.reshape(n * n, -1)


@pytest.mark.parametrize("deg,N", [(5, 5), (3, 5)])
def test_polynomial_field_recovered_exactly(deg, N):
    n, kappa = 2, 6.0
    sol = PolySolution(deg, seed=4)
    cfn = lambda x, y: kappa ** 2 * (1 - _bump(x, y))
    u, X, Y = _solve_fields(n, N, kappa, _bump, sol.t(kappa), sol.source(cfn))
    exact = sol.u(X, Y)
    corner = np.zeros((N + 1) ** 2, dtype=bool)
    for i, j in ((0, 0), (0, N), (N, 0), (N, N)):
        corner[leaf.flat(N, i, j)] = True
    scale = np.abs(exact).max()
    assert np.abs(u[:, ~corner] - exact[:, ~corner]).max() < 1e-10 * scale
    if deg <= N - 2:
        assert np.abs(u[:, corner] - exact[:, corner]).max() < 1e-10 * scale
    else:
        # degree N along the sides: the corner extrapolation is not exact
        assert np.abs(u[:, corner] - exact[:, corner]).max() > 1e-8 * scale


def test_plane_wave_field_converges_spectrally():
    n, kappa = 2, 9.0
    wave = workloads.PlaneWave(kappa, kappa)
    errs = []
    for N in (4, 6, 8, 10, 12):
        u, X, Y = _solve_fields(n, N, kappa, workloads.zero_field, wave.t)
        errs.append(np.abs(u - wave.u(X, Y)).max())
    # every two orders cut the error by more than an order of magnitude
    assert all(b < a / 10 for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-6, errs


def test_shared_edge_values_agree():
    n, N, kappa = 2, 8, 7.0
    wave = workloads.PlaneWave(kappa, kappa)
    u, X, Y = _solve_fields(n, N, kappa, _bump, wave.t)
    # elements 0 (left) and 1 (right) share x = 1/2: nodes (N, j) of 0, (0, j) of 1
    left = np.array([u[0, leaf.flat(N, N, j)] for j in range(1, N)])
    right = np.array([u[1, leaf.flat(N, 0, j)] for j in range(1, N)])
    assert np.abs(left - right).max() < 1e-4 * np.abs(left).max()
    assert np.allclose(X[0, [leaf.flat(N, N, j) for j in range(1, N)]],
                       X[1, [leaf.flat(N, 0, j) for j in range(1, N)]])
