"""Pins of the oracle's gamma-cycle (Sec. 4.3: "multiple coarse calls define a
gamma-cycle"; the reading taken is a stationary iteration on the coarse system,
y <- y + MG_{l+1}(r~ - M_{l+1} y), gamma times per level).

* With an exact coarse solve every level's MG is exact, so the gamma-cycle is
  M_1^-1 for any gamma (block-inverse identity of Sec. 4.3).
* With a k-step GMRES coarse solve the result is checked against a brute force
  built from different parts than the oracle's: dense Schur complements of the
  dense M_1 (instead of the merged box maps and sparse LU), the level split
  taken from the geometry's unknown sets, and the k-step GMRES iterate as the
  Krylov least-squares solution by QR (instead of Arnoldi).  Properties that
  hold whatever the iterate: the eliminated-face rows of M_1 z reproduce r
  exactly, and each extra coarse call cannot increase the coarse residual.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle import gll, leaf, mesh, skeleton, multigrid


def _leaves(n, N, kappa):
    xi = gll.gll_nodes(N)
    bfn = lambda x, y: 0.5 * np.exp(-((x - .35) ** 2 + (y - .6) ** 2) / .05) - 0.2 * x
    c = leaf.nodal_coefficient(N, n, kappa, bfn, xi)
    T, _ = leaf.leaves(N, 1.0 / n, kappa, kappa, c)
    return T


def _rand(m, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(m) + 1j * rng.standard_normal(m)


def _krylov_ls(S, r, k):
    """argmin ||r - S x|| over x in span{r, S r, ..., S^(k-1) r}, by QR."""
    if np.linalg.norm(r) == 0:
        return np.zeros_like(r)
    K = np.stack([np.linalg.matrix_power(S, j) @ r for j in range(k)], 1)
    Q, _ = np.linalg.qr(K)
    y, *_ = np.linalg.lstsq(S @ Q, r, rcond=None)
    return Q @ y


def _dense_levels(n, p, T, L):
    """Dense M_l for l = 1..L as successive Schur complements of the dense M_1,
    each indexed by the sorted level-l unknown slots."""
    M1, unk1 = skeleton.assemble(n, p, 1, skeleton.leaf_boxT(n, T))
    Ms, unks, splits = {1: M1.toarray()}, {1: unk1}, {}
    for level in range(1, L):
        unk, nxt = unks[level], mesh.interior_slots(n, p, level + 1)
        pos = {s: i for i, s in enumerate(unk)}
        yi = np.array([pos[s] for s in nxt])
        xi = np.array(sorted(set(range(len(unk))) - set(yi.tolist())))
        M = Ms[level]
        A, B = M[np.ix_(xi, xi)], M[np.ix_(xi, yi)]
        C, D = M[np.ix_(yi, xi)], M[np.ix_(yi, yi)]
        Ms[level + 1] = D - C @ np.linalg.solve(A, B)
        unks[level + 1] = nxt
        splits[level] = (xi, yi, A, B, C)
    return Ms, unks, splits


def _mg_brute(level, r, Ms, splits, L, k, gamma):
    if level == L:
        return _krylov_ls(Ms[L], r, k)
    xi, yi, A, B, C = splits[level]
    zx0 = np.linalg.solve(A, r[xi])
    rt = r[yi] - C @ zx0
    y = np.zeros(len(yi), dtype=complex)
    for _ in range(gamma):
        y = y + _mg_brute(level + 1, rt - Ms[level + 1] @ y, Ms, splits, L, k, gamma)
    z = np.empty(len(r), dtype=complex)
    z[xi] = zx0 - np.linalg.solve(A, B @ y)
    z[yi] = y
    return z


@pytest.mark.parametrize("levels,gamma", [(2, 2), (3, 2), (4, 3)])
def test_gamma_cycle_with_exact_coarse_is_inverse(levels, gamma):
    n, N = 4, 4
    T = _leaves(n, N, 8.0)
    hier = multigrid.Hierarchy(n, N - 1, T, levels=levels)
    M1, unk = hier.M[1], hier.unk[1]
    r = np.zeros(n * n * 4 * (N - 1), dtype=complex)
    r[unk] = _rand(len(unk), levels)
    z = hier.apply(r, None, gamma=gamma)
    ref = spla.spsolve(M1.tocsc(), r[unk])
    assert np.linalg.norm(z[unk] - ref) / np.linalg.norm(ref) < 1e-12


@pytest.mark.parametrize("levels,k,gamma", [(2, 2, 2), (3, 2, 2), (3, 3, 3), (4, 2, 2), (3, 2, 1)])
def test_gamma_cycle_matches_dense_brute_force(levels, k, gamma):
    n, N = 4, 4
    p = N - 1
    T = _leaves(n, N, 9.0)
    hier = multigrid.Hierarchy(n, p, T, levels=levels)
    Ms, unks, splits = _dense_levels(n, p, T, levels)
    r = _rand(len(unks[1]), 10 * levels + k)
    rc = np.zeros(n * n * 4 * p, dtype=complex)
    rc[unks[1]] = r
    z = hier.apply(rc, k, gamma=gamma)[unks[1]]
    zb = _mg_brute(1, r, Ms, splits, levels, k, gamma)
    assert np.linalg.norm(z - zb) / np.linalg.norm(zb) < 1e-10
    # the eliminated faces' rows of M_1 z reproduce r exactly (P and F of the
    # block-inverse identity), whatever the coarse iterate
    xi = splits[1][0]
    Mz = Ms[1] @ z
    assert np.linalg.norm(Mz[xi] - r[xi]) < 1e-11 * np.linalg.norm(r)


def test_more_coarse_calls_do_not_increase_coarse_residual():
    """Two levels: the coarse residual r~ - S y after gamma calls of k-step
    GMRES (each a minimal-residual correction from a space containing 0) is
    non-increasing in gamma."""
    n, N, k = 4, 4, 2
    p = N - 1
    T = _leaves(n, N, 7.0)
    Ms, unks, splits = _dense_levels(n, p, T, 2)
    hier = multigrid.Hierarchy(n, p, T, levels=2)
    xi, yi, A, B, C = splits[1]
    r = _rand(len(unks[1]), 3)
    rt = r[yi] - C @ np.linalg.solve(A, r[xi])
    rc = np.zeros(n * n * 4 * p, dtype=complex)
    rc[unks[1]] = r
    prev = np.linalg.norm(rt)
    for gamma in (1, 2, 3, 4):
        y = hier.apply(rc, k, gamma=gamma)[unks[1]][yi]
        res = np.linalg.norm(rt - Ms[2] @ y)
        assert res <= prev * (1 + 1e-12), (gamma, res, prev)
        prev = res
