"""Leaf (element) impedance-to-impedance map (Sec. 3.1, eq. ItIOperator).

Per element of side h with GLL order N (paper, Sec. 3.1):

* physical 1D operators D_x = (2/h) D, M_x = (h/2) diag(w), K_x = D_x^T M_x D_x
  (the paper writes D and w without the element scaling; reading: physical);
* local operator  Lt = K_x (x) M_y + M_x (x) K_y - diag(c) (M_x (x) M_y),
  c = kappa^2 (1 - b).  The paper prints "+ diag(c)"; with K = D^T M D standing
  for -Laplace, the equation -Lap u - c u = s needs the minus sign (reading);
* the four corner nodes are removed;
* the normal-derivative rows N_G = [-D_x(x)I; D_x(x)I; -I(x)D_y; I(x)D_y] on
  l, r, b, t; incoming impedance I_i = N_G + i eta E_G, outgoing
  I_o = -(N_G - i eta E_G).  The paper prints "-/+ eta I" without the
  imaginary unit and without the leading minus of I_o; both are readings: the
  impedance condition is d_n u + i eta u, and the minus makes the printed
  transmission condition I_i u^(2) = I_o u^(1) hold for a continuous field;
* L = Lt with the boundary rows replaced by I_i;
* T = I_o L^-1 I(:, iota_G),  H = I_o L^-1 I(:, iota_i) bt(iota_i), where the
  local right-hand side is bt = (M_x (x) M_y) s at the interior nodes (reading).

The solve is LAPACK's LU with partial pivoting (numpy.linalg.solve).

Test infrastructure only (see the package docstring).
"""
import numpy as np

from . import mesh
from .gll import gll
from .mesh import L_, R_, B_, T_


def flat(N, i, j):
    return i * (N + 1) + j


def index_sets(N):
    """Non-corner node list (flat order without corners) and the positions of
    iota_l, iota_r, iota_b, iota_t, iota_G and iota_i inside it."""
    corners = {flat(N, 0, 0), flat(N, 0, N), flat(N, N, 0), flat(N, N, N)}
    keep = [f for f in range((N + 1) ** 2) if f not in corners]
    pos = {f: k for k, f in enumerate(keep)}
    k = range(1, N)
    il = [pos[flat(N, 0, j)] for j in k]
    ir = [pos[flat(N, N, j)] for j in k]
    ib = [pos[flat(N, i, 0)] for i in k]
    it = [pos[flat(N, i, N)] for i in k]
    ii = [pos[flat(N, i, j)] for i in k for j in k]
    sides = {L_: il, R_: ir, B_: ib, T_: it}
    return (np.array(keep), {s: np.array(v) for s, v in sides.items()},
            np.array(il + ir + ib + it), np.array(ii))


def element_1d(N, h):
    xi, w, D = gll(N)
    Dx = (2.0 / h) * D
    Mx = (h / 2.0) * np.diag(w)
    Kx = Dx.T @ Mx @ Dx
    return xi, w, Dx, Mx, Kx


def local_operator(N, h, c):
    """Full (N+1)^2 element operator Lt for nodal coefficient c (flat order)."""
    _, _, Dx, Mx, Kx = element_1d(N, h)
    return np.kron(Kx, Mx) + np.kron(Mx, Kx) - np.diag(c) @ np.kron(Mx, Mx)


def normal_rows(N, h):
    """N_G restricted to the non-corner columns: (4(N-1)) x n_loc, real."""
    _, _, Dx, _, _ = element_1d(N, h)
    I = np.eye(N + 1)
    Gx = np.kron(Dx, I)   # (D_x (x) I)[(i,j),(i',j')] = D_x[i,i'] delta_jj'
    Gy = np.kron(I, Dx)   # (I (x) D_y)
    keep, _, _, _ = index_sets(N)
    k = range(1, N)
    rows = ([-Gx[flat(N, 0, j)] for j in k] + [Gx[flat(N, N, j)] for j in k]
            + [-Gy[flat(N, i, 0)] for i in k] + [Gy[flat(N, i, N)] for i in k])
    return np.array(rows)[:, keep]


def impedance_ops(N, h, eta):
    """(I_i, I_o) as 4(N-1) x n_loc complex matrices."""
    keep, _, iG, _ = index_sets(N)
    NG = normal_rows(N, h)
    EG = np.eye(len(keep))[iG]
    Ii = NG + 1j * eta * EG
    Io = -(NG - 1j * eta * EG)
    return Ii, Io


def leaf_system(N, h, eta, c):
    """The element matrix L (complex n_loc x n_loc) of Sec. 3.1."""
    keep, _, iG, _ = index_sets(N)
    Lt = local_operator(N, h, c)[np.ix_(keep, keep)].astype(complex)
    Ii, _ = impedance_ops(N, h, eta)
    Lt[iG, :] = Ii
    return Lt


def leaf_itI(N, h, kappa, eta, c, s=None):
    """ItI map T (4p x 4p) and load H (4p) of one element.

    c: nodal coefficient kappa^2 (1 - b) in flat order, length (N+1)^2.
    s: nodal source (flat order, complex) or None (H = 0)."""
    keep, _, iG, ii = index_sets(N)
    nloc = len(keep)
    L = leaf_system(N, h, eta, c)
    _, Io = impedance_ops(N, h, eta)
    _, w, _, _, _ = element_1d(N, h)
    rhs = np.zeros((nloc, len(iG) + 1), dtype=complex)
    rhs[iG, np.arange(len(iG))] = 1.0
    if s is not None:
        bt = (h / 2.0) ** 2 * np.outer(w, w).ravel() * np.asarray(s)   # (M (x) M) s
        rhs[ii, len(iG)] = bt[keep][ii]
    X = np.linalg.solve(L, rhs)
    T = Io @ X[:, :len(iG)]
    H = Io @ X[:, len(iG)]
    return T, H


def leaves(N, h, kappa, eta, c_all, s_all=None, chunk=256):
    """leaf_itI for every element.  c_all: [E, (N+1)^2]; s_all: [E, (N+1)^2] or
    None.  Returns T [E, 4p, 4p], H [E, 4p].  Same steps as leaf_itI, stacked."""
    keep, _, iG, ii = index_sets(N)
    nloc, nG = len(keep), len(iG)
    E = c_all.shape[0]
    _, w, _, Mx, _ = element_1d(N, h)
    base = leaf_system(N, h, eta, np.zeros((N + 1) ** 2))
    mm = np.kron(np.diag(Mx), np.diag(Mx))[keep]       # diagonal of M (x) M
    _, Io = impedance_ops(N, h, eta)
    interior_row = np.zeros(nloc, dtype=bool)
    interior_row[ii] = True
    T = np.empty((E, nG, nG), dtype=complex)
    H = np.zeros((E, nG), dtype=complex)
    for a in range(0, E, chunk):
        cb = np.asarray(c_all[a:a + chunk])[:, keep]
        nb = cb.shape[0]
        Lb = np.repeat(base[None], nb, axis=0)
        d = np.where(interior_row[None, :], -cb * mm[None, :], 0.0)
        idx = np.arange(nloc)
        Lb[:, idx, idx] += d
        rhs = np.zeros((nb, nloc, nG + 1), dtype=complex)
        rhs[:, iG, np.arange(nG)] = 1.0
        if s_all is not None:
            sb = np.asarray(s_all[a:a + chunk])[:, keep]
            bt = (h / 2.0) ** 2 * np.kron(w, w)[keep][None, :] * sb
            rhs[:, ii, nG] = bt[:, ii]
        X = np.linalg.solve(Lb, rhs)
        Y = Io[None] @ X
        T[a:a + nb] = Y[:, :, :nG]
        H[a:a + nb] = Y[:, :, nG]
    return T, H


def nodal_coefficient(N, n, kappa, b_fn, xi):
    """c = kappa^2 (1 - b) at every element node, [E, (N+1)^2] flat order."""
    from .mesh import element_node_coords
    X, Y = element_node_coords(n, N, xi)
    b = b_fn(X, Y)
    return (kappa ** 2 * (1.0 - b)).reshape(mesh.num_elements(n), (N + 1) ** 2)
