"""Element-DOF brute force (independent of every ItI map).

Unknowns: the nodal values u^(e) at all non-corner nodes of every element.
Equations, one per unknown:

* element-interior nodes: the interior rows of the local operator Lt
  (Sec. 3.1) with right-hand side bt = (M (x) M) s;
* a boundary node of element e on an interior side alpha, facing element e'
  on side beta: incoming data of e equals outgoing data of e' (Sec. 3.2),
  (N_G + i eta) u^(e)|_alpha + (N_G - i eta) u^(e')|_beta = 0;
* a boundary node on a physical side: (N_G + i eta) u^(e)|_alpha = t.

A dense LU solves it; g on an interior slot is (N_G + i eta) u^(e) there.
For tiny meshes only.

Test infrastructure only (see the package docstring).
"""
import numpy as np

from . import mesh
from .leaf import index_sets, local_operator, normal_rows, element_1d


def solve(n, N, kappa, eta, c_all, s_all, t_slots):
    p = N - 1
    h = mesh.element_size(n)
    E = mesh.num_elements(n)
    keep, sides, iG, ii = index_sets(N)
    nloc = len(keep)
    NG = normal_rows(N, h)                      # 4p x nloc, rows in [l;r;b;t] order
    _, w, _, _, _ = element_1d(N, h)
    nu = E * nloc
    A = np.zeros((nu, nu), dtype=complex)
    rhs = np.zeros(nu, dtype=complex)
    for e in range(E):
        base = e * nloc
        Lt = local_operator(N, h, c_all[e])[np.ix_(keep, keep)]
        for r in ii:
            A[base + r, base:base + nloc] = Lt[r]
        if s_all is not None:
            bt = (h / 2) ** 2 * np.kron(w, w)[keep] * s_all[e][keep]
            rhs[base + ii] = bt[ii]
        for s in range(4):
            nb = mesh.neighbour(n, e, s)
            for k in range(p):
                a = s * p + k                     # row index inside NG / iG
                row = base + iG[a]
                A[row, base:base + nloc] += NG[a]
                A[row, base + iG[a]] += 1j * eta
                if nb is None:
                    rhs[row] = t_slots[mesh.slot(n, p, e, s, k)]
                else:
                    e2, s2 = nb
                    b2 = e2 * nloc
                    a2 = s2 * p + k
                    A[row, b2:b2 + nloc] += NG[a2]
                    A[row, b2 + iG[a2]] -= 1j * eta
    u = np.linalg.solve(A, rhs)
    g = np.zeros(E * 4 * p, dtype=complex)
    phys = mesh.physical_slot_mask(n, p)
    for e in range(E):
        ue = u[e * nloc:(e + 1) * nloc]
        inc = NG @ ue + 1j * eta * ue[iG]
        g[e * 4 * p:(e + 1) * 4 * p] = inc
    g[phys] = 0.0
    return g, u
