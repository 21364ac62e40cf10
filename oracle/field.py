"""Interior field recovery (Sec. 3.1) and the corner values (a reading).

Once the skeleton unknowns g are known, every element's incoming impedance
data f on its four sides are known too: g on interior sides, the boundary
data t on physical sides.  The element's nodal field u then solves its local
system of Sec. 3.1, the interior rows of the local operator with the load bt
and the boundary rows replaced by the incoming impedance operator:

    L u = [bt on the interior nodes; f on the boundary nodes],

which determines u at every node except the four corners (they carry no
unknown: the paper removes them).  The paper does not say how a corner value
is obtained; the reading taken here: along each of the two sides meeting at
the corner, the polynomial of degree N-2 through the side's N-1 nodal values
is evaluated at the corner, and the corner value is the mean of the two.  It
is exact whenever u restricted to those sides has degree <= N-2.

Test infrastructure only (see the package docstring).
"""
import numpy as np

from . import mesh
from .gll import gll
from .leaf import element_1d, flat, index_sets, leaf_system


def _extrapolate(xs, vals, x):
    """Value at x of the polynomial through (xs, vals) (Lagrange form)."""
    out = 0.0
    for k, xk in enumerate(xs):
        others = np.delete(xs, k)
        out = out + vals[k] * np.prod((x - others) / (xk - others))
    return out


def element_field(N, h, eta, c, s, f):
    """u at the (N+1)^2 nodes (flat order) of one element.
    c: nodal coefficient kappa^2 (1 - b); s: nodal source or None; f: the
    4(N-1) incoming impedances in [l; r; b; t] order."""
    keep, _, iG, ii = index_sets(N)
    L = leaf_system(N, h, eta, c)
    _, w, _, _, _ = element_1d(N, h)
    rhs = np.zeros(len(keep), dtype=complex)
    rhs[iG] = f
    if s is not None:
        bt = (h / 2.0) ** 2 * np.outer(w, w).ravel() * np.asarray(s)   # (M (x) M) s
        rhs[ii] = bt[keep][ii]
    u = np.zeros((N + 1) ** 2, dtype=complex)
    u[keep] = np.linalg.solve(L, rhs)
    xi = gll(N)[0]
    inner = xi[1:N]
    for i, j in ((0, 0), (0, N), (N, 0), (N, N)):
        along_y = _extrapolate(inner, np.array([u[flat(N, i, jj)] for jj in range(1, N)]), xi[j])
        along_x = _extrapolate(inner, np.array([u[flat(N, ii_, j)] for ii_ in range(1, N)]), xi[i])
        u[flat(N, i, j)] = 0.5 * (along_y + along_x)
    return u


def fields(n, N, eta, c_all, s_all, g, t_slots):
    """u [E, (N+1)^2] of every element from the skeleton solution g and the
    boundary data t (both canonical vectors; t read on physical slots only)."""
    p = N - 1
    phys = mesh.physical_slot_mask(n, p)
    inc = np.where(phys, t_slots, g)
    E = mesh.num_elements(n)
    out = np.empty((E, (N + 1) ** 2), dtype=complex)
    for e in range(E):
        f = inc[e * 4 * p:(e + 1) * 4 * p]
        out[e] = element_field(N, mesh.element_size(n), eta, c_all[e], None if s_all is None else s_all[e], f)
    return out
