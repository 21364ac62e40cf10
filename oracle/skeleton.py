"""Skeleton (trace) system M g = RHS (Sec. 3.2, eq. faceequations).

Unknowns are the incoming impedances on interior sides.  For a node of the
face shared by boxes B (side gamma) and B' (side gamma'), the transmission
condition of Sec. 3.2 states: incoming data of B' at that node equals the
outgoing data of B,

    f_{B', gamma'} - sum_nu T^B_{gamma nu} f_{B, nu} = H^B_gamma
                      + sum_{nu physical} T^B_{gamma nu} t_{B, nu}.

The row of this equation is stored at the slot of the unknown it determines
(B', gamma'), so in canonical slot order M = I - Pi T_blk; this is the paper's
face system with the rows ordered like the unknowns, as in eq. faceequations.
Physical-side incoming data t are moved to the right-hand side.  The same
assembly applied to the level-l boxes gives M_l (Sec. 4.2).

Test infrastructure only (see the package docstring).
"""
import numpy as np
import scipy.sparse as sp

from . import mesh


def assemble(n, p, level, boxT):
    """Sparse M_level over `mesh.interior_slots(n, p, level)` (sorted slots).

    boxT: dict (bx, by) -> box ItI map in box-local [l; r; b; t] order."""
    unk = mesh.interior_slots(n, p, level)
    where = -np.ones(mesh.num_elements(n) * 4 * p, dtype=np.int64)
    where[unk] = np.arange(len(unk))
    partner = mesh.slot_partner(n, p)
    rows, cols, vals = [list(range(len(unk)))], [list(range(len(unk)))], [np.ones(len(unk))]
    nbx, nby = mesh.box_grid(n, level)
    for by in range(nby):
        for bx in range(nbx):
            T = boxT[(bx, by)]
            sl = mesh.box_slots(n, p, level, bx, by)
            phys = mesh.box_local_physical_mask(n, p, level, bx, by)
            inn = np.nonzero(~phys)[0]
            for a in inn:
                r = where[partner[sl[a]]]
                rows.append(np.full(len(inn), r))
                cols.append(where[sl[inn]])
                vals.append(-T[a, inn])
    rows = np.concatenate([np.asarray(r) for r in rows])
    cols = np.concatenate([np.asarray(c) for c in cols])
    vals = np.concatenate([np.asarray(v) for v in vals])
    M = sp.csr_matrix((vals, (rows, cols)), shape=(len(unk), len(unk)), dtype=complex)
    return M, unk


def rhs(n, p, leafT, leafH, t_slots):
    """Level-1 right-hand side in canonical slot layout (physical slots 0).

    leafT [E, 4p, 4p], leafH [E, 4p]; t_slots: incoming data t at every
    canonical slot (only physical slots are read)."""
    E = mesh.num_elements(n)
    phys = mesh.physical_slot_mask(n, p)
    partner = mesh.slot_partner(n, p)
    out = np.zeros(E * 4 * p, dtype=complex)
    tp = np.where(phys, t_slots, 0.0)
    for e in range(E):
        sl = np.arange(e * 4 * p, (e + 1) * 4 * p)
        o = leafH[e] + leafT[e] @ tp[sl]       # outgoing data of e driven by H and t
        for a in range(4 * p):
            if not phys[sl[a]]:
                out[partner[sl[a]]] = o[a]
    return out


def leaf_boxT(n, leafT):
    """Level-1 boxes are the elements; box-local order equals the element's."""
    nx = mesh.dims(n)[0]
    return {(e % nx, e // nx): leafT[e] for e in range(mesh.num_elements(n))}


def apply(n, p, level, boxT, g):
    """(M_level g) in canonical layout, by the assembled sparse matrix."""
    M, unk = assemble(n, p, level, boxT)
    out = np.zeros_like(g, dtype=complex)
    out[unk] = M @ g[unk]
    return out
