"""Direct HPS with an exact coarse space (Sec. 4.2; Table 1 "Exact coarse space").

Upward pass: the merge hierarchy of `merge.build_hierarchy` (with loads H).
Downward pass: the root box is the whole domain; all of its sides are
physical, so its incoming data are the boundary data t.  For a merged box with
known incoming data y on its sides, the pair's local face system gives the
shared-face data x = A^-1 (B y + h) (Sec. 4.1, eq. localfacesystem), which
completes the incoming data of both children.  Recursing to the leaves yields
every element's incoming impedances; g is their restriction to interior sides.

Test infrastructure only (see the package docstring).
"""
import numpy as np

from . import mesh
from .merge import build_hierarchy, merge_pair, merged_order


def solve(n, p, leafT, leafH, t_slots, hierarchy=None):
    """g in canonical slot layout (physical slots 0) by direct HPS.

    hierarchy: the (T, H) that build_hierarchy(n, p, leafT, leafH) returns,
    when the caller has already built it (it is not rebuilt then)."""
    Lm = mesh.lmax(n)
    if hierarchy is None:
        hierarchy = build_hierarchy(n, p, leafT, leafH, top=Lm)
    T, H = hierarchy
    root = mesh.box_slots(n, p, Lm + 1, 0, 0)
    incoming = {(0, 0): t_slots[root]}
    for level in range(Lm, 0, -1):
        nxt = {}
        perm = merged_order(level, p, n)
        for (P, Q, Mb) in mesh.pairs(n, level):
            _, _, blk = merge_pair(level, p, T[level - 1][P], T[level - 1][Q],
                                   H[level - 1][P], H[level - 1][Q], n)
            y = np.empty(len(perm), dtype=complex)
            y[perm] = incoming[Mb]
            x = np.linalg.solve(blk["A"], blk["B"] @ y + blk["h"])
            m, e1 = blk["m"], len(blk["E1"])
            bsize = T[level - 1][P].shape[0]
            fP = np.empty(bsize, dtype=complex)
            fQ = np.empty(bsize, dtype=complex)
            fP[blk["E1"]] = y[:e1]
            fP[blk["ia"]] = x[m:]
            fQ[blk["E2"]] = y[e1:]
            fQ[blk["ib"]] = x[:m]
            nxt[P], nxt[Q] = fP, fQ
        incoming = nxt
    g = np.zeros(mesh.num_elements(n) * 4 * p, dtype=complex)
    for (bx, by), f in incoming.items():
        e = mesh.element_of(n, bx, by)
        g[e * 4 * p:(e + 1) * 4 * p] = f
    g[mesh.physical_slot_mask(n, p)] = 0.0
    return g
