"""Pair merge and the merge hierarchy (Sec. 4.1, Sec. 4.2).

For a pair (P, Q) sharing side alpha of P and side beta of Q, with
x = [f^Q_beta; f^P_alpha] (eliminated) and y = [f^P_E1; f^Q_E2] (kept), the
local face system of Sec. 4.1 reads A x = B y + h with

    A = [[I, -T^P_aa], [-T^Q_bb, I]],  B = blkdiag(T^P_aE1, T^Q_bE2),
    h = [H^P_a; H^Q_b].

The outgoing data on the kept sides are g = D y + Ct x + [H^P_E1; H^Q_E2] with
D = blkdiag(T^P_E1E1, T^Q_E2E2) and Ct = [[0, T^P_E1a], [T^Q_E2b, 0]].
Substituting x = A^-1 (B y + h):

    T_pair = D + Ct A^-1 B,     H_pair = [H^P_E1; H^Q_E2] + Ct A^-1 h.

Two readings of garbled passages are taken here: Ct is block anti-diagonal (the
printed block-diagonal C does not match the order of x), and T_pair carries
"+ Ct A^-1 B" (the printed "D - C A^-1 B" holds only for the M-signed
C_M = -Ct, which the printed H_pair does not use).  Both are pinned by the
polynomial-reproduction and Schur-complement tests.

The merged box's sides are [l; r; b; t], each the concatenation of its
children's edges by increasing coordinate.

Test infrastructure only (see the package docstring).
"""
import numpy as np

from . import mesh
from .mesh import L_, R_, B_, T_


def _ranges(level, p, n=None):
    off = mesh.side_offsets(level, p, n)
    return {s: np.arange(off[s], off[s + 1]) for s in range(4)}


def pair_blocks(level, p, TP, TQ, HP=None, HQ=None, n=None):
    """The blocks A, B, Ct, D, h of one pair and the index bookkeeping (n: the
    mesh, needed only on rectangular meshes)."""
    rg = _ranges(level, p, n)
    if mesh.merge_axis(level, n) == "x":
        a, b = R_, L_
    else:
        a, b = T_, B_
    ia, ib = rg[a], rg[b]
    E1 = np.concatenate([rg[s] for s in range(4) if s != a])
    E2 = np.concatenate([rg[s] for s in range(4) if s != b])
    m = len(ia)
    e1, e2 = len(E1), len(E2)
    A = np.block([[np.eye(m), -TP[np.ix_(ia, ia)]],
                  [-TQ[np.ix_(ib, ib)], np.eye(m)]])
    Bm = np.zeros((2 * m, e1 + e2), dtype=complex)
    Bm[:m, :e1] = TP[np.ix_(ia, E1)]
    Bm[m:, e1:] = TQ[np.ix_(ib, E2)]
    Ct = np.zeros((e1 + e2, 2 * m), dtype=complex)
    Ct[:e1, m:] = TP[np.ix_(E1, ia)]
    Ct[e1:, :m] = TQ[np.ix_(E2, ib)]
    D = np.zeros((e1 + e2, e1 + e2), dtype=complex)
    D[:e1, :e1] = TP[np.ix_(E1, E1)]
    D[e1:, e1:] = TQ[np.ix_(E2, E2)]
    h = hE = None
    if HP is not None:
        h = np.concatenate([HP[ia], HQ[ib]])
        hE = np.concatenate([HP[E1], HQ[E2]])
    return dict(A=A, B=Bm, Ct=Ct, D=D, h=h, hE=hE, ia=ia, ib=ib, E1=E1, E2=E2, m=m)


def merged_order(level, p, n=None):
    """perm such that T_merged = T_pair[perm][:, perm] (y order -> [l;r;b;t])."""
    wx, wy = mesh.box_dims(level, n)
    # children's exterior sides in y order, with their lengths
    if mesh.merge_axis(level, n) == "x":
        # y = [P.l, P.b, P.t, Q.r, Q.b, Q.t]; merged l=P.l, r=Q.r, b=[P.b,Q.b], t=[P.t,Q.t]
        segs = ["Pl", "Pb", "Pt", "Qr", "Qb", "Qt"]
        lens = [wy * p, wx * p, wx * p, wy * p, wx * p, wx * p]
        target = ["Pl", "Qr", "Pb", "Qb", "Pt", "Qt"]
    else:
        # y = [P.l, P.r, P.b, Q.l, Q.r, Q.t]; merged l=[P.l,Q.l], r=[P.r,Q.r], b=P.b, t=Q.t
        segs = ["Pl", "Pr", "Pb", "Ql", "Qr", "Qt"]
        lens = [wy * p, wy * p, wx * p, wy * p, wy * p, wx * p]
        target = ["Pl", "Ql", "Pr", "Qr", "Pb", "Qt"]
    start = dict(zip(segs, np.concatenate([[0], np.cumsum(lens)[:-1]])))
    ln = dict(zip(segs, lens))
    return np.concatenate([np.arange(start[s], start[s] + ln[s]) for s in target])


def merge_pair(level, p, TP, TQ, HP=None, HQ=None, n=None):
    """(T_merged, H_merged, blocks) for one pair at merge `level`."""
    blk = pair_blocks(level, p, TP, TQ, HP, HQ, n)
    X = np.linalg.solve(blk["A"], blk["B"])
    Tpair = blk["D"] + blk["Ct"] @ X
    Hpair = None
    if HP is not None:
        Hpair = blk["hE"] + blk["Ct"] @ np.linalg.solve(blk["A"], blk["h"])
    perm = merged_order(level, p, n)
    Tm = Tpair[np.ix_(perm, perm)]
    Hm = None if Hpair is None else Hpair[perm]
    return Tm, Hm, blk


def build_hierarchy(n, p, leafT, leafH=None, top=None):
    """Box maps for levels 1..top (default L_max): list index level-1 of dicts
    (bx, by) -> T (and H if leafH is given).  Merge l produces level l+1."""
    Lm = mesh.lmax(n)
    top = Lm if top is None else top
    nx = mesh.dims(n)[0]
    E = mesh.num_elements(n)
    T = [{(e % nx, e // nx): leafT[e] for e in range(E)}]
    H = [None if leafH is None else {(e % nx, e // nx): leafH[e] for e in range(E)}]
    for level in range(1, top):
        Tn, Hn = {}, ({} if leafH is not None else None)
        for (P, Q, Mb) in mesh.pairs(n, level):
            HP = HQ = None
            if leafH is not None:
                HP, HQ = H[-1][P], H[-1][Q]
            Tm, Hm, _ = merge_pair(level, p, T[-1][P], T[-1][Q], HP, HQ, n)
            Tn[Mb] = Tm
            if Hn is not None:
                Hn[Mb] = Hm
        T.append(Tn)
        H.append(Hn)
    return T, H
