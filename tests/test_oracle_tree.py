"""Pins of the oracle's merge hierarchy (Sec. 4.1, Sec. 4.2, Fig. 1).

* exact polynomial reproduction by every box map at every level (pins the
  anti-diagonal C and the "+" of T_pair, and the merged-box side order);
* M_{l+1} equals the Schur complement D_l - C_l A_l^-1 B_l of M_l (Sec. 4.2);
* Schur associativity: a level-3 box map built by two successive merges equals
  the one-shot elimination of all of its internal faces from M_1;
* the face-block sparsity of M_1..M_4 on the 4x4 mesh equals Fig. 1.
"""
import os

import numpy as np
import pytest

from oracle import gll, leaf, mesh, merge, skeleton, multigrid
from tests.manufactured import PolySolution

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig1_sparsity.txt")


def build_leaves(n, N, kappa, b_fn, s_fn=None):
    xi = gll.gll_nodes(N)
    c = leaf.nodal_coefficient(N, n, kappa, b_fn, xi)
    s = None
    if s_fn is not None:
        X, Y = mesh.element_node_coords(n, N, xi)
        s = s_fn(X, Y).reshape(n * n, -1)
    T, H = leaf.leaves(N, 1.0 / n, kappa, kappa, c, s)
    return xi, T, H


def test_level_geometry():
    assert mesh.lmax(64) == 12 and mesh.lmax(4) == 4
    assert mesh.box_dims(1) == (1, 1) and mesh.box_dims(2) == (2, 1)
    assert mesh.box_dims(3) == (2, 2) and mesh.box_dims(12) == (64, 32)
    p = 15
    assert mesh.box_perimeter(11, p) == 1920 and mesh.box_perimeter(12, p) == 2880
    assert len(mesh.pairs(64, 1)) == 2048 and len(mesh.pairs(64, 11)) == 2
    assert len(mesh.interior_slots(4, 3, 1)) == 4 * 3 * 4 * 3     # 4(N-1) n (n-1)
    assert len(mesh.interior_slots(4, 3, 4)) == 2 * 4 * 3          # top interface, both sides


@pytest.mark.parametrize("n,N", [(4, 5), (2, 6)])
def test_every_box_reproduces_polynomial(n, N):
    kappa = 6.0
    u = PolySolution(N, seed=3, x0=0.4, y0=0.55)
    bfn = lambda x, y: 0.3 * np.sin(4 * x) * np.cos(3 * y)
    cfn = lambda x, y: kappa ** 2 * (1 - bfn(x, y))
    xi, T, H = build_leaves(n, N, kappa, bfn, u.source(cfn))
    p = N - 1
    Tl, Hl = merge.build_hierarchy(n, p, T, H)
    xs, ys, nx, ny = mesh.canonical_slot_coords(n, N, xi)
    gx, gy = u.grad(xs, ys)
    dn = gx * nx + gy * ny
    f = dn + 1j * kappa * u.u(xs, ys)
    o = -(dn - 1j * kappa * u.u(xs, ys))
    for level in range(1, mesh.lmax(n) + 1):
        for (bx, by), Tb in Tl[level - 1].items():
            sl = mesh.box_slots(n, p, level, bx, by)
            lhs = Tb @ f[sl] + Hl[level - 1][(bx, by)]
            np.testing.assert_allclose(lhs, o[sl], atol=1e-9 * np.abs(o).max(),
                                       err_msg=f"level {level} box {(bx, by)}")


def test_next_level_is_schur_complement():
    n, N, kappa = 4, 4, 8.0
    _, T, _ = build_leaves(n, N, kappa, lambda x, y: 0.5 * np.exp(-((x - .3) ** 2 + (y - .6) ** 2) / .05))
    hier = multigrid.Hierarchy(n, N - 1, T)
    for level in range(1, hier.L):
        A, B, C, D = [b.toarray() for b in hier.blocks(level)]
        S = D - C @ np.linalg.solve(A, B)
        ref = hier.M[level + 1].toarray()
        assert np.abs(S - ref).max() < 1e-12 * np.abs(ref).max()


def test_schur_associativity_one_shot():
    """Level-3 (2x2-element) box map from two merges == one-shot elimination."""
    n, N, kappa = 8, 4, 9.0
    p = N - 1
    _, T, _ = build_leaves(n, N, kappa, lambda x, y: 0.4 * np.sin(5 * x * y))
    Tl, _ = merge.build_hierarchy(n, p, T, None, top=3)
    M1, unk = skeleton.assemble(n, p, 1, skeleton.leaf_boxT(n, T))
    M1 = M1.toarray()
    where = {s: i for i, s in enumerate(unk)}
    partner = mesh.slot_partner(n, p)
    bx, by = 1, 1                                   # an interior 2x2 box
    bnd = mesh.box_slots(n, p, 3, bx, by)
    elems = [mesh.element_of(n, 2 * bx + a, 2 * by + c) for c in range(2) for a in range(2)]
    own = np.concatenate([np.arange(e * 4 * p, (e + 1) * 4 * p) for e in elems])
    internal = np.setdiff1d(own, bnd)
    ii = [where[s] for s in internal]
    ib = [where[s] for s in bnd]
    io = [where[partner[s]] for s in bnd]
    A = M1[np.ix_(ii, ii)]
    B = -M1[np.ix_(ii, ib)]
    C = -M1[np.ix_(io, ii)]
    D = -M1[np.ix_(io, ib)]
    one_shot = D + C @ np.linalg.solve(A, B)
    np.testing.assert_allclose(Tl[2][(bx, by)], one_shot, atol=1e-12)


def parse_golden():
    grids, cur = {}, None
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        tok = line.split()
        if tok[0] == "grid":
            cur = grids.setdefault(int(tok[1]), {})
        elif tok[0] == "faces":
            cur["faces"] = [tuple(int(v) for v in f.split("-")) for f in tok[1:]]
        elif tok[0] == "group":
            cur["group"] = int(tok[1])
        else:
            r, c = int(tok[1]), int(tok[2])
            blk = np.zeros((r, c), dtype=bool)
            for cell in tok[3:]:
                i, j = (int(v) for v in cell.split("/"))
                blk[i - 1, j - 1] = True
            cur[tok[0]] = blk
    return grids


def face_slots(n, p, e1, e2):
    e1, e2 = e1 - 1, e2 - 1
    if e2 == e1 + 1:
        s1, s2 = mesh.R_, mesh.L_
    elif e2 == e1 + n:
        s1, s2 = mesh.T_, mesh.B_
    else:
        raise ValueError((e1, e2))
    return ([mesh.slot(n, p, e1, s1, k) for k in range(p)]
            + [mesh.slot(n, p, e2, s2, k) for k in range(p)])


def test_fig1_sparsity_patterns():
    n, N, kappa = 4, 3, 5.0
    p = N - 1
    _, T, _ = build_leaves(n, N, kappa, lambda x, y: 0.2 + 0.1 * x * y)
    hier = multigrid.Hierarchy(n, p, T)
    for level, g in parse_golden().items():
        printed = np.block([[g["A"], g["B"]], [g["C"], g["D"]]])
        M = hier.M[level].toarray()
        where = {s: i for i, s in enumerate(hier.unk[level])}
        faces = [[where[s] for s in face_slots(n, p, *f)] for f in g["faces"]]
        assert sorted(sum(faces, [])) == list(range(len(hier.unk[level]))), level
        gs = g["group"]
        groups = [sum(faces[i:i + gs], []) for i in range(0, len(faces), gs)]
        got = np.array([[np.abs(M[np.ix_(a, b)]).max() > 0 for b in groups] for a in groups])
        np.testing.assert_array_equal(got, printed, err_msg=f"M_{level}")
        if level < hier.L:
            xi, _ = hier.split[level]
            na = g["A"].shape[0] * gs
            assert sorted(sum(faces[:na], [])) == sorted(xi.tolist()), f"F_{level}"
