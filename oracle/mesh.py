"""Mesh, side and merge-level geometry (Sec. 3, Sec. 3.2, Sec. 4.2, Fig. 1).

Conventions (the paper fixes some of them, the rest are readings):

* n x n square elements of side h = 1/n on (0,1)^2, element e = ix + n*iy
  (x fastest, as the Fig. 1 element numbering: column (e-1) mod 4, row
  floor((e-1)/4)).  A rectangular mesh of nx x ny elements (both powers of
  two; `n` given as the pair (nx, ny)) takes square elements of side
  h = 1/max(nx, ny) on (0, nx h) x (0, ny h) and e = ix + nx*iy (an extension:
  the paper's mesh is square).
* Element nodes (i, j), i the x-index, j the y-index, both 0..N; flat index
  i*(N+1) + j (x slow, matching the Kronecker order K_x (x) M_y of Sec. 3.1).
* Sides in the order l, r, b, t (Sec. 3.1); side l holds nodes (0, j),
  r (N, j), b (i, 0), t (i, N) for j or i = 1..N-1 in increasing order.  The
  corners are not unknowns.
* Canonical skeleton vector: slot (e, side, k), k = 0..N-2, flat index
  (e*4 + side)*(N-1) + k.  Physical-side slots are not unknowns.
* Merge level l (l = 1 .. L_max = log2(n^2)): boxes of level l are
  2^floor(l/2) x 2^floor((l-1)/2) elements; merge l joins pairs of level-l
  boxes along x when l is odd and along y when l is even (Fig. 1: F_1 are the
  vertical faces, Grid 2 holds 2-wide, 1-tall boxes).  On a 2^a x 2^b mesh
  (L_max = a + b) the merges alternate x, y while both directions have merges
  left (the first 2 min(a, b) levels) and then all run along the longer
  direction.  In a pair (P, Q), P is
  the left/bottom box (shared side alpha = r or t) and Q the right/top box
  (beta = l or b).
* A box's local boundary order is [l; r; b; t], each side the concatenation of
  its element edges by increasing coordinate.

Test infrastructure only (see the package docstring).
"""
import numpy as np

SIDES = ("l", "r", "b", "t")
L_, R_, B_, T_ = 0, 1, 2, 3
OPP = {L_: R_, R_: L_, B_: T_, T_: B_}


def log2i(n):
    q = int(round(np.log2(n)))
    if 2 ** q != n:
        raise ValueError("n must be a power of two")
    return q


def dims(n):
    """(nx, ny): `n` is the side of a square mesh or the pair (nx, ny)."""
    if np.isscalar(n):
        return int(n), int(n)
    return int(n[0]), int(n[1])


def num_elements(n):
    nx, ny = dims(n)
    return nx * ny


def element_size(n):
    nx, ny = dims(n)
    return 1.0 / max(nx, ny)


def lmax(n):
    nx, ny = dims(n)
    return log2i(nx) + log2i(ny)


def merge_axis(level, n=None):
    """Axis of merge `level`; n (the mesh) matters only past the alternating levels."""
    a, b = (0, 0) if n is None else (log2i(dims(n)[0]), log2i(dims(n)[1]))
    if n is None or level <= 2 * min(a, b):
        return "x" if level % 2 == 1 else "y"
    return "x" if a > b else "y"


def box_dims(level, n=None):
    """(wx, wy) in elements of a level-`level` box: 2 to the number of merges
    along x and along y among merges 1..level-1."""
    dx = sum(merge_axis(l, n) == "x" for l in range(1, level))
    return 2 ** dx, 2 ** (level - 1 - dx)


def box_grid(n, level):
    nx, ny = dims(n)
    wx, wy = box_dims(level, n)
    return nx // wx, ny // wy


def side_len(level, side, p, n=None):
    wx, wy = box_dims(level, n)
    return (wy if side in (L_, R_) else wx) * p


def box_perimeter(level, p, n=None):
    wx, wy = box_dims(level, n)
    return 2 * (wx + wy) * p


def side_offsets(level, p, n=None):
    """Start of each side in the box-local [l; r; b; t] order."""
    wx, wy = box_dims(level, n)
    lens = [wy * p, wy * p, wx * p, wx * p]
    return np.concatenate([[0], np.cumsum(lens)])


def element_of(n, ix, iy):
    return ix + dims(n)[0] * iy


def slot(n, p, e, side, k):
    return (e * 4 + side) * p + k


def neighbour(n, e, side):
    """(e', side') across `side` of element e, or None on the physical boundary."""
    nx, ny = dims(n)
    ix, iy = e % nx, e // nx
    if side == L_:
        return None if ix == 0 else (e - 1, R_)
    if side == R_:
        return None if ix == nx - 1 else (e + 1, L_)
    if side == B_:
        return None if iy == 0 else (e - nx, T_)
    return None if iy == ny - 1 else (e + nx, B_)


def box_side_slots(n, p, level, bx, by, side):
    """Canonical slots of one side of box (bx, by), increasing coordinate."""
    wx, wy = box_dims(level, n)
    out = []
    if side in (L_, R_):
        ix = bx * wx if side == L_ else bx * wx + wx - 1
        for r in range(wy):
            e = element_of(n, ix, by * wy + r)
            out.extend(slot(n, p, e, side, k) for k in range(p))
    else:
        iy = by * wy if side == B_ else by * wy + wy - 1
        for c in range(wx):
            e = element_of(n, bx * wx + c, iy)
            out.extend(slot(n, p, e, side, k) for k in range(p))
    return np.array(out, dtype=np.int64)


def box_slots(n, p, level, bx, by):
    """Canonical slots of the whole box boundary in local [l; r; b; t] order."""
    return np.concatenate([box_side_slots(n, p, level, bx, by, s) for s in range(4)])


def box_side_physical(n, level, bx, by, side):
    nbx, nby = box_grid(n, level)
    return ((side == L_ and bx == 0) or (side == R_ and bx == nbx - 1)
            or (side == B_ and by == 0) or (side == T_ and by == nby - 1))


def box_local_physical_mask(n, p, level, bx, by):
    """Boolean mask over the box-local boundary order: True on physical nodes."""
    return np.concatenate([
        np.full(side_len(level, s, p, n), box_side_physical(n, level, bx, by, s))
        for s in range(4)])


def slot_partner(n, p):
    """Array: partner[s] = slot across the face from s, -1 if s is physical."""
    E = num_elements(n)
    partner = -np.ones(E * 4 * p, dtype=np.int64)
    for e in range(E):
        for s in range(4):
            nb = neighbour(n, e, s)
            if nb is None:
                continue
            e2, s2 = nb
            for k in range(p):
                partner[slot(n, p, e, s, k)] = slot(n, p, e2, s2, k)
    return partner


def interior_slots(n, p, level):
    """Sorted canonical slots that are unknowns of the level-`level` system:
    interior (non-physical) boundary nodes of level-`level` boxes."""
    nbx, nby = box_grid(n, level)
    acc = []
    for by in range(nby):
        for bx in range(nbx):
            for s in range(4):
                if not box_side_physical(n, level, bx, by, s):
                    acc.append(box_side_slots(n, p, level, bx, by, s))
    return np.unique(np.concatenate(acc)) if acc else np.zeros(0, dtype=np.int64)


def pairs(n, level):
    """List of ((Pbx, Pby), (Qbx, Qby), (Mbx, Mby)) for merge `level`:
    P, Q in the level-`level` box grid, M the merged box at level+1."""
    nbx, nby = box_grid(n, level)
    out = []
    if merge_axis(level, n) == "x":
        for by in range(nby):
            for px in range(nbx // 2):
                out.append(((2 * px, by), (2 * px + 1, by), (px, by)))
    else:
        for py in range(nby // 2):
            for bx in range(nbx):
                out.append(((bx, 2 * py), (bx, 2 * py + 1), (bx, py)))
    return out


def element_node_coords(n, N, xi):
    """Physical node coordinates: arrays x[E, N+1, N+1], y[E, N+1, N+1]
    indexed [e, i, j] (i: x-index, j: y-index)."""
    h = element_size(n)
    nx, _ = dims(n)
    E = num_elements(n)
    ix = np.arange(E) % nx
    iy = np.arange(E) // nx
    xr = (1.0 + xi) * h / 2
    X = ix[:, None, None] * h + xr[None, :, None] + 0 * xr[None, None, :]
    Y = iy[:, None, None] * h + xr[None, None, :] + 0 * xr[None, :, None]
    return X, Y


def side_nodes_ij(N, side):
    """(i, j) index arrays of one element side's non-corner nodes."""
    k = np.arange(1, N)
    if side == L_:
        return np.zeros(N - 1, int), k
    if side == R_:
        return np.full(N - 1, N), k
    if side == B_:
        return k, np.zeros(N - 1, int)
    return k, np.full(N - 1, N)


def canonical_slot_coords(n, N, xi):
    """Coordinates (x, y) and outward normals (nx, ny) of every canonical slot."""
    p = N - 1
    X, Y = element_node_coords(n, N, xi)
    E = num_elements(n)
    xs = np.zeros(E * 4 * p)
    ys = np.zeros(E * 4 * p)
    nx = np.zeros(E * 4 * p)
    ny = np.zeros(E * 4 * p)
    normals = {L_: (-1, 0), R_: (1, 0), B_: (0, -1), T_: (0, 1)}
    for e in range(E):
        for s in range(4):
            i, j = side_nodes_ij(N, s)
            sl = slice((e * 4 + s) * p, (e * 4 + s + 1) * p)
            xs[sl] = X[e, i, j]
            ys[sl] = Y[e, i, j]
            nx[sl], ny[sl] = normals[s]
    return xs, ys, nx, ny


def physical_slot_mask(n, p):
    E = num_elements(n)
    mask = np.zeros(E * 4 * p, dtype=bool)
    for e in range(E):
        for s in range(4):
            if neighbour(n, e, s) is None:
                mask[(e * 4 + s) * p:(e * 4 + s + 1) * p] = True
    return mask
