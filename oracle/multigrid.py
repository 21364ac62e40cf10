"""Merge tree as a multigrid preconditioner (Sec. 4.3).

For M = [[A, B], [C, D]] (x: faces eliminated at this level, y: the rest) the
block-inverse identity of Sec. 4.3 reads

    M^-1 = F + P S^-1 R (I - M F),  F = [[A^-1, 0], [0, 0]],
    P = [[-A^-1 B], [I]],  R = [0, I],  S = D - C A^-1 B.

MG(M_l) applies it with S^-1 replaced by MG(M_{l+1}), where M_{l+1} is the
skeleton system of the merged boxes (its equality with D - C A^-1 B is a
test); at the coarse level L the solve is either exact or a fixed number of
unpreconditioned GMRES iterations from zero.  gamma > 1 repeats the coarse
call as a stationary iteration y <- y + MG_{l+1}(r_y - M_{l+1} y) (a reading of
the paper's "multiple coarse calls").

Everything here uses the explicitly assembled sparse M_l and its blocks.

Test infrastructure only (see the package docstring).
"""
import numpy as np
import scipy.sparse.linalg as spla

from . import mesh, skeleton
from .krylov import gmres_ksteps
from .merge import build_hierarchy


class Hierarchy:
    """Assembled M_1 .. M_L with level index sets."""

    def __init__(self, n, p, leafT, levels=None):
        self.n, self.p = n, p
        self.L = mesh.lmax(n) if not levels else levels
        T, _ = build_hierarchy(n, p, leafT, None, top=self.L)
        self.boxT = T
        self.M, self.unk = {}, {}
        for level in range(1, self.L + 1):
            self.M[level], self.unk[level] = skeleton.assemble(n, p, level, T[level - 1])
        self.split = {}
        self._lu = {}
        for level in range(1, self.L):
            pos = {s: i for i, s in enumerate(self.unk[level])}
            yi = np.array([pos[s] for s in self.unk[level + 1]], dtype=np.int64)
            xi = np.setdiff1d(np.arange(len(self.unk[level])), yi)
            self.split[level] = (xi, yi)

    def blocks(self, level):
        xi, yi = self.split[level]
        M = self.M[level].tocsr()
        return (M[xi][:, xi], M[xi][:, yi], M[yi][:, xi], M[yi][:, yi])

    def solve_A(self, level, v):
        if level not in self._lu:
            A = self.blocks(level)[0]
            self._lu[level] = spla.splu(A.tocsc())
        return self._lu[level].solve(v)

    def coarse(self, r, k):
        M = self.M[self.L]
        if k is None or k < 0:
            return spla.spsolve(M.tocsc(), r)
        return gmres_ksteps(lambda v: M @ v, r, k)

    def mg(self, level, r, k, gamma=1):
        """MG(M_level) r, r indexed like self.unk[level]."""
        if level == self.L:
            return self.coarse(r, k)
        xi, yi = self.split[level]
        _, Bb, Cb, _ = self.blocks(level)
        zx0 = self.solve_A(level, r[xi])               # F r
        ry = r[yi] - Cb @ zx0                          # R (I - M F) r
        y = np.zeros(len(yi), dtype=complex)
        for _ in range(gamma):                         # S^-1 by recursion
            res = ry if not y.any() else ry - self.M[level + 1] @ y
            y = y + self.mg(level + 1, res, k, gamma)
        z = np.empty(len(r), dtype=complex)
        z[xi] = zx0 - self.solve_A(level, Bb @ y)      # + P y
        z[yi] = y
        return z

    def apply(self, r_canon, k, gamma=1):
        """Preconditioner on canonical-layout vectors (physical slots 0)."""
        unk = self.unk[1]
        z = np.zeros_like(r_canon, dtype=complex)
        z[unk] = self.mg(1, r_canon[unk], k, gamma)
        return z
