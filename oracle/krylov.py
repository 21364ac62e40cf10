"""Krylov solvers (Sec. 4.3, Sec. 5 and the notes of Table 1).

* gmres_ksteps: the coarse solve -- k unpreconditioned GMRES iterations from
  x0 = 0 with no restart, modified Gram-Schmidt Arnoldi; returns the k-th
  iterate x_k = V_k y_k with y_k minimising ||beta e1 - H_k y||.  It stops
  early on a (lucky) breakdown h_{j+1,j} <= 1e-14 ||r||.
* fgmres: right-preconditioned flexible GMRES (the preconditioned vectors
  z_j = P(v_j) are stored, so P may change between steps), restart 60, x0 = 0,
  stops when the relative residual ||b - M x|| / ||b|| <= tol.  The least
  squares problem is updated by Givens rotations; the true residual is
  recomputed at every restart and at exit.  Iterations are counted across
  restarts.

Test infrastructure only (see the package docstring).
"""
import numpy as np


def _lstsq_hessenberg(Hm, beta):
    """Minimise ||beta e1 - Hm y|| for the (j+1) x j Hessenberg Hm."""
    rhs = np.zeros(Hm.shape[0], dtype=complex)
    rhs[0] = beta
    y, *_ = np.linalg.lstsq(Hm, rhs, rcond=None)
    return y


def gmres_ksteps(matvec, r, k):
    beta = np.linalg.norm(r)
    if beta == 0.0 or k <= 0:
        return np.zeros_like(r, dtype=complex)
    V = [r / beta]
    Hm = np.zeros((k + 1, k), dtype=complex)
    j_used = k
    for j in range(k):
        w = matvec(V[j]).astype(complex)
        for i in range(j + 1):
            Hm[i, j] = np.vdot(V[i], w)
            w = w - Hm[i, j] * V[i]
        Hm[j + 1, j] = np.linalg.norm(w)
        if abs(Hm[j + 1, j]) <= 1e-14 * beta:
            j_used = j + 1
            break
        V.append(w / Hm[j + 1, j])
    y = _lstsq_hessenberg(Hm[:j_used + 1, :j_used], beta)
    return np.array(V[:j_used]).T @ y


def fgmres(matvec, b, precond=None, tol=1e-10, restart=60, maxit=600):
    """Returns (x, iterations, history of relative residual estimates, true relres)."""
    precond = precond or (lambda v: v)
    bnorm = np.linalg.norm(b)
    x = np.zeros_like(b, dtype=complex)
    if bnorm == 0.0:
        return x, 0, [0.0], 0.0
    it = 0
    hist = [1.0]
    while True:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol or it >= maxit:
            return x, it, hist, beta / bnorm
        V = np.zeros((restart + 1, len(b)), dtype=complex)
        Z = np.zeros((restart, len(b)), dtype=complex)
        Hm = np.zeros((restart + 1, restart), dtype=complex)
        cs = np.zeros(restart, dtype=complex)
        sn = np.zeros(restart, dtype=complex)
        gvec = np.zeros(restart + 1, dtype=complex)
        gvec[0] = beta
        V[0] = r / beta
        j_end = 0
        for j in range(restart):
            Z[j] = precond(V[j])
            w = matvec(Z[j]).astype(complex)
            for i in range(j + 1):
                Hm[i, j] = np.vdot(V[i], w)
                w = w - Hm[i, j] * V[i]
            Hm[j + 1, j] = np.linalg.norm(w)
            if Hm[j + 1, j] != 0:
                V[j + 1] = w / Hm[j + 1, j]
            for i in range(j):                       # previous rotations
                # G_i = [[conj(c), conj(s)], [-s, c]]
                t = np.conj(cs[i]) * Hm[i, j] + np.conj(sn[i]) * Hm[i + 1, j]
                Hm[i + 1, j] = -sn[i] * Hm[i, j] + cs[i] * Hm[i + 1, j]
                Hm[i, j] = t
            a, bb = Hm[j, j], Hm[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(bb) ** 2)
            cs[j] = a / den if den else 1.0
            sn[j] = bb / den if den else 0.0
            Hm[j, j] = den
            Hm[j + 1, j] = 0.0
            gvec[j + 1] = -sn[j] * gvec[j]
            gvec[j] = np.conj(cs[j]) * gvec[j]
            it += 1
            j_end = j + 1
            hist.append(abs(gvec[j + 1]) / bnorm)
            if abs(gvec[j + 1]) / bnorm <= tol or it >= maxit:
                break
        y = np.linalg.solve(np.triu(Hm[:j_end, :j_end]), gvec[:j_end])
        x = x + Z[:j_end].T @ y
