"""1D Gauss-Legendre-Lobatto reference data (Sec. 3.1 of the paper).

The paper uses GLL nodes, weights w and the differentiation matrix D on each
element but does not spell them out; these are the textbook spectral-method
definitions on the reference interval [-1, 1]:

* nodes: -1, the N-1 roots of P_N', +1;
* weights: w_j = 2 / (N (N+1) P_N(x_j)^2);
* D_ij = P_N(x_i) / (P_N(x_j) (x_i - x_j)) for i != j,
  D_00 = -N(N+1)/4, D_NN = +N(N+1)/4, other diagonal entries 0.

Test infrastructure only (see the package docstring).
"""
import numpy as np


def legendre(N, x):
    """Return (P_N(x), P_{N-1}(x)) by the three-term recurrence."""
    x = np.asarray(x, dtype=np.float64)
    p_prev = np.ones_like(x)
    if N == 0:
        return p_prev, np.zeros_like(x)
    p = x.copy()
    for k in range(1, N):
        p_prev, p = p, ((2 * k + 1) * x * p - k * p_prev) / (k + 1)
    return p, p_prev


def gll_nodes(N):
    """GLL nodes on [-1, 1], increasing.

    The nodes are the zeros of f(x) = x P_N(x) - P_{N-1}(x), because
    (1 - x^2) P_N'(x) = N (P_{N-1}(x) - x P_N(x)).  Differentiating and using
    P_{N-1}' = x P_N' - N P_N gives f'(x) = (N+1) P_N(x), so Newton's method
    reads x <- x - f(x) / ((N+1) P_N(x)); it is started from the
    Chebyshev-Lobatto points.
    """
    if N < 1:
        raise ValueError("N >= 1 required")
    x = -np.cos(np.pi * np.arange(N + 1) / N)
    for _ in range(100):
        pn, pn1 = legendre(N, x)
        dx = (x * pn - pn1) / ((N + 1) * pn)
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    x[0], x[-1] = -1.0, 1.0
    return x


def gll_weights(N, x=None):
    if x is None:
        x = gll_nodes(N)
    pn, _ = legendre(N, x)
    return 2.0 / (N * (N + 1) * pn ** 2)


def gll_diff(N, x=None):
    """Differentiation matrix: (D v)_i = v'(x_i) for v in P_N."""
    if x is None:
        x = gll_nodes(N)
    pn, _ = legendre(N, x)
    D = np.zeros((N + 1, N + 1))
    for i in range(N + 1):
        for j in range(N + 1):
            if i != j:
                D[i, j] = pn[i] / (pn[j] * (x[i] - x[j]))
    D[0, 0] = -N * (N + 1) / 4.0
    D[N, N] = N * (N + 1) / 4.0
    return D


def gll(N):
    """(nodes, weights, D) on the reference interval."""
    x = gll_nodes(N)
    return x, gll_weights(N, x), gll_diff(N, x)
