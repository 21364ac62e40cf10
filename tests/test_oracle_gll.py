"""Pins of the oracle's GLL tables (closed-form identities, library cross-check)."""
import numpy as np
import numpy.polynomial.legendre as npleg
import pytest

from oracle import gll


@pytest.mark.parametrize("N", [2, 3, 4, 8, 12, 16, 20])
def test_nodes_are_roots_of_dPN(N):
    x = gll.gll_nodes(N)
    ref = np.sort(npleg.Legendre.basis(N).deriv().roots().real)
    assert x[0] == -1.0 and x[-1] == 1.0
    np.testing.assert_allclose(x[1:-1], ref, atol=1e-13)
    assert np.all(np.diff(x) > 0)


@pytest.mark.parametrize("N", [2, 4, 8, 16])
def test_weights_integrate_up_to_degree_2N_minus_1(N):
    x, w, _ = gll.gll(N)
    assert abs(w.sum() - 2.0) < 1e-14
    for k in range(2 * N):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(w @ x ** k - exact) < 1e-13
    # degree 2N is not integrated exactly: the rule gives 2/N for P_N^2, not 2/(2N+1)
    pn, _ = gll.legendre(N, x)
    assert abs(w @ pn ** 2 - 2.0 / N) < 1e-13


@pytest.mark.parametrize("N", [2, 5, 8, 16])
def test_diff_exact_on_PN(N):
    x, _, D = gll.gll(N)
    np.testing.assert_allclose(D @ np.ones(N + 1), 0.0, atol=1e-11)
    for k in range(1, N + 1):
        np.testing.assert_allclose(D @ x ** k, k * x ** (k - 1), atol=1e-10 * N ** 2)
    # a random polynomial of degree N, differentiated by numpy
    rng = np.random.default_rng(N)
    c = rng.standard_normal(N + 1)
    np.testing.assert_allclose(D @ npleg.legval(x, c), npleg.legval(x, npleg.legder(c)),
                               atol=1e-10 * N ** 2)
