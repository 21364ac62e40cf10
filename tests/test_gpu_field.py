"""Field recovery through the C ABI (hps_recover_field, Sec. 3.1) against the
oracle's element solves and the corner reading, and against a closed-form
exact solution."""
import numpy as np
import pytest

from tests.gpu_cases import oracle_case, gpu_problem, rel
from paper_2511_00735_amd import workloads

pytestmark = pytest.mark.gpu


def _bump(x, y):
    return 0.6 * np.exp(-((x - 0.4) ** 2 + (y - 0.6) ** 2) / 0.05) - 0.3 * np.sin(3 * x * y)


def _src(x, y):
    return np.exp(1j * (2 * x - y)) * (1 + x * y)


@pytest.mark.parametrize("n,N,kappa,with_src", [(4, 8, 10.0, True), (8, 12, 30.0, False), (4, 16, 25.0, True)])
def test_field_matches_oracle(hps, ctx, n, N, kappa, with_src):
    from oracle import field, gll, leaf
    print(f"[field] {n}x{n} N={N} source={with_src}", flush=True)
    wave = workloads.PlaneWave(kappa, kappa, (0.6, 0.8))
    sfn = _src if with_src else None
    oc = oracle_case(n, N, kappa, _bump, wave.t, sfn)
    prob = gpu_problem(hps, ctx, n, N, kappa, _bump, sfn, coarse_iters=-1)
    b = prob.coefficient_nodes(_bump)
    s = prob.source_nodes(sfn) if with_src else None
    t = prob.boundary_data(wave.t)
    g, info = prob.gmres_solve(prob.set_rhs(t), tol=1e-13)
    u = prob.recover_field(b, t, g, s).cpu().numpy()
    xi = gll.gll_nodes(N)
    c = leaf.nodal_coefficient(N, n, kappa, _bump, xi)
    sn = None
    if with_src:
        from oracle import mesh
        X, Y = mesh.element_node_coords(n, N, xi)
        sn = _src(X, Y).reshape(n * n, -1)
    ref = field.fields(n, N, kappa, c, sn, oc["g"], oc["t"])
    err = rel(u, ref)
    print(f"[field] vs oracle {err:.2e}", flush=True)
    assert err < 1e-10, err


def test_plane_wave_field_at_benchmark_size(hps, ctx):
    """64x64 elements, N = 16, kappa = 200, b = 0, s = 0: the exact field is the
    plane wave itself, so the recovered field's error is the discretisation
    error (plus the FGMRES tolerance); sampled elements also match the
    oracle's element solve given the same g."""
    from oracle import field, gll, leaf, mesh
    n, N, kappa = 64, 16, 200.0
    wave = workloads.PlaneWave(kappa, kappa)
    prob = gpu_problem(hps, ctx, n, N, kappa, workloads.zero_field, levels=12, coarse_iters=5)
    b = prob.coefficient_nodes(workloads.zero_field)
    t = prob.boundary_data(wave.t)
    g, info = prob.gmres_solve(prob.set_rhs(t), tol=1e-12)
    u = prob.recover_field(b, t, g).cpu().numpy()
    xi = gll.gll_nodes(N)
    X, Y = mesh.element_node_coords(n, N, xi)
    exact = wave.u(X.reshape(n * n, -1), Y.reshape(n * n, -1))
    err = np.abs(u - exact).max()
    print(f"[field] 64x64 plane wave: max nodal error {err:.2e} ({info['iterations']} its)", flush=True)
    assert err < 1e-6, err
    gc = g.cpu().numpy()
    tc = t.cpu().numpy()
    c = leaf.nodal_coefficient(N, n, kappa, workloads.zero_field, xi)
    p = N - 1
    phys = mesh.physical_slot_mask(n, p)
    inc = np.where(phys, tc, gc)
    for e in (0, 63, 2080, 4095):
        ref = field.element_field(N, 1.0 / n, kappa, c[e], None, inc[e * 4 * p:(e + 1) * 4 * p])
        assert rel(u[e], ref) < 1e-11, e
