"""The allocation-free leaf entry point (hps_leaf_maps_noalloc, for callers
that cannot allocate device memory) against hps_build_leaves on the same
inputs: two calls in a row through the C ABI, the second with fewer elements
and other data, so that it runs on the static scratch the first one left."""
import numpy as np
import pytest

from tests.gpu_cases import rel

pytestmark = pytest.mark.gpu


def _bump(x, y):
    return 0.6 * np.exp(-((x - 0.4) ** 2 + (y - 0.6) ** 2) / 0.05) - 0.3 * np.sin(3 * x * y)


def _src(x, y):
    return np.exp(1j * (2 * x - y)) * (1 + x * y)


def _partner(n, p, s):
    """Canonical slot across the face from slot s, or -1 (physical)."""
    k, side, e = s % p, (s // p) % 4, s // (4 * p)
    ix, iy = e % n, e // n
    if side == 0:
        return -1 if ix == 0 else ((e - 1) * 4 + 1) * p + k
    if side == 1:
        return -1 if ix == n - 1 else ((e + 1) * 4 + 0) * p + k
    if side == 2:
        return -1 if iy == 0 else ((e - n) * 4 + 3) * p + k
    return -1 if iy == n - 1 else ((e + n) * 4 + 2) * p + k


def test_noalloc_leaf_maps_match_build_leaves(hps):
    import torch
    ctx = hps.Context()
    # 64 elements at N = 16 (of the 102 the scratch holds), then 16 at N = 12
    for n, N, kappa, with_src in ((8, 16, 60.0, True), (4, 12, 25.0, False)):
        print(f"[noalloc] {n}x{n} elements, N={N}, source={with_src}", flush=True)
        E, p = n * n, N - 1
        m = 4 * p
        prob = hps.Problem(ctx, hps.make_desc(n, N, kappa))
        b = prob.coefficient_nodes(_bump)
        s = prob.source_nodes(_src) if with_src else None
        prob.build_leaves(b, s)
        Tm = prob.level_T(1).cpu().numpy()
        rhs = prob.set_rhs(prob.boundary_data(lambda x, y, nx, ny: 0 * x + 0j)).cpu().numpy()
        T = torch.full((E * m * m,), float("nan"), dtype=torch.complex128, device="cuda")
        H = torch.full((E * m,), float("nan"), dtype=torch.complex128, device="cuda")
        hps.leaf_maps_noalloc(ctx, N, 1.0 / n, kappa, kappa, b, s, T, H)
        Tn = T.view(E, m, m).transpose(1, 2).cpu().numpy()
        Hn = H.cpu().numpy()
        for j in range(E):
            bx, by = hps.morton_box_xy(1, j)
            e = bx + n * by
            assert rel(Tn[e], Tm[j]) <= 1e-12, (e, rel(Tn[e], Tm[j]))
        # H enters the right-hand side: with t = 0, rhs[Pi(s)] = H[s]
        inner = [(sl, _partner(n, p, sl)) for sl in range(E * m) if _partner(n, p, sl) >= 0]
        hs = np.array([Hn[a] for a, _ in inner])
        hr = np.array([rhs[b_] for _, b_ in inner])
        if with_src:
            assert rel(hs, hr) <= 1e-12
        else:
            assert np.abs(hs).max() == 0.0 and np.abs(hr).max() == 0.0


def test_noalloc_rejects_counts_beyond_its_scratch(hps):
    import torch
    ctx = hps.Context()
    b = torch.zeros((103, 17 * 17), dtype=torch.float64, device="cuda")
    T = torch.empty(103 * 60 * 60, dtype=torch.complex128, device="cuda")
    H = torch.empty(103 * 60, dtype=torch.complex128, device="cuda")
    with pytest.raises(hps.HPSError) as ei:
        hps.leaf_maps_noalloc(ctx, 16, 1.0 / 64, 200.0, 200.0, b, None, T, H)
    assert ei.value.code == -1 and "[1, 102]" in str(ei.value)
