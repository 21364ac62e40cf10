"""CPU checks of the C ABI: the library loads, exports every function that
include/hps.h declares, and its host-side helpers (no GPU calls) agree with the
oracle's geometry."""
import os
import re

import numpy as np
import pytest

from oracle import gll, mesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def hps():
    from paper_2511_00735_amd import hps as _hps
    return _hps


def declared_functions():
    text = open(os.path.join(ROOT, "include", "hps.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hps_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(hps):
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(hps.lib, name), name


def test_gll_nodes_match_oracle(hps):
    for N in (2, 5, 8, 12, 16):
        np.testing.assert_allclose(hps.gll_nodes(N), gll.gll_nodes(N), atol=2e-16)


def test_coordinates_match_oracle(hps):
    for n, N in ((4, 8), (8, 5)):
        d = hps.make_desc(n, N, 10.0)
        xi = gll.gll_nodes(N)
        x, y = hps.node_coords(d)
        X, Y = mesh.element_node_coords(n, N, xi)
        np.testing.assert_allclose(x, X.reshape(n * n, -1), atol=1e-15)
        np.testing.assert_allclose(y, Y.reshape(n * n, -1), atol=1e-15)
        got = hps.slot_coords(d)
        ref = mesh.canonical_slot_coords(n, N, xi)
        for a, b in zip(got, ref):
            np.testing.assert_allclose(a, b, atol=1e-15)


def test_workspace_sizes_and_validation(hps):
    small = hps.workspace_bytes(hps.make_desc(4, 8, 10.0))
    big = hps.workspace_bytes(hps.make_desc(64, 16, 200.0))
    assert 0 < small < big
    # the footprint is dominated by the box maps of every level: ~ L * E * (4p)^2 * 16 B
    assert big > 12 * 4096 * 60 * 60 * 16 * 0.9
    exact = hps.workspace_bytes(hps.make_desc(64, 16, 200.0, coarse_iters=-1))
    assert exact > big                      # the exact coarse space stores W_L^-1 too
    for bad in (hps.make_desc(3, 8, 10.0), hps.make_desc(4, 1, 10.0),
                hps.make_desc(4, 8, -1.0), hps.make_desc(4, 8, float("inf")),
                hps.make_desc(4, 8, 10.0, levels=9), hps.make_desc(4, 8, 10.0, levels=3, coarse_iters=-1),
                hps.make_desc(4, 8, 10.0, coarse_iters=0), hps.make_desc(4, 17, 10.0)):
        with pytest.raises(hps.HPSError):
            hps.workspace_bytes(bad)


def test_morton_box_order_is_a_bijection(hps):
    n = 16
    for level in range(1, 9):
        wx, wy = mesh.box_dims(level)
        nb = (n // wx) * (n // wy)
        seen = {hps.morton_box_xy(level, j) for j in range(nb)}
        assert seen == {(bx, by) for bx in range(n // wx) for by in range(n // wy)}
        # siblings of a merge are adjacent along the merge axis
        if level < 8:
            for j in range(nb // 2):
                (px, py), (qx, qy) = hps.morton_box_xy(level, 2 * j), hps.morton_box_xy(level, 2 * j + 1)
                if level % 2:
                    assert (qx, qy) == (px + 1, py) and px % 2 == 0
                else:
                    assert (qx, qy) == (px, py + 1) and py % 2 == 0


def test_choose_levels_is_the_most_levels_that_fit(hps):
    d = hps.make_desc(64, 16, 200.0, coarse_iters=5)
    sizes = {}
    for L in range(1, 13):
        sizes[L] = hps.workspace_bytes(hps.make_desc(64, 16, 200.0, levels=L, coarse_iters=5))
    assert all(sizes[L] < sizes[L + 1] for L in range(1, 12))   # more levels, more memory
    for L in range(1, 13):
        assert hps.choose_levels(d, sizes[L]) == L
        if L > 1:
            assert hps.choose_levels(d, sizes[L] - 1) == L - 1
    with pytest.raises(hps.HPSError):
        hps.choose_levels(d, sizes[1] - 1)
    ex = hps.make_desc(64, 16, 200.0, coarse_iters=-1)
    with pytest.raises(hps.HPSError):       # exact coarse space: only L = L_max
        hps.choose_levels(ex, hps.workspace_bytes(ex) - 1)
    assert hps.choose_levels(hps.make_desc(16, 8, 20.0), 1 << 40, count=8) == 8


def test_gamma_descriptor(hps):
    base = hps.workspace_bytes(hps.make_desc(16, 8, 20.0, levels=6))
    g2 = hps.workspace_bytes(hps.make_desc(16, 8, 20.0, levels=6, gamma=2))
    assert g2 > base                        # per-level vectors of the gamma-cycle
    for bad in (5, -1):
        with pytest.raises(hps.HPSError):
            hps.workspace_bytes(hps.make_desc(16, 8, 20.0, gamma=bad))


def test_rect_descriptor_checks(hps):
    """Rectangular meshes: both sides powers of two, at least two elements;
    ny = 0 is the square mesh; levels bounded by log2(nx ny)."""
    for nx, ny in [(3, 4), (4, 6), (1, 1), (2048, 1)]:
        with pytest.raises(hps.HPSError):
            hps.workspace_bytes(hps.make_desc(nx, 4, 5.0, ny=ny))
    assert hps.workspace_bytes(hps.make_desc(8, 4, 5.0, ny=8)) == hps.workspace_bytes(hps.make_desc(8, 4, 5.0))
    with pytest.raises(hps.HPSError):
        hps.workspace_bytes(hps.make_desc(8, 4, 5.0, ny=2, levels=5))   # L_max = 4
