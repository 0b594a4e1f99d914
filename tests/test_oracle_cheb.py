"""Pins for the oracle's Chebyshev collocation (Section 2: tensor Chebyshev
grids per leaf)."""
import os

import numpy as np

from oracle.cheb import diff_matrix, lagrange_eval, lobatto_nodes
from oracle.grid import Grid

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_diff_matrix_p3_textbook():
    D = diff_matrix(lobatto_nodes(3))
    ref = np.loadtxt(os.path.join(GOLD, "cheb_d3.txt"))
    assert np.allclose(D, ref, atol=1e-14)


def test_diff_exact_on_polynomials():
    for p in (8, 16):
        t = lobatto_nodes(p)
        D = diff_matrix(t)
        for deg in range(p):
            f = t ** deg
            df = deg * t ** (deg - 1) if deg else np.zeros_like(t)
            assert np.max(np.abs(D @ f - df)) < 1e-11 * max(1, deg) ** 2


def test_second_derivative_of_cosine_converges():
    t = lobatto_nodes(16)
    D = diff_matrix(t)
    f = np.cos(2.0 * t)
    assert np.max(np.abs(D @ (D @ f) + 4.0 * f)) < 1e-8


def test_lagrange_interpolates_polynomials():
    nodes = lobatto_nodes(16)[1:-1]
    x = np.linspace(-1, 1, 37)
    Lm = lagrange_eval(nodes, x)
    for deg in range(nodes.size):
        assert np.max(np.abs(Lm @ nodes ** deg - x ** deg)) < 1e-11


def test_grid_counts_match_table1():
    rows = np.loadtxt(os.path.join(GOLD, "table1_grid_sizes.txt"), dtype=np.int64)
    for L, N in rows[:3]:
        g = Grid(int(L), 16)
        # leaves share their Lobatto edge points: (p - 1) L + 1 per axis
        assert g.xg.size ** 2 == N
    g = Grid(4, 16)
    # unknowns = all grid points except the (L + 1)^2 leaf corners
    assert g.nu == 3721 - 25
    assert g.npde == 16 * 14 * 14
    assert g.nb == 4 * 4 * 14
