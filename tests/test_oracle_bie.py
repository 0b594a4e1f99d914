"""Pins for the oracle's layer potentials (Remark in Section 2: Green's formula
and the jump relations)."""
import numpy as np
from scipy.special import hankel1

from oracle.bie import boundary_matrices, circle_points, potential_matrices
from oracle.grid import Grid


def _point_source(g, k, x0):
    d = g.bxy - x0
    r = np.hypot(d[:, 0], d[:, 1])
    u = hankel1(0, k * r)
    du = -k * hankel1(1, k * r) * np.sum(d * g.bnormal, axis=1) / r
    return u, du


def test_exterior_calderon_and_green_representation():
    g = Grid(4, 16)
    k = 10.0
    S, K = boundary_matrices(g, k)
    x0 = np.array([0.13, -0.21])
    u, du = _point_source(g, k, x0)
    res = S @ du - (K - 0.5 * np.eye(g.nb)) @ u
    assert np.max(np.abs(res)) < 1e-9 * np.max(np.abs(u))
    X, _ = circle_points(2.0, 16)
    PS, PD = potential_matrices(g, k, X)
    dX = X - x0
    ref = hankel1(0, k * np.hypot(dX[:, 0], dX[:, 1]))
    assert np.max(np.abs(PD @ u - PS @ du - ref)) < 1e-11


def test_interior_calderon_plane_wave():
    g = Grid(4, 16)
    k = 10.0
    S, K = boundary_matrices(g, k)
    d = np.array([np.cos(0.3), np.sin(0.3)])
    u = np.exp(1j * k * g.bxy @ d)
    du = 1j * k * (g.bnormal @ d) * u
    # an entire solution: S d_n u = (K + I/2) u  (interior limit)
    assert np.max(np.abs(S @ du - (K + 0.5 * np.eye(g.nb)) @ u)) < 1e-9


def test_double_layer_vanishes_on_own_side():
    g = Grid(2, 16)
    _, K = boundary_matrices(g, 3.0)
    side = g.bnodes[:, 2]
    same = side[:, None] == side[None, :]
    assert np.all(K[same] == 0.0)
    assert np.max(np.abs(K[~same])) > 0.0
