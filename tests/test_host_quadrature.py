"""CPU check of the library's host-side boundary quadrature (its own Hankel
functions and adaptive Gauss-Legendre product integration) against the
oracle's independent quadrature: both compute the same exact integrals of
kernel x panel Lagrange basis (Remark in Section 2)."""
import os

import numpy as np
import pytest

from oracle.bie import boundary_matrices
from oracle.grid import Grid


@pytest.mark.parametrize("L,k", [(2, 3.0), (4, 10.0), (4, 37.5)])
def test_library_layer_matrices_match_oracle(L, k):
    import paper_1608_06871_amd as hps
    if not os.path.exists(hps.LIB_PATH):
        pytest.skip("libhps.so not built")
    xy, S, K = hps.boundary_operators(L, 16, k)
    g = Grid(L)
    So, Ko = boundary_matrices(g, k)
    key = lambda a: [tuple(r) for r in np.round(a * 1e9).astype(np.int64)]
    pos = {v: i for i, v in enumerate(key(xy))}
    perm = np.array([pos[v] for v in key(g.bxy)])
    assert sorted(perm) == list(range(len(perm)))
    Sl = S[np.ix_(perm, perm)]
    Kl = K[np.ix_(perm, perm)]
    assert np.max(np.abs(Sl - So)) < 1e-12 * np.max(np.abs(So))
    assert np.max(np.abs(Kl - Ko)) < 1e-11 * np.max(np.abs(Ko))


@pytest.mark.parametrize("L,k", [(2, 3.0), (4, 10.0), (4, 37.5)])
def test_library_combined_field_operators_match_oracle(L, k):
    """K' and the hypersingular T of the combined-field exterior relation:
    the library's own-panel principal value and end terms against the
    oracle's."""
    import paper_1608_06871_amd as hps
    if not os.path.exists(hps.LIB_PATH):
        pytest.skip("libhps.so not built")
    from oracle.bie import bm_matrices
    xy, _, _ = hps.boundary_operators(L, 16, k)
    Kp, T = hps.combined_field_operators(L, 16, k)
    g = Grid(L)
    Kpo, To = bm_matrices(g, k)
    key = lambda a: [tuple(r) for r in np.round(a * 1e9).astype(np.int64)]
    pos = {v: i for i, v in enumerate(key(xy))}
    perm = np.array([pos[v] for v in key(g.bxy)])
    assert np.max(np.abs(Kp[np.ix_(perm, perm)] - Kpo)) < 1e-11 * np.max(np.abs(Kpo))
    assert np.max(np.abs(T[np.ix_(perm, perm)] - To)) < 1e-11 * np.max(np.abs(To))
