"""Parity at the benchmark's full size (k = 80, 64 x 64 leaves of 16 x 16,
256 directions x 256 angles, R = 2) by properties that hold at any size:
a radial contrast against the separation-of-variables reference of the
oracle (exact up to the contrast's 1e-11 tail), and zero contrast."""
import numpy as np
import pytest

import os

import synth
from oracle.radial import scattered_from_modes

GOLD = os.path.join(os.path.dirname(__file__), "golden", "radial_k80.txt")

pytestmark = pytest.mark.gpu

K, L, M, P, R = 80.0, 64, 256, 256, 2.0


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def solver():
    _torch()
    import paper_1608_06871_amd as hps
    s = hps.Solver(nleaf=L, p=16, keep_derivs=False)
    s.set_wavenumber(K)
    return s


def test_radial_contrast_k80_full_size(solver):
    torch = _torch()
    amp, sig = 0.4, 0.2
    print("full-size radial parity: k=80, 64x64 leaves, 256 x 256", flush=True)
    q = synth.radial_gaussian(solver.node_coords(), amp, sig)
    solver.factor(torch.from_numpy(q).cuda(), K)
    dirs = synth.equispaced_angles(M)
    th = synth.equispaced_angles(P)
    solver.solve(dirs)
    uf = solver.far_field(th, R).cpu().numpy()
    tab = np.loadtxt(GOLD)  # written by tests/golden/make_radial_k80.py (oracle only)
    coef = tab[:, 1] + 1j * tab[:, 2]
    ref = scattered_from_modes(coef, th[None, :] - dirs[:, None])
    err = np.max(np.abs(uf - ref)) / np.max(np.abs(ref))
    print(f"max relative error {err:.2e}", flush=True)
    assert err < 1e-8


def test_zero_contrast_k80_full_size(solver):
    torch = _torch()
    solver.factor(torch.zeros(solver.npde, dtype=torch.float64, device="cuda"), K)
    solver.solve(synth.equispaced_angles(16))
    uf = solver.far_field(synth.equispaced_angles(P), R).cpu().numpy()
    assert np.max(np.abs(uf)) < 1e-8


def test_radial_contrast_k160_largest_grid():
    """The largest grid tested: 128 x 128 leaves of 16 x 16 (4.0M unknowns,
    outer boundary 7168 nodes, a 14-level tree, the 7168-order top inverse),
    k = 160 (38 points per wavelength), against the oracle's separation-of-
    variables reference (tests/golden/radial_k160.txt, written by
    tests/golden/make_radial_k160.py from oracle/radial.py only); then zero
    contrast on the same factorised grid."""
    torch = _torch()
    import paper_1608_06871_amd as hps
    K2, L2, M2, P2 = 160.0, 128, 16, 64
    print("largest grid: k=160, 128x128 leaves, 16 x 64", flush=True)
    s = hps.Solver(nleaf=L2, p=16, keep_derivs=False)
    amp, sig = 0.4, 0.2
    q = synth.radial_gaussian(s.node_coords(), amp, sig)
    s.factor(torch.from_numpy(q).cuda(), K2)
    dirs = synth.equispaced_angles(M2)
    th = synth.equispaced_angles(P2)
    s.solve(dirs)
    uf = s.far_field(th, R).cpu().numpy()
    tab = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "radial_k160.txt"))
    coef = tab[:, 1] + 1j * tab[:, 2]
    ref = scattered_from_modes(coef, th[None, :] - dirs[:, None])
    err = np.max(np.abs(uf - ref)) / np.max(np.abs(ref))
    print(f"max relative error {err:.2e}", flush=True)
    assert err < 1e-8
    s.factor(torch.zeros(s.npde, dtype=torch.float64, device="cuda"), K2)
    s.solve(dirs)
    assert np.max(np.abs(s.far_field(th, R).cpu().numpy())) < 1e-8
    del s
    torch.cuda.empty_cache()
