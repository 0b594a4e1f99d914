"""Pins for the oracle's Frechet derivative (Theorem 1) and adjoint
(Theorem 2, discrete transpose), and for the Gauss-Newton step."""
import numpy as np

import synth
from oracle import gn, sine
from oracle.bie import circle_points
from oracle.forward import Problem, directions


def _setup(L=2, k=5.0, M=3, P=8, seed=1):
    prob = Problem(L, k)
    xy = prob.grid.pde_coords()
    q = synth.gaussian_bumps(xy, 5, seed)
    prob.factor(q)
    prob.solve(directions(M))
    _, th = circle_points(2.0, P)
    prob.set_measurement(th, 2.0)
    return prob, q


def _F(prob, q, M):
    prob.factor(q)
    prob.solve(directions(M))
    return prob.far_field()


def test_jvp_matches_central_differences():
    prob, q = _setup()
    dq = synth.gaussian_bumps(prob.grid.pde_coords(), 3, 7)
    jv = prob.jvp(dq)
    h = 1e-4
    fd = (_F(prob, q + h * dq, 3) - _F(prob, q - h * dq, 3)) / (2 * h)
    assert np.max(np.abs(fd - jv)) < 1e-6 * np.max(np.abs(jv))


def test_vjp_is_adjoint_of_jvp():
    prob, q = _setup()
    rng = np.random.default_rng(0)
    dq = rng.standard_normal(prob.grid.npde)
    r = rng.standard_normal((3, 8)) + 1j * rng.standard_normal((3, 8))
    lhs = np.real(np.vdot(r, prob.jvp(dq)))
    rhs = dq @ prob.vjp(r)
    assert abs(lhs - rhs) < 1e-11 * abs(lhs)


def test_explicit_jacobian_columns():
    prob = Problem(1, 3.0, p=8)
    q = synth.gaussian_bumps(prob.grid.pde_coords(), 2, 3)
    prob.factor(q)
    prob.solve(directions(2))
    _, th = circle_points(2.0, 6)
    prob.set_measurement(th, 2.0)
    J = prob.jacobian()
    rng = np.random.default_rng(1)
    x = rng.standard_normal(prob.grid.npde)
    assert np.allclose(J @ x, prob.jvp(x).ravel(), rtol=0, atol=1e-12 * np.max(np.abs(J)))
    y = rng.standard_normal(J.shape[0]) + 1j * rng.standard_normal(J.shape[0])
    assert np.allclose(np.real(J.conj().T @ y), prob.vjp(y.reshape(2, 6)), atol=1e-11)


def test_sine_adjoint_is_transpose():
    rng = np.random.default_rng(2)
    xy = rng.uniform(-1, 1, size=(50, 2))
    C = rng.standard_normal((4, 4))
    g = rng.standard_normal(50)
    assert abs(g @ sine.evaluate(xy, C) - np.sum(C * sine.adjoint(xy, g, 4))) < 1e-12
    # sin(m pi (x+1)/2) vanishes on the boundary of [-1, 1]^2
    edge = np.array([[-1.0, 0.3], [1.0, -0.2], [0.1, -1.0], [0.4, 1.0]])
    assert np.max(np.abs(sine.evaluate(edge, C))) < 1e-14


def test_gauss_newton_recovers_linearised_data():
    L, k, M, P, S = 2, 4.0, 4, 8, 3
    rng = np.random.default_rng(3)
    C0 = 0.05 * rng.standard_normal((S, S))
    dC = 0.01 * rng.standard_normal((S, S))
    prob = Problem(L, k)
    xy = prob.grid.pde_coords()
    prob.factor(sine.evaluate(xy, C0))
    prob.solve(directions(M))
    _, th = circle_points(2.0, P)
    prob.set_measurement(th, 2.0)
    data = prob.far_field() + prob.jvp(sine.evaluate(xy, dC))
    C1, r, Jc, _ = gn.gauss_newton_step(L, k, C0, data, directions(M), P, 2.0)
    assert np.max(np.abs(C1 - (C0 + dC))) < 1e-9


def test_gauss_newton_reduces_misfit():
    L, k, M, P, S = 2, 4.0, 4, 8, 3
    rng = np.random.default_rng(4)
    Ct = 0.1 * rng.standard_normal((S, S))
    prob = Problem(L, k)
    xy = prob.grid.pde_coords()
    _, th = circle_points(2.0, P)
    prob.set_measurement(th, 2.0)
    data = _F(prob, sine.evaluate(xy, Ct), M)
    C0 = np.zeros((S, S))
    C1, r0, _, _ = gn.gauss_newton_step(L, k, C0, data, directions(M), P, 2.0)
    r1 = data - _F(prob, sine.evaluate(xy, C1), M)
    assert np.linalg.norm(r1) < 0.2 * np.linalg.norm(r0)


def test_sine_mode_values_at_known_points():
    """Single modes at points where both factors are exact fractions of pi
    (tests/golden/sine_mode_values.txt; a doubled or halved frequency, a
    swapped axis or a shifted origin changes some of these values)."""
    import os
    tab = np.loadtxt(os.path.join(os.path.dirname(__file__), "golden", "sine_mode_values.txt"))
    for m, n, x, y, val in tab:
        S = int(max(m, n))
        C = np.zeros((S, S))
        C[int(m) - 1, int(n) - 1] = 1.0
        got = sine.evaluate(np.array([[x, y]]), C)[0]
        assert abs(got - val) < 1e-14, (m, n, x, y, got, val)


def test_sine_modes_orthonormal_under_gauss_quadrature():
    """int_Omega phi_mn phi_m'n' = delta (each factor has unit L2 norm on
    [-1, 1]): the Gram matrix of the modes under a tensor Gauss-Legendre rule
    that integrates these trigonometric products to rounding is the identity."""
    S = 6
    x, w = np.polynomial.legendre.leggauss(40)
    X, Y = np.meshgrid(x, x, indexing="ij")
    W = np.outer(w, w).ravel()
    B = sine.basis(np.stack([X.ravel(), Y.ravel()], axis=1), S)
    G = B.T @ (W[:, None] * B)
    assert np.max(np.abs(G - np.eye(S * S))) < 1e-13


def test_gauss_newton_band_recovers_in_band_perturbation():
    """With the triangular band (eq. sineseries, modes m + n <= S), linearised
    data of an in-band perturbation are recovered exactly and the coefficients
    outside the band keep their values."""
    L, k, M, P, S, band = 2, 3.0, 6, 12, 3, 3
    prob = Problem(L, k)
    xy = prob.grid.pde_coords()
    _, th = circle_points(2.0, P)
    prob.set_measurement(th, 2.0)
    rng = np.random.default_rng(4)
    C0 = 0.05 * rng.standard_normal((S, S))
    keep = gn.band_mask(S, band)
    assert keep.sum() == band * (band - 1) // 2
    dC = np.where(keep, 1e-7 * rng.standard_normal((S, S)), 0.0)
    prob.factor(sine.evaluate(xy, C0))
    prob.solve(directions(M))
    data = prob.far_field() + prob.jvp(sine.evaluate(xy, dC))
    C1, _, _, _ = gn.gauss_newton_step(L, k, C0, data, directions(M), P, 2.0, band=band)
    assert np.array_equal(C1[~keep], C0[~keep])
    assert np.max(np.abs(C1 - (C0 + dC))) < 1e-6 * np.max(np.abs(dC))
