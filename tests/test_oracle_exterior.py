"""Pins for the oracle's combined-field (Burton-Miller) exterior relation.

The Remark of Section 2 couples the interior solver to the exterior through
the Green relation S t = (K - I/2) s and assumes k^2 is not a Dirichlet
eigenvalue of the box.  The combined field adds i/k times the normal
derivative of that relation, (S + i/k (K' + I/2)) t = (K - I/2 + i/k T) s,
which has no such exceptional wavenumbers.  Checked here:
* the two jump relations of the normal derivative of Green's formula on the
  discrete operators: (K' + I/2) d_n v = T v for a field radiating from a
  source inside the box, (K' - I/2) d_n u = T u for an interior solution
  (a plane wave) -- a sign slip in K', a missing jump term or a wrong T
  fails one of them;
* at the lowest Dirichlet eigenvalue k = pi/sqrt(2) of [-1, 1]^2 the Green
  relation gives a wrong far field while the combined field matches the
  radial reference by separation of variables;
* away from eigenvalues both relations give the same far field, and the
  derivative of the combined-field map passes the central-difference and
  adjoint checks."""
import numpy as np
import pytest
from scipy.special import hankel1

import synth
from oracle.bie import bm_matrices, boundary_matrices, circle_points
from oracle.forward import Problem, directions, plane_wave
from oracle.grid import Grid
from oracle.radial import scattered_on_circle

K_EIG = np.pi / np.sqrt(2.0)  # (pi/2) sqrt(1^2 + 1^2)


def _point_source(g, k, z):
    d = g.bxy - z[None, :]
    r = np.hypot(d[:, 0], d[:, 1])
    v = 0.25j * hankel1(0, k * r)
    dv = -0.25j * k * hankel1(1, k * r) * np.sum(d * g.bnormal, axis=1) / r
    return v, dv


@pytest.mark.parametrize("L,k,tol", [(2, 5.0, 2e-7), (4, 10.0, 1e-8)])
def test_exterior_jump_relation(L, k, tol):
    g = Grid(L)
    Kp, T = bm_matrices(g, k)
    v, dv = _point_source(g, k, np.array([0.13, -0.21]))
    e = (Kp + 0.5 * np.eye(g.nb)) @ dv - T @ v
    assert np.max(np.abs(e)) < tol * np.max(np.abs(T @ v))


def test_interior_jump_relation_converges():
    errs = []
    for L in (2, 4):
        g = Grid(L)
        Kp, T = bm_matrices(g, 5.0)
        u, grad = plane_wave(5.0, 0.3, g.bxy)
        du = np.sum(grad * g.bnormal, axis=1)
        e = (Kp - 0.5 * np.eye(g.nb)) @ du - T @ u
        errs.append(np.max(np.abs(e)) / np.max(np.abs(T @ u)))
    assert errs[1] < 1e-11 and errs[1] < 1e-3 * errs[0]


def test_own_panel_blocks_are_translation_invariant():
    """The block of T on a target's own panel depends only on the panel's
    length, the node positions and k (principal value, Cauchy-part
    subtraction and end terms); every panel of the box has the same length,
    so all own-panel blocks must agree."""
    g = Grid(2)
    _, T = bm_matrices(g, 5.0)
    pan = g.bnodes[:, 2] * g.L + g.bnodes[:, 3]
    blocks = []
    for P in range(4 * g.L):
        rows = np.flatnonzero(pan == P)
        rows = rows[np.argsort(g.bnodes[rows, 4])]
        blocks.append(T[np.ix_(rows, rows)])
    for b in blocks[1:]:
        assert np.max(np.abs(b - blocks[0])) < 1e-11 * np.max(np.abs(blocks[0]))


def _radial_case(k, L, exterior):
    amp, sig = 0.4, 0.2
    th = 2 * np.pi * np.arange(16) / 16
    ref = scattered_on_circle(k, lambda r: amp * np.exp(-r * r / sig ** 2), 1.0, 0.7, 2.0, th)
    prob = Problem(L, k, exterior=exterior)
    q = synth.radial_gaussian(prob.grid.pde_coords(), amp, sig)
    prob.factor(q)
    prob.solve(np.array([0.7]))
    prob.set_measurement(th, 2.0)
    uf = prob.far_field()[0]
    return np.max(np.abs(uf - ref)) / np.max(np.abs(ref))


def test_combined_field_is_correct_at_a_dirichlet_eigenvalue():
    assert _radial_case(K_EIG, 4, "calderon") > 1e-2
    assert _radial_case(K_EIG, 4, "burton_miller") < 1e-6


def test_combined_field_agrees_with_green_relation_off_resonance():
    L, k, M, P = 4, 7.0, 3, 16
    xy = Grid(L).pde_coords()
    q = synth.gaussian_bumps(xy, 5, 3)
    _, th = circle_points(2.0, P)
    out = []
    for ext in ("calderon", "burton_miller"):
        prob = Problem(L, k, exterior=ext)
        prob.factor(q)
        prob.solve(directions(M))
        prob.set_measurement(th, 2.0)
        out.append(prob.far_field())
    assert np.max(np.abs(out[0] - out[1])) < 1e-7 * np.max(np.abs(out[0]))


def test_combined_field_derivatives():
    L, k, M, P = 2, 5.0, 3, 8
    prob = Problem(L, k, exterior="burton_miller")
    xy = prob.grid.pde_coords()
    q = synth.gaussian_bumps(xy, 5, 1)
    _, th = circle_points(2.0, P)
    prob.set_measurement(th, 2.0)

    def F(qq):
        prob.factor(qq)
        prob.solve(directions(M))
        return prob.far_field()

    dq = synth.gaussian_bumps(xy, 3, 7)
    h = 1e-4
    fd = (F(q + h * dq) - F(q - h * dq)) / (2 * h)
    F(q)
    jv = prob.jvp(dq)
    assert np.max(np.abs(fd - jv)) < 1e-6 * np.max(np.abs(jv))
    rng = np.random.default_rng(0)
    r = rng.standard_normal((M, P)) + 1j * rng.standard_normal((M, P))
    jv = prob.jvp(dq)
    lhs = np.real(np.vdot(r, jv))
    # rounding in both sides scales with |r| |J dq|, not with the inner product
    assert abs(lhs - dq @ prob.vjp(r)) < 1e-12 * np.linalg.norm(r) * np.linalg.norm(jv)


def test_unknown_exterior_rejected():
    with pytest.raises(ValueError):
        Problem(1, 3.0, exterior="dirichlet")
