"""Independent reference for radially symmetric contrasts (used only to pin the
forward oracle): separation of variables in polar coordinates.

For q = q(r) supported in r <= a, plane-wave incidence from angle phi_d
(u_inc = sum_n i^n J_n(k r) e^{i n (phi - phi_d)}, the Jacobi-Anger expansion)
each angular mode of the total field is c_n psi_n(r) inside, where psi_n is
the regular solution (psi_n ~ r^n at 0) of
    psi'' + psi'/r + (k^2 (1 - q(r)) - n^2 / r^2) psi = 0,
and i^n J_n(k r) + b_n H_n(k r) outside (the Sommerfeld condition of eq.
(srad) keeps only H_n^(1)).  Continuity of u and d_r u at r = a gives b_n, and
u_s(R, theta) = sum_n b_n H_n(k R) e^{i n (theta - phi_d)} (Section 1 data).
"""
import numpy as np
from scipy.integrate import solve_ivp
from scipy.special import hankel1, h1vp, jv, jvp


def _regular_log_derivative(k, q_of_r, n, a, r0=1e-4):
    """psi_n'(a) / psi_n(a) for the regular solution.  Writing psi = r^n phi,
    phi solves phi'' + (2n+1)/r phi' + k^2 (1 - q) phi = 0 with phi(0) = 1,
    phi'(0) = 0; it stays O(1) for every n, so high modes neither under- nor
    overflow.  Started from its series at r0 (q is flat there)."""
    k2 = k * k
    c = k2 * (1.0 - q_of_r(0.0)) / (2.0 * (2 * n + 2))
    y0 = [1.0 - c * r0 * r0, -2.0 * c * r0]

    def rhs(r, y):
        return [y[1], -(2 * n + 1) / r * y[1] - k2 * (1.0 - q_of_r(r)) * y[0]]

    sol = solve_ivp(rhs, (r0, a), y0, method='DOP853', rtol=1e-13, atol=1e-300)
    phi, dphi = sol.y[0, -1], sol.y[1, -1]
    return n / a + dphi / phi


def mode_coefficients(k, q_of_r, a, R, nmax=None):
    """b_n H_n(k R) for n = 0..nmax (radial contrast supported in r <= a)."""
    if nmax is None:
        nmax = int(np.ceil(k * max(a, R))) + 25
    out = np.zeros(nmax + 1, dtype=np.complex128)
    for n in range(0, nmax + 1):
        ld = _regular_log_derivative(k, q_of_r, n, a)
        J, dJ = jv(n, k * a), jvp(n, k * a)
        H, dH = hankel1(n, k * a), h1vp(n, k * a)
        b = (1j ** n) * (J * ld - k * dJ) / (k * dH - H * ld)
        out[n] = b * hankel1(n, k * R)
    return out


def scattered_from_modes(coef, angle_diff):
    """u_s at measurement angle theta for incidence phi_d, as a function of
    theta - phi_d (rotational symmetry of a radial contrast)."""
    d = np.asarray(angle_diff, dtype=np.float64)
    out = np.full(d.shape, coef[0], dtype=np.complex128)
    for n in range(1, coef.size):
        out += 2.0 * coef[n] * np.cos(n * d)
    return out


def scattered_on_circle(k, q_of_r, a, phi_d, R, thetas, nmax=None):
    """u_s(R cos theta, R sin theta) for a radial contrast supported in r <= a."""
    if nmax is None:
        nmax = int(np.ceil(k * max(a, R))) + 25
    thetas = np.asarray(thetas, dtype=np.float64)
    out = np.zeros(thetas.shape, dtype=np.complex128)
    for n in range(0, nmax + 1):
        ld = _regular_log_derivative(k, q_of_r, n, a)
        J, dJ = jv(n, k * a), jvp(n, k * a)
        H, dH = hankel1(n, k * a), h1vp(n, k * a)
        b = (1j ** n) * (J * ld - k * dJ) / (k * dH - H * ld)
        term = b * hankel1(n, k * R)
        if n == 0:
            out += term
        else:
            # mode -n has the same radial equation; b_{-n} = b_n and
            # H_{-n} = (-1)^n H_n, i^{-n} J_{-n} = i^n J_n, so the pair
            # contributes 2 b_n H_n(kR) cos(n (theta - phi_d))
            out += 2.0 * term * np.cos(n * (thetas - phi_d))
    return out
