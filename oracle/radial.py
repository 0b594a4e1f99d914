"""Independent reference for radially symmetric contrasts (used only to pin the
forward oracle): separation of variables in polar coordinates.

For q = q(r) supported in r <= a, plane-wave incidence from angle phi_d
(u_inc = sum_n i^n J_n(k r) e^{i n (phi - phi_d)}, the Jacobi-Anger expansion)
each angular mode of the total field is c_n psi_n(r) inside, where psi_n is
the regular solution of
    psi'' + psi'/r + (k^2 (1 - q(r)) - n^2 / r^2) psi = 0,
and i^n J_n(k r) + b_n H_n(k r) outside (the Sommerfeld condition of eq.
(srad) keeps only H_n^(1)).  Continuity of u and d_r u at r = a gives b_n, and
u_s(R, theta) = sum_n b_n H_n(k R) e^{i n (theta - phi_d)} (Section 1 data).
"""
import numpy as np
from scipy.integrate import solve_ivp
from scipy.special import hankel1, h1vp, jv, jvp


def _regular_log_derivative(k, q_of_r, n, a, r0=1e-4):
    """psi_n'(a) / psi_n(a) for the regular solution, started from the
    constant-coefficient Bessel solution at r0 (q is flat there)."""
    k1 = k * np.sqrt(1.0 - q_of_r(0.0))
    y0 = [jv(n, k1 * r0), k1 * jvp(n, k1 * r0)]
    scale = max(abs(y0[0]), abs(y0[1]))
    y0 = [y0[0] / scale, y0[1] / scale]

    def rhs(r, y):
        return [y[1], -y[1] / r - (k * k * (1.0 - q_of_r(r)) - n * n / (r * r)) * y[0]]

    sol = solve_ivp(rhs, (r0, a), y0, method='DOP853', rtol=1e-13, atol=1e-300)
    psi, dpsi = sol.y[0, -1], sol.y[1, -1]
    return psi, dpsi


def scattered_on_circle(k, q_of_r, a, phi_d, R, thetas, nmax=None):
    """u_s(R cos theta, R sin theta) for a radial contrast supported in r <= a."""
    if nmax is None:
        nmax = int(np.ceil(k * max(a, R))) + 25
    thetas = np.asarray(thetas, dtype=np.float64)
    out = np.zeros(thetas.shape, dtype=np.complex128)
    for n in range(0, nmax + 1):
        psi, dpsi = _regular_log_derivative(k, q_of_r, n, a)
        J, dJ = jv(n, k * a), jvp(n, k * a)
        H, dH = hankel1(n, k * a), h1vp(n, k * a)
        b = (1j ** n) * (J * dpsi - k * dJ * psi) / (k * dH * psi - H * dpsi)
        term = b * hankel1(n, k * R)
        if n == 0:
            out += term
        else:
            # mode -n has the same radial equation; b_{-n} = b_n and
            # H_{-n} = (-1)^n H_n, i^{-n} J_{-n} = i^n J_n, so the pair
            # contributes 2 b_n H_n(kR) cos(n (theta - phi_d))
            out += 2.0 * term * np.cos(n * (thetas - phi_d))
    return out
