"""One Gauss-Newton step of the Newton iteration of Section 3.3 on the
band-limited model (eq. normaleq): solve
    min || J E dc - (u_far - F[q]) ||
in the least-squares sense for real coefficients dc (real and imaginary parts
stacked), then c <- c + dc.  The oracle forms the explicit Jacobian of the
sine coefficients (one derivative solve per coefficient, Theorem 1) and calls
a dense least-squares routine; the library instead runs conjugate gradients on
the normal equations with derivative/adjoint solves, which Section 4 notes is
algebraically identical to LSQR.
"""
import numpy as np

from . import sine
from .bie import circle_points
from .forward import Problem


def band_mask(S, band):
    """[S, S] boolean: the modes (m, n) with m + n <= band (eq. sineseries'
    triangular index set); band = 0 keeps all S x S modes."""
    m = np.arange(1, S + 1)
    keep = (m[:, None] + m[None, :]) <= band if band > 0 else np.ones((S, S), dtype=bool)
    return keep


def gauss_newton_step(L, k, C0, data, dir_angles, P, R, p=16, box=(-1.0, 1.0, -1.0, 1.0), band=0):
    """Returns (C1, residual_before, J_c) for one step from coefficients C0;
    with band > 0 only the modes with m + n <= band are unknowns (the other
    coefficients keep their values)."""
    prob = Problem(L, k, p, box)
    xy = prob.grid.pde_coords()
    S = C0.shape[0]
    q0 = sine.evaluate(xy, C0, box)
    prob.factor(q0)
    prob.solve(np.asarray(dir_angles))
    _, th = circle_points(R, P)
    prob.set_measurement(th, R)
    r = np.asarray(data) - prob.far_field()
    E = sine.basis(xy, S, box)
    cols = np.flatnonzero(band_mask(S, band).ravel())
    Jc = np.stack([prob.jvp(E[:, c]).ravel() for c in cols], axis=1)
    A = np.concatenate([Jc.real, Jc.imag], axis=0)
    b = np.concatenate([r.ravel().real, r.ravel().imag])
    dcs, *_ = np.linalg.lstsq(A, b, rcond=None)
    dc = np.zeros(S * S)
    dc[cols] = dcs
    return C0 + dc.reshape(S, S), r, Jc, prob
