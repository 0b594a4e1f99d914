"""Band-limited sine model of the contrast (eq. sineseries, Section 3.2) and
its adjoint, in the form sin(m pi (x - x0)/(x1 - x0)) sin(n pi (y - y0)/(y1 - y0))
on Omega = [x0, x1] x [y0, y1] with the square index set 1 <= m, n <= S.

E maps coefficients C [S, S] (row m = x mode, column n = y mode) to values at
points; E^T is its transpose (real).  Pinned by tests: single-mode values at
points where they are exact fractions of pi (tests/golden/sine_mode_values.txt),
orthonormality of the modes under a tensor Gauss-Legendre rule, E^T as the
exact transpose, and vanishing on the boundary of Omega.
"""
import numpy as np


def basis(xy, S, box=(-1.0, 1.0, -1.0, 1.0)):
    """Dense matrix [n_points, S * S]; column (m - 1) * S + (n - 1)."""
    x0, x1, y0, y1 = box
    xy = np.asarray(xy, dtype=np.float64)
    m = np.arange(1, S + 1)
    sx = np.sin(np.pi * m[None, :] * (xy[:, 0:1] - x0) / (x1 - x0))
    sy = np.sin(np.pi * m[None, :] * (xy[:, 1:2] - y0) / (y1 - y0))
    return (sx[:, :, None] * sy[:, None, :]).reshape(xy.shape[0], S * S)


def evaluate(xy, C, box=(-1.0, 1.0, -1.0, 1.0)):
    """q at points xy for coefficients C [S, S]."""
    C = np.asarray(C, dtype=np.float64)
    return basis(xy, C.shape[0], box) @ C.ravel()


def adjoint(xy, g, S, box=(-1.0, 1.0, -1.0, 1.0)):
    """E^T g as an [S, S] array."""
    return (basis(xy, S, box).T @ np.asarray(g, dtype=np.float64)).reshape(S, S)
