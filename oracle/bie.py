"""Layer potentials on the outer boundary of Omega (Remark in Section 2: the
scattered field satisfies u_s = D u_s - S d_n u_s outside Omega, with
G(x, y) = (i/4) H_0^(1)(k |x - y|); the jump relations give the exterior
Calderon relation S t = (K - I/2) s on the boundary).

Discretisation reading: the boundary densities are represented on every leaf
edge of the outer boundary (a panel) by the Lagrange interpolant through the
panel's p - 2 non-corner Lobatto nodes.  The matrices are the exact integrals
of kernel x Lagrange basis over the panel,
    S_ij  = int G(x_i, y) ell_j(y) ds_y,
    K_ij  = p.v. int d/dn_y G(x_i, y) ell_j(y) ds_y,
and the same integrals with the target on the measurement circle give the
far-field (finite-R) matrices.  The integrals are computed by composite
Gauss-Legendre quadrature on panel pieces refined dyadically until each piece
is no longer than its distance to the target and short on the wavelength
scale (k * length <= 4), graded towards the target for the weakly singular
self-panel integrals.

Pinned by tests/test_oracle_bie.py: exterior Calderon identity and Green's
representation for an interior point source, interior Calderon identity for
a plane wave.
"""
import math

import numpy as np
from scipy.special import hankel1

from .cheb import bary_weights

_NG = 20
_GX, _GW = np.polynomial.legendre.leggauss(_NG)
_MIN_LEN = 1e-15  # pieces touching the target below this length are dropped


def kernel_G(k, x, y):
    """Single-layer kernel (i/4) H0(k|x-y|); x [2], y [n, 2]."""
    r = np.hypot(x[0] - y[:, 0], x[1] - y[:, 1])
    return 0.25j * hankel1(0, k * r)


def kernel_dG(k, x, y, n):
    """Double-layer kernel d/dn_y G = (ik/4) H1(k r) ((x - y) . n) / r."""
    dx = x[0] - y[:, 0]
    dy = x[1] - y[:, 1]
    r = np.hypot(dx, dy)
    return 0.25j * k * hankel1(1, k * r) * (dx * n[0] + dy * n[1]) / r


def _lagrange_rows(nodes, w, tau):
    d = tau[:, None] - nodes[None, :]
    d = np.where(d == 0.0, 1e-300, d)
    c = w[None, :] / d
    return c / c.sum(axis=1, keepdims=True)


def _pieces(x, A, B, k):
    """Dyadic pieces [a, b] of the parameter interval [-1, 1] of panel A -> B,
    each no longer than its distance to x and with kernel phase k * length
    at most 4 (pieces that touch x are split until shorter than a tiny
    length and then dropped)."""
    ax, ay = float(A[0]), float(A[1])
    vx, vy = float(B[0]) - ax, float(B[1]) - ay
    L2 = vx * vx + vy * vy
    half = 0.5 * math.sqrt(L2)
    px, py = float(x[0]) - ax, float(x[1]) - ay
    sx = (px * vx + py * vy) / L2          # projection parameter in [0, 1] units
    perp = abs(px * vy - py * vx) / math.sqrt(L2)
    out = []
    stack = [(-1.0, 1.0)]
    while stack:
        a, b = stack.pop()
        s0, s1 = (1 + a) / 2, (1 + b) / 2
        along = 0.0 if s0 <= sx <= s1 else min(abs(sx - s0), abs(sx - s1)) * 2 * half
        d = math.hypot(along, perp)
        length = (b - a) * half
        if d >= length and k * length <= 4.0:
            out.append((a, b))
        elif d == 0.0 and length < _MIN_LEN:
            continue
        else:
            m = 0.5 * (a + b)
            stack.append((a, m))
            stack.append((m, b))
    return out, half


def panel_moments(k, x, A, B, n, nodes):
    """Integrals over one panel of kernel(x, y) * ell_j(y) for all basis
    functions j: returns (S moments, D moments)."""
    pieces, half = _pieces(x, A, B, k)
    a = np.array([p[0] for p in pieces])
    b = np.array([p[1] for p in pieces])
    tau = (0.5 * (a + b))[:, None] + (0.5 * (b - a))[:, None] * _GX[None, :]
    wt = (0.5 * (b - a))[:, None] * _GW[None, :] * half
    tau = tau.ravel()
    wt = wt.ravel()
    y = A[None, :] + (B - A)[None, :] * ((1 + tau) / 2)[:, None]
    lag = _lagrange_rows(nodes, bary_weights(nodes), tau)
    ms = (kernel_G(k, x, y) * wt) @ lag
    md = (kernel_dG(k, x, y, n) * wt) @ lag
    return ms, md


def _panel_arrays(grid):
    P = grid.panels()
    A = np.array([p[0] for p in P])
    B = np.array([p[1] for p in P])
    N = np.array([p[2] for p in P])
    return A, B, N


def _moments_all_panels(k, x, A, B, N, nodes, lag_far):
    """S and D moments of every panel for one target x: [n_panels, nloc] each.
    Panels no longer than their distance to x take one Gauss rule (vectorised);
    the others go through the adaptive piece refinement."""
    v = B - A
    L2 = np.einsum('ij,ij->i', v, v)
    s = np.clip(np.einsum('ij,ij->i', x[None, :] - A, v) / L2, 0.0, 1.0)
    c = A + s[:, None] * v
    dist = np.hypot(x[0] - c[:, 0], x[1] - c[:, 1])
    length = np.sqrt(L2)
    far = (dist >= length) & (k * length <= 4.0)
    nloc = nodes.size
    MS = np.zeros((len(A), nloc), dtype=np.complex128)
    MD = np.zeros_like(MS)
    if np.any(far):
        fA, fv, fN = A[far], v[far], N[far]
        y = fA[:, None, :] + fv[:, None, :] * ((1 + _GX) / 2)[None, :, None]
        dx = x[0] - y[..., 0]
        dy = x[1] - y[..., 1]
        r = np.hypot(dx, dy)
        w = (0.5 * length[far])[:, None] * _GW[None, :]
        kG = 0.25j * hankel1(0, k * r)
        kD = 0.25j * k * hankel1(1, k * r) * (dx * fN[:, 0:1] + dy * fN[:, 1:2]) / r
        MS[far] = (kG * w) @ lag_far
        MD[far] = (kD * w) @ lag_far
    for j in np.nonzero(~far)[0]:
        MS[j], MD[j] = panel_moments(k, x, A[j], B[j], N[j], nodes)
    return MS, MD


def boundary_matrices(grid, k):
    """S and K (N_b x N_b, complex) on the outer-boundary nodes of `grid`,
    ordered like grid.bnodes (panel-major, panel order of grid.panels())."""
    nodes = grid.t[1:-1]
    A, B, N = _panel_arrays(grid)
    lag_far = _lagrange_rows(nodes, bary_weights(nodes), _GX)
    nb = grid.nb
    S = np.zeros((nb, nb), dtype=np.complex128)
    K = np.zeros((nb, nb), dtype=np.complex128)
    for i in range(nb):
        MS, MD = _moments_all_panels(k, grid.bxy[i], A, B, N, nodes, lag_far)
        S[i] = MS.ravel()
        K[i] = MD.ravel()
    return S, K


def potential_matrices(grid, k, targets):
    """Single- and double-layer potential matrices from the boundary nodes to
    arbitrary targets off the boundary: returns (PhiS, PhiD), each
    [n_targets, N_b]."""
    nodes = grid.t[1:-1]
    A, B, N = _panel_arrays(grid)
    lag_far = _lagrange_rows(nodes, bary_weights(nodes), _GX)
    targets = np.atleast_2d(targets)
    PS = np.zeros((len(targets), grid.nb), dtype=np.complex128)
    PD = np.zeros_like(PS)
    for i, x in enumerate(targets):
        MS, MD = _moments_all_panels(k, np.asarray(x, dtype=np.float64), A, B, N, nodes, lag_far)
        PS[i] = MS.ravel()
        PD[i] = MD.ravel()
    return PS, PD


def kernel_dGx(k, x, y, v):
    """Derivative of G(x, y) in x along the unit vector v (the target's normal
    or tangent): -(ik/4) H1(k r) ((x - y) . v) / r; x [2], y [n, 2]."""
    dx = x[0] - y[:, 0]
    dy = x[1] - y[:, 1]
    r = np.hypot(dx, dy)
    return -0.25j * k * hankel1(1, k * r) * (dx * v[0] + dy * v[1]) / r


def _dlagrange_rows(nodes, w, tau):
    """d ell_j / dt at points tau (none equal to a node): ell_j(t) times
    sum_{m != j} 1 / (t - t_m)."""
    lag = _lagrange_rows(nodes, w, tau)
    d = tau[:, None] - nodes[None, :]
    tot = np.sum(1.0 / d, axis=1)
    return lag * (tot[:, None] - 1.0 / d)


def _piece_points(x, A, B, k):
    """Gauss points (parameter t, weight in t) of the adaptive pieces of
    panel A -> B for target x (the refinement rule of _pieces)."""
    pieces, _ = _pieces(x, A, B, k)
    a = np.array([p[0] for p in pieces])
    b = np.array([p[1] for p in pieces])
    t = ((0.5 * (a + b))[:, None] + (0.5 * (b - a))[:, None] * _GX[None, :]).ravel()
    wt = ((0.5 * (b - a))[:, None] * _GW[None, :]).ravel()
    return t, wt


def bm_matrices(grid, k):
    """The two further operators of the combined-field (Burton-Miller) form of
    the exterior relation, on the outer-boundary nodes (ordering of
    boundary_matrices): the adjoint double layer
        K'_ij = int d/dn_x G(x_i, y) ell_j(y) ds_y
    and the hypersingular operator T = d/dn_x of the double layer, written by
    Maue's identity for the panel-wise density s = sum_j s_j ell_j:
        T s (x) = d/dsigma_x int G(x, y) (ds/dsigma)(y) dsigma_y
                  + k^2 int G(x, y) (n_x . n_y) s(y) ds_y,
    sigma the arclength along the boundary in the counter-clockwise sense
    (tangent tau = (-n_y, n_x)).  ds/dsigma of a panel's interpolant includes
    point masses at the panel ends (the interpolant's jumps), so a panel P
    from A to B with orientation o = +1 (A -> B counter-clockwise) or -1
    contributes
        o [ int d/dtau_x G(x, y(t)) ell_j'(t) dt + ell_j(-1) d/dtau_x G(x, A)
            - ell_j(1) d/dtau_x G(x, B) ]
    (t the panel parameter).  On the target's own (straight) panel
    d/dtau_x G = -1 / (pi h (t_x - t)) + a bounded remainder, so the
    principal value is
        -1/(pi h) [int (ell'(t) - ell'(t_x)) / (t_x - t) dt
                   + ell'(t_x) log((1 + t_x) / (1 - t_x))]
    and the remainder takes the adaptive rule.  The second term of Maue's
    identity is k^2 (n_x . n_y) S_ij (straight panels)."""
    nodes = grid.t[1:-1]
    w = bary_weights(nodes)
    nloc = nodes.size
    A, B, N = _panel_arrays(grid)
    nP = len(A)
    orient = np.array([1.0 if side in (0, 1) else -1.0 for side in range(4) for _ in range(grid.L)])
    S, _ = boundary_matrices(grid, k)
    nb = grid.nb
    Kp = np.zeros((nb, nb), dtype=np.complex128)
    T1 = np.zeros((nb, nb), dtype=np.complex128)
    lag_end = _lagrange_rows(nodes, w, np.array([-1.0, 1.0]))  # [2, nloc]
    # ell_j'(t_i) on the panel's own nodes: the differentiation matrix
    Dn = np.zeros((nloc, nloc))
    for i in range(nloc):
        for j in range(nloc):
            if i != j:
                Dn[i, j] = (w[j] / w[i]) / (nodes[i] - nodes[j])
        Dn[i, i] = -np.sum(Dn[i])
    gdl = _dlagrange_rows(nodes, w, _GX)  # ell'(t) at the plain Gauss points
    for i in range(nb):
        x = grid.bxy[i]
        nx = grid.bnormal[i]
        tx = np.array([-nx[1], nx[0]])
        Pi = int(grid.bnodes[i, 2]) * grid.L + int(grid.bnodes[i, 3])
        li = int(grid.bnodes[i, 4])
        for P in range(nP):
            cols = slice(P * nloc, (P + 1) * nloc)
            h = float(np.hypot(*(B[P] - A[P])))
            t, wt = _piece_points(x, A[P], B[P], k)
            y = A[P][None, :] + (B[P] - A[P])[None, :] * ((1 + t) / 2)[:, None]
            lag = _lagrange_rows(nodes, w, t)
            Kp[i, cols] = (kernel_dGx(k, x, y, nx) * wt * 0.5 * h) @ lag
            dl = _dlagrange_rows(nodes, w, t)
            jumps = lag_end[0] * kernel_dGx(k, x, A[P][None, :], tx)[0] - lag_end[1] * kernel_dGx(k, x, B[P][None, :], tx)[0]
            if P != Pi:
                T1[i, cols] = orient[P] * ((kernel_dGx(k, x, y, tx) * wt) @ dl + jumps)
                continue
            # own panel: principal value + remainder + the end terms
            t0 = nodes[li]
            dlx = Dn[li]  # ell_j'(t_x)
            dd = (gdl - dlx[None, :]) / (t0 - _GX)[:, None]
            pv = -(1.0 / (np.pi * h)) * (_GW @ dd + dlx * np.log((1 + t0) / (1 - t0)))
            delta = t0 - t
            rem = -0.25j * k * hankel1(1, k * 0.5 * h * np.abs(delta)) * np.sign(delta) + 1.0 / (np.pi * h * delta)
            T1[i, cols] = pv + (rem * wt) @ dl + orient[P] * jumps
    nn = grid.bnormal @ grid.bnormal.T
    T = T1 + k * k * nn * S
    return Kp, T


def circle_points(R, P):
    """Measurement points x_p = R (cos theta_p, sin theta_p), theta_p = 2 pi p / P
    (Section 4 uses equispaced angles on the circle of radius R)."""
    th = 2.0 * np.pi * np.arange(P) / P
    return np.stack([R * np.cos(th), R * np.sin(th)], axis=1), th
