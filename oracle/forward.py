"""Forward scattering problem, Frechet derivative and adjoint, assembled as one
global sparse system and solved by SuperLU (plain definition; no hierarchy).

Paper passages followed:
* eq. (origpde) / (fscatprob), Section 1: Delta u + k^2 (1 - q) u = 0 for the
  total field u = u_inc + u_s, u_inc = exp(i k x . d), u_s radiating;
* Section 2, interior problem on Omega coupled to the exterior; the Remark's
  Green formula gives the exterior relation S d_n u_s = (K - I/2) u_s on the
  boundary, used here without inverting S;
* Section 1: data u_far(theta) = u_s(R cos theta, R sin theta);
* Theorem 1 (eq. Jdef / vdef): J dq = v_far, Delta v + k^2 (1 - q) v =
  k^2 dq u_0, v radiating -- here the exact derivative of the discrete map;
* Theorem 2 / eq. (adjfrechetdef): the adjoint, here the discrete conjugate
  transpose (sum over incident directions).

Discrete system (rows):
  E1  each leaf-interior node: spectral Laplacian (tensor Lobatto
      differentiation of its own leaf) + k^2 (1 - q) u = 0;
  E2  each interior shared-edge node: sum of the outward normal derivatives
      from the two leaves = 0 (u is single valued there);
  E3  each outer-boundary node: d_nu u (leaf spectral) - t = d_nu u_inc;
  E4  outer boundary: S t - (K - I/2) (u - u_inc) = 0.
With exterior="burton_miller" the E4 rows are instead the combined-field
relation (S + i beta (K' + I/2)) t - ((K - I/2) + i beta T) (u - u_inc) = 0,
beta = 1/k: the Green relation plus i beta times its normal derivative, which
stays uniquely solvable at the Dirichlet eigenvalues of the box where the plain
relation does not (the Remark of Section 2 assumes k is not one of them).
Unknowns: u at all non-corner grid nodes, then t at the boundary nodes.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .bie import bm_matrices, boundary_matrices, circle_points, potential_matrices
from .cheb import diff_matrix
from .grid import Grid


def plane_wave(k, d_angle, xy):
    """u_inc = exp(i k x . d) and its gradient at points xy [n, 2]."""
    d = np.array([np.cos(d_angle), np.sin(d_angle)])
    u = np.exp(1j * k * (xy @ d))
    return u, 1j * k * u[:, None] * d[None, :]


class Problem:
    """Discrete forward problem for one (grid, k)."""

    def __init__(self, L, k, p=16, box=(-1.0, 1.0, -1.0, 1.0), exterior="calderon"):
        if exterior not in ("calderon", "burton_miller"):
            raise ValueError("exterior must be 'calderon' or 'burton_miller'")
        self.grid = Grid(L, p, box)
        self.k = float(k)
        self.exterior = exterior
        D = diff_matrix(self.grid.t) * (2.0 / self.grid.h)
        self.D1 = D
        self.D2 = D @ D
        self.S, self.K = boundary_matrices(self.grid, self.k)
        # E4 coefficients: Mt t - Ms (u - u_inc) = 0
        nb = self.grid.nb
        self.Mt = self.S.copy()
        self.Ms = self.K - 0.5 * np.eye(nb)
        if exterior == "burton_miller":
            Kp, T = bm_matrices(self.grid, self.k)
            beta = 1.0 / self.k
            self.Mt = self.Mt + 1j * beta * (Kp + 0.5 * np.eye(nb))
            self.Ms = self.Ms + 1j * beta * T
        self._base = self._assemble_q_independent()
        self.nrow = self._base[3]
        self.ncol = self.grid.nu + self.grid.nb

    # ---------------------------------------------------------------- assembly
    def _assemble_q_independent(self):
        g, p, pm = self.grid, self.grid.p, self.grid.p - 1
        L, G, U = g.L, g.G, g.uidx
        D1, D2 = self.D1, self.D2
        rows, cols, vals = [], [], []
        ar = np.arange(p)
        # E1: rows 0..npde-1 in PDE-node order
        gy, gx = g.pde_g[:, 0], g.pde_g[:, 1]
        i, a = gx // pm, gx % pm
        j, b = gy // pm, gy % pm
        r = np.arange(g.npde)
        cx = U[gy[:, None], pm * i[:, None] + ar[None, :]]
        cy = U[pm * j[:, None] + ar[None, :], gx[:, None]]
        rows += [np.repeat(r, p), np.repeat(r, p)]
        cols += [cx.ravel(), cy.ravel()]
        vals += [D2[a].ravel(), D2[b].ravel()]
        nrow = g.npde
        # E2: vertical interior edges, then horizontal interior edges
        s = np.array([v for v in range(1, G) if v % pm])
        for ie in range(1, L):
            r = nrow + np.arange(s.size)
            left = U[s[:, None], pm * (ie - 1) + ar[None, :]]
            right = U[s[:, None], pm * ie + ar[None, :]]
            rows += [np.repeat(r, p)] * 2
            cols += [left.ravel(), right.ravel()]
            vals += [np.tile(D1[pm], s.size), np.tile(-D1[0], s.size)]
            nrow += s.size
        for je in range(1, L):
            r = nrow + np.arange(s.size)
            below = U[pm * (je - 1) + ar[None, :], s[:, None]]
            above = U[pm * je + ar[None, :], s[:, None]]
            rows += [np.repeat(r, p)] * 2
            cols += [below.ravel(), above.ravel()]
            vals += [np.tile(D1[pm], s.size), np.tile(-D1[0], s.size)]
            nrow += s.size
        # E3: outer-boundary normal derivative minus t
        self.e3_row0 = nrow
        for bi, (gyb, gxb, side, _, _) in enumerate(g.bnodes):
            if side == 0:
                c, v = U[ar, gxb], -D1[0]
            elif side == 1:
                c, v = U[gyb, pm * (L - 1) + ar], D1[pm]
            elif side == 2:
                c, v = U[pm * (L - 1) + ar, gxb], D1[pm]
            else:
                c, v = U[gyb, ar], -D1[0]
            rows += [np.full(p + 1, nrow + bi)]
            cols += [np.append(c, g.nu + bi)]
            vals += [np.append(v, -1.0)]
        nrow += g.nb
        # E4: dense Calderon rows
        self.e4_row0 = nrow
        bu = U[g.bnodes[:, 0], g.bnodes[:, 1]]
        self.bu = bu
        rr = nrow + np.repeat(np.arange(g.nb), g.nb)
        rows += [rr, rr]
        cols += [np.tile(g.nu + np.arange(g.nb), g.nb), np.tile(bu, g.nb)]
        vals += [self.Mt.ravel(), -self.Ms.ravel()]
        nrow += g.nb
        rows = np.concatenate(rows)
        cols = np.concatenate(cols)
        vals = np.concatenate([np.asarray(v, dtype=np.complex128) for v in vals])
        return rows, cols, vals, nrow

    def matrix(self, q):
        """Global sparse matrix for contrast q given at the PDE nodes."""
        q = np.asarray(q, dtype=np.float64)
        if q.shape != (self.grid.npde,):
            raise ValueError("q must have one value per PDE node")
        rows, cols, vals, nrow = self._base
        r = np.arange(self.grid.npde)
        rows = np.concatenate([rows, r])
        cols = np.concatenate([cols, self.grid.pde_u])
        vals = np.concatenate([vals, self.k ** 2 * (1.0 - q)])
        return sp.csc_matrix((vals, (rows, cols)), shape=(nrow, self.ncol))

    def rhs(self, dir_angles):
        """Right-hand sides (one column per incident direction)."""
        g = self.grid
        B = np.zeros((self.nrow, len(dir_angles)), dtype=np.complex128)
        for m, th in enumerate(dir_angles):
            u, grad = plane_wave(self.k, th, g.bxy)
            B[self.e3_row0:self.e3_row0 + g.nb, m] = np.sum(grad * g.bnormal, axis=1)
            B[self.e4_row0:self.e4_row0 + g.nb, m] = -self.Ms @ u
        return B

    # ------------------------------------------------------------------ solves
    def factor(self, q):
        self.q = np.asarray(q, dtype=np.float64)
        self.lu = spla.splu(self.matrix(self.q))
        return self

    def solve(self, dir_angles):
        """Total-field solve for every direction; keeps the solutions."""
        self.dirs = np.asarray(dir_angles, dtype=np.float64)
        self.X = self.lu.solve(self.rhs(self.dirs))
        return self.X

    def set_measurement(self, thetas, R):
        X = np.stack([R * np.cos(thetas), R * np.sin(thetas)], axis=1)
        self.PS, self.PD = potential_matrices(self.grid, self.k, X)

    def boundary_data(self, X, incident=True):
        """(s, t): scattered trace and scattered normal derivative on the outer
        boundary for solution columns X."""
        g = self.grid
        ub = X[self.bu, :]
        t = X[g.nu:g.nu + g.nb, :]
        if incident:
            inc = np.stack([plane_wave(self.k, th, g.bxy)[0] for th in self.dirs], axis=1)
            ub = ub - inc
        return ub, t

    def far_field(self, X=None, incident=True):
        """u_far [M, P]: the scattered field on the measurement circle,
        D s - S t evaluated there."""
        if X is None:
            X = self.X
        s, t = self.boundary_data(X, incident)
        return (self.PD @ s - self.PS @ t).T

    def u_pde(self, X=None):
        """Total field at the PDE nodes [npde, M]."""
        if X is None:
            X = self.X
        return X[self.grid.pde_u, :]

    def jvp(self, dq):
        """Frechet derivative applied to a real perturbation dq at the PDE
        nodes (Theorem 1): returns dU_far [M, P]."""
        dq = np.asarray(dq, dtype=np.float64)
        B = np.zeros((self.nrow, self.X.shape[1]), dtype=np.complex128)
        B[:self.grid.npde, :] = self.k ** 2 * dq[:, None] * self.u_pde()
        V = self.lu.solve(B)
        return self.far_field(V, incident=False)

    def vjp(self, r):
        """Re(J^H r) for r [M, P] (Theorem 2 in its discrete form): the
        adjoint solve with A^H, restricted to the PDE rows, times
        k^2 conj(u_0), summed over directions."""
        r = np.asarray(r, dtype=np.complex128)
        g = self.grid
        Y = np.zeros((self.ncol, r.shape[0]), dtype=np.complex128)
        Y[self.bu, :] = self.PD.conj().T @ r.T
        Y[g.nu:g.nu + g.nb, :] = -self.PS.conj().T @ r.T
        Lam = self.lu.solve(Y, trans='H')
        w = self.k ** 2 * np.conj(self.u_pde()) * Lam[:g.npde, :]
        return np.real(np.sum(w, axis=1))

    def jacobian(self):
        """Explicit Jacobian [M * P, npde] (complex), one JVP per PDE node;
        for tiny grids only."""
        cols = []
        for n in range(self.grid.npde):
            e = np.zeros(self.grid.npde)
            e[n] = 1.0
            cols.append(self.jvp(e).ravel())
        return np.stack(cols, axis=1)


def directions(M):
    """Incident angles 2 pi m / M, m = 0..M-1 (Section 4)."""
    return 2.0 * np.pi * np.arange(M) / M


def forward(L, k, q, M, P, R, p=16, box=(-1.0, 1.0, -1.0, 1.0)):
    """u_far [M, P] for contrast q at the PDE nodes."""
    prob = Problem(L, k, p, box).factor(q)
    prob.solve(directions(M))
    _, th = circle_points(R, P)
    prob.set_measurement(th, R)
    return prob.far_field(), prob
