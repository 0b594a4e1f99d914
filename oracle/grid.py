"""Geometry of the discretisation (Section 2: a uniform quad-tree of leaves, each
carrying a p x p tensor Chebyshev grid; Section 4: 2^l x 2^l leaves of 16 x 16
points).

Reading used (the paper defers details to the HPS reference it cites):
* Omega = [x0, x1] x [y0, y1] with square leaves, L x L of them;
* Chebyshev-Lobatto points per leaf (the node count (15 * 2^l + 1)^2 of
  Table 1 requires leaves to share their edge points);
* leaf corner points are dropped: they enter no equation;
* unknowns are the total field u at every distinct non-corner grid point
  (shared edge points are single valued) and the scattered normal
  derivative t at every point of the outer boundary.

PDE-node layout shared with the library's interface (test contract, not
code): leaves in Morton order (x bit below y bit), and inside a leaf the
(p-2) x (p-2) interior points row-major with y as the slow index.
"""
import numpy as np

from .cheb import lobatto_nodes


def morton(i, j):
    """Interleave the bits of leaf column i (even bits) and row j (odd bits)."""
    z = 0
    b = 0
    while (i >> b) or (j >> b):
        z |= ((i >> b) & 1) << (2 * b)
        z |= ((j >> b) & 1) << (2 * b + 1)
        b += 1
    return z


class Grid:
    """Global collocation grid of L x L leaves with p points per leaf side."""

    def __init__(self, L, p=16, box=(-1.0, 1.0, -1.0, 1.0)):
        x0, x1, y0, y1 = map(float, box)
        if abs((x1 - x0) - (y1 - y0)) > 1e-15 * abs(x1 - x0):
            raise ValueError("square domain expected")
        self.L, self.p = int(L), int(p)
        self.x0, self.y0 = x0, y0
        self.h = (x1 - x0) / L
        self.t = lobatto_nodes(p)
        pm = p - 1
        self.G = pm * L  # last global index per axis
        n = self.G + 1
        g = np.arange(n)
        frac = (1.0 + self.t[g % pm]) / 2.0
        self.xg = x0 + self.h * (g // pm + frac)
        self.yg = y0 + self.h * (g // pm + frac)
        # unknown index of every global point (gy, gx); -1 at leaf corners
        corner = (g[:, None] % pm == 0) & (g[None, :] % pm == 0)
        self.uidx = -np.ones((n, n), dtype=np.int64)
        self.uidx[~corner] = np.arange(np.count_nonzero(~corner))
        self.nu = int(np.count_nonzero(~corner))

        # outer-boundary points: four sides, each a run of leaf edges (panels)
        # side 0 bottom (y = y0), 1 right, 2 top, 3 left; parameter increasing
        # in x (sides 0, 2) or y (sides 1, 3)
        bnodes = []  # (gy, gx, side, panel_on_side, local_index)
        for side in range(4):
            for i in range(L):
                for m in range(1, pm):
                    s = pm * i + m
                    if side == 0:
                        gy, gx = 0, s
                    elif side == 1:
                        gy, gx = s, self.G
                    elif side == 2:
                        gy, gx = self.G, s
                    else:
                        gy, gx = s, 0
                    bnodes.append((gy, gx, side, i, m - 1))
        self.bnodes = np.array(bnodes, dtype=np.int64)
        self.nb = len(bnodes)
        self.normals = np.array([[0.0, -1.0], [1.0, 0.0], [0.0, 1.0], [-1.0, 0.0]])
        self.bxy = np.stack([self.xg[self.bnodes[:, 1]], self.yg[self.bnodes[:, 0]]], axis=1)
        self.bnormal = self.normals[self.bnodes[:, 2]]

        # PDE (leaf-interior) nodes in the interface layout
        pdx = []
        for z in range(L * L):
            i, j = self.leaf_of_morton(z)
            for b in range(1, pm):
                for a in range(1, pm):
                    pdx.append((pm * j + b, pm * i + a))
        self.pde_g = np.array(pdx, dtype=np.int64)
        self.npde = len(pdx)
        self.pde_u = self.uidx[self.pde_g[:, 0], self.pde_g[:, 1]]

    def leaf_of_morton(self, z):
        i = j = 0
        b = 0
        while z >> (2 * b):
            i |= ((z >> (2 * b)) & 1) << b
            j |= ((z >> (2 * b + 1)) & 1) << b
            b += 1
        return i, j

    def pde_coords(self):
        """[npde, 2] coordinates of the PDE nodes in the interface layout."""
        return np.stack([self.xg[self.pde_g[:, 1]], self.yg[self.pde_g[:, 0]]], axis=1)

    def panels(self):
        """List of (A, B, normal) for the leaf edges on the outer boundary, in
        the order (side, index along side); A -> B is the increasing
        parameter direction, boundary nodes of a panel sit at
        A + (B - A) (1 + t_m) / 2 for the interior Lobatto nodes t_m."""
        out = []
        x0, y0, h, L = self.x0, self.y0, self.h, self.L
        X1, Y1 = x0 + h * L, y0 + h * L
        for side in range(4):
            n = self.normals[side]
            for i in range(L):
                if side == 0:
                    A, B = (x0 + h * i, y0), (x0 + h * (i + 1), y0)
                elif side == 1:
                    A, B = (X1, y0 + h * i), (X1, y0 + h * (i + 1))
                elif side == 2:
                    A, B = (x0 + h * i, Y1), (x0 + h * (i + 1), Y1)
                else:
                    A, B = (x0, y0 + h * i), (x0, y0 + h * (i + 1))
                out.append((np.array(A), np.array(B), n.copy()))
        return out
