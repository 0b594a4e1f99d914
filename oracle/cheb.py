"""Chebyshev-Lobatto collocation on one leaf (Section 2: tensor-product
Chebyshev grids on each leaf represent both u and q).

Pinned by tests/test_oracle_cheb.py: exact differentiation of polynomials of
degree < p, the textbook p = 3 matrix (golden fixture), interpolation of
polynomials of degree < number of nodes.
"""
import numpy as np


def lobatto_nodes(p):
    """p Chebyshev extreme points on [-1, 1] in ascending order,
    t_m = -cos(pi m / (p - 1))."""
    m = np.arange(p, dtype=np.float64)
    return -np.cos(np.pi * m / (p - 1))


def bary_weights(t):
    """Barycentric weights w_j = 1 / prod_{k != j} (t_j - t_k), computed
    directly from the definition (no closed form), normalised to max |w| = 1."""
    t = np.asarray(t, dtype=np.float64)
    n = t.size
    w = np.empty(n)
    for j in range(n):
        d = t[j] - np.delete(t, j)
        w[j] = 1.0 / np.prod(d)
    return w / np.max(np.abs(w))


def diff_matrix(t):
    """Spectral differentiation matrix on the nodes t: (D f)_i = p'(t_i) where
    p interpolates f.  Off-diagonal D_ij = (w_j / w_i) / (t_i - t_j); the
    diagonal makes each row annihilate constants."""
    t = np.asarray(t, dtype=np.float64)
    w = bary_weights(t)
    n = t.size
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            if i != j:
                D[i, j] = (w[j] / w[i]) / (t[i] - t[j])
        D[i, i] = -np.sum(D[i, :])
    return D


def lagrange_eval(nodes, x):
    """Values of the Lagrange basis through `nodes` at points x.
    Returns array [len(x), len(nodes)] with entry (m, j) = ell_j(x_m)
    (barycentric second form; exact at the nodes)."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    w = bary_weights(nodes)
    out = np.zeros((x.size, nodes.size))
    for m, xm in enumerate(x):
        d = xm - nodes
        hit = np.nonzero(d == 0.0)[0]
        if hit.size:
            out[m, hit[0]] = 1.0
            continue
        c = w / d
        out[m, :] = c / np.sum(c)
    return out
