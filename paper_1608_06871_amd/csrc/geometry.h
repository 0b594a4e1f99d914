// Host-side geometry of the hierarchical discretisation: Chebyshev-Lobatto
// leaves in Morton order, the binary merge tree with its per-level index
// patterns, and the quadrature of the boundary layer potentials.
#pragma once
#include <complex>
#include <cstdint>
#include <vector>

namespace hps {

typedef std::complex<double> cplx;

struct LevelPattern {
  int count = 0;  // merges at this level
  int nc = 0;     // boundary size of each child box
  int m = 0;      // n1 = n2: exterior nodes of each child
  int s = 0;      // n3: nodes on the shared edge
  int np = 0;     // boundary size of the parent (= 2 m)
  // positions inside the children's boundary lists; pos3b follows the
  // order of pos3a (same physical nodes)
  std::vector<int> pos1a, pos3a, pos2b, pos3b;
};

struct BoundaryNode {
  double x, y, nx, ny;  // coordinates and outward normal of Omega
  int panel;            // leaf edge on the outer boundary: side * L + index
  int local;            // position among the panel's p - 2 nodes (ascending)
};

struct Geometry {
  int L = 0, p = 0, mi = 0, ne = 0, nleaf = 0, nlev = 0;
  double x0 = 0, y0 = 0, h = 0;
  std::vector<double> t;   // Lobatto nodes on [-1, 1], ascending
  std::vector<double> D;   // p x p differentiation matrix, row-major
  std::vector<LevelPattern> lev;     // lev[1..nlev]
  std::vector<BoundaryNode> root;    // outer boundary in root order

  void build(double x0, double x1, double y0, int L, int p);
  // coordinates of the PDE nodes in interface order ([leaf Morton][b][a])
  void pde_coords(double* xy) const;
  // leaf-local unknown index of grid point (a, b), -1 at corners
  int lidx(int a, int b) const;
};

// Leaf operators for wavenumber k and impedance eta (row-major complex):
//   A0   [n x n]   collocation matrix with q = 0: PDE rows at the interior
//                  nodes, incoming-impedance rows d_nu u + i eta u at the edges
//   Mout [ne x n]  outgoing impedance d_nu u - i eta u at the edge nodes
void leaf_operators(const Geometry& g, double k, double eta, std::vector<cplx>& A0,
                    std::vector<cplx>& Mout);

// Single- and double-layer moments: S[i][j] = int G(x_i, y) ell_j(y) ds,
// K[i][j] = p.v. int dG/dn_y(x_i, y) ell_j(y) ds over the panel of column j,
// for targets x_i (row-major, [ntarget x nb]).  Targets on the boundary are
// handled by graded refinement towards the singular point.
void layer_moments(const Geometry& g, double k, const std::vector<double>& tx,
                   const std::vector<double>& ty, std::vector<cplx>& S, std::vector<cplx>& K,
                   int nthreads);

// Moments of the combined-field (Burton-Miller) exterior relation on the
// outer-boundary nodes (row-major [nb x nb], root order):
//   Kp[i][j] = int dG/dn_x(x_i, y) ell_j(y) ds (adjoint double layer),
//   T1[i][j] = d/dsigma_x int G(x_i, y) d(ell_j)/dsigma ds (the tangential
//              part of the hypersingular operator in Maue's form, including
//              the interpolant's jumps at the panel ends; principal value on
//              the target's own panel).
// The full hypersingular operator is T1 + k^2 (n_i . n_j) S.
void combined_field_moments(const Geometry& g, double k, std::vector<cplx>& Kp, std::vector<cplx>& T1,
                            int nthreads);

}  // namespace hps
