// Host geometry, merge-tree patterns, leaf operators and layer-potential
// quadrature for the HPS solver.
#include "geometry.h"

#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <thread>

namespace hps {

namespace {

const double PI = 3.14159265358979323846;
const double EULER_GAMMA = 0.57721566490153286061;

// Hankel functions H0^(1)(x), H1^(1)(x) for x > 0.
//  * x < 17: J_n by Miller's backward recurrence normalised with
//    J0 + 2 sum J_2k = 1, then Y0, Y1 from the Neumann series
//      Y0 = (2/pi)(ln(x/2) + gamma) J0 - (4/pi) sum_k (-1)^k J_2k / k,
//      Y1 = -(2/(pi x)) J0 + (2/pi)(ln(x/2) + gamma) J1
//           + (2/pi) sum_k (-1)^k (J_{2k-1} - J_{2k+1}) / k
//    (the second is minus the derivative of the first);
//  * x >= 17: Hankel's asymptotic expansion
//      H_nu(x) ~ sqrt(2/(pi x)) e^{i(x - nu pi/2 - pi/4)} sum_k i^k a_k(nu) / x^k,
//    a_k = prod_{j<=k} (4 nu^2 - (2j-1)^2) / (k! 8^k), summed to the smallest term.
void hankel01(double x, cplx& h0, cplx& h1) {
  if (x < 17.0) {
    int N = (int)(x + 10.0 * std::cbrt(x) + 30.0);
    N += N & 1;
    double J[160];
    double jp1 = 0.0, jn = 1e-300;
    J[N] = jn;
    for (int n = N; n > 0; --n) {
      double jm1 = (2.0 * n / x) * jn - jp1;
      jp1 = jn;
      jn = jm1;
      J[n - 1] = jn;
      if (std::fabs(jn) > 1e250) {
        for (int q = n - 1; q <= N; ++q) J[q] *= 1e-250;
        jp1 *= 1e-250;
        jn *= 1e-250;
      }
    }
    double norm = J[0];
    for (int q = 2; q <= N; q += 2) norm += 2.0 * J[q];
    for (int q = 0; q <= N; ++q) J[q] /= norm;
    const double lg = std::log(0.5 * x) + EULER_GAMMA;
    double s0 = 0.0, s1 = 0.0;
    for (int k = 1; 2 * k + 1 <= N; ++k) {
      const double sg = (k & 1) ? -1.0 : 1.0;
      s0 += sg * J[2 * k] / k;
      s1 += sg * (J[2 * k - 1] - J[2 * k + 1]) / k;
    }
    const double Y0 = (2.0 / PI) * lg * J[0] - (4.0 / PI) * s0;
    const double Y1 = -2.0 / (PI * x) * J[0] + (2.0 / PI) * lg * J[1] + (2.0 / PI) * s1;
    h0 = cplx(J[0], Y0);
    h1 = cplx(J[1], Y1);
    return;
  }
  for (int nu = 0; nu <= 1; ++nu) {
    const double mu = 4.0 * nu * nu;
    cplx sum(1.0, 0.0);
    double a = 1.0, prev = 1e300;
    cplx ik(1.0, 0.0);
    for (int k = 1; k < 60; ++k) {
      a *= (mu - (2.0 * k - 1) * (2.0 * k - 1)) / (8.0 * k * x);
      ik *= cplx(0.0, 1.0);
      if (std::fabs(a) >= prev) break;
      prev = std::fabs(a);
      sum += a * ik;
    }
    const double ph = x - nu * 0.5 * PI - 0.25 * PI;
    const cplx v = std::sqrt(2.0 / (PI * x)) * cplx(std::cos(ph), std::sin(ph)) * sum;
    if (nu == 0)
      h0 = v;
    else
      h1 = v;
  }
}

// Gauss-Legendre rule on [-1, 1] (Newton iteration on P_n).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) {
        x[n - 1 - i] = z;
        w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
        break;
      }
      if (it == 99) {
        x[n - 1 - i] = z;
        w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
      }
    }
  }
}

struct Panel {
  double ax, ay, bx, by, nx, ny;
};

struct Quad {
  int nloc;
  std::vector<double> nodes, bw;  // interpolation nodes and barycentric weights
  std::vector<double> gx, gw;     // Gauss rule
  double k;
};

inline void lagrange(const Quad& Q, double tau, double* out) {
  double den = 0.0;
  for (int j = 0; j < Q.nloc; ++j) {
    const double d = tau - Q.nodes[j];
    if (d == 0.0) {
      for (int q = 0; q < Q.nloc; ++q) out[q] = (q == j) ? 1.0 : 0.0;
      return;
    }
    out[j] = Q.bw[j] / d;
    den += out[j];
  }
  for (int j = 0; j < Q.nloc; ++j) out[j] /= den;
}

// Accumulates moments over the parameter piece [a, b] of panel P, refining
// until each piece is no longer than 4/3 of its distance to the target and
// short on the wavelength scale.
void piece(const Quad& Q, const Panel& P, double x, double y, double a, double b, int depth,
           cplx* mS, cplx* mD) {
  const double vx = P.bx - P.ax, vy = P.by - P.ay;
  const double len_full = std::sqrt(vx * vx + vy * vy);
  const double len = 0.5 * (b - a) * len_full;
  // parameter of the orthogonal projection of the target, in [-1, 1] units
  const double px = x - P.ax, py = y - P.ay;
  const double tp = 2.0 * (px * vx + py * vy) / (len_full * len_full) - 1.0;
  const double tc = std::min(std::max(tp, a), b);
  const double cx = P.ax + vx * 0.5 * (1.0 + tc), cy = P.ay + vy * 0.5 * (1.0 + tc);
  const double d = std::hypot(x - cx, y - cy);
  // accept a piece when it is no longer than 4/3 of its distance to the
  // target and the kernel's phase k * len across it is at most 4 (a 16-point
  // rule then resolves the oscillation of the Hankel functions)
  if ((d >= 0.75 * len && Q.k * len <= 4.0) || depth > 200) {
    const double half = 0.5 * (b - a), mid = 0.5 * (a + b);
    double lag[64];
    for (size_t g = 0; g < Q.gx.size(); ++g) {
      const double tau = mid + half * Q.gx[g];
      const double wq = half * Q.gw[g] * 0.5 * len_full;
      const double yx = P.ax + vx * 0.5 * (1.0 + tau), yy = P.ay + vy * 0.5 * (1.0 + tau);
      const double dx = x - yx, dy = y - yy;
      const double r = std::hypot(dx, dy);
      cplx h0, h1;
      hankel01(Q.k * r, h0, h1);
      const cplx gS = cplx(0.0, 0.25) * h0 * wq;
      const cplx gD = cplx(0.0, 0.25 * Q.k) * h1 * ((dx * P.nx + dy * P.ny) / r) * wq;
      lagrange(Q, tau, lag);
      for (int j = 0; j < Q.nloc; ++j) {
        mS[j] += gS * lag[j];
        mD[j] += gD * lag[j];
      }
    }
    return;
  }
  if (d == 0.0 && len < 1e-15) return;  // negligible piece touching a log singularity
  double split = 0.5 * (a + b);
  if (tp > a + 0.05 * (b - a) && tp < b - 0.05 * (b - a)) split = tp;
  piece(Q, P, x, y, a, split, depth + 1, mS, mD);
  piece(Q, P, x, y, split, b, depth + 1, mS, mD);
}

}  // namespace

void Geometry::build(double x0_, double x1_, double y0_, int L_, int p_) {
  L = L_;
  p = p_;
  if (L < 1 || (L & (L - 1))) throw std::invalid_argument("nleaf must be a power of two");
  if (p < 4 || p > 32) throw std::invalid_argument("p must be in [4, 32]");
  x0 = x0_;
  y0 = y0_;
  h = (x1_ - x0_) / L;
  mi = (p - 2) * (p - 2);
  ne = 4 * (p - 2);
  nleaf = L * L;
  nlev = 0;
  while ((1 << nlev) < nleaf) ++nlev;

  // Chebyshev extreme points and the closed-form differentiation matrix
  // (Trefethen, Spectral Methods in MATLAB, ch. 6) written for ascending
  // points t_i = -cos(pi i / N); the diagonal is minus the row sum.
  const int N = p - 1;
  t.assign(p, 0.0);
  for (int i = 0; i < p; ++i) t[i] = -std::cos(PI * i / N);
  D.assign((size_t)p * p, 0.0);
  for (int i = 0; i < p; ++i) {
    double rs = 0.0;
    for (int j = 0; j < p; ++j) {
      if (i == j) continue;
      const double ci = (i == 0 || i == N) ? 2.0 : 1.0;
      const double cj = (j == 0 || j == N) ? 2.0 : 1.0;
      // t_i - t_j = 2 sin((i + j) pi / 2N) sin((i - j) pi / 2N)
      const double diff = 2.0 * std::sin((i + j) * PI / (2.0 * N)) * std::sin((i - j) * PI / (2.0 * N));
      const double v = (ci / cj) * (((i + j) & 1) ? -1.0 : 1.0) / diff;
      D[(size_t)i * p + j] = v;
      rs += v;
    }
    D[(size_t)i * p + i] = -rs;
  }

  // Global edge-node ids: horizontal leaf edges then vertical ones.
  const int m1 = p - 2;
  const long NH = (long)(L + 1) * L * m1;
  auto hid = [&](int jy, int i, int a) { return ((long)jy * L + i) * m1 + (a - 1); };
  auto vid = [&](int ix, int j, int b) { return NH + ((long)ix * L + j) * m1 + (b - 1); };
  std::vector<std::vector<long>> boxes(nleaf);
  for (int z = 0; z < nleaf; ++z) {
    int i = 0, j = 0;
    for (int b = 0; (z >> (2 * b)) != 0; ++b) {
      i |= ((z >> (2 * b)) & 1) << b;
      j |= ((z >> (2 * b + 1)) & 1) << b;
    }
    auto& v = boxes[z];
    v.reserve(ne);
    for (int a = 1; a <= m1; ++a) v.push_back(hid(j, i, a));      // S
    for (int b = 1; b <= m1; ++b) v.push_back(vid(i + 1, j, b));  // E
    for (int a = 1; a <= m1; ++a) v.push_back(hid(j + 1, i, a));  // N
    for (int b = 1; b <= m1; ++b) v.push_back(vid(i, j, b));      // W
  }
  const long nid = 2 * NH;
  std::vector<int> posB(nid, -1), stampB(nid, -1), stampA(nid, -1);
  lev.assign(nlev + 1, LevelPattern());
  for (int l = 1; l <= nlev; ++l) {
    const int count = (int)boxes.size() / 2;
    std::vector<std::vector<long>> parents(count);
    LevelPattern& P = lev[l];
    for (int mg = 0; mg < count; ++mg) {
      const auto& A = boxes[2 * mg];
      const auto& B = boxes[2 * mg + 1];
      const int stamp = l * 1000003 + mg;
      for (size_t q = 0; q < B.size(); ++q) {
        posB[B[q]] = (int)q;
        stampB[B[q]] = stamp;
      }
      for (size_t q = 0; q < A.size(); ++q) stampA[A[q]] = stamp;
      std::vector<int> p1a, p3a, p2b, p3b;
      for (size_t q = 0; q < A.size(); ++q) {
        if (stampB[A[q]] == stamp) {
          p3a.push_back((int)q);
          p3b.push_back(posB[A[q]]);
        } else {
          p1a.push_back((int)q);
        }
      }
      for (size_t q = 0; q < B.size(); ++q)
        if (stampA[B[q]] != stamp) p2b.push_back((int)q);
      auto& par = parents[mg];
      for (int q : p1a) par.push_back(A[q]);
      for (int q : p2b) par.push_back(B[q]);
      if (mg == 0) {
        P.count = count;
        P.nc = (int)A.size();
        P.m = (int)p1a.size();
        P.s = (int)p3a.size();
        P.np = (int)par.size();
        P.pos1a = p1a;
        P.pos3a = p3a;
        P.pos2b = p2b;
        P.pos3b = p3b;
        if ((int)p2b.size() != P.m || (int)B.size() != P.nc)
          throw std::runtime_error("unbalanced merge");
      } else if (p1a != P.pos1a || p3a != P.pos3a || p2b != P.pos2b || p3b != P.pos3b) {
        throw std::runtime_error("merge patterns differ within a level");
      }
    }
    boxes.swap(parents);
  }

  // outer boundary in root order
  root.clear();
  for (long id : boxes[0]) {
    BoundaryNode bn;
    if (id < NH) {
      const long r = id / m1;
      const int a = (int)(id % m1) + 1;
      const int jy = (int)(r / L), i = (int)(r % L);
      bn.x = x0 + h * (i + 0.5 * (1.0 + t[a]));
      bn.y = y0 + h * jy;
      bn.nx = 0.0;
      bn.ny = (jy == 0) ? -1.0 : 1.0;
      bn.panel = (jy == 0 ? 0 : 2) * L + i;
      bn.local = a - 1;
      if (jy != 0 && jy != L) throw std::runtime_error("interior node at the root");
    } else {
      const long r = (id - NH) / m1;
      const int b = (int)((id - NH) % m1) + 1;
      const int ix = (int)(r / L), j = (int)(r % L);
      bn.x = x0 + h * ix;
      bn.y = y0 + h * (j + 0.5 * (1.0 + t[b]));
      bn.nx = (ix == 0) ? -1.0 : 1.0;
      bn.ny = 0.0;
      bn.panel = (ix == 0 ? 3 : 1) * L + j;
      bn.local = b - 1;
      if (ix != 0 && ix != L) throw std::runtime_error("interior node at the root");
    }
    root.push_back(bn);
  }
}

int Geometry::lidx(int a, int b) const {
  const int m1 = p - 2, pm = p - 1;
  const bool ea = (a == 0 || a == pm), eb = (b == 0 || b == pm);
  if (ea && eb) return -1;
  if (!ea && !eb) return (b - 1) * m1 + (a - 1);
  if (b == 0) return mi + (a - 1);
  if (a == pm) return mi + m1 + (b - 1);
  if (b == pm) return mi + 2 * m1 + (a - 1);
  return mi + 3 * m1 + (b - 1);
}

void Geometry::pde_coords(double* xy) const {
  const int m1 = p - 2;
  size_t o = 0;
  for (int z = 0; z < nleaf; ++z) {
    int i = 0, j = 0;
    for (int b = 0; (z >> (2 * b)) != 0; ++b) {
      i |= ((z >> (2 * b)) & 1) << b;
      j |= ((z >> (2 * b + 1)) & 1) << b;
    }
    for (int b = 1; b <= m1; ++b)
      for (int a = 1; a <= m1; ++a) {
        xy[o++] = x0 + h * (i + 0.5 * (1.0 + t[a]));
        xy[o++] = y0 + h * (j + 0.5 * (1.0 + t[b]));
      }
  }
}

void leaf_operators(const Geometry& g, double k, double eta, std::vector<cplx>& A0,
                    std::vector<cplx>& Mout) {
  const int p = g.p, pm = p - 1, m1 = p - 2;
  const int n = g.mi + g.ne;
  const double s1 = 2.0 / g.h;
  std::vector<double> D2((size_t)p * p, 0.0);
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < p; ++j) {
      double acc = 0.0;
      for (int q = 0; q < p; ++q) acc += g.D[(size_t)i * p + q] * g.D[(size_t)q * p + j];
      D2[(size_t)i * p + j] = acc * s1 * s1;
    }
  A0.assign((size_t)n * n, cplx(0.0, 0.0));
  Mout.assign((size_t)g.ne * n, cplx(0.0, 0.0));
  for (int b = 1; b <= m1; ++b)
    for (int a = 1; a <= m1; ++a) {
      const int r = g.lidx(a, b);
      for (int q = 0; q < p; ++q) {
        A0[(size_t)r * n + g.lidx(q, b)] += D2[(size_t)a * p + q];
        A0[(size_t)r * n + g.lidx(a, q)] += D2[(size_t)b * p + q];
      }
      A0[(size_t)r * n + r] += k * k;
    }
  // edge rows: outward normal derivative along the normal grid line
  for (int e = 0; e < g.ne; ++e) {
    const int side = e / m1, c = e % m1 + 1;
    int a = 0, b = 0;
    double sgn = 1.0;
    int endrow = 0;
    bool alongx = false;  // derivative in x (east/west) or in y (south/north)
    if (side == 0) { a = c; b = 0; sgn = -1.0; endrow = 0; alongx = false; }
    if (side == 1) { a = pm; b = c; sgn = 1.0; endrow = pm; alongx = true; }
    if (side == 2) { a = c; b = pm; sgn = 1.0; endrow = pm; alongx = false; }
    if (side == 3) { a = 0; b = c; sgn = -1.0; endrow = 0; alongx = true; }
    const int r = g.mi + e;
    for (int q = 0; q < p; ++q) {
      const int col = alongx ? g.lidx(q, b) : g.lidx(a, q);
      const double v = sgn * s1 * g.D[(size_t)endrow * p + q];
      A0[(size_t)r * n + col] += v;
      Mout[(size_t)e * n + col] += v;
    }
    A0[(size_t)r * n + r] += cplx(0.0, eta);
    Mout[(size_t)e * n + r] += cplx(0.0, -eta);
  }
}

namespace {

// The 4 L outer-boundary panels (leaf edges), side * L + index, each from A
// to B in increasing x (sides 0, 2) or y (sides 1, 3), with outward normal.
std::vector<Panel> outer_panels(const Geometry& g) {
  const int L = g.L;
  const double X1 = g.x0 + g.h * L, Y1 = g.y0 + g.h * L;
  std::vector<Panel> pan(4 * L);
  for (int side = 0; side < 4; ++side)
    for (int i = 0; i < L; ++i) {
      Panel P;
      const double lo = g.h * i, hi = g.h * (i + 1);
      if (side == 0) P = {g.x0 + lo, g.y0, g.x0 + hi, g.y0, 0.0, -1.0};
      if (side == 1) P = {X1, g.y0 + lo, X1, g.y0 + hi, 1.0, 0.0};
      if (side == 2) P = {g.x0 + lo, Y1, g.x0 + hi, Y1, 0.0, 1.0};
      if (side == 3) P = {g.x0, g.y0 + lo, g.x0, g.y0 + hi, -1.0, 0.0};
      pan[side * L + i] = P;
    }
  return pan;
}

// Interpolation on a panel's p - 2 interior Lobatto nodes, 16-point Gauss rule.
Quad panel_quad(const Geometry& g, double k) {
  const int m1 = g.p - 2;
  Quad Q;
  Q.nloc = m1;
  Q.k = k;
  Q.nodes.assign(g.t.begin() + 1, g.t.end() - 1);
  Q.bw.assign(m1, 1.0);
  for (int j = 0; j < m1; ++j) {
    double prod = 1.0;
    for (int q = 0; q < m1; ++q)
      if (q != j) prod *= (Q.nodes[j] - Q.nodes[q]);
    Q.bw[j] = 1.0 / prod;
  }
  gauss_legendre(16, Q.gx, Q.gw);
  return Q;
}

// Runs work(lo, hi) over [0, n) on up to nthreads threads.
template <class F>
void parallel_rows(size_t n, int nthreads, F work) {
  if (nthreads < 1) nthreads = 1;
  if ((size_t)nthreads > n) nthreads = (int)std::max<size_t>(1, n);
  std::vector<std::thread> th;
  const size_t chunk = (n + nthreads - 1) / nthreads;
  for (int w = 0; w < nthreads; ++w) {
    const size_t lo = w * chunk, hi = std::min(n, lo + chunk);
    if (lo >= hi) break;
    th.emplace_back(work, lo, hi);
  }
  for (auto& x : th) x.join();
}

// Derivatives ell_j'(tau) of the Lagrange basis (tau not a node), from the
// barycentric form ell_j = u_j / sum_m u_m, u_j = bw_j / (tau - t_j):
// ell_j' = ell_j (sum_m ell_m / (tau - t_m) - 1 / (tau - t_j)).
void dlagrange(const Quad& Q, double tau, const double* lag, double* out) {
  double s = 0.0;
  for (int m = 0; m < Q.nloc; ++m) s += lag[m] / (tau - Q.nodes[m]);
  for (int j = 0; j < Q.nloc; ++j) out[j] = lag[j] * (s - 1.0 / (tau - Q.nodes[j]));
}

// Target data of the combined-field moments: boundary node (x, y) with
// outward normal (nx, ny), counter-clockwise tangent (-ny, nx); on its own
// panel (own = true) at parameter t0.
struct BmTarget {
  double x, y, nx, ny;
  bool own;
  double t0;
};

// Accumulates, over the parameter piece [a, b] of panel P (orientation o =
// +1 when A -> B runs counter-clockwise), with the refinement rule of piece():
//   mKp[j] += int dG/dn_x ell_j ds,
//   mT[j]  += int o dG/dtau_x ell_j'(t) dt  (plus, on the target's own panel,
//             1 / (pi h (t0 - t)): the kernel minus its Cauchy part).
void piece_bm(const Quad& Q, const Panel& P, const BmTarget& X, double o, double a, double b, int depth,
              cplx* mKp, cplx* mT) {
  const double vx = P.bx - P.ax, vy = P.by - P.ay;
  const double len_full = std::sqrt(vx * vx + vy * vy);
  const double len = 0.5 * (b - a) * len_full;
  // On the target's own panel everything is taken in the panel parameter:
  // the kernel's Cauchy part is subtracted at t0, so the kernel must be
  // singular at exactly t0 (coordinates would move it by rounding, and near
  // the target that mismatch grows like 1 / (t0 - t)).
  double tp, d;
  if (X.own) {
    tp = X.t0;
    d = 0.5 * len_full * std::max(0.0, std::max(a - tp, tp - b));
  } else {
    const double px = X.x - P.ax, py = X.y - P.ay;
    tp = 2.0 * (px * vx + py * vy) / (len_full * len_full) - 1.0;
    const double tc = std::min(std::max(tp, a), b);
    const double cx = P.ax + vx * 0.5 * (1.0 + tc), cy = P.ay + vy * 0.5 * (1.0 + tc);
    d = std::hypot(X.x - cx, X.y - cy);
  }
  if ((d >= 0.75 * len && Q.k * len <= 4.0) || depth > 200) {
    const double half = 0.5 * (b - a), mid = 0.5 * (a + b);
    const double tx = -X.ny, ty = X.nx;
    double lag[64], dl[64];
    for (size_t g = 0; g < Q.gx.size(); ++g) {
      const double tau = mid + half * Q.gx[g];
      const double wt = half * Q.gw[g];
      cplx gK, gT;
      if (X.own) {
        // x - y = (t0 - t) (B - A) / 2: normal component 0, o times the
        // tangential one (t0 - t) h / 2
        const double dt = X.t0 - tau;
        const double r = 0.5 * len_full * std::fabs(dt);
        cplx h0, h1;
        hankel01(Q.k * r, h0, h1);
        gK = 0.0;
        gT = cplx(0.0, -0.25 * Q.k) * h1 * (dt > 0.0 ? 1.0 : -1.0) + 1.0 / (PI * len_full * dt);
      } else {
        const double yx = P.ax + vx * 0.5 * (1.0 + tau), yy = P.ay + vy * 0.5 * (1.0 + tau);
        const double dx = X.x - yx, dy = X.y - yy;
        const double r = std::hypot(dx, dy);
        cplx h0, h1;
        hankel01(Q.k * r, h0, h1);
        const cplx c1 = cplx(0.0, -0.25 * Q.k) * h1 / r;  // grad_x G = c1 (x - y)
        gK = c1 * (dx * X.nx + dy * X.ny) * (wt * 0.5 * len_full);
        gT = o * c1 * (dx * tx + dy * ty);
      }
      gT *= wt;
      lagrange(Q, tau, lag);
      dlagrange(Q, tau, lag, dl);
      for (int j = 0; j < Q.nloc; ++j) {
        mKp[j] += gK * lag[j];
        mT[j] += gT * dl[j];
      }
    }
    return;
  }
  if (d == 0.0 && len < 1e-15) return;
  double split = 0.5 * (a + b);
  if (tp > a + 0.05 * (b - a) && tp < b - 0.05 * (b - a)) split = tp;
  piece_bm(Q, P, X, o, a, split, depth + 1, mKp, mT);
  piece_bm(Q, P, X, o, split, b, depth + 1, mKp, mT);
}

}  // namespace

void layer_moments(const Geometry& g, double k, const std::vector<double>& tx,
                   const std::vector<double>& ty, std::vector<cplx>& S, std::vector<cplx>& K,
                   int nthreads) {
  const int L = g.L, m1 = g.p - 2;
  const int npan = 4 * L;
  const std::vector<Panel> pan = outer_panels(g);
  const int nb = (int)g.root.size();
  std::vector<int> col((size_t)npan * m1, -1);
  for (int q = 0; q < nb; ++q) col[(size_t)g.root[q].panel * m1 + g.root[q].local] = q;
  const Quad Q = panel_quad(g, k);
  const size_t nt = tx.size();
  S.assign(nt * nb, cplx(0.0, 0.0));
  K.assign(nt * nb, cplx(0.0, 0.0));
  auto work = [&](size_t lo, size_t hi) {
    std::vector<cplx> mS(m1), mD(m1);
    for (size_t i = lo; i < hi; ++i)
      for (int pp = 0; pp < npan; ++pp) {
        std::fill(mS.begin(), mS.end(), cplx(0.0, 0.0));
        std::fill(mD.begin(), mD.end(), cplx(0.0, 0.0));
        piece(Q, pan[pp], tx[i], ty[i], -1.0, 1.0, 0, mS.data(), mD.data());
        for (int j = 0; j < m1; ++j) {
          const int c = col[(size_t)pp * m1 + j];
          S[i * nb + c] = mS[j];
          K[i * nb + c] = mD[j];
        }
      }
  };
  parallel_rows(nt, nthreads, work);
}

void combined_field_moments(const Geometry& g, double k, std::vector<cplx>& Kp, std::vector<cplx>& T1,
                            int nthreads) {
  const int L = g.L, m1 = g.p - 2;
  const int npan = 4 * L;
  const std::vector<Panel> pan = outer_panels(g);
  const int nb = (int)g.root.size();
  std::vector<int> col((size_t)npan * m1, -1);
  for (int q = 0; q < nb; ++q) col[(size_t)g.root[q].panel * m1 + g.root[q].local] = q;
  const Quad Q = panel_quad(g, k);
  // ell_j'(t_i) on the nodes: off the diagonal (bw_j / bw_i) / (t_i - t_j),
  // on it sum_{m != i} 1 / (t_i - t_m) (log-derivative of the node polynomial)
  std::vector<double> Dn((size_t)m1 * m1);
  for (int i = 0; i < m1; ++i)
    for (int j = 0; j < m1; ++j) {
      double v = 0.0;
      if (i != j) {
        v = (Q.bw[j] / Q.bw[i]) / (Q.nodes[i] - Q.nodes[j]);
      } else {
        for (int m = 0; m < m1; ++m)
          if (m != i) v += 1.0 / (Q.nodes[i] - Q.nodes[m]);
      }
      Dn[(size_t)i * m1 + j] = v;
    }
  // ell_j at the panel ends t = -1, +1
  std::vector<double> lA(m1), lB(m1);
  lagrange(Q, -1.0, lA.data());
  lagrange(Q, 1.0, lB.data());
  Kp.assign((size_t)nb * nb, cplx(0.0, 0.0));
  T1.assign((size_t)nb * nb, cplx(0.0, 0.0));
  auto dGdtau = [&](const BmTarget& X, double yx, double yy) {
    const double dx = X.x - yx, dy = X.y - yy;
    const double r = std::hypot(dx, dy);
    cplx h0, h1;
    hankel01(k * r, h0, h1);
    return cplx(0.0, -0.25 * k) * h1 * ((dx * -X.ny + dy * X.nx) / r);
  };
  auto work = [&](size_t lo, size_t hi) {
    std::vector<cplx> mK(m1), mT(m1);
    std::vector<double> lag(m1), dl(m1);
    for (size_t i = lo; i < hi; ++i) {
      const BoundaryNode& bn = g.root[i];
      for (int pp = 0; pp < npan; ++pp) {
        const Panel& P = pan[pp];
        const double o = (pp / L) < 2 ? 1.0 : -1.0;  // sides 0, 1 run counter-clockwise
        BmTarget X{bn.x, bn.y, bn.nx, bn.ny, pp == bn.panel, Q.nodes[bn.local]};
        std::fill(mK.begin(), mK.end(), cplx(0.0, 0.0));
        std::fill(mT.begin(), mT.end(), cplx(0.0, 0.0));
        piece_bm(Q, P, X, o, -1.0, 1.0, 0, mK.data(), mT.data());
        // point masses of d s / d sigma at the panel ends (jumps of the
        // panel-wise interpolant): o [ell_j(-1) dG/dtau(x, A) - ell_j(1) dG/dtau(x, B)]
        const cplx gA = o * dGdtau(X, P.ax, P.ay), gB = o * dGdtau(X, P.bx, P.by);
        for (int j = 0; j < m1; ++j) mT[j] += gA * lA[j] - gB * lB[j];
        if (X.own) {
          // principal value of -1/(pi h) int ell_j'(t) / (t0 - t) dt: the
          // divided difference is a polynomial (Gauss rule exact) plus the
          // closed-form p.v. integral of 1 / (t0 - t)
          const double t0 = X.t0;
          const double hl = std::hypot(P.bx - P.ax, P.by - P.ay);
          const double lg = std::log((1.0 + t0) / (1.0 - t0));
          const double* d0 = &Dn[(size_t)bn.local * m1];
          std::vector<double> acc(m1, 0.0);
          for (size_t q = 0; q < Q.gx.size(); ++q) {
            lagrange(Q, Q.gx[q], lag.data());
            dlagrange(Q, Q.gx[q], lag.data(), dl.data());
            for (int j = 0; j < m1; ++j) acc[j] += Q.gw[q] * (dl[j] - d0[j]) / (t0 - Q.gx[q]);
          }
          for (int j = 0; j < m1; ++j) mT[j] += -(acc[j] + d0[j] * lg) / (PI * hl);
        }
        for (int j = 0; j < m1; ++j) {
          const int c = col[(size_t)pp * m1 + j];
          Kp[i * nb + c] = mK[j];
          T1[i * nb + c] = mT[j];
        }
      }
    }
  };
  parallel_rows((size_t)nb, nthreads, work);
}

}  // namespace hps
