// Data-movement and pointwise kernels of the HPS solver.  All heavy
// arithmetic (leaf inversions, merges, sweeps, far field) goes through the
// complex GEMM / inverse; these kernels assemble leaf matrices, move blocks
// between the boxes of adjacent tree levels, and form boundary data.
#include "common.h"
#include "hps_kernels.h"

namespace hps {
namespace {

constexpr int NT = 256;

inline unsigned blocks_for(ll n) {
  ll b = (n + NT - 1) / NT;
  if (b > 1048576) b = 1048576;
  return (unsigned)(b < 1 ? 1 : b);
}

// Quotient of n < 2^31 by the divisor that (mul, shift) encode (make_fastdiv).
__device__ __forceinline__ unsigned fdiv(unsigned n, unsigned mul, int shift) {
  return mul ? (__umulhi(n, mul) >> shift) : n;
}

// Grid of a batched move: x covers the per (< 2^31) elements of one batch
// entry, y the entries (the kernels loop over y with stride gridDim.y).
dim3 move_grid(ll per, int batch) {
  ll gx = (per + NT - 1) / NT;
  ll gy = batch < 65535 ? batch : 65535;
  if (gx < 1) gx = 1;
  if (gy < 1) gy = 1;
  while (gx * gy > 1048576 && gy > 1) gy = (gy + 1) / 2;
  if (gx * gy > 1048576) gx = 1048576 / gy;
  return dim3((unsigned)gx, (unsigned)gy);
}

// Leaf z belongs to problem z / lpp, whose base matrix is A0 + problem sA0 and
// whose k^2 is k2v[problem].
__global__ void k_leaf_assemble(const double2* A0, ll sA0, const double* q, const double* k2v, int n,
                                unsigned fdm, int fds, int mi, double2* out, int nleaf, int lpp) {
  const unsigned per = (unsigned)n * (unsigned)n;
  for (int z = blockIdx.y; z < nleaf; z += gridDim.y) {
    const int pb = z / lpp;
    const double2* a = A0 + (ll)pb * sA0;
    double2* o = out + (ll)z * per;
    const double* qz = q + (ll)z * mi;
    const double k2 = k2v[pb];
    for (unsigned e = blockIdx.x * NT + threadIdx.x; e < per; e += gridDim.x * NT) {
      double2 v = a[e];
      const unsigned c = fdiv(e, fdm, fds), r = e - c * (unsigned)n;
      if (r == c && (int)r < mi) v.x -= k2 * qz[r];
      o[e] = v;
    }
  }
}

template <typename T2, typename T>
__global__ void k_gather2d(int M, int N, unsigned fdm, int fds, const T2* in, ll ldi, ll si, const int* ridx,
                           const int* cidx, T2* out, ll ldo, ll so, T sc, int batch) {
  const unsigned per = (unsigned)M * (unsigned)N;
  for (int b = blockIdx.y; b < batch; b += gridDim.y) {
    const T2* ib = in + (ll)b * si;
    T2* ob = out + (ll)b * so;
    for (unsigned e = blockIdx.x * NT + threadIdx.x; e < per; e += gridDim.x * NT) {
      const unsigned j = fdiv(e, fdm, fds), i = e - j * (unsigned)M;
      const int ri = ridx ? ridx[i] : (int)i;
      const int cj = cidx ? cidx[j] : (int)j;
      const T2 v = ib[(ll)ri + (ll)cj * ldi];
      T2 o;
      o.x = sc * v.x;
      o.y = sc * v.y;
      ob[(ll)i + (ll)j * ldo] = o;
    }
  }
}

__global__ void k_gather_perm(int M, int N, unsigned fdm, int fds, const double2* in, ll ldi, ll si, int idiv,
                              const int* ridx, ll sri, int rlim, const int* cidx, ll sci, int clim, double2* out,
                              ll ldo, ll so, int batch) {
  const unsigned per = (unsigned)M * (unsigned)N;
  for (int b = blockIdx.y; b < batch; b += gridDim.y) {
    const double2* ib = in + (ll)(b / idiv) * si;
    const int* rb = ridx ? ridx + (ll)b * sri : nullptr;
    const int* cb = cidx ? cidx + (ll)b * sci : nullptr;
    double2* ob = out + (ll)b * so;
    for (unsigned e = blockIdx.x * NT + threadIdx.x; e < per; e += gridDim.x * NT) {
      const unsigned j = fdiv(e, fdm, fds), i = e - j * (unsigned)M;
      const int ri = rb ? rb[i] : (int)i;
      const int cj = cb ? cb[j] : (int)j;
      const bool ok = (unsigned)ri < (unsigned)rlim && (unsigned)cj < (unsigned)clim;
      ob[(ll)i + (ll)j * ldo] = ok ? ib[(ll)ri + (ll)cj * ldi] : make_double2(0.0, 0.0);
    }
  }
}

template <typename T2>
__global__ void k_scatter_rows(int M, int N, unsigned fdm, int fds, const T2* in, ll ldi, ll si, const int* ridx,
                               T2* out, ll ldo, ll so, int batch) {
  const unsigned per = (unsigned)M * (unsigned)N;
  for (int b = blockIdx.y; b < batch; b += gridDim.y) {
    const T2* ib = in + (ll)b * si;
    T2* ob = out + (ll)b * so;
    for (unsigned e = blockIdx.x * NT + threadIdx.x; e < per; e += gridDim.x * NT) {
      const unsigned j = fdiv(e, fdm, fds), i = e - j * (unsigned)M;
      ob[(ll)ridx[i] + (ll)j * ldo] = ib[(ll)i + (ll)j * ldi];
    }
  }
}

__global__ void k_set2d(int M, int N, unsigned fdm, int fds, double2* out, ll ldo, ll so, double2 diag,
                        double2 off, int batch) {
  const unsigned per = (unsigned)M * (unsigned)N;
  for (int b = blockIdx.y; b < batch; b += gridDim.y) {
    double2* ob = out + (ll)b * so;
    for (unsigned e = blockIdx.x * NT + threadIdx.x; e < per; e += gridDim.x * NT) {
      const unsigned j = fdiv(e, fdm, fds), i = e - j * (unsigned)M;
      ob[(ll)i + (ll)j * ldo] = (i == j) ? diag : off;
    }
  }
}

struct RowMoves4 {
  RowMove m[4];
  unsigned fdm[4];
  int fds[4];
};

// Move blockIdx.y of the list (selected by uniform branches, so the list stays
// in the kernel arguments): z (stride gridDim.z) runs over the batch, x over
// the elements of one matrix.
__global__ void k_row_moves(RowMoves4 d, int N, int batch) {
  const int y = blockIdx.y;
  const RowMove mv = y == 0 ? d.m[0] : y == 1 ? d.m[1] : y == 2 ? d.m[2] : d.m[3];
  const unsigned fdm = y == 0 ? d.fdm[0] : y == 1 ? d.fdm[1] : y == 2 ? d.fdm[2] : d.fdm[3];
  const int fds = y == 0 ? d.fds[0] : y == 1 ? d.fds[1] : y == 2 ? d.fds[2] : d.fds[3];
  const unsigned per = (unsigned)mv.M * (unsigned)N;
  if (blockIdx.x * NT >= per) return;
  for (int b = blockIdx.z; b < batch; b += gridDim.z) {
    const double2* ib = mv.in + (ll)b * mv.si;
    double2* ob = mv.out + (ll)b * mv.so;
    for (unsigned e = blockIdx.x * NT + threadIdx.x; e < per; e += gridDim.x * NT) {
      const unsigned j = fdiv(e, fdm, fds), i = e - j * (unsigned)mv.M;
      const int r = mv.ridx[i];
      if (mv.scatter)
        ob[(ll)r + (ll)j * mv.ldo] = ib[(ll)i + (ll)j * mv.ldi];
      else
        ob[(ll)i + (ll)j * mv.ldo] = ib[(ll)r + (ll)j * mv.ldi];
    }
  }
}

// Move desc[blockIdx.y]: z (stride gridDim.z) runs over the batch, x over the
// elements of one matrix.
__global__ void k_multi_move(const MoveDesc* desc, int batch) {
  const MoveDesc d = desc[blockIdx.y];
  const unsigned per = (unsigned)d.M * (unsigned)d.N;
  if (blockIdx.x * NT >= per) return;
  for (int b = blockIdx.z; b < batch; b += gridDim.z) {
    const double2* ib = d.in + (ll)b * d.si;
    double2* ob = d.out + (ll)b * d.so;
    for (unsigned e = blockIdx.x * NT + threadIdx.x; e < per; e += gridDim.x * NT) {
      const unsigned j = fdiv(e, d.fdm, d.fds), i = e - j * (unsigned)d.M;
      double2 v;
      if (d.set) {
        v = (i == j) ? d.diag : d.off;
      } else {
        const int ri = d.ridx ? d.ridx[i] : (int)i;
        const int cj = d.cidx ? d.cidx[j] : (int)j;
        const double2 x = ib[(ll)ri + (ll)cj * d.ldi];
        v = make_double2(d.sc * x.x, d.sc * x.y);
      }
      ob[(ll)i + (ll)j * d.ldo] = v;
    }
  }
}

// Rows [0, nb): d_nu u_inc; rows [nb, 2 nb): u_inc, one column per direction;
// column m belongs to problem m / ndir (wavenumber kv[m / ndir]).
__global__ void k_incident(const double4* bnode, int nb, const double2* dirs, int ndir, const double* kv,
                           double2* G, int nprob) {
  const ll total = (ll)nb * ndir * nprob;
  for (ll idx = blockIdx.x * (ll)NT + threadIdx.x; idx < total; idx += (ll)gridDim.x * NT) {
    const int i = (int)(idx % nb);
    const ll m = idx / nb;
    const double k = kv[m / ndir];
    const double4 b = bnode[i];
    const double2 d = dirs[m];
    double s, c;
    sincos(k * (b.x * d.x + b.y * d.y), &s, &c);
    const double kn = k * (b.z * d.x + b.w * d.y);
    G[(ll)m * 2 * nb + i] = make_double2(-kn * s, kn * c);
    G[(ll)m * 2 * nb + nb + i] = make_double2(c, s);
  }
}

// From the incoming/outgoing impedance (f, g) on the outer boundary:
//   s = (f - g) / (2 i eta) - u_inc,  t = (f + g) / 2 - d_nu u_inc
// (the incident terms are skipped when G is null).  Output [s; t] per column;
// column m belongs to problem m / ncol (eta = etav[m / ncol]).
__global__ void k_boundary_st(const double2* f, const double2* g, const double2* G, int nb,
                              int ncol, const double* etav, double2* ST, int nprob) {
  const ll total = (ll)nb * ncol * nprob;
  for (ll idx = blockIdx.x * (ll)NT + threadIdx.x; idx < total; idx += (ll)gridDim.x * NT) {
    const int i = (int)(idx % nb);
    const ll m = idx / nb;
    const double eta = etav[m / ncol];
    const double2 fv = f[(ll)m * nb + i], gv = g[(ll)m * nb + i];
    const double2 dmin = make_double2(fv.x - gv.x, fv.y - gv.y);
    // (a + ib) / (2 i eta) = (b - i a) / (2 eta)
    double2 s = make_double2(dmin.y / (2.0 * eta), -dmin.x / (2.0 * eta));
    double2 t = make_double2(0.5 * (fv.x + gv.x), 0.5 * (fv.y + gv.y));
    if (G) {
      const double2 du = G[(ll)m * 2 * nb + i], u = G[(ll)m * 2 * nb + nb + i];
      s.x -= u.x;
      s.y -= u.y;
      t.x -= du.x;
      t.y -= du.y;
    }
    ST[(ll)m * 2 * nb + i] = s;
    ST[(ll)m * 2 * nb + nb + i] = t;
  }
}

// Adjoint of k_boundary_st without incident terms: from (sbar, tbar)
//   fbar = conj(1/(2 i eta)) sbar + tbar / 2,  gbar = -conj(1/(2 i eta)) sbar + tbar / 2.
__global__ void k_boundary_st_adj(const double2* STb, int nb, int ncol, const double* etav, double2* fb,
                                  double2* gb, int nprob) {
  const ll total = (ll)nb * ncol * nprob;
  for (ll idx = blockIdx.x * (ll)NT + threadIdx.x; idx < total; idx += (ll)gridDim.x * NT) {
    const int i = (int)(idx % nb);
    const ll m = idx / nb;
    const double eta = etav[m / ncol];
    const double2 sb = STb[(ll)m * 2 * nb + i], tb = STb[(ll)m * 2 * nb + nb + i];
    // conj(1/(2 i eta)) = i / (2 eta):  i (a + ib) / (2 eta) = (-b + i a) / (2 eta)
    const double2 c = make_double2(-sb.y / (2.0 * eta), sb.x / (2.0 * eta));
    fb[(ll)m * nb + i] = make_double2(c.x + 0.5 * tb.x, c.y + 0.5 * tb.y);
    gb[(ll)m * nb + i] = make_double2(-c.x + 0.5 * tb.x, -c.y + 0.5 * tb.y);
  }
}

// b[z][n + m mi] = k^2 dq[z mi + n] u0[z][n + m mi]  (k^2 of leaf z's problem)
// Body-load operator of the Frechet derivative, folded into the leaf maps:
// Hs[z][e + n ne] = k^2 dq[z mi + n] H[z][e + n ne] (H: ne x mi per leaf), so
// that the outgoing impedance of the load k^2 dq u0 is Hs u0.
__global__ void k_scale_leaf_cols(const double* dq, const double2* H, const double* k2v, int ne, int mi,
                                  ll nleaf, ll lpp, double2* Hs) {
  const ll per = (ll)ne * mi;
  const ll total = per * nleaf;
  for (ll idx = blockIdx.x * (ll)NT + threadIdx.x; idx < total; idx += (ll)gridDim.x * NT) {
    const ll z = idx / per;
    const int n = (int)(idx % per) / ne;
    const double s = k2v[z / lpp] * dq[z * mi + n];
    const double2 h = H[idx];
    Hs[idx] = make_double2(s * h.x, s * h.y);
  }
}

// Adjoint reduction over the directions, from Q^T = g u0^H (ne x mi per leaf,
// g the leaf-edge adjoint data): grad[z mi + n] = k^2 Re sum_e conj(H[e][n])
// Q^T[e][n], which equals Re sum_m k^2 conj(u0[n][m]) (H^H g)[n][m].  Sixteen
// lanes per node read the node's column in contiguous runs and are summed by
// lane exchanges in a fixed order.
__global__ __launch_bounds__(NT) void k_grad_leaf(const double2* H, const double2* QT, const double* k2v, int ne,
                                                  int mi, ll nleaf, ll lpp, double* grad) {
  const ll total = (ll)mi * nleaf;
  const int sub = threadIdx.x & 15;
  for (ll base = (ll)blockIdx.x * (NT / 16); base < total; base += (ll)gridDim.x * (NT / 16)) {
    const ll idx = base + (threadIdx.x >> 4);
    double acc = 0.0;
    ll z = 0;
    if (idx < total) {
      z = idx / mi;
      const int n = (int)(idx % mi);
      const ll col = z * (ll)ne * mi + (ll)n * ne;
      for (int e = sub; e < ne; e += 16) {
        const double2 h = H[col + e], q = QT[col + e];
        acc += h.x * q.x + h.y * q.y;
      }
    }
#pragma unroll
    for (int o = 8; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 16);
    if (idx < total && sub == 0) grad[idx] = k2v[z / lpp] * acc;
  }
}

// out[m][z mi + n] = u0[z][n + m mi]
__global__ void k_export_field(const double2* u0, int mi, int ndir, ll nleaf, double2* out) {
  const ll npde = (ll)mi * nleaf;
  const ll total = npde * ndir;
  for (ll idx = blockIdx.x * (ll)NT + threadIdx.x; idx < total; idx += (ll)gridDim.x * NT) {
    const ll m = idx / npde, node = idx % npde;
    const ll z = node / mi;
    const int n = (int)(node % mi);
    out[idx] = u0[z * (ll)mi * ndir + m * mi + n];
  }
}

__global__ void k_real_to_complex(const double* x, ll n, double2* y) {
  for (ll idx = blockIdx.x * (ll)NT + threadIdx.x; idx < n; idx += (ll)gridDim.x * NT)
    y[idx] = make_double2(x[idx], 0.0);
}

__global__ void k_complex_real_part(const double2* x, ll n, double* y) {
  for (ll idx = blockIdx.x * (ll)NT + threadIdx.x; idx < n; idx += (ll)gridDim.x * NT)
    y[idx] = x[idx].x;
}

// partial[block] = sum of x[i] y[i] over the block's grid-stride share
__global__ void k_dot_partial(const double* x, const double* y, ll n, double* partial) {
  __shared__ double sh[NT];
  double acc = 0.0;
  for (ll i = blockIdx.x * (ll)NT + threadIdx.x; i < n; i += (ll)gridDim.x * NT) acc += x[i] * y[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void k_sum_partials(const double* partial, int nb, double* out) {
  __shared__ double sh[NT];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += NT) acc += partial[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

__global__ void k_to_f32(const double2* x, ll n, float2* y) {
  for (ll i = blockIdx.x * (ll)NT + threadIdx.x; i < n; i += (ll)gridDim.x * NT)
    y[i] = make_float2((float)x[i].x, (float)x[i].y);
}

__global__ void k_add_f32(const float2* x, ll n, double2* y) {
  for (ll i = blockIdx.x * (ll)NT + threadIdx.x; i < n; i += (ll)gridDim.x * NT)
    y[i] = make_double2(y[i].x + (double)x[i].x, y[i].y + (double)x[i].y);
}

__global__ void k_to_f64(const float2* x, ll n, double2* y) {
  for (ll i = blockIdx.x * (ll)NT + threadIdx.x; i < n; i += (ll)gridDim.x * NT)
    y[i] = make_double2((double)x[i].x, (double)x[i].y);
}

__global__ void k_add_to_f32(const double2* x, ll n, float2* y) {
  for (ll i = blockIdx.x * (ll)NT + threadIdx.x; i < n; i += (ll)gridDim.x * NT)
    y[i] = make_float2(y[i].x + (float)x[i].x, y[i].y + (float)x[i].y);
}

__global__ void k_zadd(const double2* x, const double2* y, double2* z, ll n) {
  for (ll i = blockIdx.x * (ll)NT + threadIdx.x; i < n; i += (ll)gridDim.x * NT)
    z[i] = make_double2(x[i].x + y[i].x, x[i].y + y[i].y);
}

// Skeleton data addressing: leaf-edge data X is [leaf][ne][M] (column-major
// per leaf, leading dimension ne); a slot is (leaf offset inside a box) * ne +
// (edge position).  Box b of a level owns the leaves [b lpb, (b + 1) lpb).
__device__ inline ll slot_addr(int slot, ll box_leaf0, int ne, int M, int col) {
  const int lo = slot / ne, e = slot - lo * ne;
  return (box_leaf0 + lo) * (ll)ne * M + e + (ll)col * ne;
}

// Interface residual of one level: for merge t and shared node j with slots
// sa[j] (alpha side) and sb[j] (beta side),
//   rho[t][j][col]     = F[sb[j]] + G[sa[j]]   (f of beta + g of alpha),
//   rho[t][s + j][col] = F[sa[j]] + G[sb[j]],
// rho column-major per merge with leading dimension 2 s.
__global__ void k_skel_residual(int s, int M, int ne, int lpm, const int* sab, const double2* F,
                                const double2* G, double2* rho, ll total) {
  const int s2 = 2 * s;
  for (ll idx = blockIdx.x * (ll)NT + threadIdx.x; idx < total; idx += (ll)gridDim.x * NT) {
    const int r = (int)(idx % s2);
    const ll rest = idx / s2;
    const int col = (int)(rest % M);
    const ll t = rest / M;
    const int j = r < s ? r : r - s;
    const int fs = r < s ? sab[s + j] : sab[j];
    const int gs = r < s ? sab[j] : sab[s + j];
    const ll l0 = t * lpm;
    const double2 f = F[slot_addr(fs, l0, ne, M, col)];
    const double2 g = G[slot_addr(gs, l0, ne, M, col)];
    rho[t * s2 * M + r + (ll)col * s2] = make_double2(f.x + g.x, f.y + g.y);
  }
}

// out[b][i][col] = X[slot[i]] of box b (n slots per box, column-major per
// box with leading dimension n).
__global__ void k_skel_gather(int n, int M, int ne, int lpb, const int* slot, const double2* X,
                              double2* out, ll total) {
  for (ll idx = blockIdx.x * (ll)NT + threadIdx.x; idx < total; idx += (ll)gridDim.x * NT) {
    const int i = (int)(idx % n);
    const ll rest = idx / n;
    const int col = (int)(rest % M);
    const ll b = rest / M;
    out[idx] = X[slot_addr(slot[i], b * lpb, ne, M, col)];
  }
}

// out = in^H for square n x n matrices (column-major), 32 x 32 tiles through
// LDS so that both the reads and the writes are coalesced.
__global__ __launch_bounds__(256) void k_conj_transpose(int n, const double2* in, ll ldi, ll si, double2* out,
                                                        ll ldo, ll so) {
  __shared__ double2 tile[32][33];
  const ll b = blockIdx.z;
  const int r0 = blockIdx.x * 32, c0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int j = ty; j < 32; j += 8) {
    const int r = r0 + tx, c = c0 + j;
    if (r < n && c < n) tile[j][tx] = in[b * si + (ll)r + (ll)c * ldi];
  }
  __syncthreads();
  for (int j = ty; j < 32; j += 8) {
    const int r = c0 + tx, c = r0 + j;  // out(r, c) = conj(in(c, r))
    if (r < n && c < n) {
      const double2 v = tile[tx][j];
      out[b * so + (ll)r + (ll)c * ldo] = make_double2(v.x, -v.y);
    }
  }
}

// y = a x + b y
__global__ void k_axpby(double a, const double* x, double b, double* y, ll n) {
  for (ll i = blockIdx.x * (ll)NT + threadIdx.x; i < n; i += (ll)gridDim.x * NT) y[i] = a * x[i] + b * y[i];
}

__global__ void k_axpby_dev(const double* ap, double sa, const double* x, const double* bp, double* y, ll n) {
  const double a = ap ? sa * *ap : sa, b = bp ? *bp : 1.0;
  for (ll i = blockIdx.x * (ll)NT + threadIdx.x; i < n; i += (ll)gridDim.x * NT) y[i] = a * x[i] + b * y[i];
}

__global__ void k_cg_init(double* s, int* f) {
  if (threadIdx.x != 0) return;
  s[CG_REL] = 1.0;
  f[CG_DONE] = 0;
  f[CG_ACTIVE] = 0;
  f[CG_ITERS] = 0;
}

__global__ void k_cg_alpha(double* s, int* f) {
  if (threadIdx.x != 0) return;
  const double pAp = s[CG_PAP];
  if (f[CG_DONE] || !(pAp > 0.0)) {
    f[CG_DONE] = 1;
    f[CG_ACTIVE] = 0;
    s[CG_ALPHA] = 0.0;
    return;
  }
  f[CG_ACTIVE] = 1;
  s[CG_ALPHA] = s[CG_RR] / pAp;
}

__global__ void k_cg_beta(double* s, int* f, double bnorm, double tol) {
  if (threadIdx.x != 0) return;
  if (!f[CG_ACTIVE]) {
    s[CG_BETA] = 0.0;
    return;
  }
  f[CG_ITERS] += 1;
  const double rr_new = s[CG_RRNEW];
  const double rel = sqrt(rr_new) / bnorm;
  s[CG_REL] = rel;
  if (rel <= tol) {
    f[CG_DONE] = 1;
    s[CG_BETA] = 0.0;
    return;
  }
  s[CG_BETA] = rr_new / s[CG_RR];
  s[CG_RR] = rr_new;
}

// z = x - y (complex)
__global__ void k_zsub(const double2* x, const double2* y, double2* z, ll n) {
  for (ll i = blockIdx.x * (ll)NT + threadIdx.x; i < n; i += (ll)gridDim.x * NT)
    z[i] = make_double2(x[i].x - y[i].x, x[i].y - y[i].y);
}

}  // namespace

constexpr int DOT_BLOCKS = 256;

// *flag |= bit if any of the n doubles of x is NaN or infinite (one atomic
// per workgroup that saw one).
__global__ __launch_bounds__(256) void k_flag_nonfinite(const double* x, ll n, int bit, int* flag) {
  int bad = 0;
  for (ll i = (ll)blockIdx.x * 256 + threadIdx.x; i < n; i += (ll)gridDim.x * 256) bad |= !isfinite(x[i]);
  if (__syncthreads_or(bad) && threadIdx.x == 0) atomicOr(flag, bit);
}

hipError_t flag_nonfinite(hipStream_t st, const double* x, ll n, int bit, int* flag) {
  if (n <= 0) return hipSuccess;
  ll blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  KernelTimer kt(st, K_POINT, 0.0, 8.0 * n);
  hipLaunchKernelGGL(k_flag_nonfinite, dim3((unsigned)blocks), dim3(256), 0, st, x, n, bit, flag);
  return hipGetLastError();
}

hipError_t dot(hipStream_t st, const double* x, const double* y, ll n, double* partial, double* out) {
  {
    KernelTimer kt(st, K_POINT, 2.0 * n, 16.0 * n);
    hipLaunchKernelGGL(k_dot_partial, dim3(DOT_BLOCKS), dim3(NT), 0, st, x, y, n, partial);
  }
  HPS_HIP_TRY(hipGetLastError());
  KernelTimer kt(st, K_POINT, (double)DOT_BLOCKS, 8.0 * DOT_BLOCKS);
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(NT), 0, st, partial, DOT_BLOCKS, out);
  return hipGetLastError();
}

// Zeroes the sine coefficients outside the band: x[(m - 1) S + (n - 1)] = 0
// when m + n > band (1-based mode numbers).
__global__ void k_band_mask(double* x, int S, int band) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= S * S) return;
  const int m = e / S + 1, n = e % S + 1;
  if (m + n > band) x[e] = 0.0;
}

hipError_t band_mask(hipStream_t st, double* x, int S, int band) {
  if (band <= 0 || S <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_band_mask, dim3((S * S + 255) / 256), dim3(256), 0, st, x, S, band);
  return hipGetLastError();
}

hipError_t axpby(hipStream_t st, double a, const double* x, double b, double* y, ll n) {
  KernelTimer kt(st, K_POINT, 3.0 * n, 24.0 * n);
  hipLaunchKernelGGL(k_axpby, dim3(blocks_for(n)), dim3(NT), 0, st, a, x, b, y, n);
  return hipGetLastError();
}

hipError_t axpby_dev(hipStream_t st, const double* a, double sa, const double* x, const double* b, double* y,
                     ll n) {
  KernelTimer kt(st, K_POINT, 3.0 * n, 24.0 * n);
  hipLaunchKernelGGL(k_axpby_dev, dim3(blocks_for(n)), dim3(NT), 0, st, a, sa, x, b, y, n);
  return hipGetLastError();
}

hipError_t cg_init(hipStream_t st, double* s, int* f) {
  hipLaunchKernelGGL(k_cg_init, dim3(1), dim3(64), 0, st, s, f);
  return hipGetLastError();
}

hipError_t cg_alpha(hipStream_t st, double* s, int* f) {
  hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(64), 0, st, s, f);
  return hipGetLastError();
}

hipError_t cg_beta(hipStream_t st, double* s, int* f, double bnorm, double tol) {
  hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(64), 0, st, s, f, bnorm, tol);
  return hipGetLastError();
}

hipError_t zsub(hipStream_t st, const double2* x, const double2* y, double2* z, ll n) {
  KernelTimer kt(st, K_POINT, 2.0 * n, 48.0 * n);
  hipLaunchKernelGGL(k_zsub, dim3(blocks_for(n)), dim3(NT), 0, st, x, y, z, n);
  return hipGetLastError();
}

hipError_t leaf_assemble(hipStream_t st, const double2* A0, ll sA0, const double* q, const double* k2v,
                         int n, int mi, double2* out, ll nleaf, ll lpp) {
  if (n <= 0 || nleaf <= 0) return hipSuccess;
  if ((ll)n * n > 0x7fffffffLL || nleaf > 0x7fffffffLL || lpp < 1 || lpp > 0x7fffffffLL) return hipErrorInvalidValue;
  KernelTimer kt(st, K_LEAF, 0.0, 16.0 * (double)n * n * nleaf + 8.0 * mi * (double)nleaf);
  const FastDiv f = make_fastdiv(n);
  hipLaunchKernelGGL(k_leaf_assemble, move_grid((ll)n * n, (int)nleaf), dim3(NT), 0, st, A0, sA0, q, k2v, n, f.mul,
                     f.shift, mi, out, (int)nleaf, (int)lpp);
  return hipGetLastError();
}

FastDiv make_fastdiv(int d) {
  if (d <= 1) return FastDiv{0u, 0};
  const int l = 32 - __builtin_clz((unsigned)(d - 1));  // ceil(log2 d), d >= 2
  const unsigned long long p = 1ULL << (31 + l);
  return FastDiv{(unsigned)((p + (unsigned long long)d - 1) / (unsigned long long)d), l - 1};
}

hipError_t row_moves(hipStream_t st, const RowMove* moves, int nmoves, int N, int batch) {
  if (nmoves < 1 || nmoves > 4 || N <= 0 || batch <= 0) return nmoves == 0 ? hipSuccess : hipErrorInvalidValue;
  RowMoves4 d{};
  ll maxper = 0;
  double bytes = 0.0;
  for (int i = 0; i < nmoves; ++i) {
    const ll per = (ll)moves[i].M * N;
    if (moves[i].M <= 0 || per > 0x7fffffffLL) return hipErrorInvalidValue;
    d.m[i] = moves[i];
    const FastDiv f = make_fastdiv(moves[i].M);
    d.fdm[i] = f.mul;
    d.fds[i] = f.shift;
    maxper = per > maxper ? per : maxper;
    bytes += 32.0 * (double)per * batch;
  }
  KernelTimer kt(st, K_MOVE, 0.0, bytes);
  ll gx = (maxper + NT - 1) / NT, gz = batch;
  while (gx * nmoves * gz > 1048576 && gz > 1) gz = (gz + 1) / 2;
  if (gz > 65535) gz = 65535;
  hipLaunchKernelGGL(k_row_moves, dim3((unsigned)gx, nmoves, (unsigned)gz), dim3(NT), 0, st, d, N, batch);
  return hipGetLastError();
}

void multi_move_prepare(MoveDesc* desc, int ndesc) {
  for (int i = 0; i < ndesc; ++i) {
    const FastDiv f = make_fastdiv(desc[i].M);
    desc[i].fdm = f.mul;
    desc[i].fds = f.shift;
  }
}

hipError_t multi_move(hipStream_t st, const MoveDesc* desc, int ndesc, ll max_elems, int batch) {
  if (ndesc <= 0 || max_elems <= 0 || batch <= 0) return hipSuccess;
  if (ndesc > 65535) return hipErrorInvalidValue;
  const ll per = (max_elems + batch - 1) / batch;  // largest M * N
  if (per > 0x7fffffffLL) return hipErrorInvalidValue;
  KernelTimer kt(st, K_MOVE, 0.0, 0.0);
  // x covers the largest move (blocks beyond a smaller move's elements exit
  // at once), z the batch (stride loop beyond)
  ll gx = (per + NT - 1) / NT, gz = batch;
  if (gx > 4096) gx = 4096;
  while (gx * ndesc * gz > 1048576 && gz > 1) gz = (gz + 1) / 2;
  if (gz > 65535) gz = 65535;
  hipLaunchKernelGGL(k_multi_move, dim3((unsigned)gx, ndesc, (unsigned)gz), dim3(NT), 0, st, desc, batch);
  return hipGetLastError();
}

hipError_t gather2d(hipStream_t st, int M, int N, const double2* in, ll ldi, ll si,
                    const int* ridx, const int* cidx, double2* out, ll ldo, ll so, double sc,
                    int batch) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  if ((ll)M * N > 0x7fffffffLL) return hipErrorInvalidValue;
  KernelTimer kt(st, K_MOVE, 0.0, 32.0 * (double)M * N * batch);
  const FastDiv f = make_fastdiv(M);
  hipLaunchKernelGGL((k_gather2d<double2, double>), move_grid((ll)M * N, batch), dim3(NT), 0, st, M, N, f.mul,
                     f.shift, in, ldi, si, ridx, cidx, out, ldo, so, sc, batch);
  return hipGetLastError();
}

hipError_t gather2d(hipStream_t st, int M, int N, const float2* in, ll ldi, ll si, const int* ridx,
                    const int* cidx, float2* out, ll ldo, ll so, float sc, int batch) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  if ((ll)M * N > 0x7fffffffLL) return hipErrorInvalidValue;
  KernelTimer kt(st, K_MOVE, 0.0, 16.0 * (double)M * N * batch);
  const FastDiv f = make_fastdiv(M);
  hipLaunchKernelGGL((k_gather2d<float2, float>), move_grid((ll)M * N, batch), dim3(NT), 0, st, M, N, f.mul,
                     f.shift, in, ldi, si, ridx, cidx, out, ldo, so, sc, batch);
  return hipGetLastError();
}

hipError_t gather_perm(hipStream_t st, int M, int N, const double2* in, ll ldi, ll si, int idiv,
                       const int* ridx, ll sri, int rlim, const int* cidx, ll sci, int clim, double2* out, ll ldo,
                       ll so, int batch) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  if (idiv < 1 || (ll)M * N > 0x7fffffffLL) return hipErrorInvalidValue;
  KernelTimer kt(st, K_MOVE, 0.0, 32.0 * (double)M * N * batch);
  const FastDiv f = make_fastdiv(M);
  hipLaunchKernelGGL(k_gather_perm, move_grid((ll)M * N, batch), dim3(NT), 0, st, M, N, f.mul, f.shift, in, ldi,
                     si, idiv, ridx, sri, rlim, cidx, sci, clim, out, ldo, so, batch);
  return hipGetLastError();
}

hipError_t scatter_rows(hipStream_t st, int M, int N, const double2* in, ll ldi, ll si,
                        const int* ridx, double2* out, ll ldo, ll so, int batch) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  if ((ll)M * N > 0x7fffffffLL) return hipErrorInvalidValue;
  KernelTimer kt(st, K_MOVE, 0.0, 32.0 * (double)M * N * batch);
  const FastDiv f = make_fastdiv(M);
  hipLaunchKernelGGL(k_scatter_rows<double2>, move_grid((ll)M * N, batch), dim3(NT), 0, st, M, N, f.mul, f.shift,
                     in, ldi, si, ridx, out, ldo, so, batch);
  return hipGetLastError();
}

hipError_t scatter_rows(hipStream_t st, int M, int N, const float2* in, ll ldi, ll si, const int* ridx,
                        float2* out, ll ldo, ll so, int batch) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  if ((ll)M * N > 0x7fffffffLL) return hipErrorInvalidValue;
  KernelTimer kt(st, K_MOVE, 0.0, 16.0 * (double)M * N * batch);
  const FastDiv f = make_fastdiv(M);
  hipLaunchKernelGGL(k_scatter_rows<float2>, move_grid((ll)M * N, batch), dim3(NT), 0, st, M, N, f.mul, f.shift,
                     in, ldi, si, ridx, out, ldo, so, batch);
  return hipGetLastError();
}

hipError_t to_f32(hipStream_t st, const double2* x, ll n, float2* y) {
  KernelTimer kt(st, K_POINT, 0.0, 24.0 * (double)n);
  hipLaunchKernelGGL(k_to_f32, dim3(blocks_for(n)), dim3(NT), 0, st, x, n, y);
  return hipGetLastError();
}

hipError_t add_f32(hipStream_t st, const float2* x, ll n, double2* y) {
  KernelTimer kt(st, K_POINT, 2.0 * (double)n, 40.0 * (double)n);
  hipLaunchKernelGGL(k_add_f32, dim3(blocks_for(n)), dim3(NT), 0, st, x, n, y);
  return hipGetLastError();
}

hipError_t to_f64(hipStream_t st, const float2* x, ll n, double2* y) {
  KernelTimer kt(st, K_POINT, 0.0, 24.0 * (double)n);
  hipLaunchKernelGGL(k_to_f64, dim3(blocks_for(n)), dim3(NT), 0, st, x, n, y);
  return hipGetLastError();
}

hipError_t add_to_f32(hipStream_t st, const double2* x, ll n, float2* y) {
  KernelTimer kt(st, K_POINT, 2.0 * (double)n, 32.0 * (double)n);
  hipLaunchKernelGGL(k_add_to_f32, dim3(blocks_for(n)), dim3(NT), 0, st, x, n, y);
  return hipGetLastError();
}

hipError_t conj_transpose(hipStream_t st, int n, const double2* in, ll ldi, ll si, double2* out, ll ldo, ll so,
                          int batch) {
  if (n <= 0 || batch <= 0) return hipSuccess;
  KernelTimer kt(st, K_MOVE, 0.0, 32.0 * (double)n * n * batch);
  const unsigned t = (unsigned)((n + 31) / 32);
  hipLaunchKernelGGL(k_conj_transpose, dim3(t, t, batch), dim3(256), 0, st, n, in, ldi, si, out, ldo, so);
  return hipGetLastError();
}

hipError_t skel_residual(hipStream_t st, int s, int M, int ne, int lpm, const int* sab, const double2* F,
                         const double2* G, double2* rho, int cnt) {
  const ll total = (ll)cnt * 2 * s * M;
  if (total <= 0) return hipSuccess;
  KernelTimer kt(st, K_MOVE, 2.0 * (double)total, 48.0 * (double)total);
  hipLaunchKernelGGL(k_skel_residual, dim3(blocks_for(total)), dim3(NT), 0, st, s, M, ne, lpm, sab, F, G, rho,
                     total);
  return hipGetLastError();
}

hipError_t skel_gather(hipStream_t st, int n, int M, int ne, int lpb, const int* slot, const double2* X,
                       double2* out, int nbox) {
  const ll total = (ll)nbox * n * M;
  if (total <= 0) return hipSuccess;
  KernelTimer kt(st, K_MOVE, 0.0, 32.0 * (double)total);
  hipLaunchKernelGGL(k_skel_gather, dim3(blocks_for(total)), dim3(NT), 0, st, n, M, ne, lpb, slot, X, out,
                     total);
  return hipGetLastError();
}

hipError_t zadd(hipStream_t st, const double2* x, const double2* y, double2* z, ll n) {
  KernelTimer kt(st, K_POINT, 2.0 * (double)n, 48.0 * (double)n);
  hipLaunchKernelGGL(k_zadd, dim3(blocks_for(n)), dim3(NT), 0, st, x, y, z, n);
  return hipGetLastError();
}

hipError_t set2d(hipStream_t st, int M, int N, double2* out, ll ldo, ll so, double2 diag,
                 double2 off, int batch) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  if ((ll)M * N > 0x7fffffffLL) return hipErrorInvalidValue;
  KernelTimer kt(st, K_MOVE, 0.0, 16.0 * (double)M * N * batch);
  const FastDiv f = make_fastdiv(M);
  hipLaunchKernelGGL(k_set2d, move_grid((ll)M * N, batch), dim3(NT), 0, st, M, N, f.mul, f.shift, out, ldo, so,
                     diag, off, batch);
  return hipGetLastError();
}

hipError_t incident(hipStream_t st, const double4* bnode, int nb, const double2* dirs, int ndir,
                    const double* kv, double2* G, int nprob) {
  KernelTimer kt(st, K_POINT, 0.0, (32.0 + 32.0 * ndir) * (double)nb * nprob);
  hipLaunchKernelGGL(k_incident, dim3(blocks_for((ll)nb * ndir * nprob)), dim3(NT), 0, st, bnode, nb,
                     dirs, ndir, kv, G, nprob);
  return hipGetLastError();
}

hipError_t boundary_st(hipStream_t st, const double2* f, const double2* g, const double2* G,
                       int nb, int ncol, const double* etav, double2* ST, int nprob) {
  KernelTimer kt(st, K_POINT, 0.0, 16.0 * 5.0 * nb * (double)ncol * nprob);
  hipLaunchKernelGGL(k_boundary_st, dim3(blocks_for((ll)nb * ncol * nprob)), dim3(NT), 0, st, f, g, G,
                     nb, ncol, etav, ST, nprob);
  return hipGetLastError();
}

hipError_t boundary_st_adj(hipStream_t st, const double2* STb, int nb, int ncol, const double* etav,
                           double2* fb, double2* gb, int nprob) {
  KernelTimer kt(st, K_POINT, 0.0, 16.0 * 4.0 * nb * (double)ncol * nprob);
  hipLaunchKernelGGL(k_boundary_st_adj, dim3(blocks_for((ll)nb * ncol * nprob)), dim3(NT), 0, st, STb,
                     nb, ncol, etav, fb, gb, nprob);
  return hipGetLastError();
}

hipError_t scale_leaf_cols(hipStream_t st, const double* dq, const double2* H, const double* k2v, int ne, int mi,
                           ll nleaf, ll lpp, double2* Hs) {
  const ll total = (ll)ne * mi * nleaf;
  KernelTimer kt(st, K_POINT, 2.0 * (double)total, 40.0 * (double)total);
  hipLaunchKernelGGL(k_scale_leaf_cols, dim3(blocks_for(total)), dim3(NT), 0, st, dq, H, k2v, ne, mi, nleaf, lpp,
                     Hs);
  return hipGetLastError();
}

// Few directions: the body load k^2 dq u0 itself (mi x M per leaf, the
// layout of u0), so that H is read once by the product H (k^2 dq u0) instead
// of being scaled into a copy.
__global__ void k_scale_leaf_rows(const double* dq, const double2* u0, const double* k2v, int mi, int M, ll nleaf,
                                  ll lpp, double2* out) {
  const ll per = (ll)mi * M;
  const ll total = per * nleaf;
  for (ll idx = blockIdx.x * (ll)NT + threadIdx.x; idx < total; idx += (ll)gridDim.x * NT) {
    const ll z = idx / per;
    const int n = (int)(idx % per) % mi;
    const double s = k2v[z / lpp] * dq[z * mi + n];
    const double2 u = u0[idx];
    out[idx] = make_double2(s * u.x, s * u.y);
  }
}

// Few directions: grad[z mi + n] = k^2 Re sum_m conj(u0[n][m]) W[n][m] with
// W = H^H g formed by a product (mi x M per leaf); one thread per node, the
// directions summed in order.
__global__ void k_grad_rows(const double2* u0, const double2* W, const double* k2v, int mi, int M, ll nleaf, ll lpp,
                            double* grad) {
  const ll total = (ll)mi * nleaf;
  for (ll idx = blockIdx.x * (ll)NT + threadIdx.x; idx < total; idx += (ll)gridDim.x * NT) {
    const ll z = idx / mi;
    const int n = (int)(idx % mi);
    const ll base = z * (ll)mi * M + n;
    double acc = 0.0;
    for (int m = 0; m < M; ++m) {
      const double2 u = u0[base + (ll)m * mi], w = W[base + (ll)m * mi];
      acc += u.x * w.x + u.y * w.y;
    }
    grad[idx] = k2v[z / lpp] * acc;
  }
}

hipError_t scale_leaf_rows(hipStream_t st, const double* dq, const double2* u0, const double* k2v, int mi, int M,
                           ll nleaf, ll lpp, double2* out) {
  const ll total = (ll)mi * M * nleaf;
  KernelTimer kt(st, K_POINT, 6.0 * (double)total, 40.0 * (double)total);
  hipLaunchKernelGGL(k_scale_leaf_rows, dim3(blocks_for(total)), dim3(NT), 0, st, dq, u0, k2v, mi, M, nleaf, lpp,
                     out);
  return hipGetLastError();
}

hipError_t grad_rows(hipStream_t st, const double2* u0, const double2* W, const double* k2v, int mi, int M,
                     ll nleaf, ll lpp, double* grad) {
  KernelTimer kt(st, K_POINT, 4.0 * M * (double)mi * nleaf, (32.0 * M + 8.0) * mi * (double)nleaf);
  hipLaunchKernelGGL(k_grad_rows, dim3(blocks_for((ll)mi * nleaf)), dim3(NT), 0, st, u0, W, k2v, mi, M, nleaf, lpp,
                     grad);
  return hipGetLastError();
}

hipError_t grad_leaf(hipStream_t st, const double2* H, const double2* QT, const double* k2v, int ne, int mi,
                     ll nleaf, ll lpp, double* grad) {
  KernelTimer kt(st, K_POINT, 4.0 * ne * (double)mi * nleaf, (32.0 * ne + 8.0) * mi * (double)nleaf);
  hipLaunchKernelGGL(k_grad_leaf, dim3(blocks_for((ll)mi * nleaf * 16)), dim3(NT), 0, st, H, QT, k2v, ne, mi,
                     nleaf, lpp, grad);
  return hipGetLastError();
}

hipError_t export_field(hipStream_t st, const double2* u0, int mi, int ndir, ll nleaf,
                        double2* out) {
  KernelTimer kt(st, K_POINT, 0.0, 32.0 * mi * (double)ndir * nleaf);
  hipLaunchKernelGGL(k_export_field, dim3(blocks_for((ll)mi * ndir * nleaf)), dim3(NT), 0, st, u0,
                     mi, ndir, nleaf, out);
  return hipGetLastError();
}

hipError_t real_to_complex(hipStream_t st, const double* x, ll n, double2* y) {
  KernelTimer kt(st, K_POINT, 0.0, 24.0 * (double)n);
  hipLaunchKernelGGL(k_real_to_complex, dim3(blocks_for(n)), dim3(NT), 0, st, x, n, y);
  return hipGetLastError();
}

hipError_t complex_real_part(hipStream_t st, const double2* x, ll n, double* y) {
  KernelTimer kt(st, K_POINT, 0.0, 24.0 * (double)n);
  hipLaunchKernelGGL(k_complex_real_part, dim3(blocks_for(n)), dim3(NT), 0, st, x, n, y);
  return hipGetLastError();
}

}  // namespace hps
