// libhps: the C ABI of include/hps.h and include/hps_blocks.h on top of the HIP kernels.
//
// Factorisation (per contrast q, wavenumber k):
//   leaf stage   the leaf collocation matrix A = [A_ii A_ie; A_ei A_ee]
//                (PDE rows at the interior nodes, incoming-impedance rows at
//                the edge nodes; unknowns interior then edge) changes with q
//                only on the diagonal of A_ii.  The edge unknowns are folded
//                in per wavenumber (A_ee is diagonally dominant), leaving the
//                leaf's impedance problem on the interior,
//                  S = A_ii - A_ie A_ee^-1 A_ei - k^2 diag(q),
//                uniquely solvable for real k like A itself (det A =
//                det A_ee det S), which one batched call inverts.  With the
//                per-k blocks P1 = A_ie A_ee^-1, V = Mout_i - Mout_e A_ee^-1 A_ei,
//                R0 = Mout_e A_ee^-1 (Mout the outgoing impedance rows):
//                  Y = -S^-1 P1        interior field from incoming impedance,
//                  R = R0 + V Y        leaf impedance-to-impedance map,
//                  H = V S^-1          outgoing impedance from a body load;
//   merge tree   per level, all merges are batched: with child maps
//                Ra = [A11 A13; A31 A33], Rb = [B22 B23; B32 B33] on
//                (exterior, shared) nodes and the matching f3a = -g3b,
//                f3b = -g3a,
//                  W  = I - B33 A33,
//                  X  = W^-1 [B33 A31, -B32]         (f3a from [f1; f2])
//                  Yb = -[A31, 0] - A33 X             (f3b from [f1; f2])
//                  R  = blkdiag(A11, B22) + [A13 X; B23 Yb],
//                D = [X; Yb] is kept for the down-sweep and
//                U = [A13 V; -B23 (A33 V + [I, 0])], V = W^-1 [B33, -I],
//                for the upward propagation of body-load data (derivatives);
//   top          the outer-boundary system Z = A1 + A2 R_root with
//                A1 = Mt/2 - Ms/(2 i eta), A2 = Mt/2 + Ms/(2 i eta)
//                from the exterior relation Mt t = Ms s (Mt = S, Ms = K - I/2
//                for the Green relation; S + i beta (K' + I/2) and
//                K - I/2 + i beta T for the combined field), inverted.
// Solve: f_root = Z^-1 [Mt, -Ms] [d_nu u_inc; u_inc], then the
// down-sweep f3 = D f through the levels and u = Y f at the leaves.
#include "../../include/hps_blocks.h"

#include <chrono>
#include <memory>
#include <cmath>
#include <cstring>
#include <new>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "common.h"
#include "geometry.h"
#include "hps_kernels.h"

using namespace hps;

namespace {

struct HpsError {
  hps_status code;
  std::string msg;
};

#define CK(expr)                                                                          \
  do {                                                                                    \
    hipError_t _e = (expr);                                                               \
    if (_e != hipSuccess)                                                                 \
      throw HpsError{HPS_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e)};     \
  } while (0)

struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), bytes(o.bytes) {
    o.p = nullptr;
    o.bytes = 0;
  }
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  void ensure(size_t n) {
    if (n <= bytes && p) return;
    release();
    if (n == 0) n = 256;
    if (hipMalloc(&p, n) != hipSuccess) {
      p = nullptr;
      throw HpsError{HPS_ENOMEM, "device allocation of " + std::to_string(n) + " bytes failed"};
    }
    bytes = n;
  }
  double2* z() const { return (double2*)p; }
  double* d() const { return (double*)p; }
  int* i() const { return (int*)p; }
};

const double2 ONE = {1.0, 0.0};
const double2 ZERO = {0.0, 0.0};
const double2 MONE = {-1.0, 0.0};

inline size_t zb(size_t n) { return n * sizeof(double2); }

}  // namespace

struct hps_ctx {
  hps_opts o{};
  hipStream_t st = nullptr;
  int device = 0;
  Geometry g;
  std::string err;
  int nthreads = 1;
  int n = 0, nb = 0;
  int P = 1;  // problems in the batch (same grid, own q and k)

  // per wavenumber (one slot per problem)
  bool have_k = false;
  std::vector<double> kv, etav;
  // per problem, n^2 entries: the leaf blocks S0 = A_ii - A_ie A_ee^-1 A_ei
  // at q = 0 [mi x mi], P1 [mi x ne], V [ne x mi], R0 [ne x ne] (column-major,
  // consecutive)
  DBuf dLeaf;
  // top blocks scaled by A2^-1 (per problem): C1 = A2^-1 A1 and, in dBop,
  // A2^-1 [Mt, -Ms]; the outer-boundary system is then Z' = C1 + R_root
  DBuf dBop, dC1, dbnode;
  DBuf dPk;  // device [k (P) | k^2 (P) | eta (P)]
  std::vector<DBuf> didx;  // 4 index arrays per level
  // leaf-edge slots: [1 .. nlev] the shared nodes of a merge ([alpha; beta]
  // sides), [0] the outer boundary in root order
  std::vector<DBuf> dSlot;
  // per level: [pos3a; pos3b], the shared-edge rows of the two children
  std::vector<DBuf> dMap3;

  // mixed precision
  bool mixed = false;
  int refine_iters = 0;
  double refine_res = 0.0;
  int refine_fallback = 0;  // last solve fell back to the complex128 sweep
  int cg_graph_iters = 0;   // last GN step: CG iterations replayed from a graph
  DBuf dRleaf;                              // leaf ItI maps (complex128)
  std::vector<DBuf> dD32, dU32, dE32;       // complex64 sweep operators per level
  DBuf sE;                                  // h-to-f3 maps before conversion
  DBuf mF0, mF1, mF3, mTmp;                 // complex64 sweep vectors
  std::vector<DBuf> mH3;                    // complex64 shared-edge sources per level
  std::vector<DBuf> dRho;                   // interface residuals per level (complex128)
  DBuf dFl, dGl, rF0, rF1, rG0, rG1, rT0, rT1, dRb, sNorm;

  // factorisation
  bool factored = false;
  int singular = 0;
  int nonfinite = 0;  // last factorisation: 1 non-finite contrast, 2 non-finite top inverse
  DBuf dY, dH, dRroot, dZinv;
  // conjugate transposes of the top operators for the adjoint (read as plain
  // column-major operands, which the matrix cores stream faster)
  DBuf dRrootH, dZinvH;
  std::vector<DBuf> dD, dU;
  DBuf sA, sInv, sZws, sR0, sR1, sBlk, sW, sWinv, sQ, sVin, sV, sTmp, sInfo, sRbt;
  // second set of the merge scratch that a level's operator products for the
  // sweeps (V, U) read on the second stream while the next level runs (odd
  // levels; allocated when those products are formed)
  DBuf sBlk2, sWinv2, sVin2, sTmp2;
  // per merge level, the block moves that depend only on the children's maps
  // (one launch per level; built and uploaded once per factorisation)
  std::vector<MoveDesc> hMoves;
  std::vector<int> moveOff;
  DBuf dMoves;

  // solve
  bool solved = false;
  int ndir = 0;
  std::vector<double> h_dirs;
  DBuf d_dirs, dG, dRhs, dF0, dF1, dF3, du0, dST, dg;

  // measurement set
  bool have_meas = false;
  std::vector<double> theta;
  double R = 0.0;
  DBuf dPhi;

  // derivative scratch
  DBuf sB, sST2;
  // Gauss-Newton scratch
  DBuf sGn, sGnZ;

  // sine model
  int sine_S = 0;
  DBuf dSx, dSy, dNodeGrid, sS1, sS2, sS3;

  hipEvent_t ev[16] = {};  // start/end pairs: factor, solve, far field, jvp, vjp, and the factor's
                           // leaf stage, merge tree and top system
  // second stream of the leaf stage and its fork / join events (created on
  // first use, default priority)
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  hipEvent_t lev_ready = nullptr, lev_done[2] = {};  // merge levels: main -> second stream, and back
  hipEvent_t q_ready = nullptr, q_done = nullptr;     // a level's Q product on the second stream
  bool capturing = false;  // the stream is being captured into a graph: no stage timers
  double t_wave = 0.0;
  bool ev_used[8] = {};
};

namespace {

double elapsed_ms(hps_ctx* c, int a) {
  if (!c->ev_used[a]) return 0.0;
  float ms = 0.0f;
  if (hipEventElapsedTime(&ms, c->ev[2 * a], c->ev[2 * a + 1]) != hipSuccess) return 0.0;
  return ms;
}

void mark(hps_ctx* c, int a, int end) {
  if (c->capturing) return;
  CK(hipEventRecord(c->ev[2 * a + end], c->st));
  if (end) c->ev_used[a] = true;
}

template <class F>
hps_status guard(hps_ctx* c, F&& f) {
  try {
    if (c) CK(hipSetDevice(c->device));
    f();
    if (c) c->err.clear();
    return HPS_OK;
  } catch (const HpsError& e) {
    if (c) c->err = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    if (c) c->err = "host allocation failed";
    return HPS_ENOMEM;
  } catch (const std::exception& e) {
    if (c) c->err = e.what();
    return HPS_EINVAL;
  }
}

void require(bool cond, hps_status code, const char* msg) {
  if (!cond) throw HpsError{code, msg};
}

void upload(DBuf& b, const void* src, size_t bytes, hipStream_t st) {
  b.ensure(bytes);
  CK(hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, st));
  CK(hipStreamSynchronize(st));
}

// Host-side operators of one wavenumber: the leaf blocks (layout of
// hps_ctx::dLeaf), the boundary right-hand-side operator [Mt, -Ms] and the
// top blocks A1, A2.
struct WaveOps {
  std::vector<cplx> Leaf, Bop, A1, A2;
};

// In-place inverse of the row-major n x n matrix a (Gauss-Jordan with
// partial pivoting; host, small orders).
void host_inverse(int n, std::vector<cplx>& a) {
  std::vector<int> perm(n);
  for (int i = 0; i < n; ++i) perm[i] = i;
  for (int c = 0; c < n; ++c) {
    int pr = c;
    for (int r = c + 1; r < n; ++r)
      if (std::abs(a[(size_t)r * n + c]) > std::abs(a[(size_t)pr * n + c])) pr = r;
    require(std::abs(a[(size_t)pr * n + c]) > 0.0, HPS_ESINGULAR, "singular leaf edge block");
    if (pr != c) {
      for (int j = 0; j < n; ++j) std::swap(a[(size_t)pr * n + j], a[(size_t)c * n + j]);
      std::swap(perm[pr], perm[c]);
    }
    const cplx piv = 1.0 / a[(size_t)c * n + c];
    a[(size_t)c * n + c] = 1.0;
    for (int j = 0; j < n; ++j) a[(size_t)c * n + j] *= piv;
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const cplx f = a[(size_t)r * n + c];
      if (f == 0.0) continue;
      a[(size_t)r * n + c] = 0.0;
      for (int j = 0; j < n; ++j) a[(size_t)r * n + j] -= f * a[(size_t)c * n + j];
    }
  }
  // columns come out in the pivot order: undo the row exchanges
  std::vector<cplx> t(n);
  for (int r = 0; r < n; ++r) {
    for (int j = 0; j < n; ++j) t[perm[j]] = a[(size_t)r * n + j];
    for (int j = 0; j < n; ++j) a[(size_t)r * n + j] = t[j];
  }
}

// The per-wavenumber leaf blocks from the collocation matrix A0 (q = 0) and
// the outgoing rows Mout (both row-major, unknowns interior then edge).
void leaf_blocks(const Geometry& g, const std::vector<cplx>& A0, const std::vector<cplx>& Mout,
                 std::vector<cplx>& out) {
  const int mi = g.mi, ne = g.ne, n = mi + ne;
  auto a = [&](int r, int j) { return A0[(size_t)r * n + j]; };
  auto mo = [&](int e, int j) { return Mout[(size_t)e * n + j]; };
  std::vector<cplx> E((size_t)ne * ne);
  for (int i = 0; i < ne; ++i)
    for (int j = 0; j < ne; ++j) E[(size_t)i * ne + j] = a(mi + i, mi + j);
  host_inverse(ne, E);  // A_ee^-1
  std::vector<cplx> P2((size_t)ne * mi);  // A_ee^-1 A_ei
  for (int i = 0; i < ne; ++i)
    for (int b = 0; b < ne; ++b) {
      const cplx e = E[(size_t)i * ne + b];
      for (int j = 0; j < mi; ++j) P2[(size_t)i * mi + j] += e * a(mi + b, j);
    }
  out.assign((size_t)n * n, cplx());
  cplx* S0 = out.data();
  cplx* P1 = S0 + (size_t)mi * mi;
  cplx* V = P1 + (size_t)mi * ne;
  cplx* R0 = V + (size_t)ne * mi;
  for (int r = 0; r < mi; ++r)
    for (int j = 0; j < mi; ++j) {
      cplx v = a(r, j);
      for (int b = 0; b < ne; ++b) v -= a(r, mi + b) * P2[(size_t)b * mi + j];
      S0[r + (size_t)j * mi] = v;
    }
  for (int r = 0; r < mi; ++r)
    for (int j = 0; j < ne; ++j) {
      cplx v = 0.0;
      for (int b = 0; b < ne; ++b) v += a(r, mi + b) * E[(size_t)b * ne + j];
      P1[r + (size_t)j * mi] = v;
    }
  for (int e = 0; e < ne; ++e) {
    for (int j = 0; j < mi; ++j) {
      cplx v = mo(e, j);
      for (int b = 0; b < ne; ++b) v -= mo(e, mi + b) * P2[(size_t)b * mi + j];
      V[e + (size_t)j * ne] = v;
    }
    for (int j = 0; j < ne; ++j) {
      cplx v = 0.0;
      for (int b = 0; b < ne; ++b) v += mo(e, mi + b) * E[(size_t)b * ne + j];
      R0[e + (size_t)j * ne] = v;
    }
  }
}

void wave_ops(const hps_ctx* c, double k, double eta, WaveOps& w) {
  const Geometry& g = c->g;
  const int nb = c->nb;
  std::vector<cplx> A0, Mout;
  leaf_operators(g, k, eta, A0, Mout);
  leaf_blocks(g, A0, Mout, w.Leaf);
  std::vector<double> tx(nb), ty(nb);
  for (int i = 0; i < nb; ++i) {
    tx[i] = g.root[i].x;
    ty[i] = g.root[i].y;
  }
  std::vector<cplx> S, K;
  layer_moments(g, k, tx, ty, S, K, c->nthreads);
  // exterior relation Mt t = Ms s: (S, K - I/2), or the combined field
  // (S + i beta (K' + I/2), K - I/2 + i beta T), beta = 1/k
  std::vector<cplx>& Mt = S;
  std::vector<cplx>& Ms = K;
  for (int i = 0; i < nb; ++i) Ms[(size_t)i * nb + i] -= 0.5;
  if (c->o.exterior == HPS_EXT_BURTON_MILLER) {
    std::vector<cplx> Kp, T1;
    combined_field_moments(g, k, Kp, T1, c->nthreads);
    const cplx ib = cplx(0.0, 1.0 / k);
    for (int i = 0; i < nb; ++i)
      for (int j = 0; j < nb; ++j) {
        const size_t ij = (size_t)i * nb + j;
        const double nn = g.root[i].nx * g.root[j].nx + g.root[i].ny * g.root[j].ny;
        const cplx Tij = T1[ij] + k * k * nn * S[ij];
        Ms[ij] += ib * Tij;
        Mt[ij] += ib * (Kp[ij] + (i == j ? 0.5 : 0.0));
      }
  }
  const cplx cinv = cplx(0.0, -1.0 / (2.0 * eta));  // 1 / (2 i eta)
  w.Bop.assign((size_t)nb * 2 * nb, cplx());
  w.A1.assign((size_t)nb * nb, cplx());
  w.A2.assign((size_t)nb * nb, cplx());
  for (int i = 0; i < nb; ++i)
    for (int j = 0; j < nb; ++j) {
      const cplx sv = Mt[(size_t)i * nb + j];
      const cplx kmi = Ms[(size_t)i * nb + j];
      w.Bop[i + (size_t)j * nb] = sv;
      w.Bop[i + (size_t)(nb + j) * nb] = -kmi;
      w.A1[i + (size_t)j * nb] = 0.5 * sv - cinv * kmi;
      w.A2[i + (size_t)j * nb] = 0.5 * sv + cinv * kmi;
    }
}

void upload_at(DBuf& b, size_t off_bytes, const void* src, size_t bytes, hipStream_t st) {
  CK(hipMemcpyAsync((char*)b.p + off_bytes, src, bytes, hipMemcpyHostToDevice, st));
  CK(hipStreamSynchronize(st));
}

void set_wavenumbers(hps_ctx* c, const double* k) {
  const int P = c->P;
  for (int b = 0; b < P; ++b)
    require(std::isfinite(k[b]) && k[b] > 0.0, HPS_EINVAL, "wavenumbers must be positive and finite");
  const auto t0 = std::chrono::steady_clock::now();
  const Geometry& g = c->g;
  const int n = c->n, ne = g.ne, nb = c->nb;
  const double es = c->o.eta_scale > 0.0 ? c->o.eta_scale : 1.0;
  const size_t sA0 = (size_t)n * n, sBo = (size_t)nb * 2 * nb, sA = (size_t)nb * nb;
  if (!c->have_k) {
    c->dLeaf.ensure(zb(sA0 * P));
    c->dBop.ensure(zb(sBo * P));
    c->dC1.ensure(zb(sA * P));
    c->kv.assign(P, 0.0);
    c->etav.assign(P, 0.0);
    std::vector<double> bn(4 * (size_t)nb);
    for (int i = 0; i < nb; ++i) {
      const BoundaryNode& bd = g.root[i];
      bn[4 * i] = bd.x;
      bn[4 * i + 1] = bd.y;
      bn[4 * i + 2] = bd.nx;
      bn[4 * i + 3] = bd.ny;
    }
    upload(c->dbnode, bn.data(), bn.size() * sizeof(double), c->st);
  }
  bool changed = false;
  DBuf tA2, tInv, tRaw, tWs, tInfo;  // device temporaries of the A2^-1 scaling
  for (int b = 0; b < P; ++b) {
    if (c->have_k && k[b] == c->kv[b]) continue;
    changed = true;
    // reuse the operators of an earlier problem with the same wavenumber
    int src = -1;
    for (int a = 0; a < P && src < 0; ++a)
      if (a != b && c->have_k && c->kv[a] == k[b]) src = a;
    for (int a = 0; a < b && src < 0; ++a)
      if (k[a] == k[b]) src = a;
    if (src >= 0) {
      CK(hipMemcpyAsync(c->dLeaf.z() + sA0 * b, c->dLeaf.z() + sA0 * src, zb(sA0), hipMemcpyDeviceToDevice,
                        c->st));
      CK(hipMemcpyAsync(c->dBop.z() + sBo * b, c->dBop.z() + sBo * src, zb(sBo), hipMemcpyDeviceToDevice,
                        c->st));
      CK(hipMemcpyAsync(c->dC1.z() + sA * b, c->dC1.z() + sA * src, zb(sA), hipMemcpyDeviceToDevice, c->st));
    } else {
      WaveOps w;
      wave_ops(c, k[b], es * k[b], w);
      upload_at(c->dLeaf, zb(sA0 * b), w.Leaf.data(), zb(sA0), c->st);
      // C1 = A2^-1 A1 and A2^-1 [Mt, -Ms] on the device
      tA2.ensure(zb(sA));
      tInv.ensure(zb(sA));
      tRaw.ensure(zb(sBo));
      tWs.ensure(zinv_workspace(nb, 1));
      tInfo.ensure(sizeof(int));
      upload(tA2, w.A2.data(), zb(sA), c->st);
      CK(hipMemsetAsync(tInfo.p, 0, sizeof(int), c->st));
      CK(zinv(c->st, nb, tA2.z(), nb, (ll)sA, tInv.z(), nb, (ll)sA, 1, tWs.p, tInfo.i()));
      upload(tRaw, w.A1.data(), zb(sA), c->st);
      CK(zgemm(c->st, OP_N, OP_N, nb, nb, nb, ONE, tInv.z(), nb, 0, tRaw.z(), nb, 0, ZERO, c->dC1.z() + sA * b, nb,
               0, 1));
      upload(tRaw, w.Bop.data(), zb(sBo), c->st);
      CK(zgemm(c->st, OP_N, OP_N, nb, 2 * nb, nb, ONE, tInv.z(), nb, 0, tRaw.z(), nb, 0, ZERO,
               c->dBop.z() + sBo * b, nb, 0, 1));
      int info = 0;
      CK(hipMemcpyAsync(&info, tInfo.p, sizeof(int), hipMemcpyDeviceToHost, c->st));
      CK(hipStreamSynchronize(c->st));
      require(info == 0, HPS_ESINGULAR, "the exterior impedance block A2 is singular at this wavenumber");
    }
    c->kv[b] = k[b];
    c->etav[b] = es * k[b];
  }
  std::vector<double> pk(3 * (size_t)P);
  for (int b = 0; b < P; ++b) {
    pk[b] = c->kv[b];
    pk[P + b] = c->kv[b] * c->kv[b];
    pk[2 * P + b] = c->etav[b];
  }
  upload(c->dPk, pk.data(), pk.size() * sizeof(double), c->st);
  c->have_k = true;
  if (changed) {
    c->factored = false;
    c->solved = false;
    c->have_meas = false;
  }
  c->t_wave = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

void set_wavenumber(hps_ctx* c, double k) {
  std::vector<double> kv(c->P, k);
  set_wavenumbers(c, kv.data());
}

// All per-level counts below are for the whole batch: the P problems' trees
// form a forest whose nodes are numbered problem-major, so at every level
// node i has children 2 i and 2 i + 1 one level down, exactly as in one tree.
// The leaf stage runs in two parts on two streams, so that one part's panel
// eliminations (vector ALU, latency-bound) overlap the other's products
// (matrix cores).  Returns the first leaf of the second part (0: one part):
// half the problems, or half the leaves of a single problem; small stages
// stay on one stream.
int leaf_split(int nl, int lpp, int P) {
  if (nl < 512) return 0;
  return P >= 2 ? (P / 2) * lpp : nl / 2;
}

size_t align_ws(size_t x) { return (x + 255) & ~(size_t)255; }

void plan_factor_buffers(hps_ctx* c) {
  const Geometry& g = c->g;
  const size_t P = c->P;
  const size_t nl = (size_t)g.nleaf * P, ne = g.ne, mi = g.mi, nb = c->nb;
  size_t zws = zinv_workspace((int)mi, (int)nl);
  const int h = c->o.streams > 1 ? leaf_split((int)nl, g.nleaf, (int)P) : 0;
  if (h > 0) zws = std::max(zws, align_ws(zinv_workspace((int)mi, h)) + zinv_workspace((int)mi, (int)nl - h));
  size_t rmax = nl * ne * ne, blk = 0, w = 0, q = 0, v = 0;
  for (int l = 1; l <= g.nlev; ++l) {
    const LevelPattern& L = g.lev[l];
    const size_t cnt = L.count * P, m = L.m, s = L.s, np = L.np;
    zws = std::max(zws, zinv_workspace((int)s, (int)cnt));
    rmax = std::max(rmax, cnt * np * np);
    blk = std::max(blk, cnt * (2 * m * s + s * m + 2 * s * s));
    w = std::max(w, cnt * s * s);
    q = std::max(q, cnt * 2 * s * m);
    v = std::max(v, cnt * 2 * s * s);
  }
  zws = std::max(zws, zinv_workspace((int)nb, (int)P));
  c->sA.ensure(zb(std::max(nl * mi * mi, P * nb * nb)));  // leaf impedance problems, then Z
  c->sInv.ensure(zb(nl * mi * mi));  // leaf stage: S^-1
  c->sZws.ensure(zws);
  c->sR0.ensure(zb(rmax));
  c->sR1.ensure(zb(rmax));
  c->sBlk.ensure(zb(blk));
  if ((c->o.keep_derivs || c->mixed) && c->o.streams > 1) {
    c->sBlk2.ensure(zb(blk));
    c->sWinv2.ensure(zb(w));
    c->sVin2.ensure(zb(v));
    c->sTmp2.ensure(zb(v));
  }
  c->sW.ensure(zb(w));
  c->sWinv.ensure(zb(w));
  c->sQ.ensure(zb(q));
  c->sVin.ensure(zb(v));
  c->sV.ensure(zb(v));
  c->sTmp.ensure(zb(v));
  c->sInfo.ensure(sizeof(int) * (std::max<size_t>(nl, P) + 1));
  c->dY.ensure(zb(nl * mi * ne));
  if (c->o.keep_derivs) c->dH.ensure(zb(nl * ne * mi));
  c->dRroot.ensure(zb(P * nb * nb));
  c->dZinv.ensure(zb(P * nb * nb));
  if (c->o.keep_derivs) {
    c->dRrootH.ensure(zb(P * nb * nb));
    c->dZinvH.ensure(zb(P * nb * nb));
  }
  c->dD.resize(g.nlev + 1);
  c->dU.resize(g.nlev + 1);
  const bool needU = c->o.keep_derivs || c->mixed;
  for (int l = 1; l <= g.nlev; ++l) {
    const LevelPattern& L = g.lev[l];
    c->dD[l].ensure(zb(P * L.count * 2 * L.s * 2 * L.m));
    if (needU) c->dU[l].ensure(zb(P * L.count * 2 * L.m * 2 * L.s));
  }
  if (c->mixed) {
    c->dRleaf.ensure(zb(nl * ne * ne));
    c->dD32.resize(g.nlev + 1);
    c->dU32.resize(g.nlev + 1);
    c->dE32.resize(g.nlev + 1);
    size_t emax = 1;
    for (int l = 1; l <= g.nlev; ++l) {
      const LevelPattern& L = g.lev[l];
      const size_t cnt = P * L.count;
      c->dD32[l].ensure(cnt * 2 * L.s * 2 * L.m * sizeof(float2));
      c->dU32[l].ensure(cnt * 2 * L.m * 2 * L.s * sizeof(float2));
      c->dE32[l].ensure(cnt * 2 * L.s * 2 * L.s * sizeof(float2));
      emax = std::max(emax, cnt * 2 * L.s * 2 * L.s);
    }
    c->sE.ensure(zb(emax));
  }
}

// Scratch set of merge level l: with sweep operators, odd levels take the
// second set, so that a level's V and U products (second stream) read their
// blocks while the next level fills the other set.
struct MergeScratch {
  double2 *blk, *winv, *vin, *tmp;
};
MergeScratch merge_scratch(hps_ctx* c, int l) {
  if ((c->o.keep_derivs || c->mixed) && c->o.streams > 1 && (l & 1))
    return MergeScratch{c->sBlk2.z(), c->sWinv2.z(), c->sVin2.z(), c->sTmp2.z()};
  return MergeScratch{c->sBlk.z(), c->sWinv.z(), c->sVin.z(), c->sTmp.z()};
}

// The context's second stream and its events (default priority; created on
// first use).
void ensure_side(hps_ctx* c) {
  if (!c->side) CK(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
  for (hipEvent_t* e : {&c->fork, &c->join, &c->lev_ready, &c->lev_done[0], &c->lev_done[1], &c->q_ready,
                        &c->q_done})
    if (!*e) CK(hipEventCreateWithFlags(e, hipEventDisableTiming));
}

// The block moves of every merge level that depend only on the children's
// maps (gathers of the child blocks, the identity of W, the -B32 part of Q,
// the -A31 and zero parts of D's lower half, the parent map's diagonal and
// zero blocks, and V's and Tm's fixed parts), as one list per level, uploaded
// to the device.  The moves of a level write disjoint elements; they run at
// the start of the level, before the products that read or complete them.
void build_merge_moves(hps_ctx* c) {
  const Geometry& g = c->g;
  const int P = c->P;
  const bool derivs = c->o.keep_derivs || c->mixed;
  c->hMoves.clear();
  c->moveOff.assign(g.nlev + 2, 0);
  const double2 one = make_double2(1.0, 0.0), zero = make_double2(0.0, 0.0), mone = make_double2(-1.0, 0.0);
  const double2* Rc = c->sR0.z();
  for (int l = 1; l <= g.nlev; ++l) {
    c->moveOff[l] = (int)c->hMoves.size();
    const LevelPattern& L = g.lev[l];
    const int cnt = L.count * P, m = L.m, s = L.s, nc = L.nc, np = L.np;
    (void)cnt;
    const int* i1a = c->didx[4 * l].i();
    const int* i3a = c->didx[4 * l + 1].i();
    const int* i2b = c->didx[4 * l + 2].i();
    const int* i3b = c->didx[4 * l + 3].i();
    const ll sc = 2LL * nc * nc;
    const double2* Ra = Rc;
    const double2* Rb = Rc + (ll)nc * nc;
    double2* Rn = (Rc == c->sR0.z()) ? c->sR1.z() : c->sR0.z();
    const ll ms = (ll)m * s, ss = (ll)s * s, sp = (ll)np * np, sd = 4 * ms, sq = 2 * ms, sv = 2 * ss;
    const MergeScratch scr = merge_scratch(c, l);
    double2* A13 = scr.blk;
    double2* A31 = A13 + (ll)cnt * ms;
    double2* A33 = A31 + (ll)cnt * ms;
    double2* B23 = A33 + (ll)cnt * ss;
    double2* B33 = B23 + (ll)cnt * ms;
    double2* D = c->dD[l].z();
    auto gather = [&](int M, int N, const double2* in, const int* ri, const int* ci, double2* out, ll ldo,
                      ll so, double scale) {
      c->hMoves.push_back(MoveDesc{in, nc, sc, ri, ci, out, ldo, so, M, N, 0, 0, scale, zero, zero});
    };
    auto fill = [&](int M, int N, double2* out, ll ldo, ll so, double2 diag, double2 off) {
      c->hMoves.push_back(MoveDesc{nullptr, 0, 0, nullptr, nullptr, out, ldo, so, M, N, 1, 0, 0.0, diag, off});
    };
    gather(m, s, Ra, i1a, i3a, A13, m, ms, 1.0);
    gather(s, m, Ra, i3a, i1a, A31, s, ms, 1.0);
    gather(s, s, Ra, i3a, i3a, A33, s, ss, 1.0);
    gather(m, s, Rb, i2b, i3b, B23, m, ms, 1.0);
    gather(s, s, Rb, i3b, i3b, B33, s, ss, 1.0);
    fill(s, s, c->sW.z(), s, ss, one, zero);                                   // W = I (- B33 A33 below)
    gather(s, m, Rb, i3b, i2b, c->sQ.z() + ms, s, sq, -1.0);                   // Q = [., -B32]
    gather(s, m, Ra, i3a, i1a, D + s, 2 * s, sd, -1.0);                        // Yb = [-A31, 0] (- A33 X)
    fill(s, m, D + s + (ll)m * 2 * s, 2 * s, sd, zero, zero);
    gather(m, m, Ra, i1a, i1a, Rn, np, sp, 1.0);                               // R = blkdiag(A11, B22) + ...
    gather(m, m, Rb, i2b, i2b, Rn + m + (ll)m * np, np, sp, 1.0);
    fill(m, m, Rn + (ll)m * np, np, sp, zero, zero);
    fill(m, m, Rn + m, np, sp, zero, zero);
    if (derivs) {
      gather(s, s, Rb, i3b, i3b, scr.vin, s, sv, 1.0);                         // V_in = [B33, -I]
      fill(s, s, scr.vin + ss, s, sv, mone, zero);
      fill(s, 2 * s, scr.tmp, s, sv, one, zero);                               // Tm = [I, 0] (+ A33 V)
    }
    Rc = Rn;
  }
  c->moveOff[g.nlev + 1] = (int)c->hMoves.size();
  multi_move_prepare(c->hMoves.data(), (int)c->hMoves.size());
  c->dMoves.ensure(std::max<size_t>(1, c->hMoves.size()) * sizeof(MoveDesc));
  CK(hipMemcpyAsync(c->dMoves.p, c->hMoves.data(), c->hMoves.size() * sizeof(MoveDesc), hipMemcpyHostToDevice,
                    c->st));
}

// One factorisation pass.  With defer, the butterfly inverses report their
// probe checks through the device flag read at this pass's single
// synchronisation; returns false (nothing reported) when a check failed, so
// that the caller redoes the pass on the pivoted path.
bool factor_pass(hps_ctx* c, const double* q, bool defer) {
  plan_factor_buffers(c);
  c->sRbt.ensure(16);  // [int verdict flag | pad | u64 largest probe error]
  const Geometry& g = c->g;
  hipStream_t st = c->st;
  const int P = c->P;
  const int n = c->n, ne = g.ne, mi = g.mi, lpp = g.nleaf, nl = g.nleaf * P, nb = c->nb;
  const ll nn = (ll)n * n;
  const double* k2v = c->dPk.d() + P;
  c->factored = false;
  c->solved = false;
  mark(c, 0, 0);
  mark(c, 5, 0);
  profile_set_phase(PH_LEAF);
  const int ninfo = std::max(nl, P);
  // info[0 .. ninfo): zero pivots per matrix; info[ninfo]: non-finite flags
  // (1: the contrast, 2: the top inverse)
  int* nonfinite = c->sInfo.i() + ninfo;
  // work left on the second stream by an interrupted pass ends before this one
  if (c->side) {
    CK(hipEventRecord(c->join, c->side));
    CK(hipStreamWaitEvent(st, c->join, 0));
  }
  CK(hipMemsetAsync(c->sInfo.p, 0, sizeof(int) * (ninfo + 1), st));
  CK(hipMemsetAsync(c->sRbt.p, 0, 16, st));
  CK(flag_nonfinite(st, q, (ll)P * g.nleaf * mi, 1, nonfinite));
  std::unique_ptr<RbtDeferScope> defer_scope;
  if (defer) defer_scope.reset(new RbtDeferScope(c->sRbt.i(), (unsigned long long*)((char*)c->sRbt.p + 8)));

  // leaf stage (all leaves of all problems)
  // S = S0 - k^2 diag(q) per leaf, inverted (the blocks of problem z / lpp)
  const double2* S0 = c->dLeaf.z();
  const double2* P1 = S0 + (ll)mi * mi;
  const double2* V = P1 + (ll)mi * ne;
  const double2* R0 = V + (ll)ne * mi;
  const ll smm = (ll)mi * mi;
  CK(leaf_assemble(st, S0, nn, q, k2v, mi, mi, c->sA.z(), nl, lpp));
  double2* Si = c->sInv.z();
  double2* Rc = c->sR0.z();
  // leaves [z0, z1) on stream s with inverse workspace ws; the per-problem
  // operands are those of problem z0 / lpp, indexed by leaf / lpp when the
  // part starts a problem, else shared by the whole part (one problem)
  auto leaf_part = [&](hipStream_t s, int z0, int z1, void* ws) {
    const int b = z1 - z0;
    const ll pz = (ll)(z0 / lpp) * nn;
    const int dv = (z0 % lpp == 0) ? lpp : b;
    double2* Sz = Si + (ll)z0 * smm;
    double2* Yz = c->dY.z() + (ll)z0 * mi * ne;
    double2* Rz = Rc + (ll)z0 * ne * ne;
    CK(zinv(s, mi, c->sA.z() + (ll)z0 * smm, mi, smm, Sz, mi, smm, b, ws, c->sInfo.i() + z0));
    // Y = -S^-1 P1
    CK(zgemm_div(s, OP_N, OP_N, mi, ne, mi, MONE, Sz, mi, smm, 1, P1 + pz, mi, nn, dv, ZERO, Yz, mi, (ll)mi * ne,
                 b));
    // R = R0 + V Y
    CK(gather_perm(s, ne, ne, R0 + pz, ne, nn, dv, nullptr, 0, ne, nullptr, 0, ne, Rz, ne, (ll)ne * ne, b));
    CK(zgemm_div(s, OP_N, OP_N, ne, ne, mi, ONE, V + pz, ne, nn, dv, Yz, mi, (ll)mi * ne, 1, ONE, Rz, ne,
                 (ll)ne * ne, b));
    // H = V S^-1
    if (c->o.keep_derivs)
      CK(zgemm_div(s, OP_N, OP_N, ne, mi, mi, ONE, V + pz, ne, nn, dv, Sz, mi, smm, 1, ZERO,
                   c->dH.z() + (ll)z0 * ne * mi, ne, (ll)ne * mi, b));
  };
  const int h = c->o.streams > 1 ? leaf_split(nl, lpp, P) : 0;
  if (h > 0) {
    ensure_side(c);
    CK(hipEventRecord(c->fork, st));
    CK(hipStreamWaitEvent(c->side, c->fork, 0));
    leaf_part(st, 0, h, c->sZws.p);
    leaf_part(c->side, h, nl, (char*)c->sZws.p + align_ws(zinv_workspace(mi, h)));
    CK(hipEventRecord(c->join, c->side));
    CK(hipStreamWaitEvent(st, c->join, 0));
  } else {
    leaf_part(st, 0, nl, c->sZws.p);
  }
  if (c->mixed) CK(hipMemcpyAsync(c->dRleaf.p, Rc, zb((size_t)nl * ne * ne), hipMemcpyDeviceToDevice, st));
  mark(c, 5, 1);

  // merge tree
  mark(c, 6, 0);
  profile_set_phase(PH_MERGE);
  const bool derivs = c->o.keep_derivs || c->mixed;
  const bool overlap = derivs && c->o.streams > 1;  // V, U products on the second stream
  if (overlap && g.nlev > 0) ensure_side(c);
  build_merge_moves(c);
  for (int l = 1; l <= g.nlev; ++l) {
    const LevelPattern& L = g.lev[l];
    const int cnt = L.count * P, m = L.m, s = L.s, np = L.np;
    const MergeScratch scr = merge_scratch(c, l);
    double2* A13 = scr.blk;
    double2* A31 = A13 + (ll)cnt * m * s;
    double2* A33 = A31 + (ll)cnt * s * m;
    double2* B23 = A33 + (ll)cnt * s * s;
    double2* B33 = B23 + (ll)cnt * m * s;
    const ll ms = (ll)m * s, ss = (ll)s * s;
    // this level's scratch set was last read by level l - 2's products on
    // the second stream
    if (overlap && l >= 3) CK(hipStreamWaitEvent(st, c->lev_done[l & 1], 0));
    // the child blocks, the identity of W, the -B32 and -A31 parts of Q and D,
    // the parent map's diagonal blocks and zero blocks (and V's and Tm's fixed
    // parts): one launch of independent moves
    {
      const int o0 = c->moveOff[l], o1 = c->moveOff[l + 1];
      ll mx = 0;
      for (int t = o0; t < o1; ++t)
        mx = std::max(mx, (ll)c->hMoves[t].M * c->hMoves[t].N * cnt);
      CK(multi_move(st, (const MoveDesc*)c->dMoves.p + o0, o1 - o0, mx, cnt));
    }
    // Q = [B33 A31, -B32] needs no W: where W's inverse is a latency-bound
    // look-ahead chain (butterfly orders), Q runs beside it on the second
    // stream
    double2* Q = c->sQ.z();
    const ll sq = 2 * ms;
    const bool q_side = overlap && s >= 224;
    if (q_side) {
      CK(hipEventRecord(c->q_ready, st));
      CK(hipStreamWaitEvent(c->side, c->q_ready, 0));
      CK(zgemm(c->side, OP_N, OP_N, s, m, s, ONE, B33, s, ss, A31, s, ms, ZERO, Q, s, sq, cnt));
      CK(hipEventRecord(c->q_done, c->side));
    }
    // W = I - B33 A33, inverted
    double2* W = c->sW.z();
    double2* Wi = scr.winv;
    CK(zgemm(st, OP_N, OP_N, s, s, s, MONE, B33, s, ss, A33, s, ss, ONE, W, s, ss, cnt));
    CK(zinv(st, s, W, s, ss, Wi, s, ss, cnt, c->sZws.p, c->sInfo.i()));
    if (q_side)
      CK(hipStreamWaitEvent(st, c->q_done, 0));
    else
      CK(zgemm(st, OP_N, OP_N, s, m, s, ONE, B33, s, ss, A31, s, ms, ZERO, Q, s, sq, cnt));
    // D = [X; Yb]
    double2* D = c->dD[l].z();
    const ll sd = 4 * ms;
    CK(zgemm(st, OP_N, OP_N, s, 2 * m, s, ONE, Wi, s, ss, Q, s, sq, ZERO, D, 2 * s, sd, cnt));
    CK(zgemm(st, OP_N, OP_N, s, 2 * m, s, MONE, A33, s, ss, D, 2 * s, sd, ONE, D + s, 2 * s, sd,
             cnt));
    // parent map
    double2* Rn = (Rc == c->sR0.z()) ? c->sR1.z() : c->sR0.z();
    const ll sp = (ll)np * np;
    CK(zgemm(st, OP_N, OP_N, m, 2 * m, s, ONE, A13, m, ms, D, 2 * s, sd, ONE, Rn, np, sp, cnt));
    CK(zgemm(st, OP_N, OP_N, m, 2 * m, s, ONE, B23, m, ms, D + s, 2 * s, sd, ONE, Rn + m, np, sp,
             cnt));
    // the sweeps' operators V and U (and the complex64 copies) need nothing
    // of the next level: they run on the second stream meanwhile
    if (derivs) {
      hipStream_t xs = st;
      if (overlap) {
        CK(hipEventRecord(c->lev_ready, st));
        CK(hipStreamWaitEvent(c->side, c->lev_ready, 0));
        xs = c->side;
      }
      double2* Vin = scr.vin;
      double2* V = c->sV.z();
      double2* Tm = scr.tmp;
      const ll sv = 2 * ss;
      CK(zgemm(xs, OP_N, OP_N, s, 2 * s, s, ONE, Wi, s, ss, Vin, s, sv, ZERO, V, s, sv, cnt));
      double2* U = c->dU[l].z();
      CK(zgemm(xs, OP_N, OP_N, m, 2 * s, s, ONE, A13, m, ms, V, s, sv, ZERO, U, 2 * m, sd, cnt));
      CK(zgemm(xs, OP_N, OP_N, s, 2 * s, s, ONE, A33, s, ss, V, s, sv, ONE, Tm, s, sv, cnt));
      CK(zgemm(xs, OP_N, OP_N, m, 2 * s, s, MONE, B23, m, ms, Tm, s, sv, ZERO, U + m, 2 * m, sd,
               cnt));
      if (c->mixed) {
        // E = [V; -Tm]: shared-edge sources h3 to f3 (the down-sweep's h term)
        double2* E = c->sE.z();
        const ll se = 4 * ss;
        CK(gather2d(xs, s, 2 * s, V, s, sv, nullptr, nullptr, E, 2 * s, se, 1.0, cnt));
        CK(gather2d(xs, s, 2 * s, Tm, s, sv, nullptr, nullptr, E + s, 2 * s, se, -1.0, cnt));
        CK(to_f32(xs, E, (ll)cnt * se, (float2*)c->dE32[l].p));
        CK(to_f32(xs, D, (ll)cnt * sd, (float2*)c->dD32[l].p));
        CK(to_f32(xs, U, (ll)cnt * sd, (float2*)c->dU32[l].p));
      }
      if (overlap) CK(hipEventRecord(c->lev_done[l & 1], xs));
    }
    Rc = Rn;
  }
  mark(c, 6, 1);

  // top: Z' = A2^-1 (A1 + A2 R_root) = C1 + R_root per problem, inverted
  mark(c, 7, 0);
  profile_set_phase(PH_TOP);
  const ll sbb = (ll)nb * nb;
  CK(hipMemcpyAsync(c->dRroot.p, Rc, zb((size_t)P * sbb), hipMemcpyDeviceToDevice, st));
  double2* Z = c->sA.z();
  CK(zadd(st, c->dC1.z(), Rc, Z, (ll)P * sbb));
  CK(zinv(st, nb, Z, nb, sbb, c->dZinv.z(), nb, sbb, P, c->sZws.p, c->sInfo.i()));
  if (c->o.keep_derivs) {
    CK(conj_transpose(st, nb, c->dRroot.z(), nb, sbb, c->dRrootH.z(), nb, sbb, P));
    CK(conj_transpose(st, nb, c->dZinv.z(), nb, sbb, c->dZinvH.z(), nb, sbb, P));
  }
  CK(flag_nonfinite(st, (const double*)c->dZinv.p, 2 * (ll)P * sbb, 2, nonfinite));
  // the last merge levels' sweep operators (second stream) overlap the top
  if (overlap && g.nlev > 0) CK(hipStreamWaitEvent(st, c->lev_done[g.nlev & 1], 0));
  mark(c, 7, 1);
  mark(c, 0, 1);
  profile_set_phase(PH_OTHER);
  std::vector<int> info(ninfo + 1);
  unsigned long long rbt[2] = {0, 0};
  CK(hipMemcpyAsync(info.data(), c->sInfo.p, sizeof(int) * (ninfo + 1), hipMemcpyDeviceToHost, st));
  CK(hipMemcpyAsync(rbt, c->sRbt.p, 16, hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  defer_scope.reset();
  c->nonfinite = info[ninfo];
  if (c->nonfinite & 1) throw HpsError{HPS_ENONFINITE, "the contrast q holds a NaN or infinite value"};
  if (defer) {
    int flag = 0;
    double max_err = 0.0;
    std::memcpy(&flag, &rbt[0], sizeof(int));
    std::memcpy(&max_err, &rbt[1], sizeof(double));
    zinv_note_deferred(max_err, flag != 0);
    if (flag) return false;
  }
  c->singular = 0;
  for (int i = 0; i < ninfo; ++i) c->singular |= (info[i] != 0);
  if (c->singular) throw HpsError{HPS_ESINGULAR, "zero pivot in the factorisation"};
  if (c->nonfinite) throw HpsError{HPS_ENONFINITE, "the factorisation produced a NaN or infinite value"};
  c->factored = true;
  return true;
}

void factor(hps_ctx* c, const double* q, const double* kv) {
  require(q != nullptr, HPS_EINVAL, "q_nodes is NULL");
  bool same = c->have_k;
  for (int b = 0; b < c->P && same; ++b) same = (kv[b] == c->kv[b]);
  if (!same) set_wavenumbers(c, kv);
  // the butterfly inverses' checks are read once per pass; a failed check
  // (not met so far on any workload) redoes the pass with pivoting
  if (factor_pass(c, q, true)) return;
  RbtOffScope pivoted;
  factor_pass(c, q, false);
}

void plan_sweep_buffers(hps_ctx* c, int M) {
  const Geometry& g = c->g;
  const size_t P = c->P;
  size_t fmax = (size_t)g.nleaf * g.ne, f3 = 0;
  for (int l = 1; l <= g.nlev; ++l) {
    const LevelPattern& L = g.lev[l];
    fmax = std::max(fmax, (size_t)L.count * L.np);
    f3 = std::max(f3, (size_t)L.count * 2 * L.s);
  }
  fmax = std::max(fmax, (size_t)c->nb);
  c->dF0.ensure(zb(P * fmax * M));
  c->dF1.ensure(zb(P * fmax * M));
  c->dF3.ensure(zb(P * std::max<size_t>(f3, 1) * M));
  c->dG.ensure(zb(P * 2 * c->nb * M));
  c->dRhs.ensure(zb(P * c->nb * M));
  c->dg.ensure(zb(P * c->nb * M));
  c->dST.ensure(zb(P * 2 * c->nb * M));
  c->du0.ensure(zb(P * g.nleaf * g.mi * M));
}

// Down-sweep step of one level: F3 = Op [f1; f2] per merge (Op: D, or U^H
// for the adjoint sweep) written straight into the two children's boundary
// orderings (rows pos3a of child alpha, pos3b of child beta), then the
// parent data [f1; f2] copied to the children's exterior rows.
void down_level(hps_ctx* c, int l, int op, const double2* Op, const double2* Fp, double2* Fch, int M) {
  const LevelPattern& L = c->g.lev[l];
  const int cnt = L.count * c->P, m = L.m, s = L.s, nc = L.nc, np = L.np;
  const ll sp = (ll)np * M, sc = 2LL * nc * M;
  hipStream_t st = c->st;
  if (op == OP_N)
    CK(zgemm_rowmap(st, OP_N, OP_N, 2 * s, M, np, ONE, Op, 2 * s, 4LL * m * s, Fp, np, sp, ZERO, Fch, nc, sc,
                    c->dMap3[l].i(), s, (ll)nc * M, cnt));
  else
    CK(zgemm_rowmap(st, OP_C, OP_N, 2 * s, M, np, ONE, Op, np, 4LL * m * s, Fp, np, sp, ZERO, Fch, nc, sc,
                    c->dMap3[l].i(), s, (ll)nc * M, cnt));
  const RowMove mv[2] = {{Fp, np, sp, c->didx[4 * l].i(), Fch, nc, sc, m, 1},
                         {Fp + m, np, sp, c->didx[4 * l + 2].i(), Fch + (ll)nc * M, nc, sc, m, 1}};
  CK(row_moves(st, mv, 2, M, cnt));
}

// ---- mixed precision: complex64 sweeps refined on the skeleton system ----
//
// Skeleton unknowns: the incoming impedance data f on every leaf edge.  The
// leaf maps give g = R_leaf f; the equations are the matching f3a = -g3b,
// f3b = -g3a at the shared edge of every merge, and A1 f + A2 g = rhs on
// the outer boundary.  The residual is formed in complex128; a correction
// solves the same system with the residuals as sources: an interface
// residual enters a merge exactly like the h data of a body load, with
// h3a += rho_b and h3b += rho_a, so the correction is an up-sweep of sources
// (U), the top solve and a down-sweep that adds E h3 at every level.

void plan_mixed_buffers(hps_ctx* c, int M) {
  const Geometry& g = c->g;
  const size_t P = c->P, Ms = M;
  const size_t leaf = P * g.nleaf * g.ne * Ms;
  size_t up = 1, sh = 1;
  c->dRho.resize(g.nlev + 1);
  c->mH3.resize(g.nlev + 1);
  for (int l = 1; l <= g.nlev; ++l) {
    const LevelPattern& L = g.lev[l];
    const size_t cnt = P * L.count;
    up = std::max(up, cnt * L.np * Ms);
    sh = std::max(sh, cnt * 2 * L.s * Ms);
    c->dRho[l].ensure(zb(cnt * 2 * L.s * Ms));
    c->mH3[l].ensure(cnt * 2 * L.s * Ms * sizeof(float2));
  }
  const size_t top = P * c->nb * Ms;
  c->dFl.ensure(zb(leaf));
  c->dGl.ensure(zb(leaf));
  c->rF0.ensure(zb(up));
  c->rF1.ensure(zb(up));
  c->rG0.ensure(zb(up));
  c->rG1.ensure(zb(up));
  c->rT0.ensure(zb(std::max(sh, top)));
  c->rT1.ensure(zb(std::max(sh, top)));
  c->dRb.ensure(zb(top));
  c->mF0.ensure(std::max(leaf, up) * sizeof(float2));
  c->mF1.ensure(std::max(leaf, up) * sizeof(float2));
  c->mF3.ensure(sh * sizeof(float2));
  c->sNorm.ensure(sizeof(double) * (256 + g.nlev + 8));
}

// complex64 down-sweep from root data Fr (complex64 [P][nb][M]) to leaf-edge
// data (returned buffer, complex64 [nl][ne][M]); with_h adds E h3 per level.
float2* mixed_down(hps_ctx* c, int M, float2* Fr, bool with_h) {
  const Geometry& g = c->g;
  hipStream_t st = c->st;
  const float2 one = make_float2(1.0f, 0.0f), zero = make_float2(0.0f, 0.0f);
  float2* Fc = Fr;
  float2* Fo = (Fr == (float2*)c->mF0.p) ? (float2*)c->mF1.p : (float2*)c->mF0.p;
  float2* F3 = (float2*)c->mF3.p;
  for (int l = g.nlev; l >= 1; --l) {
    const LevelPattern& L = g.lev[l];
    const int cnt = L.count * c->P, m = L.m, s = L.s, nc = L.nc, np = L.np;
    const ll s3 = 2LL * s * M;
    CK(cgemm(st, OP_N, OP_N, 2 * s, M, 2 * m, one, (const float2*)c->dD32[l].p, 2 * s, 4LL * m * s, Fc, np,
             (ll)np * M, zero, F3, 2 * s, s3, cnt));
    if (with_h)
      CK(cgemm(st, OP_N, OP_N, 2 * s, M, 2 * s, one, (const float2*)c->dE32[l].p, 2 * s, 4LL * s * s,
               (const float2*)c->mH3[l].p, 2 * s, s3, one, F3, 2 * s, s3, cnt));
    const ll sp = (ll)np * M, sc = 2LL * nc * M;
    CK(scatter_rows(st, m, M, Fc, np, sp, c->didx[4 * l].i(), Fo, nc, sc, cnt));
    CK(scatter_rows(st, s, M, F3, 2 * s, s3, c->didx[4 * l + 1].i(), Fo, nc, sc, cnt));
    CK(scatter_rows(st, m, M, Fc + m, np, sp, c->didx[4 * l + 2].i(), Fo + (ll)nc * M, nc, sc, cnt));
    CK(scatter_rows(st, s, M, F3 + s, 2 * s, s3, c->didx[4 * l + 3].i(), Fo + (ll)nc * M, nc, sc, cnt));
    std::swap(Fc, Fo);
  }
  return Fc;
}

// Residual of the skeleton system at the leaf data dFl (complex128):
// dRho[l] = [f3b + g3a; f3a + g3b] per level, dRb = A1 f + A2 g - rhs on
// the outer boundary.  Returns the relative residual
// max(||rho|| / ||f||, ||r_b|| / ||rhs||); froot / groot receive the outer
// boundary data.
double mixed_residual(hps_ctx* c, int M, const double2*& froot, const double2*& groot) {
  const Geometry& g = c->g;
  hipStream_t st = c->st;
  const int P = c->P, ne = g.ne, nb = c->nb, nl = g.nleaf * P;
  CK(zgemm(st, OP_N, OP_N, ne, M, ne, ONE, c->dRleaf.z(), ne, (ll)ne * ne, c->dFl.z(), ne, (ll)ne * M, ZERO,
           c->dGl.z(), ne, (ll)ne * M, nl));
  double* partial = c->sNorm.d();
  double* nrm = partial + 256;  // [0] f, [1] rhs, [2] r_b, [3 ..] rho per level
  for (int l = 1; l <= g.nlev; ++l) {
    const LevelPattern& L = g.lev[l];
    const int cnt = L.count * P, s = L.s;
    const ll nr = (ll)cnt * 2 * s * M;
    CK(skel_residual(st, s, M, ne, 1 << l, c->dSlot[l].i(), c->dFl.z(), c->dGl.z(), c->dRho[l].z(), cnt));
    CK(dot(st, (const double*)c->dRho[l].p, (const double*)c->dRho[l].p, 2 * nr, partial, nrm + 2 + l));
  }
  // outer-boundary data in root order
  double2* fc = c->rF0.z();
  double2* gc = c->rG0.z();
  CK(skel_gather(st, nb, M, ne, g.nleaf, c->dSlot[0].i(), c->dFl.z(), fc, P));
  CK(skel_gather(st, nb, M, ne, g.nleaf, c->dSlot[0].i(), c->dGl.z(), gc, P));
  froot = fc;
  groot = gc;
  const ll sF = (ll)nb * M, sbb = (ll)nb * nb, ntop = (ll)P * sF;
  CK(hipMemcpyAsync(c->dRb.p, c->dRhs.p, zb((size_t)ntop), hipMemcpyDeviceToDevice, st));
  // outer-boundary residual in the scaled form C1 f + g - A2^-1 rhs
  CK(zgemm(st, OP_N, OP_N, nb, M, nb, ONE, c->dC1.z(), nb, sbb, froot, nb, sF, MONE, c->dRb.z(), nb, sF, P));
  CK(zadd(st, c->dRb.z(), groot, c->dRb.z(), ntop));
  const ll nleaf = (ll)nl * ne * M;
  CK(dot(st, (const double*)c->dFl.p, (const double*)c->dFl.p, 2 * nleaf, partial, nrm));
  CK(dot(st, (const double*)c->dRhs.p, (const double*)c->dRhs.p, 2 * ntop, partial, nrm + 1));
  CK(dot(st, (const double*)c->dRb.p, (const double*)c->dRb.p, 2 * ntop, partial, nrm + 2));
  std::vector<double> h(g.nlev + 3);
  CK(hipMemcpyAsync(h.data(), nrm, sizeof(double) * h.size(), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  double rho = 0.0;
  for (int l = 1; l <= g.nlev; ++l) rho += h[2 + l];
  const double rf = h[0] > 0.0 ? std::sqrt(rho / h[0]) : std::sqrt(rho);
  const double rb = h[1] > 0.0 ? std::sqrt(h[2] / h[1]) : std::sqrt(h[2]);
  return std::max(rf, rb);
}

// One correction of the leaf data dFl from the residuals dRho, dRb.
void mixed_correct(hps_ctx* c, int M) {
  const Geometry& g = c->g;
  hipStream_t st = c->st;
  const int P = c->P, nb = c->nb;
  const float2 one = make_float2(1.0f, 0.0f), zero = make_float2(0.0f, 0.0f);
  // up-sweep of sources (complex64); the leaves carry none
  const float2* hc = nullptr;
  float2* ho[2] = {(float2*)c->mF0.p, (float2*)c->mF1.p};
  int pp = 0;
  for (int l = 1; l <= g.nlev; ++l) {
    const LevelPattern& L = g.lev[l];
    const int cnt = L.count * P, m = L.m, s = L.s, nc = L.nc, np = L.np;
    const ll sc = 2LL * nc * M, sp = (ll)np * M, s3 = 2LL * s * M, nr = (ll)cnt * s3;
    float2* H3 = (float2*)c->mH3[l].p;
    float2* hp = ho[pp];
    if (hc == nullptr) {
      CK(to_f32(st, c->dRho[l].z(), nr, H3));
      CK(cgemm(st, OP_N, OP_N, np, M, 2 * s, one, (const float2*)c->dU32[l].p, np, 4LL * m * s, H3, 2 * s, s3,
               zero, hp, np, sp, cnt));
    } else {
      const float2* ha = hc;
      const float2* hb = hc + (ll)nc * M;
      CK(gather2d(st, m, M, ha, nc, sc, c->didx[4 * l].i(), nullptr, hp, np, sp, 1.0f, cnt));
      CK(gather2d(st, m, M, hb, nc, sc, c->didx[4 * l + 2].i(), nullptr, hp + m, np, sp, 1.0f, cnt));
      CK(gather2d(st, s, M, ha, nc, sc, c->didx[4 * l + 1].i(), nullptr, H3, 2 * s, s3, 1.0f, cnt));
      CK(gather2d(st, s, M, hb, nc, sc, c->didx[4 * l + 3].i(), nullptr, H3 + s, 2 * s, s3, 1.0f, cnt));
      CK(add_to_f32(st, c->dRho[l].z(), nr, H3));
      CK(cgemm(st, OP_N, OP_N, np, M, 2 * s, one, (const float2*)c->dU32[l].p, np, 4LL * m * s, H3, 2 * s, s3,
               one, hp, np, sp, cnt));
    }
    hc = hp;
    pp ^= 1;
  }
  // top: delta f = Z'^-1 (-r_b - h)
  const ll sF = (ll)nb * M, sbb = (ll)nb * nb, ntop = (ll)P * sF;
  double2* hr = c->rT0.z();
  double2* w = c->rT1.z();
  CK(to_f64(st, hc, ntop, hr));
  CK(gather2d(st, (int)ntop, 1, c->dRb.z(), ntop, 0, nullptr, nullptr, w, ntop, 0, -1.0, 1));
  CK(zsub(st, w, hr, w, ntop));
  CK(zgemm(st, OP_N, OP_N, nb, M, nb, ONE, c->dZinv.z(), nb, sbb, w, nb, sF, ZERO, hr, nb, sF, P));
  float2* dr = (hc == (float2*)c->mF0.p) ? (float2*)c->mF1.p : (float2*)c->mF0.p;
  CK(to_f32(st, hr, ntop, dr));
  float2* dfl = mixed_down(c, M, dr, true);
  CK(add_f32(st, dfl, (ll)P * g.nleaf * g.ne * M, c->dFl.z()));
}

// Mixed-precision forward solve from the root data Fc = Z^-1 rhs
// (complex128).  Leaves dST and du0 as the complex128 path does.
void solve_mixed(hps_ctx* c, int M, const double2* Fc) {
  const Geometry& g = c->g;
  hipStream_t st = c->st;
  const int P = c->P, nb = c->nb;
  plan_mixed_buffers(c, M);
  const ll ntop = (ll)P * nb * M;
  float2* fr = (float2*)c->mF0.p;
  CK(to_f32(st, Fc, ntop, fr));
  float2* fl = mixed_down(c, M, fr, false);
  CK(to_f64(st, fl, (ll)P * g.nleaf * g.ne * M, c->dFl.z()));
  const double2* froot = nullptr;
  const double2* groot = nullptr;
  int it = 0;
  double res = mixed_residual(c, M, froot, groot);
  while (res > c->o.refine_tol && it < c->o.max_refine) {
    mixed_correct(c, M);
    ++it;
    res = mixed_residual(c, M, froot, groot);
  }
  c->refine_iters = it;
  c->refine_res = res;
  CK(boundary_st(st, froot, groot, c->dG.z(), nb, M, c->dPk.d() + 2 * P, c->dST.z(), P));
  CK(zgemm(st, OP_N, OP_N, g.mi, M, g.ne, ONE, c->dY.z(), g.mi, (ll)g.mi * g.ne, c->dFl.z(), g.ne,
           (ll)g.ne * M, ZERO, c->du0.z(), g.mi, (ll)g.mi * M, g.nleaf * P));
}

// complex128 sweep from the root data Fc (= Z^-1 rhs): boundary (s, t), the
// down-sweep through the levels and u0 = Y f at the leaves.  Fo is scratch.
void solve_fp64(hps_ctx* c, int M, double2* Fc, double2* Fo) {
  const Geometry& g = c->g;
  hipStream_t st = c->st;
  const int P = c->P, nb = c->nb;
  const ll sF = (ll)nb * M, sbb = (ll)nb * nb;
  CK(zgemm(st, OP_N, OP_N, nb, M, nb, ONE, c->dRroot.z(), nb, sbb, Fc, nb, sF, ZERO, c->dg.z(), nb, sF,
           P));
  CK(boundary_st(st, Fc, c->dg.z(), c->dG.z(), nb, M, c->dPk.d() + 2 * P, c->dST.z(), P));
  for (int l = g.nlev; l >= 1; --l) {
    down_level(c, l, OP_N, c->dD[l].z(), Fc, Fo, M);
    std::swap(Fc, Fo);
  }
  CK(zgemm(st, OP_N, OP_N, g.mi, M, g.ne, ONE, c->dY.z(), g.mi, (ll)g.mi * g.ne, Fc, g.ne,
           (ll)g.ne * M, ZERO, c->du0.z(), g.mi, (ll)g.mi * M, g.nleaf * P));
}

// ang: P x M direction angles (problem-major).
void solve(hps_ctx* c, int M, const double* ang) {
  require(c->factored, HPS_ESTATE, "hps_solve before hps_factor");
  require(M >= 1 && M <= 65535 && ang != nullptr, HPS_EINVAL, "bad direction list");
  const int P = c->P;
  for (ll i = 0; i < (ll)M * P; ++i) require(std::isfinite(ang[i]), HPS_EINVAL, "non-finite angle");
  plan_sweep_buffers(c, M);
  const Geometry& g = c->g;
  hipStream_t st = c->st;
  const int nb = c->nb;
  c->h_dirs.resize(2 * (size_t)M * P);
  for (ll i = 0; i < (ll)M * P; ++i) {
    c->h_dirs[2 * i] = std::cos(ang[i]);
    c->h_dirs[2 * i + 1] = std::sin(ang[i]);
  }
  upload(c->d_dirs, c->h_dirs.data(), c->h_dirs.size() * sizeof(double), st);
  c->solved = false;
  mark(c, 1, 0);
  profile_set_phase(PH_SOLVE);
  const double* kv = c->dPk.d();
  const double* etav = c->dPk.d() + 2 * P;
  const ll sG = 2LL * nb * M, sF = (ll)nb * M, sbb = (ll)nb * nb;
  CK(incident(st, (const double4*)c->dbnode.p, nb, c->d_dirs.z(), M, kv, c->dG.z(), P));
  CK(zgemm(st, OP_N, OP_N, nb, M, 2 * nb, ONE, c->dBop.z(), nb, 2 * sbb, c->dG.z(), 2 * nb, sG, ZERO,
           c->dRhs.z(), nb, sF, P));
  double2* Fc = c->dF0.z();
  double2* Fo = c->dF1.z();
  CK(zgemm(st, OP_N, OP_N, nb, M, nb, ONE, c->dZinv.z(), nb, sbb, c->dRhs.z(), nb, sF, ZERO, Fc, nb, sF,
           P));
  c->refine_fallback = 0;
  if (c->mixed) {
    solve_mixed(c, M, Fc);
    if (!(c->refine_res <= c->o.refine_tol) && c->o.fallback_fp64) {
      // refinement stopped above its target: the complex128 sweep from the
      // same top solution (Fc is untouched by the mixed sweeps)
      solve_fp64(c, M, Fc, Fo);
      c->refine_fallback = 1;
    }
    mark(c, 1, 1);
    profile_set_phase(PH_OTHER);
    c->ndir = M;
    c->solved = true;
    if (!c->refine_fallback && !(c->refine_res <= c->o.refine_tol))
      throw HpsError{HPS_ENOCONV, "refinement stopped at relative residual " + std::to_string(c->refine_res)};
    return;
  }
  solve_fp64(c, M, Fc, Fo);
  mark(c, 1, 1);
  profile_set_phase(PH_OTHER);
  c->ndir = M;
  c->solved = true;
}

void set_measurement(hps_ctx* c, int nt, const double* th, double R) {
  bool same = c->have_meas && nt == (int)c->theta.size() && R == c->R;
  if (same)
    for (int i = 0; i < nt; ++i) same = same && th[i] == c->theta[i];
  if (same) return;
  const Geometry& g = c->g;
  const double half = 0.5 * g.h * g.L;
  const double xc = g.x0 + half, yc = g.y0 + half;
  std::vector<double> tx(nt), ty(nt);
  for (int i = 0; i < nt; ++i) {
    require(std::isfinite(th[i]), HPS_EINVAL, "non-finite angle");
    tx[i] = R * std::cos(th[i]);
    ty[i] = R * std::sin(th[i]);
    require(std::max(std::fabs(tx[i] - xc), std::fabs(ty[i] - yc)) > half * (1.0 + 1e-12),
            HPS_EINVAL, "measurement point inside Omega");
  }
  const int nb = c->nb, P = c->P;
  const size_t sphi = (size_t)nt * 2 * nb;
  c->dPhi.ensure(zb(sphi * P));
  for (int b = 0; b < P; ++b) {
    int src = -1;
    for (int a = 0; a < b && src < 0; ++a)
      if (c->kv[a] == c->kv[b]) src = a;
    if (src >= 0) {
      CK(hipMemcpyAsync(c->dPhi.z() + sphi * b, c->dPhi.z() + sphi * src, zb(sphi), hipMemcpyDeviceToDevice,
                        c->st));
      continue;
    }
    std::vector<cplx> PS, PD;
    layer_moments(g, c->kv[b], tx, ty, PS, PD, c->nthreads);
    std::vector<cplx> Phi(sphi);
    for (int p = 0; p < nt; ++p)
      for (int j = 0; j < nb; ++j) {
        Phi[p + (size_t)j * nt] = PD[(size_t)p * nb + j];
        Phi[p + (size_t)(nb + j) * nt] = -PS[(size_t)p * nb + j];
      }
    upload_at(c->dPhi, zb(sphi * b), Phi.data(), zb(sphi), c->st);
  }
  c->theta.assign(th, th + nt);
  c->R = R;
  c->have_meas = true;
}

void far_field(hps_ctx* c, int nt, const double* th, double R, double* out) {
  require(c->solved, HPS_ESTATE, "hps_far_field before hps_solve");
  require(nt >= 1 && th != nullptr && out != nullptr && std::isfinite(R) && R > 0.0, HPS_EINVAL,
          "bad measurement arguments");
  set_measurement(c, nt, th, R);
  const int nb = c->nb, M = c->ndir, P = c->P;
  mark(c, 2, 0);
  profile_set_phase(PH_FAR);
  CK(zgemm(c->st, OP_N, OP_N, nt, M, 2 * nb, ONE, c->dPhi.z(), nt, (ll)nt * 2 * nb, c->dST.z(), 2 * nb,
           2LL * nb * M, ZERO, (double2*)out, nt, (ll)nt * M, P));
  mark(c, 2, 1);
  profile_set_phase(PH_OTHER);
}

void jvp(hps_ctx* c, const double* dq, double* out) {
  require(c->solved && c->have_meas, HPS_ESTATE, "hps_jvp needs hps_solve and hps_far_field");
  require(c->o.keep_derivs != 0, HPS_ESTATE, "context created without keep_derivs");
  require(dq != nullptr && out != nullptr, HPS_EINVAL, "NULL argument");
  const Geometry& g = c->g;
  hipStream_t st = c->st;
  const int M = c->ndir, nb = c->nb, nt = (int)c->theta.size(), P = c->P;
  const int nl = g.nleaf * P;
  const ll sF = (ll)nb * M, sbb = (ll)nb * nb;
  c->sB.ensure(zb((size_t)nl * g.ne * g.mi));
  c->sST2.ensure(zb((size_t)2 * P * nb * M));
  mark(c, 3, 0);
  profile_set_phase(PH_JVP);
  // leaf outgoing data of the body load k^2 dq u0: H (k^2 dq u0).  With many
  // directions H diag(k^2 dq) is formed (ne x mi per leaf, fewer bytes than
  // the scaled fields); with fewer than ne directions the fields are scaled
  // (mi x M per leaf) and H is read once.
  double2* Hc = c->dF0.z();
  double2* Ho = c->dF1.z();
  if (M < g.ne) {
    CK(scale_leaf_rows(st, dq, c->du0.z(), c->dPk.d() + P, g.mi, M, nl, g.nleaf, c->sB.z()));
    CK(zgemm(st, OP_N, OP_N, g.ne, M, g.mi, ONE, c->dH.z(), g.ne, (ll)g.ne * g.mi, c->sB.z(), g.mi,
             (ll)g.mi * M, ZERO, Hc, g.ne, (ll)g.ne * M, nl));
  } else {
    CK(scale_leaf_cols(st, dq, c->dH.z(), c->dPk.d() + P, g.ne, g.mi, nl, g.nleaf, c->sB.z()));
    CK(zgemm(st, OP_N, OP_N, g.ne, M, g.mi, ONE, c->sB.z(), g.ne, (ll)g.ne * g.mi, c->du0.z(), g.mi,
             (ll)g.mi * M, ZERO, Hc, g.ne, (ll)g.ne * M, nl));
  }
  for (int l = 1; l <= g.nlev; ++l) {
    const LevelPattern& L = g.lev[l];
    const int cnt = L.count * P, m = L.m, s = L.s, nc = L.nc, np = L.np;
    const ll sc = 2LL * nc * M, sp = (ll)np * M, s3 = 2LL * s * M;
    const double2* Ha = Hc;
    const double2* Hb = Hc + (ll)nc * M;
    double2* H3 = c->dF3.z();
    // the children's exterior data to the parent ordering, their shared-edge
    // data to H3: one launch
    const RowMove mv[4] = {{Ha, nc, sc, c->didx[4 * l].i(), Ho, np, sp, m, 0},
                           {Hb, nc, sc, c->didx[4 * l + 2].i(), Ho + m, np, sp, m, 0},
                           {Ha, nc, sc, c->didx[4 * l + 1].i(), H3, 2 * s, s3, s, 0},
                           {Hb, nc, sc, c->didx[4 * l + 3].i(), H3 + s, 2 * s, s3, s, 0}};
    CK(row_moves(st, mv, 4, M, cnt));
    CK(zgemm(st, OP_N, OP_N, np, M, 2 * s, ONE, c->dU[l].z(), np, 4LL * m * s, H3, 2 * s, s3, ONE,
             Ho, np, sp, cnt));
    std::swap(Hc, Ho);
  }
  // root: f = -Z'^-1 h (Z' = A2^-1 Z),  g = R f + h
  CK(zgemm(st, OP_N, OP_N, nb, M, nb, MONE, c->dZinv.z(), nb, sbb, Hc, nb, sF, ZERO, Ho, nb, sF, P));
  CK(hipMemcpyAsync(c->dg.p, Hc, zb((size_t)P * nb * M), hipMemcpyDeviceToDevice, st));
  CK(zgemm(st, OP_N, OP_N, nb, M, nb, ONE, c->dRroot.z(), nb, sbb, Ho, nb, sF, ONE, c->dg.z(), nb, sF,
           P));
  CK(boundary_st(st, Ho, c->dg.z(), nullptr, nb, M, c->dPk.d() + 2 * P, c->sST2.z(), P));
  CK(zgemm(st, OP_N, OP_N, nt, M, 2 * nb, ONE, c->dPhi.z(), nt, (ll)nt * 2 * nb, c->sST2.z(), 2 * nb,
           2LL * nb * M, ZERO, (double2*)out, nt, (ll)nt * M, P));
  mark(c, 3, 1);
  profile_set_phase(PH_OTHER);
}

void vjp(hps_ctx* c, const double* r, double* grad) {
  require(c->solved && c->have_meas, HPS_ESTATE, "hps_vjp needs hps_solve and hps_far_field");
  require(c->o.keep_derivs != 0, HPS_ESTATE, "context created without keep_derivs");
  require(r != nullptr && grad != nullptr, HPS_EINVAL, "NULL argument");
  const Geometry& g = c->g;
  hipStream_t st = c->st;
  const int M = c->ndir, nb = c->nb, nt = (int)c->theta.size(), P = c->P;
  const int nl = g.nleaf * P;
  const ll sF = (ll)nb * M, sbb = (ll)nb * nb;
  c->sB.ensure(zb((size_t)nl * g.ne * g.mi));
  c->sST2.ensure(zb((size_t)2 * P * nb * M));
  mark(c, 4, 0);
  profile_set_phase(PH_VJP);
  // [sbar; tbar] = Phi^H r
  CK(zgemm(st, OP_C, OP_N, 2 * nb, M, nt, ONE, c->dPhi.z(), nt, (ll)nt * 2 * nb, (const double2*)r, nt,
           (ll)nt * M, ZERO, c->sST2.z(), 2 * nb, 2LL * nb * M, P));
  double2* Hc = c->dF0.z();
  double2* Ho = c->dF1.z();
  double2* fb = Ho;
  double2* gb = Hc;
  CK(boundary_st_adj(st, c->sST2.z(), nb, M, c->dPk.d() + 2 * P, fb, gb, P));
  CK(zgemm(st, OP_N, OP_N, nb, M, nb, ONE, c->dRrootH.z(), nb, sbb, gb, nb, sF, ONE, fb, nb, sF, P));
  CK(zgemm(st, OP_N, OP_N, nb, M, nb, MONE, c->dZinvH.z(), nb, sbb, fb, nb, sF, ONE, gb, nb, sF, P));
  for (int l = g.nlev; l >= 1; --l) {
    down_level(c, l, OP_C, c->dU[l].z(), Hc, Ho, M);
    std::swap(Hc, Ho);
  }
  // grad = k^2 Re sum_dir conj(u0) (H^H g).  Many directions: summed over the
  // directions first, Q^T = g u0^H per leaf (ne x mi), then
  // grad_n = k^2 Re sum_e conj(H_en) Q^T_en.  Fewer than ne directions:
  // W = H^H g (mi x M per leaf, H read once), then the sum over directions.
  if (M < g.ne) {
    CK(zgemm(st, OP_C, OP_N, g.mi, M, g.ne, ONE, c->dH.z(), g.ne, (ll)g.ne * g.mi, Hc, g.ne, (ll)g.ne * M, ZERO,
             c->sB.z(), g.mi, (ll)g.mi * M, nl));
    CK(grad_rows(st, c->du0.z(), c->sB.z(), c->dPk.d() + P, g.mi, M, nl, g.nleaf, grad));
  } else {
    CK(zgemm(st, OP_N, OP_C, g.ne, g.mi, M, ONE, Hc, g.ne, (ll)g.ne * M, c->du0.z(), g.mi, (ll)g.mi * M, ZERO,
             c->sB.z(), g.ne, (ll)g.ne * g.mi, nl));
    CK(grad_leaf(st, c->dH.z(), c->sB.z(), c->dPk.d() + P, g.ne, g.mi, nl, g.nleaf, grad));
  }
  mark(c, 4, 1);
  profile_set_phase(PH_OTHER);
}

void sine_setup(hps_ctx* c, int S) {
  require(c->P == 1, HPS_EINVAL, "the sine model takes a single-problem context");
  if (S == c->sine_S) return;
  const Geometry& g = c->g;
  const int m1 = g.p - 2, nX = g.L * m1;
  const double PI = 3.14159265358979323846;
  const double Lx = g.h * g.L;
  std::vector<cplx> Sx((size_t)nX * S), Sy((size_t)nX * S);
  for (int i = 0; i < nX; ++i) {
    const int leaf = i / m1, a = i % m1 + 1;
    const double u = (leaf + 0.5 * (1.0 + g.t[a])) / g.L;  // (x - x0) / Lx
    for (int m = 1; m <= S; ++m) {
      const double v = std::sin(m * PI * u);
      Sx[i + (size_t)(m - 1) * nX] = v;
      Sy[i + (size_t)(m - 1) * nX] = v;
    }
  }
  (void)Lx;
  std::vector<int> node(g.nleaf * (size_t)g.mi);
  size_t o = 0;
  for (int z = 0; z < g.nleaf; ++z) {
    int i = 0, j = 0;
    for (int b = 0; (z >> (2 * b)) != 0; ++b) {
      i |= ((z >> (2 * b)) & 1) << b;
      j |= ((z >> (2 * b + 1)) & 1) << b;
    }
    for (int b = 1; b <= m1; ++b)
      for (int a = 1; a <= m1; ++a) node[o++] = (i * m1 + a - 1) + (j * m1 + b - 1) * nX;
  }
  upload(c->dSx, Sx.data(), Sx.size() * sizeof(cplx), c->st);
  upload(c->dSy, Sy.data(), Sy.size() * sizeof(cplx), c->st);
  upload(c->dNodeGrid, node.data(), node.size() * sizeof(int), c->st);
  c->sS1.ensure(zb((size_t)nX * nX));
  c->sS2.ensure(zb((size_t)nX * S));
  c->sS3.ensure(zb((size_t)S * S + nX * (size_t)nX));
  c->sine_S = S;
}

void sine_eval(hps_ctx* c, int S, const double* coef, double* q) {
  require(S >= 1 && S <= 4096 && coef && q, HPS_EINVAL, "bad sine-model arguments");
  sine_setup(c, S);
  const Geometry& g = c->g;
  const int nX = g.L * (g.p - 2);
  hipStream_t st = c->st;
  double2* Cc = c->sS3.z();
  CK(real_to_complex(st, coef, (ll)S * S, Cc));
  // T1 = Sy Cc (nX x S);  Q = Sx T1^T (nX x nX)
  CK(zgemm(st, OP_N, OP_N, nX, S, S, ONE, c->dSy.z(), nX, 0, Cc, S, 0, ZERO, c->sS2.z(), nX, 0, 1));
  CK(zgemm(st, OP_N, OP_T, nX, nX, S, ONE, c->dSx.z(), nX, 0, c->sS2.z(), nX, 0, ZERO, c->sS1.z(), nX,
           0, 1));
  // gather grid values into node order, keep the real part
  const ll npde = (ll)g.nleaf * g.mi;
  double2* tmp = c->sS3.z() + (ll)S * S;
  CK(gather2d(st, (int)npde, 1, c->sS1.z(), npde, 0, c->dNodeGrid.i(), nullptr, tmp, npde, 0, 1.0, 1));
  CK(complex_real_part(st, tmp, npde, q));
}

void sine_adjoint(hps_ctx* c, int S, const double* gv, double* coef) {
  require(S >= 1 && S <= 4096 && gv && coef, HPS_EINVAL, "bad sine-model arguments");
  sine_setup(c, S);
  const Geometry& g = c->g;
  const int nX = g.L * (g.p - 2);
  hipStream_t st = c->st;
  const ll npde = (ll)g.nleaf * g.mi;
  double2* tmp = c->sS3.z() + (ll)S * S;
  CK(real_to_complex(st, gv, npde, tmp));
  // G (nX x nX grid) from node values
  CK(scatter_rows(st, (int)npde, 1, tmp, npde, 0, c->dNodeGrid.i(), c->sS1.z(), (ll)nX * nX, 0, 1));
  // T3 = G^T Sx (nX x S);  Out = Sy^T T3 (S x S)
  CK(zgemm(st, OP_T, OP_N, nX, S, nX, ONE, c->sS1.z(), nX, 0, c->dSx.z(), nX, 0, ZERO, c->sS2.z(), nX,
           0, 1));
  CK(zgemm(st, OP_T, OP_N, S, S, nX, ONE, c->dSy.z(), nX, 0, c->sS2.z(), nX, 0, ZERO, c->sS3.z(), S, 0,
           1));
  CK(complex_real_part(st, c->sS3.z(), (ll)S * S, coef));
}

// One Gauss-Newton step on the sine model (Section 3.3, eq. normaleq, with
// conjugate gradients on the normal equations in place of LSQR).
struct GnResult {
  int iters;
  double cg_rel_res;
  double misfit;
};

GnResult gn_step(hps_ctx* c, double k, int M, const double* ang, int nt, const double* th, double R,
                 int S, int band, const double* coef, const double* data, int max_iter, double tol,
                 double* coef_out) {
  require(c->o.keep_derivs != 0, HPS_ESTATE, "context created without keep_derivs");
  require(c->P == 1, HPS_EINVAL, "the Gauss-Newton step takes a single-problem context");
  require(S >= 1 && band >= 0 && coef && data && coef_out && max_iter >= 0 && tol >= 0.0, HPS_EINVAL,
          "bad Gauss-Newton arguments");
  const ll npde = (ll)c->g.nleaf * c->g.mi, ns = (ll)S * S, nd = (ll)M * nt;
  hipStream_t st = c->st;
  c->cg_graph_iters = 0;
  // work vectors: q | g | x r p Ap | partial(256) | scalars(4) | CG scalars | CG flags
  c->sGn.ensure(sizeof(double) * (2 * npde + 4 * ns + 256 + 4 + CG_NS) + sizeof(int) * CG_NF);
  c->sGnZ.ensure(zb(2 * nd));
  double* q = c->sGn.d();
  double* gv = q + npde;
  double* x = gv + npde;
  double* r = x + ns;
  double* pv = r + ns;
  double* Ap = pv + ns;
  double* partial = Ap + ns;
  double* sc = partial + 256;
  double* cs = sc + 4;
  int* cf = (int*)(cs + CG_NS);
  double2* res = c->sGnZ.z();
  double2* jv = res + nd;
  auto dotv = [&](const double* a, const double* b) {
    double h = 0.0;
    CK(dot(st, a, b, ns, partial, sc));
    CK(hipMemcpyAsync(&h, sc, sizeof(double), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    return h;
  };
  sine_eval(c, S, coef, q);
  factor(c, q, &k);
  solve(c, M, ang);
  far_field(c, nt, th, R, (double*)jv);
  CK(zsub(st, (const double2*)data, jv, res, nd));
  // misfit ||data - F[q]||
  double misfit = 0.0;
  {
    CK(dot(st, (const double*)res, (const double*)res, 2 * nd, partial, sc));
    CK(hipMemcpyAsync(&misfit, sc, sizeof(double), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    misfit = std::sqrt(misfit);
  }
  // b = E^T Re(J^H res)
  vjp(c, (const double*)res, gv);
  sine_adjoint(c, S, gv, r);
  CK(band_mask(st, r, S, band));  // unknowns: the modes in the band only
  CK(hipMemsetAsync(x, 0, sizeof(double) * ns, st));
  CK(hipMemcpyAsync(pv, r, sizeof(double) * ns, hipMemcpyDeviceToDevice, st));
  const double bnorm = std::sqrt(dotv(r, r));
  int it = 0;
  double rel = bnorm > 0.0 ? 1.0 : 0.0;
  if (it < max_iter && rel > tol) {
    // CG with its scalars on the device: rr, then per iteration
    // Ap = E^T Re(J^H J E p), alpha, x += alpha p, r -= alpha Ap, rr_new,
    // beta, p = r + beta p (cg_alpha / cg_beta stop the updates once done).
    // The iterations after the first replay one captured iteration.  The
    // legacy default stream cannot be captured: the loop then runs on the
    // context's second stream (forked here, joined when the block ends), with
    // the library's calls issued on it meanwhile, from the first iteration on
    // (which also sets up that stream's GEMM workspaces and tile choices).
    struct StreamSwap {
      hps_ctx* c;
      hipStream_t saved;
      ~StreamSwap() {
        if (c->st != saved) {
          (void)hipEventRecord(c->join, c->st);
          c->st = saved;
          (void)hipStreamWaitEvent(saved, c->join, 0);
        }
      }
    } swap{c, st};
    const bool try_graph = !profile_active();
    if (try_graph && st == nullptr) {
      ensure_side(c);
      CK(hipEventRecord(c->fork, st));
      CK(hipStreamWaitEvent(c->side, c->fork, 0));
      c->st = c->side;
    }
    CK(dot(c->st, r, r, ns, partial, cs + CG_RR));
    CK(cg_init(c->st, cs, cf));
    auto iteration = [&]() {
      sine_eval(c, S, pv, q);
      jvp(c, q, (double*)jv);
      vjp(c, (const double*)jv, gv);
      sine_adjoint(c, S, gv, Ap);
      hipStream_t s = c->st;  // the context's stream, or the second stream for replays
      CK(band_mask(s, Ap, S, band));
      CK(dot(s, pv, Ap, ns, partial, cs + CG_PAP));
      CK(cg_alpha(s, cs, cf));
      CK(axpby_dev(s, cs + CG_ALPHA, 1.0, pv, nullptr, x, ns));
      CK(axpby_dev(s, cs + CG_ALPHA, -1.0, Ap, nullptr, r, ns));
      CK(dot(s, r, r, ns, partial, cs + CG_RRNEW));
      CK(cg_beta(s, cs, cf, bnorm, tol));
      CK(axpby_dev(s, nullptr, 1.0, r, cs + CG_BETA, pv, ns));
    };
    int fl[CG_NF] = {0, 0, 0};
    auto read_state = [&]() {
      CK(hipMemcpyAsync(fl, cf, sizeof(fl), hipMemcpyDeviceToHost, c->st));
      CK(hipMemcpyAsync(&rel, cs + CG_REL, sizeof(double), hipMemcpyDeviceToHost, c->st));
      CK(hipStreamSynchronize(c->st));
      it = fl[CG_ITERS];
    };
    // the first iteration runs directly; the state is read back every few
    // replays (an iteration after the stop changes nothing)
    iteration();
    read_state();
    struct Exec {
      hipGraphExec_t e = nullptr;
      ~Exec() {
        if (e) (void)hipGraphExecDestroy(e);
      }
    } exec;
    const int it_direct = it;
    if (!fl[CG_DONE] && it < max_iter && try_graph) {
      hipGraph_t graph = nullptr;
      c->capturing = true;
      hipError_t e = hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal);
      if (e == hipSuccess) {
        try {
          iteration();
        } catch (...) {
          e = hipErrorUnknown;
        }
        const hipError_t e2 = hipStreamEndCapture(c->st, &graph);
        if (e == hipSuccess) e = e2;
      }
      c->capturing = false;
      if (e == hipSuccess && graph) e = hipGraphInstantiate(&exec.e, graph, nullptr, nullptr, 0);
      if (graph) (void)hipGraphDestroy(graph);
      if (e != hipSuccess) {
        // capture not possible: the remaining iterations run directly (the
        // captured launches never executed); leave the stream out of capture
        // mode and clear the error the attempt left behind
        if (exec.e) (void)hipGraphExecDestroy(exec.e);
        exec.e = nullptr;
        hipStreamCaptureStatus cs_status = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(c->st, &cs_status) == hipSuccess && cs_status != hipStreamCaptureStatusNone) {
          hipGraph_t g2 = nullptr;
          (void)hipStreamEndCapture(c->st, &g2);
          if (g2) (void)hipGraphDestroy(g2);
        }
        (void)hipGetLastError();
      }
    }
    while (!fl[CG_DONE] && it < max_iter) {
      const int chunk = std::min(4, max_iter - it);
      for (int j = 0; j < chunk; ++j) {
        if (exec.e)
          CK(hipGraphLaunch(exec.e, c->st));
        else
          iteration();
      }
      read_state();
    }
    if (exec.e) c->cg_graph_iters = it - it_direct;
  }
  CK(hipMemcpyAsync(coef_out, coef, sizeof(double) * ns, hipMemcpyDeviceToDevice, st));
  CK(axpby(st, 1.0, x, 1.0, coef_out, ns));
  CK(hipStreamSynchronize(st));
  return GnResult{it, rel, misfit};
}

int64_t device_bytes(const hps_ctx* c) {
  int64_t s = 0;
  const DBuf* bufs[] = {&c->dLeaf, &c->dBop, &c->dC1, &c->dbnode, &c->dPk, &c->dY, &c->dH,
                        &c->dRroot, &c->dZinv, &c->dRrootH, &c->dZinvH, &c->sA, &c->sInv, &c->sZws, &c->sR0, &c->sR1,
                        &c->sBlk, &c->sW, &c->sWinv, &c->sQ, &c->sVin, &c->sV, &c->sTmp, &c->sInfo,
                        &c->sBlk2, &c->sWinv2, &c->sVin2, &c->sTmp2,
                        &c->d_dirs, &c->dG, &c->dRhs, &c->dF0, &c->dF1, &c->dF3, &c->du0, &c->dST,
                        &c->dg, &c->dPhi, &c->sB, &c->sST2, &c->dSx, &c->dSy,
                        &c->dNodeGrid, &c->sS1, &c->sS2, &c->sS3, &c->sGn, &c->sGnZ};
  for (const DBuf* b : bufs) s += (int64_t)b->bytes;
  for (const auto& b : c->didx) s += (int64_t)b.bytes;
  for (const auto& b : c->dD) s += (int64_t)b.bytes;
  for (const auto& b : c->dU) s += (int64_t)b.bytes;
  const DBuf* mb[] = {&c->dRleaf, &c->sE, &c->mF0, &c->mF1, &c->mF3, &c->mTmp, &c->dFl, &c->dGl, &c->rF0,
                      &c->rF1, &c->rG0, &c->rG1, &c->rT0, &c->rT1, &c->dRb, &c->sNorm};
  for (const DBuf* b : mb) s += (int64_t)b->bytes;
  for (const auto* v : {&c->dD32, &c->dU32, &c->dE32, &c->mH3, &c->dRho})
    for (const auto& b : *v) s += (int64_t)b.bytes;
  return s;
}

}  // namespace

extern "C" {

void hps_default_opts(hps_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->x0 = -1.0;
  o->x1 = 1.0;
  o->y0 = -1.0;
  o->y1 = 1.0;
  o->nleaf = 4;
  o->p = 16;
  o->eta_scale = 1.0;
  o->keep_derivs = 1;
  o->precision = HPS_FP64;
  o->host_threads = 0;
  o->stream = nullptr;
  o->nprob = 1;
  o->max_refine = 8;
  o->refine_tol = 1e-10;
  o->fallback_fp64 = 1;
  o->exterior = HPS_EXT_GREEN;
  o->streams = 2;
}

hps_status hps_create(const hps_opts* opts, hps_ctx** out) {
  if (!opts || !out) return HPS_EINVAL;
  *out = nullptr;
  const hps_opts& o = *opts;
  const double lx = o.x1 - o.x0, ly = o.y1 - o.y0;
  if (!(lx > 0.0) || std::fabs(lx - ly) > 1e-14 * lx) return HPS_EINVAL;
  if (o.nleaf < 1 || o.nleaf > 256 || (o.nleaf & (o.nleaf - 1))) return HPS_EINVAL;
  if (o.p < 4 || o.p > 20) return HPS_EINVAL;
  if (o.precision != HPS_FP64 && o.precision != HPS_MIXED) return HPS_EINVAL;
  if (o.exterior != HPS_EXT_GREEN && o.exterior != HPS_EXT_BURTON_MILLER) return HPS_EINVAL;
  if (o.streams != 1 && o.streams != 2) return HPS_EINVAL;
  if (o.nprob < 1 || o.nprob > 4096) return HPS_EINVAL;
  if (o.precision == HPS_MIXED && (o.max_refine < 0 || o.max_refine > 100 || !(o.refine_tol > 0.0)))
    return HPS_EINVAL;
  hps_ctx* c = nullptr;
  try {
    c = new hps_ctx();
  } catch (...) {
    return HPS_ENOMEM;
  }
  hps_status s = guard(nullptr, [&] {
    c->o = o;
    c->P = o.nprob;
    c->mixed = (o.precision == HPS_MIXED);
    c->st = (hipStream_t)o.stream;
    CK(hipGetDevice(&c->device));
    unsigned hw = std::thread::hardware_concurrency();
    c->nthreads = o.host_threads > 0 ? o.host_threads : (int)std::min(16u, std::max(1u, hw));
    c->g.build(o.x0, o.x1, o.y0, o.nleaf, o.p);
    c->n = c->g.mi + c->g.ne;
    c->nb = (int)c->g.root.size();
    c->didx.resize(4 * (size_t)(c->g.nlev + 1));
    c->dMap3.resize(c->g.nlev + 1);
    for (int l = 1; l <= c->g.nlev; ++l) {
      const LevelPattern& P = c->g.lev[l];
      const std::vector<int>* v[4] = {&P.pos1a, &P.pos3a, &P.pos2b, &P.pos3b};
      for (int a = 0; a < 4; ++a)
        upload(c->didx[4 * l + a], v[a]->data(), v[a]->size() * sizeof(int), c->st);
      std::vector<int> m3(P.pos3a);
      m3.insert(m3.end(), P.pos3b.begin(), P.pos3b.end());
      upload(c->dMap3[l], m3.data(), m3.size() * sizeof(int), c->st);
    }
    // leaf-edge slot (leaf offset inside the box * ne + edge position) of
    // every boundary position of a box, level by level: a box lists the
    // exterior nodes of its alpha child, then those of its beta child
    {
      const Geometry& g = c->g;
      std::vector<int> prev(g.ne), cur;
      for (int e = 0; e < g.ne; ++e) prev[e] = e;
      c->dSlot.resize(g.nlev + 1);
      for (int l = 1; l <= g.nlev; ++l) {
        const LevelPattern& P = g.lev[l];
        const int half = (1 << (l - 1)) * g.ne;  // slots of the alpha child
        std::vector<int> sab(2 * (size_t)P.s);
        for (int j = 0; j < P.s; ++j) {
          sab[j] = prev[P.pos3a[j]];
          sab[P.s + j] = prev[P.pos3b[j]] + half;
        }
        upload(c->dSlot[l], sab.data(), sab.size() * sizeof(int), c->st);
        cur.assign(P.np, 0);
        for (int i = 0; i < P.m; ++i) {
          cur[i] = prev[P.pos1a[i]];
          cur[P.m + i] = prev[P.pos2b[i]] + half;
        }
        prev.swap(cur);
      }
      if ((int)prev.size() != c->nb) throw HpsError{HPS_EINVAL, "root boundary size mismatch"};
      upload(c->dSlot[0], prev.data(), prev.size() * sizeof(int), c->st);
    }
    for (auto& e : c->ev) CK(hipEventCreate(&e));
  });
  if (s != HPS_OK) {
    hps_destroy(c);
    return s;
  }
  *out = c;
  return HPS_OK;
}

void hps_destroy(hps_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->st);
  if (c->side) {
    (void)hipStreamSynchronize(c->side);
    (void)hipStreamDestroy(c->side);
  }
  if (c->fork) (void)hipEventDestroy(c->fork);
  if (c->join) (void)hipEventDestroy(c->join);
  if (c->lev_ready) (void)hipEventDestroy(c->lev_ready);
  if (c->q_ready) (void)hipEventDestroy(c->q_ready);
  if (c->q_done) (void)hipEventDestroy(c->q_done);
  for (auto& e : c->lev_done)
    if (e) (void)hipEventDestroy(e);
  for (auto& e : c->ev)
    if (e) (void)hipEventDestroy(e);
  delete c;
}

const char* hps_last_error(const hps_ctx* c) { return c ? c->err.c_str() : "NULL context"; }

int64_t hps_num_nodes(const hps_ctx* c) { return c ? (int64_t)c->g.nleaf * c->g.mi : 0; }

int64_t hps_num_boundary_nodes(const hps_ctx* c) { return c ? (int64_t)c->nb : 0; }

hps_status hps_node_coords(const hps_ctx* c, double* xy) {
  if (!c || !xy) return HPS_EINVAL;
  c->g.pde_coords(xy);
  return HPS_OK;
}

hps_status hps_set_wavenumber(hps_ctx* c, double k) {
  if (!c) return HPS_EINVAL;
  return guard(c, [&] { set_wavenumber(c, k); });
}

hps_status hps_set_streams(hps_ctx* c, int streams) {
  if (!c || (streams != 1 && streams != 2)) return HPS_EINVAL;
  c->o.streams = streams;
  return HPS_OK;
}

hps_status hps_set_wavenumbers(hps_ctx* c, const double* k) {
  if (!c || !k) return HPS_EINVAL;
  return guard(c, [&] { set_wavenumbers(c, k); });
}

hps_status hps_factor(hps_ctx* c, const double* q, double k) {
  if (!c) return HPS_EINVAL;
  return guard(c, [&] {
    std::vector<double> kv(c->P, k);
    factor(c, q, kv.data());
  });
}

hps_status hps_factor_batch(hps_ctx* c, const double* q, const double* k) {
  if (!c || !k) return HPS_EINVAL;
  return guard(c, [&] { factor(c, q, k); });
}

hps_status hps_solve(hps_ctx* c, int ndir, const double* ang) {
  if (!c) return HPS_EINVAL;
  return guard(c, [&] {
    require(ndir >= 1 && ndir <= 65535 && ang != nullptr, HPS_EINVAL, "bad direction list");
    std::vector<double> all((size_t)ndir * c->P);
    for (int b = 0; b < c->P; ++b) std::memcpy(all.data() + (size_t)b * ndir, ang, sizeof(double) * ndir);
    solve(c, ndir, all.data());
  });
}

hps_status hps_solve_batch(hps_ctx* c, int ndir, const double* ang) {
  if (!c) return HPS_EINVAL;
  return guard(c, [&] { solve(c, ndir, ang); });
}

hps_status hps_far_field(hps_ctx* c, int nt, const double* th, double R, double* out) {
  if (!c) return HPS_EINVAL;
  return guard(c, [&] { far_field(c, nt, th, R, out); });
}

hps_status hps_total_field(hps_ctx* c, double* u) {
  if (!c) return HPS_EINVAL;
  return guard(c, [&] {
    require(c->solved, HPS_ESTATE, "hps_total_field before hps_solve");
    require(u != nullptr, HPS_EINVAL, "NULL output");
    const ll per = (ll)c->g.nleaf * c->g.mi * c->ndir;
    for (int b = 0; b < c->P; ++b)
      CK(export_field(c->st, c->du0.z() + per * b, c->g.mi, c->ndir, c->g.nleaf, (double2*)u + per * b));
  });
}

hps_status hps_jvp(hps_ctx* c, const double* dq, double* out) {
  if (!c) return HPS_EINVAL;
  return guard(c, [&] { jvp(c, dq, out); });
}

hps_status hps_vjp(hps_ctx* c, const double* r, double* grad) {
  if (!c) return HPS_EINVAL;
  return guard(c, [&] { vjp(c, r, grad); });
}

hps_status hps_sine_eval(hps_ctx* c, int S, const double* coef, double* q) {
  if (!c) return HPS_EINVAL;
  return guard(c, [&] { sine_eval(c, S, coef, q); });
}

hps_status hps_sine_adjoint(hps_ctx* c, int S, const double* g, double* coef) {
  if (!c) return HPS_EINVAL;
  return guard(c, [&] { sine_adjoint(c, S, g, coef); });
}

hps_status hps_gn_step(hps_ctx* c, double k, int ndir, const double* dir_angle_host, int ntheta,
                       const double* theta_host, double R, int S, int band, const double* coef,
                       const double* data, int max_iter, double tol, double* coef_out,
                       int* iters_host, double* cg_rel_res_host, double* misfit_host) {
  if (!c) return HPS_EINVAL;
  return guard(c, [&] {
    const GnResult g = gn_step(c, k, ndir, dir_angle_host, ntheta, theta_host, R, S, band, coef, data,
                               max_iter, tol, coef_out);
    if (iters_host) *iters_host = g.iters;
    if (cg_rel_res_host) *cg_rel_res_host = g.cg_rel_res;
    if (misfit_host) *misfit_host = g.misfit;
  });
}

hps_status hps_get_stats(hps_ctx* c, hps_stats* out) {
  if (!c || !out) return HPS_EINVAL;
  return guard(c, [&] {
    CK(hipStreamSynchronize(c->st));
    std::memset(out, 0, sizeof(*out));
    out->t_wavenumber_ms = c->t_wave;
    out->t_factor_ms = elapsed_ms(c, 0);
    out->t_solve_ms = elapsed_ms(c, 1);
    out->t_far_field_ms = elapsed_ms(c, 2);
    out->t_jvp_ms = elapsed_ms(c, 3);
    out->t_vjp_ms = elapsed_ms(c, 4);
    out->t_leaf_ms = elapsed_ms(c, 5);
    out->t_merge_ms = elapsed_ms(c, 6);
    out->t_top_ms = elapsed_ms(c, 7);
    out->device_bytes = device_bytes(c);
    out->ndir = c->ndir;
    out->singular = c->singular;
    out->nonfinite = c->nonfinite;
    out->refine_iters = c->refine_iters;
    out->refine_residual = c->refine_res;
    out->refine_fallback = c->refine_fallback;
    out->cg_graph_iters = c->cg_graph_iters;
  });
}

hps_status hps_boundary_operators(const hps_opts* opts, double k, double* xy_host, double* S_host,
                                  double* K_host) {
  if (!opts || !(k > 0.0) || !S_host || !K_host) return HPS_EINVAL;
  try {
    Geometry g;
    g.build(opts->x0, opts->x1, opts->y0, opts->nleaf, opts->p);
    const int nb = (int)g.root.size();
    std::vector<double> tx(nb), ty(nb);
    for (int i = 0; i < nb; ++i) {
      tx[i] = g.root[i].x;
      ty[i] = g.root[i].y;
      if (xy_host) {
        xy_host[2 * i] = tx[i];
        xy_host[2 * i + 1] = ty[i];
      }
    }
    std::vector<cplx> S, K;
    unsigned hw = std::thread::hardware_concurrency();
    const int nth = opts->host_threads > 0 ? opts->host_threads : (int)std::min(16u, std::max(1u, hw));
    layer_moments(g, k, tx, ty, S, K, nth);
    std::memcpy(S_host, S.data(), S.size() * sizeof(cplx));
    std::memcpy(K_host, K.data(), K.size() * sizeof(cplx));
  } catch (...) {
    return HPS_EINVAL;
  }
  return HPS_OK;
}

hps_status hps_combined_field_operators(const hps_opts* opts, double k, double* Kp_host, double* T_host) {
  if (!opts || !(k > 0.0) || !std::isfinite(k) || !Kp_host || !T_host) return HPS_EINVAL;
  try {
    Geometry g;
    g.build(opts->x0, opts->x1, opts->y0, opts->nleaf, opts->p);
    const int nb = (int)g.root.size();
    std::vector<double> tx(nb), ty(nb);
    for (int i = 0; i < nb; ++i) {
      tx[i] = g.root[i].x;
      ty[i] = g.root[i].y;
    }
    unsigned hw = std::thread::hardware_concurrency();
    const int nth = opts->host_threads > 0 ? opts->host_threads : (int)std::min(16u, std::max(1u, hw));
    std::vector<cplx> S, K, Kp, T1;
    layer_moments(g, k, tx, ty, S, K, nth);
    combined_field_moments(g, k, Kp, T1, nth);
    for (int i = 0; i < nb; ++i)
      for (int j = 0; j < nb; ++j) {
        const size_t ij = (size_t)i * nb + j;
        T1[ij] += k * k * (g.root[i].nx * g.root[j].nx + g.root[i].ny * g.root[j].ny) * S[ij];
      }
    std::memcpy(Kp_host, Kp.data(), Kp.size() * sizeof(cplx));
    std::memcpy(T_host, T1.data(), T1.size() * sizeof(cplx));
  } catch (...) {
    return HPS_EINVAL;
  }
  return HPS_OK;
}

hps_status hps_zgemm(void* stream, int opA, int opB, int M, int N, int K, const double* alpha,
                     const double* A, int64_t lda, int64_t sA, const double* B, int64_t ldb,
                     int64_t sB, const double* beta, double* C, int64_t ldc, int64_t sC,
                     int batch) {
  if (!alpha || !beta || M < 0 || N < 0 || K < 0 || batch < 0) return HPS_EINVAL;
  if (opA < 0 || opA > 2 || opB < 0 || opB > 2) return HPS_EINVAL;
  if (M == 0 || N == 0 || batch == 0) return HPS_OK;
  if (!A || !B || !C) return HPS_EINVAL;
  const ll rowsA = opA == OP_N ? M : K, rowsB = opB == OP_N ? K : N;
  if (lda < std::max<ll>(1, rowsA) || ldb < std::max<ll>(1, rowsB) || ldc < std::max(1, M))
    return HPS_EINVAL;
  const hipError_t e = zgemm((hipStream_t)stream, opA, opB, M, N, K, make_double2(alpha[0], alpha[1]),
                             (const double2*)A, lda, sA, (const double2*)B, ldb, sB,
                             make_double2(beta[0], beta[1]), (double2*)C, ldc, sC, batch);
  return e == hipSuccess ? HPS_OK : HPS_EDEVICE;
}

hps_status hps_gemm_tuning(int mode, int force) {
  if (mode < 0 || mode > 1 || force < -1 || force >= gemm_variant_count()) return HPS_EINVAL;
  gemm_set_tuning(mode, force);
  return HPS_OK;
}

hps_status hps_zinv_blocking(int mode) {
  if (mode < -1 || mode > 1) return HPS_EINVAL;
  zinv_set_blocking(mode);
  return HPS_OK;
}

hps_status hps_zinv_pivoting(int mode, double tol) {
  if (mode < -1 || mode > 1 || !(tol >= 0.0 || tol == -1.0)) return HPS_EINVAL;
  zinv_set_pivoting(mode, tol);
  return HPS_OK;
}

hps_status hps_zinv_pivoting_info(int64_t* calls, int64_t* fallbacks, double* max_err) {
  long c = 0, f = 0;
  double e = 0.0;
  zinv_pivoting_info(&c, &f, &e);
  if (calls) *calls = c;
  if (fallbacks) *fallbacks = f;
  if (max_err) *max_err = e;
  return HPS_OK;
}

hps_status hps_gemm_tuning_info(int* variants, int* shapes_tuned, double* seconds) {
  if (variants) *variants = gemm_variant_count();
  gemm_tuning_info(shapes_tuned, seconds);
  return HPS_OK;
}

hps_status hps_zinv(void* stream, int n, int batch, double* A, double* inv) {
  if (n < 0 || batch < 0 || batch > 65535) return HPS_EINVAL;
  if (n == 0 || batch == 0) return HPS_OK;
  if (!A || !inv) return HPS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  void* ws = nullptr;
  int* info = nullptr;
  if (hipMalloc(&ws, zinv_workspace(n, batch)) != hipSuccess) return HPS_ENOMEM;
  if (hipMalloc((void**)&info, sizeof(int) * batch) != hipSuccess) {
    (void)hipFree(ws);
    return HPS_ENOMEM;
  }
  hps_status s = HPS_OK;
  std::vector<int> h(batch, 0);
  if (hipMemsetAsync(info, 0, sizeof(int) * batch, st) != hipSuccess ||
      zinv(st, n, (double2*)A, n, (ll)n * n, (double2*)inv, n, (ll)n * n, batch, ws, info) !=
          hipSuccess ||
      hipMemcpyAsync(h.data(), info, sizeof(int) * batch, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    s = HPS_EDEVICE;
  } else {
    for (int v : h)
      if (v) s = HPS_ESINGULAR;
  }
  (void)hipFree(ws);
  (void)hipFree(info);
  return s;
}

hps_status hps_zinv_noalloc(void* stream, int n, int batch, double* A, double* inv, int* status_dev) {
  if (n < 0 || batch < 0 || batch > 65535) return HPS_EINVAL;
  if (n == 0 || batch == 0) return HPS_OK;
  if (!A || !inv) return HPS_EINVAL;
  if (n > 512 || zinv_noalloc_bytes(n, batch) > zinv_noalloc_capacity()) return HPS_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  if (zinv_noalloc(st, n, (double2*)A, (double2*)inv, batch, status_dev) != hipSuccess) return HPS_EDEVICE;
  if (status_dev) return HPS_OK;
  int* slot = nullptr;
  int h = 0;
  if (zinv_noalloc_status_slot(&slot) != hipSuccess ||
      hipMemcpyAsync(&h, slot, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return HPS_EDEVICE;
  return h ? HPS_ESINGULAR : HPS_OK;
}

}  // extern "C"
