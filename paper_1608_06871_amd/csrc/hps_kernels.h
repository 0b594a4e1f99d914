// Launchers for the pointwise / data-movement kernels (hps_kernels.hip).
#pragma once
#include "common.h"

namespace hps {

// Several problems share one leaf grid: leaf z belongs to problem z / lpp.
// Per-problem scalars (k, k^2, eta) are device arrays indexed by problem.

// out[z] = A0[problem] with -k^2 q[z][r] added to the diagonal of the first
// mi rows.
hipError_t leaf_assemble(hipStream_t st, const double2* A0, ll sA0, const double* q, const double* k2v,
                         int n, int mi, double2* out, ll nleaf, ll lpp);
// out(i, j) = sc * in(ridx[i], cidx[j]) (null index array = identity).
hipError_t gather2d(hipStream_t st, int M, int N, const double2* in, ll ldi, ll si,
                    const int* ridx, const int* cidx, double2* out, ll ldo, ll so, double sc,
                    int batch);
// out_b(i, j) = in_{b / idiv}(r, c) with per-matrix index maps
// r = ridx ? ridx[b sri + i] : i and c = cidx ? cidx[b sci + j] : j; an
// index outside [0, rlim) / [0, clim) gives 0 (maps of a singular matrix).
hipError_t gather_perm(hipStream_t st, int M, int N, const double2* in, ll ldi, ll si, int idiv,
                       const int* ridx, ll sri, int rlim, const int* cidx, ll sci, int clim, double2* out, ll ldo,
                       ll so, int batch);
// out(ridx[i], j) = in(i, j).
hipError_t scatter_rows(hipStream_t st, int M, int N, const double2* in, ll ldi, ll si,
                        const int* ridx, double2* out, ll ldo, ll so, int batch);
// FP32 versions (mixed-precision sweeps).
hipError_t gather2d(hipStream_t st, int M, int N, const float2* in, ll ldi, ll si, const int* ridx,
                    const int* cidx, float2* out, ll ldo, ll so, float sc, int batch);
hipError_t scatter_rows(hipStream_t st, int M, int N, const float2* in, ll ldi, ll si, const int* ridx,
                        float2* out, ll ldo, ll so, int batch);
// y = (float) x;  y += (double) x;  y = (double) x;  y += (float) x;  z = x + y
hipError_t to_f32(hipStream_t st, const double2* x, ll n, float2* y);
hipError_t add_f32(hipStream_t st, const float2* x, ll n, double2* y);
hipError_t to_f64(hipStream_t st, const float2* x, ll n, double2* y);
hipError_t add_to_f32(hipStream_t st, const double2* x, ll n, float2* y);
hipError_t zadd(hipStream_t st, const double2* x, const double2* y, double2* z, ll n);
// out_b = in_b^H for batch square n x n matrices (column-major).
hipError_t conj_transpose(hipStream_t st, int n, const double2* in, ll ldi, ll si, double2* out, ll ldo, ll so,
                          int batch);
// Interface residual of one level from leaf-edge data F, G ([leaf][ne][M]):
// sab = [alpha slots (s); beta slots (s)] relative to a merge's first leaf,
// lpm leaves per merge, cnt merges; rho = [F(beta) + G(alpha); F(alpha) +
// G(beta)] per merge, leading dimension 2 s.
hipError_t skel_residual(hipStream_t st, int s, int M, int ne, int lpm, const int* sab, const double2* F,
                         const double2* G, double2* rho, int cnt);
// out[b] (n x M, leading dimension n) = X at the n slots of box b (lpb leaves
// per box).
hipError_t skel_gather(hipStream_t st, int n, int M, int ne, int lpb, const int* slot, const double2* X,
                       double2* out, int nbox);
// One batched block move: out_b(i, j) = sc * in_b(ridx[i], cidx[j]) (null
// index arrays = identity), or, when set != 0, out_b(i, j) = diag on the
// diagonal and off elsewhere (in unused).  Batch strides si, so.
// Exact unsigned division by a fixed d >= 1 for numerators below 2^31
// (Granlund and Montgomery, PLDI 1994): q = umulhi(n, mul) >> shift with
// mul = ceil(2^(31 + l) / d), l = ceil(log2 d), shift = l - 1; mul = 0 encodes
// d = 1 (q = n).
struct FastDiv {
  unsigned mul;
  int shift;
};
FastDiv make_fastdiv(int d);

struct MoveDesc {
  const double2* in;
  ll ldi, si;
  const int* ridx;
  const int* cidx;
  double2* out;
  ll ldo, so;
  int M, N, set, pad;
  double sc;
  double2 diag, off;
  unsigned fdm;  // division by M (make_fastdiv; set by multi_move_prepare)
  int fds;
};
// Fills the division parameters of host-side descriptors before their copy
// to the device.
void multi_move_prepare(MoveDesc* desc, int ndesc);

// A row move of M rows by N columns over a batch: gather (out row i = in row
// ridx[i]) or scatter (out row ridx[i] = in row i).
struct RowMove {
  const double2* in;
  ll ldi, si;
  const int* ridx;
  double2* out;
  ll ldo, so;
  int M;
  int scatter;
};
// Up to four independent row moves with the same N and batch in one launch
// (passed by value: no device copy of the list, so the launch can be
// captured); the moves must write disjoint elements.
hipError_t row_moves(hipStream_t st, const RowMove* moves, int nmoves, int N, int batch);
// Applies ndesc independent moves (device array `desc`, over `batch` matrices
// each) in one launch; the moves must write disjoint elements.  max_elems:
// the largest M * N * batch among them.
hipError_t multi_move(hipStream_t st, const MoveDesc* desc, int ndesc, ll max_elems, int batch);

// out = off everywhere, diag on the diagonal.
hipError_t set2d(hipStream_t st, int M, int N, double2* out, ll ldo, ll so, double2 diag,
                 double2 off, int batch);
// ndir (ncol) columns per problem, nprob problems.
hipError_t incident(hipStream_t st, const double4* bnode, int nb, const double2* dirs, int ndir,
                    const double* kv, double2* G, int nprob);
hipError_t boundary_st(hipStream_t st, const double2* f, const double2* g, const double2* G,
                       int nb, int ncol, const double* etav, double2* ST, int nprob);
hipError_t boundary_st_adj(hipStream_t st, const double2* STb, int nb, int ncol, const double* etav,
                           double2* fb, double2* gb, int nprob);
// Hs = H diag(k^2 dq) per leaf (H: ne x mi): the Frechet body load folded into
// the outgoing-impedance maps.
hipError_t scale_leaf_cols(hipStream_t st, const double* dq, const double2* H, const double* k2v, int ne, int mi,
                           ll nleaf, ll lpp, double2* Hs);
// out = k^2 dq u0 per leaf (mi x M, u0's layout): the Frechet body load for
// the product H (k^2 dq u0) when few directions make that cheaper.
hipError_t scale_leaf_rows(hipStream_t st, const double* dq, const double2* u0, const double* k2v, int mi, int M,
                           ll nleaf, ll lpp, double2* out);
// grad[z mi + n] = k^2 Re sum_m conj(u0[n][m]) W[n][m] per leaf (W = H^H g).
hipError_t grad_rows(hipStream_t st, const double2* u0, const double2* W, const double* k2v, int mi, int M,
                     ll nleaf, ll lpp, double* grad);
// grad[z mi + n] = k^2 Re sum_e conj(H[e][n]) QT[e][n] per leaf.
hipError_t grad_leaf(hipStream_t st, const double2* H, const double2* QT, const double* k2v, int ne, int mi,
                     ll nleaf, ll lpp, double* grad);
hipError_t export_field(hipStream_t st, const double2* u0, int mi, int ndir, ll nleaf,
                        double2* out);
hipError_t real_to_complex(hipStream_t st, const double* x, ll n, double2* y);
hipError_t complex_real_part(hipStream_t st, const double2* x, ll n, double* y);
// *out = sum x[i] y[i] (deterministic two-stage reduction; partial holds 256 doubles).
hipError_t dot(hipStream_t st, const double* x, const double* y, ll n, double* partial, double* out);
// *flag |= bit when any of x[0 .. n) is NaN or infinite.
hipError_t flag_nonfinite(hipStream_t st, const double* x, ll n, int bit, int* flag);
// x[(m - 1) S + (n - 1)] = 0 for m + n > band (band <= 0: no-op).
hipError_t band_mask(hipStream_t st, double* x, int S, int band);
// y = a x + b y
hipError_t axpby(hipStream_t st, double a, const double* x, double b, double* y, ll n);

// Conjugate-gradient scalars kept on the device (so that an iteration can be
// captured in a graph and replayed without reading them back).  s holds
// doubles [CG_RR, CG_PAP, CG_ALPHA, CG_RRNEW, CG_BETA, CG_REL], f the ints
// [CG_DONE, CG_ACTIVE, CG_ITERS].
enum { CG_RR = 0, CG_PAP, CG_ALPHA, CG_RRNEW, CG_BETA, CG_REL, CG_NS };
enum { CG_DONE = 0, CG_ACTIVE, CG_ITERS, CG_NF };
// rel = 1 and the flags cleared (rr is written by dot).
hipError_t cg_init(hipStream_t st, double* s, int* f);
// alpha = rr / pAp, or 0 with the iteration inactive once done or when
// pAp <= 0 (which also sets done).
hipError_t cg_alpha(hipStream_t st, double* s, int* f);
// For an active iteration: iterations + 1, rel = sqrt(rr_new) / bnorm; done
// when rel <= tol (beta 0), else beta = rr_new / rr and rr = rr_new.
hipError_t cg_beta(hipStream_t st, double* s, int* f, double bnorm, double tol);
// y = (sa * *a) x + (b ? *b : 1) y (a null: 1), the same arithmetic as axpby.
hipError_t axpby_dev(hipStream_t st, const double* a, double sa, const double* x, const double* b, double* y,
                     ll n);
// z = x - y (complex)
hipError_t zsub(hipStream_t st, const double2* x, const double2* y, double2* z, ll n);

}  // namespace hps
