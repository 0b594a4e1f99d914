// Batched complex FP64 matrix inverse by blocked Gauss-Jordan elimination with
// partial (row) pivoting.
//
// For each column panel [c0, c0 + b):
//   1. a panel kernel (one workgroup per matrix) eliminates the b pivot
//      columns in place: pivot search over the rows not yet used, a full-row
//      swap, and the in-place inverse update of the panel columns, which
//      leaves inv(A_PP) in the pivot rows and -A_QP inv(A_PP) in the others.
//      It then emits E = that panel and T = the pivot rows with the panel
//      columns zeroed;
//   2. the other columns are updated by batched complex GEMMs on the matrix
//      cores: A_Q += E_Q T for the non-pivot rows (two row ranges) and
//      A_P = inv(A_PP) T on the non-panel columns of the pivot rows (two
//      column ranges, overwriting).  The pivot rows are never formed as
//      A_P + (inv - I) A_P, which would cancel catastrophically when the
//      pivots are large.
// The row interchanges turn into a column permutation of the result, applied
// out of place at the end.  Panels of matrices up to ~300 rows live in LDS;
// larger ones are updated in global memory.
#include "common.h"

namespace hps {
namespace {

constexpr int NT = 256;
constexpr int BMAX = 32;
constexpr size_t LDS_BUDGET = 150 * 1024;

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double2 crecip(double2 a) {
  const double d = a.x * a.x + a.y * a.y;
  return make_double2(a.x / d, -a.y / d);
}

// Arg-max of (value, index) over the workgroup: wave shuffles, then one
// exchange of the per-wave winners through LDS.  Ties go to the lower index.
// rv / ri hold NT / 64 entries; the caller synchronises before reusing them.
__device__ inline int block_argmax(double v, int i, double* rv, int* ri, double* best) {
  for (int off = 32; off > 0; off >>= 1) {
    const double ov = __shfl_xor(v, off, 64);
    const int oi = __shfl_xor(i, off, 64);
    if (ov > v || (ov == v && oi < i)) {
      v = ov;
      i = oi;
    }
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    rv[w] = v;
    ri[w] = i;
  }
  __syncthreads();
  double bv = rv[0];
  int bi = ri[0];
  for (int q = 1; q < NT / 64; ++q)
    if (rv[q] > bv || (rv[q] == bv && ri[q] < bi)) {
      bv = rv[q];
      bi = ri[q];
    }
  *best = bv;
  return bi;
}

template <bool L>
__device__ inline double2& pel(double2* sm, double2* A, ll lda, int n, int c0, int r, int c) {
  if constexpr (L)
    return sm[r + c * n];
  else
    return A[(ll)r + (ll)(c0 + c) * lda];
}

template <bool L>
__global__ __launch_bounds__(NT) void gj_panel(double2* Aall, ll lda, ll sA, int n, int c0, int b,
                                              int bstride, int* ipiv_all, double2* Eall,
                                              double2* Tall, int* info) {
  extern __shared__ double2 sm[];
  __shared__ double2 prow[BMAX];
  __shared__ double rv[NT];
  __shared__ int ri[NT];
  const ll bi = blockIdx.x;
  const int t = threadIdx.x;
  double2* A = Aall + bi * sA;
  int* ipiv = ipiv_all + bi * n;
  double2* E = Eall + bi * (ll)n * bstride;
  double2* T = Tall + bi * (ll)n * bstride;

  if constexpr (L) {
    for (int idx = t; idx < n * b; idx += NT) {
      const int r = idx % n, c = idx / n;
      sm[idx] = A[(ll)r + (ll)(c0 + c) * lda];
    }
    __syncthreads();
  }

  for (int c = 0; c < b; ++c) {
    const int gc = c0 + c;
    double best = -1.0;
    int bidx = gc;
    for (int r = gc + t; r < n; r += NT) {
      const double2 v = pel<L>(sm, A, lda, n, c0, r, c);
      const double m = fabs(v.x) + fabs(v.y);
      if (m > best) {
        best = m;
        bidx = r;
      }
    }
    double bestv;
    const int p = block_argmax(best, bidx, rv, ri, &bestv);
    const bool zero = !(bestv > 0.0);
    if (t == 0) {
      ipiv[gc] = p;
      if (zero) info[bi] = 1;
    }
    if (p != gc) {
      for (int j = t; j < n; j += NT) {
        if (L && j >= c0 && j < c0 + b) {
          double2& x = pel<L>(sm, A, lda, n, c0, gc, j - c0);
          double2& y = pel<L>(sm, A, lda, n, c0, p, j - c0);
          const double2 tmp = x;
          x = y;
          y = tmp;
        } else {
          double2* x = A + (ll)gc + (ll)j * lda;
          double2* y = A + (ll)p + (ll)j * lda;
          const double2 tmp = *x;
          *x = *y;
          *y = tmp;
        }
      }
      __syncthreads();
    }
    const double2 piv = pel<L>(sm, A, lda, n, c0, gc, c);
    const double2 inv = zero ? make_double2(0.0, 0.0) : crecip(piv);
    if (t < b) prow[t] = (t == c) ? inv : cmul(pel<L>(sm, A, lda, n, c0, gc, t), inv);
    __syncthreads();
    for (int r = t; r < n; r += NT) {
      if (r == gc) {
        for (int j = 0; j < b; ++j) pel<L>(sm, A, lda, n, c0, gc, j) = prow[j];
        continue;
      }
      const double2 f = pel<L>(sm, A, lda, n, c0, r, c);
      for (int j = 0; j < b; ++j) {
        if (j == c) continue;
        double2& x = pel<L>(sm, A, lda, n, c0, r, j);
        const double2 d = cmul(f, prow[j]);
        x.x -= d.x;
        x.y -= d.y;
      }
      const double2 nf = cmul(f, inv);
      pel<L>(sm, A, lda, n, c0, r, c) = make_double2(-nf.x, -nf.y);
    }
    __syncthreads();
  }

  if constexpr (L) {
    for (int idx = t; idx < n * b; idx += NT) {
      const int r = idx % n, c = idx / n;
      A[(ll)r + (ll)(c0 + c) * lda] = sm[idx];
    }
  }
  for (int idx = t; idx < n * b; idx += NT) {
    const int r = idx % n, c = idx / n;
    E[idx] = pel<L>(sm, A, lda, n, c0, r, c);
  }
  __syncthreads();
  for (int idx = t; idx < n * b; idx += NT) {
    const int i = idx % b, j = idx / b;
    T[idx] = (j >= c0 && j < c0 + b) ? make_double2(0.0, 0.0) : A[(ll)(c0 + i) + (ll)j * lda];
  }
}

// perm[j] = original column that ends up in column j after undoing the row
// interchanges (column swaps applied in reverse pivot order).
__global__ void gj_perm(const int* ipiv_all, int* perm_all, int n, int batch) {
  const int bi = blockIdx.x * blockDim.x + threadIdx.x;
  if (bi >= batch) return;
  const int* ipiv = ipiv_all + (ll)bi * n;
  int* perm = perm_all + (ll)bi * n;
  for (int j = 0; j < n; ++j) perm[j] = j;
  for (int c = n - 1; c >= 0; --c) {
    const int p = ipiv[c];
    if (p != c) {
      const int tmp = perm[c];
      perm[c] = perm[p];
      perm[p] = tmp;
    }
  }
}

__global__ __launch_bounds__(NT) void gj_gather(const double2* W, ll lda, ll sA, double2* O,
                                                ll ldo, ll sO, const int* perm_all, int n) {
  const ll bi = blockIdx.y;
  const int* perm = perm_all + bi * n;
  const int j = blockIdx.x;
  const double2* src = W + bi * sA + (ll)perm[j] * lda;
  double2* dst = O + bi * sO + (ll)j * ldo;
  for (int r = threadIdx.x; r < n; r += NT) dst[r] = src[r];
}

// ---------------------------------------------------------------------------
// Tournament pivoting for matrices whose panels do not fit in LDS
// (communication-avoiding LU, Grigori, Demmel and Xiang 2011): the candidate
// rows [c0, n) are split into chunks of TR rows; each chunk picks b pivot
// candidates by partial-pivoting elimination of its panel rows; groups of TF
// candidate sets are reduced the same way until one set of b rows remains.
// Those rows become the pivot rows of the block step, which is then all
// matrix products.

constexpr int TR = 256;  // rows per tournament leaf (one per thread)
constexpr int TF = 4;    // candidate sets merged per reduction workgroup

// Partial-pivoting elimination of an nr x b block in LDS (column-major,
// leading dimension ld); ids[] follows the row interchanges.  After it the
// first min(nr, b) entries of ids are the selected rows.
__device__ void select_rows(double2* blk, int ld, int nr, int b, int* ids, double* rv, int* ri) {
  const int t = threadIdx.x;
  const int steps = nr < b ? nr : b;
  for (int c = 0; c < steps; ++c) {
    double best = -1.0;
    int bidx = c;
    for (int r = c + t; r < nr; r += NT) {
      const double2 v = blk[r + c * ld];
      const double m = fabs(v.x) + fabs(v.y);
      if (m > best) {
        best = m;
        bidx = r;
      }
    }
    double bestv;
    const int p = block_argmax(best, bidx, rv, ri, &bestv);
    const bool zero = !(bestv > 0.0);
    __syncthreads();
    if (p != c) {
      for (int j = t; j < b; j += NT) {
        const double2 x = blk[c + j * ld];
        blk[c + j * ld] = blk[p + j * ld];
        blk[p + j * ld] = x;
      }
      if (t == 0) {
        const int x = ids[c];
        ids[c] = ids[p];
        ids[p] = x;
      }
    }
    __syncthreads();
    if (!zero) {
      const double2 inv = crecip(blk[c + c * ld]);
      for (int r = c + 1 + t; r < nr; r += NT) {
        const double2 l = cmul(blk[r + c * ld], inv);
        for (int j = c + 1; j < b; ++j) {
          const double2 d = cmul(l, blk[c + j * ld]);
          blk[r + j * ld].x -= d.x;
          blk[r + j * ld].y -= d.y;
        }
      }
    }
    __syncthreads();
  }
}

// Leaves: chunk g of rows [c0, n) selects up to b candidate rows.
__global__ __launch_bounds__(NT) void tp_leaf(const double2* Aall, ll lda, ll sA, int n, int c0,
                                              int b, int G, int* cand_all) {
  extern __shared__ double2 blk[];
  __shared__ double rv[NT];
  __shared__ int ri[NT];
  __shared__ int ids[TR];
  const ll bi = blockIdx.y;
  const int g = blockIdx.x, t = threadIdx.x;
  const double2* A = Aall + bi * sA;
  const int r0 = c0 + g * TR;
  const int nr = (n - r0) < TR ? (n - r0) : TR;
  for (int idx = t; idx < nr * b; idx += NT) {
    const int r = idx % nr, c = idx / nr;
    blk[r + c * TR] = A[(ll)(r0 + r) + (ll)(c0 + c) * lda];
  }
  for (int r = t; r < TR; r += NT) ids[r] = (r < nr) ? r0 + r : -1;
  __syncthreads();
  select_rows(blk, TR, nr, b, ids, rv, ri);
  int* cand = cand_all + (bi * G + g) * (ll)b;
  for (int i = t; i < b; i += NT) cand[i] = (i < nr) ? ids[i] : -1;
}

// Reduction: workgroup g merges candidate sets [TF g, TF g + TF) of Gin
// (entries -1 mark missing candidates of short chunks).
__global__ __launch_bounds__(NT) void tp_reduce(const double2* Aall, ll lda, ll sA, int c0, int b,
                                                int Gin, const int* cin_all, int Gout,
                                                int* cout_all) {
  extern __shared__ double2 blk[];
  __shared__ double rv[NT];
  __shared__ int ri[NT];
  __shared__ int ids[TF * BMAX];
  __shared__ int nsel;
  const ll bi = blockIdx.y;
  const int g = blockIdx.x, t = threadIdx.x;
  const double2* A = Aall + bi * sA;
  const int* cin = cin_all + bi * (ll)Gin * b;
  if (t == 0) {
    int k = 0;
    for (int s = TF * g; s < TF * g + TF && s < Gin; ++s)
      for (int i = 0; i < b; ++i)
        if (cin[(ll)s * b + i] >= 0) ids[k++] = cin[(ll)s * b + i];
    nsel = k;
  }
  __syncthreads();
  const int nr = nsel;
  const int ld = TF * BMAX;
  for (int idx = t; idx < nr * b; idx += NT) {
    const int r = idx % nr, c = idx / nr;
    blk[r + c * ld] = A[(ll)ids[r] + (ll)(c0 + c) * lda];
  }
  __syncthreads();
  select_rows(blk, ld, nr, b, ids, rv, ri);
  int* cout = cout_all + (bi * Gout + g) * (ll)b;
  for (int i = t; i < b; i += NT) cout[i] = (i < nr) ? ids[i] : -1;
}

// Plans the interchanges that bring the selected rows (in order) to rows
// c0..c0+b-1: the sequence of swaps is recorded in ipiv (same convention as
// the unblocked panel), and their net effect -- a permutation of at most 2b
// rows -- as (destination, source) pairs for tp_apply.  One workgroup per
// matrix; dense maps over the rows [c0, n) live in LDS.
__global__ __launch_bounds__(NT) void tp_plan(int n, int c0, int b, const int* sel_all,
                                              int* ipiv_all, int* plan_all) {
  extern __shared__ int maps[];  // row_at[n - c0], pos_of[n - c0]
  __shared__ int touched[2 * BMAX];
  const ll bi = blockIdx.x;
  const int t = threadIdx.x, nr = n - c0;
  const int* sel = sel_all + bi * b;
  int* plan = plan_all + bi * (1 + 4 * BMAX);
  int* row_at = maps;
  int* pos_of = maps + nr;
  for (int x = t; x < nr; x += NT) {
    row_at[x] = x;
    pos_of[x] = x;
  }
  __syncthreads();
  if (t == 0) {
    for (int i = 0; i < b; ++i) {
      const int want = sel[i] - c0, tgt = i;
      // always in range: the tournament returns >= b rows of [c0, n)
      const int s = (want >= 0 && want < nr) ? pos_of[want] : tgt;
      ipiv_all[bi * n + c0 + tgt] = c0 + s;
      touched[2 * i] = tgt;
      touched[2 * i + 1] = s;
      if (s == tgt) continue;
      const int rt = row_at[tgt], rs = row_at[s];
      row_at[tgt] = rs;
      row_at[s] = rt;
      pos_of[rs] = tgt;
      pos_of[rt] = s;
    }
    int m = 0;
    for (int q = 0; q < 2 * b; ++q) {
      const int x = touched[q];
      if (row_at[x] != x) {
        plan[1 + 2 * m] = c0 + x;
        plan[2 + 2 * m] = c0 + row_at[x];
        row_at[x] = x;  // emitted
        ++m;
      }
    }
    plan[0] = m;
  }
}

// Applies the planned row permutation to 64 columns per workgroup: all moved
// rows are read into LDS first, then written to their destinations.
__global__ __launch_bounds__(NT) void tp_apply(double2* Aall, ll lda, ll sA, int n,
                                               const int* plan_all) {
  __shared__ double2 buf[2 * BMAX][64];
  const ll bi = blockIdx.y;
  const int t = threadIdx.x;
  double2* A = Aall + bi * sA;
  const int* plan = plan_all + bi * (1 + 4 * BMAX);
  const int m = plan[0];
  const int j0 = blockIdx.x * 64;
  for (int idx = t; idx < m * 64; idx += NT) {
    const int q = idx % m, jj = idx / m;
    const int j = j0 + jj;
    if (j < n) buf[q][jj] = A[(ll)plan[2 + 2 * q] + (ll)j * lda];
  }
  __syncthreads();
  for (int idx = t; idx < m * 64; idx += NT) {
    const int q = idx % m, jj = idx / m;
    const int j = j0 + jj;
    if (j < n) A[(ll)plan[1 + 2 * q] + (ll)j * lda] = buf[q][jj];
  }
}

// Inverse of the b x b pivot block by Gauss-Jordan elimination without
// interchanges: the tournament ordered the pivot rows by partial pivoting, so
// elimination in that order makes the same pivot choices.  BMAX x BMAX
// threads, one element each (the block padded with the identity); the
// matrix is exchanged through LDS once per elimination step.
__global__ __launch_bounds__(BMAX * BMAX) void tp_block(const double2* Aall, ll lda, ll sA, int c0,
                                                        int b, double2* IB_all, int* info) {
  __shared__ double2 m[BMAX * BMAX];  // column-major: (r, j) at r + j * BMAX
  const ll bi = blockIdx.x;
  const int t = threadIdx.x;
  const int r = t % BMAX, j = t / BMAX;
  const double2* A = Aall + bi * sA;
  double2* IB = IB_all + bi * (ll)BMAX * BMAX;
  const bool act = (r < b && j < b);
  double2 v = act ? A[(ll)(c0 + r) + (ll)(c0 + j) * lda] : make_double2((r == j) ? 1.0 : 0.0, 0.0);
  bool singular = false;
  for (int c = 0; c < b; ++c) {
    m[t] = v;
    __syncthreads();
    const double2 piv = m[c + c * BMAX], f = m[r + c * BMAX], pc = m[c + j * BMAX];
    __syncthreads();
    const bool zero = (piv.x == 0.0 && piv.y == 0.0);
    singular |= zero;
    const double2 inv = zero ? make_double2(0.0, 0.0) : crecip(piv);
    if (r == c) {
      v = (j == c) ? inv : cmul(pc, inv);
    } else if (j == c) {
      const double2 nf = cmul(f, inv);
      v = make_double2(-nf.x, -nf.y);
    } else {
      const double2 d = cmul(f, cmul(pc, inv));
      v.x -= d.x;
      v.y -= d.y;
    }
  }
  if (act) IB[r + j * b] = v;
  if (t == 0 && singular) info[bi] = 1;
}

// T = pivot rows c0.. of A, with the panel columns zeroed (b x n, ld b).
__global__ __launch_bounds__(NT) void tp_copy_t(const double2* Aall, ll lda, ll sA, int n, int c0,
                                                int b, int bstride, double2* Tall) {
  const ll bi = blockIdx.y;
  const double2* A = Aall + bi * sA;
  double2* T = Tall + bi * (ll)n * bstride;
  for (ll idx = blockIdx.x * (ll)NT + threadIdx.x; idx < (ll)n * b; idx += (ll)gridDim.x * NT) {
    const int i = (int)(idx % b);
    const int j = (int)(idx / b);
    T[idx] = (j >= c0 && j < c0 + b) ? make_double2(0.0, 0.0) : A[(ll)(c0 + i) + (ll)j * lda];
  }
}

// After E = -A[:, panel] IB: the pivot rows of E become IB, and the panel
// columns of A take their eliminated values (IB on the pivot rows, E
// elsewhere).
__global__ __launch_bounds__(NT) void tp_fix(double2* Aall, ll lda, ll sA, int n, int c0, int b,
                                             int bstride, const double2* IB_all, double2* Eall) {
  const ll bi = blockIdx.y;
  double2* A = Aall + bi * sA;
  double2* E = Eall + bi * (ll)n * bstride;
  const double2* IB = IB_all + bi * (ll)BMAX * BMAX;
  for (ll idx = blockIdx.x * (ll)NT + threadIdx.x; idx < (ll)n * b; idx += (ll)gridDim.x * NT) {
    const int r = (int)(idx % n);
    const int c = (int)(idx / n);
    if (r >= c0 && r < c0 + b) {
      const double2 v = IB[(r - c0) + c * b];
      A[(ll)r + (ll)(c0 + c) * lda] = v;
      E[idx] = v;
    } else {
      A[(ll)r + (ll)(c0 + c) * lda] = E[idx];
    }
  }
}

int panel_width(int n) { return n < BMAX ? n : BMAX; }

// Dynamic LDS available to one workgroup of the panel kernel (bytes).
size_t lds_limit() {
  static size_t cached = 0;
  if (cached == 0) {
    int dev = 0, v = 0;
    size_t lim = 64 * 1024;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        v > 0)
      lim = (size_t)v;
    const size_t static_lds = BMAX * sizeof(double2) + NT * (sizeof(double) + sizeof(int));
    lim = lim > static_lds + 512 ? lim - static_lds - 512 : 0;
    cached = lim < LDS_BUDGET ? lim : LDS_BUDGET;
  }
  return cached;
}

// Applies the eliminations of panel [c0, c0 + bw) to the other columns (see
// the file comment): rows outside the panel accumulate E_Q T, the pivot rows
// are overwritten by inv(A_PP) T outside the panel columns.
hipError_t apply_panel(hipStream_t st, int n, int c0, int bw, int bmax, double2* work, ll lda, ll sA,
                       const double2* E, const double2* T, int batch) {
  const double2 one = make_double2(1.0, 0.0), zero = make_double2(0.0, 0.0);
  const ll se = (ll)n * bmax;
  const int c1 = c0 + bw;
  // non-pivot rows [0, c0) and [c1, n), all columns (T is zero on the panel)
  HPS_HIP_TRY(zgemm(st, OP_N, OP_N, c0, n, bw, one, E, n, se, T, bw, se, one, work, lda, sA, batch));
  HPS_HIP_TRY(zgemm(st, OP_N, OP_N, n - c1, n, bw, one, E + c1, n, se, T, bw, se, one, work + c1, lda,
                    sA, batch));
  // pivot rows, columns [0, c0) and [c1, n)
  HPS_HIP_TRY(zgemm(st, OP_N, OP_N, bw, c0, bw, one, E + c0, n, se, T, bw, se, zero, work + c0, lda, sA,
                    batch));
  HPS_HIP_TRY(zgemm(st, OP_N, OP_N, bw, n - c1, bw, one, E + c0, n, se, T + (ll)c1 * bw, bw, se, zero,
                    work + c0 + (ll)c1 * lda, lda, sA, batch));
  return hipSuccess;
}

}  // namespace

constexpr int TOURNAMENT_MIN_N = 512;

size_t cand_ints(int n, int batch) { return (size_t)batch * ((n + TR - 1) / TR) * BMAX; }

size_t zinv_workspace(int n, int batch) {
  const int b = panel_width(n);
  size_t bytes = 0;
  bytes += (size_t)batch * n * sizeof(int) * 2;         // ipiv + perm
  bytes = (bytes + 255) & ~(size_t)255;
  bytes += (size_t)batch * n * b * sizeof(double2) * 2;  // E + T
  bytes += (size_t)batch * BMAX * BMAX * sizeof(double2);  // pivot-block inverses
  bytes += 2 * cand_ints(n, batch) * sizeof(int);          // tournament candidates
  bytes += (size_t)batch * (1 + 4 * BMAX) * sizeof(int);   // row-permutation plans
  return bytes;
}

hipError_t zinv(hipStream_t st, int n, double2* work, ll lda, ll sA, double2* out, ll ldo, ll sO,
                int batch, void* ws, int* info) {
  if (n <= 0 || batch <= 0) return hipSuccess;
  if (batch > 65535) return hipErrorInvalidValue;
  const int bmax = panel_width(n);
  // panel in LDS when at least min(8, n) columns fit, else in global memory
  const int b_lds = (int)(lds_limit() / ((size_t)n * sizeof(double2)));
  const bool in_lds = b_lds >= (n < 8 ? n : 8);
  const int b = in_lds ? (b_lds < bmax ? b_lds : bmax) : bmax;
  int* ipiv = (int*)ws;
  int* perm = ipiv + (size_t)batch * n;
  size_t off = ((size_t)batch * n * sizeof(int) * 2 + 255) & ~(size_t)255;
  double2* E = (double2*)((char*)ws + off);
  double2* T = E + (size_t)batch * n * bmax;
  if (n > TOURNAMENT_MIN_N) {
    double2* IB = T + (size_t)batch * n * bmax;
    int* candA = (int*)(IB + (size_t)batch * BMAX * BMAX);
    int* candB = candA + cand_ints(n, batch);
    int* plan = candB + cand_ints(n, batch);
    const int bt = bmax;
    HPS_HIP_TRY(hipFuncSetAttribute((const void*)tp_leaf, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)(TR * bt * sizeof(double2))));
    HPS_HIP_TRY(hipFuncSetAttribute((const void*)tp_reduce,
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)(TF * BMAX * bt * sizeof(double2))));
    HPS_HIP_TRY(hipFuncSetAttribute((const void*)tp_plan, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)(2 * n * sizeof(int))));
    const unsigned eblocks = (unsigned)(((ll)n * bt + NT - 1) / NT);
    for (int c0 = 0; c0 < n; c0 += bt) {
      const int bw = (n - c0) < bt ? (n - c0) : bt;
      const int G = (n - c0 + TR - 1) / TR;
      {
        KernelTimer kt(st, K_GJ_PANEL, 8.0 * (n - c0) * (double)bw * bw * batch,
                       16.0 * (n - c0) * (double)bw * batch);
        hipLaunchKernelGGL(tp_leaf, dim3(G, batch), dim3(NT), TR * bw * sizeof(double2), st, work, lda,
                           sA, n, c0, bw, G, candA);
      }
      HPS_HIP_TRY(hipGetLastError());
      int* cin = candA;
      int* cout = candB;
      int Gin = G;
      while (Gin > 1) {
        const int Gout = (Gin + TF - 1) / TF;
        KernelTimer kt(st, K_GJ_PANEL, 8.0 * Gin * (double)bw * bw * bw * batch,
                       16.0 * Gin * (double)bw * bw * batch);
        hipLaunchKernelGGL(tp_reduce, dim3(Gout, batch), dim3(NT), TF * BMAX * bw * sizeof(double2), st,
                           work, lda, sA, c0, bw, Gin, cin, Gout, cout);
        HPS_HIP_TRY(hipGetLastError());
        int* tmp = cin;
        cin = cout;
        cout = tmp;
        Gin = Gout;
      }
      {
        KernelTimer kt(st, K_GJ_PERM, 0.0, 8.0 * bw * (double)batch);
        hipLaunchKernelGGL(tp_plan, dim3(batch), dim3(NT), 2 * (n - c0) * sizeof(int), st, n, c0, bw, cin,
                           ipiv, plan);
      }
      HPS_HIP_TRY(hipGetLastError());
      {
        KernelTimer kt(st, K_GJ_PERM, 0.0, 64.0 * n * (double)bw * batch);
        hipLaunchKernelGGL(tp_apply, dim3((n + 63) / 64, batch), dim3(NT), 0, st, work, lda, sA, n, plan);
      }
      HPS_HIP_TRY(hipGetLastError());
      {
        KernelTimer kt(st, K_GJ_PANEL, 8.0 * bw * (double)bw * bw * batch, 32.0 * bw * (double)bw * batch);
        hipLaunchKernelGGL(tp_block, dim3(batch), dim3(BMAX * BMAX), 0, st, work, lda, sA, c0, bw, IB,
                           info);
      }
      HPS_HIP_TRY(hipGetLastError());
      {
        KernelTimer kt(st, K_MOVE, 0.0, 32.0 * n * (double)bw * batch);
        hipLaunchKernelGGL(tp_copy_t, dim3(eblocks, batch), dim3(NT), 0, st, work, lda, sA, n, c0, bw, bmax,
                           T);
      }
      HPS_HIP_TRY(hipGetLastError());
      HPS_HIP_TRY(zgemm(st, OP_N, OP_N, n, bw, bw, make_double2(-1.0, 0.0), work + (ll)c0 * lda, lda, sA,
                        IB, bw, (ll)BMAX * BMAX, make_double2(0.0, 0.0), E, n, (ll)n * bmax, batch));
      {
        KernelTimer kt(st, K_MOVE, 0.0, 48.0 * n * (double)bw * batch);
        hipLaunchKernelGGL(tp_fix, dim3(eblocks, batch), dim3(NT), 0, st, work, lda, sA, n, c0, bw, bmax,
                           IB, E);
      }
      HPS_HIP_TRY(hipGetLastError());
      if (bw < n) HPS_HIP_TRY(apply_panel(st, n, c0, bw, bmax, work, lda, sA, E, T, batch));
    }
    {
      KernelTimer kt(st, K_GJ_PERM, 0.0, 8.0 * n * batch);
      hipLaunchKernelGGL(gj_perm, dim3((batch + 63) / 64), dim3(64), 0, st, ipiv, perm, n, batch);
    }
    HPS_HIP_TRY(hipGetLastError());
    {
      KernelTimer kt(st, K_GJ_PERM, 0.0, 32.0 * n * (double)n * batch);
      hipLaunchKernelGGL(gj_gather, dim3(n, batch), dim3(NT), 0, st, work, lda, sA, out, ldo, sO, perm, n);
    }
    return hipGetLastError();
  }
  const size_t lds = (size_t)n * b * sizeof(double2);
  if (in_lds) {
    HPS_HIP_TRY(hipFuncSetAttribute((const void*)gj_panel<true>,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  }
  for (int c0 = 0; c0 < n; c0 += b) {
    const int bw = (n - c0) < b ? (n - c0) : b;
    KernelTimer kt(st, K_GJ_PANEL, 8.0 * n * (double)bw * bw * batch, 64.0 * n * (double)bw * batch);
    if (in_lds) {
      hipLaunchKernelGGL(gj_panel<true>, dim3(batch), dim3(NT), (size_t)n * bw * sizeof(double2),
                         st, work, lda, sA, n, c0, bw, bmax, ipiv, E, T, info);
    } else {
      hipLaunchKernelGGL(gj_panel<false>, dim3(batch), dim3(NT), 0, st, work, lda, sA, n, c0, bw,
                         bmax, ipiv, E, T, info);
    }
    HPS_HIP_TRY(hipGetLastError());
    if (bw < n) HPS_HIP_TRY(apply_panel(st, n, c0, bw, bmax, work, lda, sA, E, T, batch));
  }
  {
    KernelTimer kt(st, K_GJ_PERM, 0.0, 8.0 * n * batch);
    hipLaunchKernelGGL(gj_perm, dim3((batch + 63) / 64), dim3(64), 0, st, ipiv, perm, n, batch);
  }
  HPS_HIP_TRY(hipGetLastError());
  {
    KernelTimer kt(st, K_GJ_PERM, 0.0, 32.0 * n * (double)n * batch);
    hipLaunchKernelGGL(gj_gather, dim3(n, batch), dim3(NT), 0, st, work, lda, sA, out, ldo, sO, perm, n);
  }
  return hipGetLastError();
}

}  // namespace hps
