// Batched complex FP64 matrix inverse by blocked Gauss-Jordan elimination with
// partial (row) pivoting.
//
// For each column panel [c0, c0 + b):
//   1. a panel kernel (one workgroup per matrix) eliminates the b pivot
//      columns in place: pivot search over the rows not yet used, a full-row
//      swap, and the in-place inverse update of the panel columns, which
//      leaves inv(A_PP) in the pivot rows and -A_QP inv(A_PP) in the others.
//      It then emits E = panel - [0; I; 0] and T = pivot rows with the panel
//      columns zeroed;
//   2. the rank-b update A += E T on all other columns is one batched
//      complex GEMM on the matrix cores.
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
    rv[t] = best;
    ri[t] = bidx;
    __syncthreads();
    for (int s = NT / 2; s > 0; s >>= 1) {
      if (t < s) {
        const double o = rv[t + s];
        const int oi = ri[t + s];
        if (o > rv[t] || (o == rv[t] && oi < ri[t])) {
          rv[t] = o;
          ri[t] = oi;
        }
      }
      __syncthreads();
    }
    const int p = ri[0];
    const bool zero = !(rv[0] > 0.0);
    __syncthreads();
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
    double2 v = pel<L>(sm, A, lda, n, c0, r, c);
    if (r == c0 + c) v.x -= 1.0;
    E[idx] = v;
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

}  // namespace

size_t zinv_workspace(int n, int batch) {
  const int b = panel_width(n);
  size_t bytes = 0;
  bytes += (size_t)batch * n * sizeof(int) * 2;         // ipiv + perm
  bytes = (bytes + 255) & ~(size_t)255;
  bytes += (size_t)batch * n * b * sizeof(double2) * 2;  // E + T
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
    if (bw < n) {
      HPS_HIP_TRY(zgemm(st, OP_N, OP_N, n, n, bw, make_double2(1.0, 0.0), E, n, (ll)n * bmax, T, bw,
                        (ll)n * bmax, make_double2(1.0, 0.0), work, lda, sA, batch));
    }
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
