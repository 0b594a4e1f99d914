// Batched complex FP64 GEMM on CDNA4 matrix cores.
//
// Complex products are done as real split products on the FP64 MFMA
// (v_mfma_f64_16x16x4f64): Re += ar*br - ai*bi, Im += ar*bi + ai*br.
// A 256-thread workgroup (4 wave64s) owns a 64 x 64 tile of C; each wave
// owns a 32 x 32 quarter as 2 x 2 MFMA blocks of 16 x 16.  The K loop steps
// by 16: the A (64 x 16) and B (16 x 64) tiles are loaded from HBM with
// coalesced 16-byte accesses, split into real/imaginary planes in LDS, and
// the next tile is prefetched into registers while the current one is
// multiplied.  Operands may be used as stored (N), transposed (T) or
// conjugate-transposed (C); all shapes are bounds-checked (zero fill).
#include "common.h"

namespace hps {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int TM = 64;
constexpr int TN = 64;
constexpr int TK = 16;
constexpr int PAD = 1;

struct Args {
  int M, N, K, opA, opB;
  const double2* A;
  ll lda, sA;
  const double2* B;
  ll ldb, sB;
  double2* C;
  ll ldc, sC;
  double2 alpha, beta;
};

__device__ inline double2 ld_op(const double2* p, bool conj) {
  double2 v = *p;
  if (conj) v.y = -v.y;
  return v;
}

// Loads this thread's 4 elements of the A tile (rows m0.., cols k0..).
__device__ inline void load_a(const Args& a, const double2* A, int m0, int k0, int t,
                              double2 r[4]) {
  if (a.opA == OP_N) {
    const int m = m0 + (t & 63);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + (t >> 6) + 4 * j;
      r[j] = (m < a.M && k < a.K) ? A[(ll)m + (ll)k * a.lda] : make_double2(0.0, 0.0);
    }
  } else {
    const int k = k0 + (t & 15);
    const bool cj = a.opA == OP_C;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int m = m0 + (t >> 4) + 16 * j;
      r[j] = (m < a.M && k < a.K) ? ld_op(A + (ll)k + (ll)m * a.lda, cj) : make_double2(0.0, 0.0);
    }
  }
}

__device__ inline void store_a(const Args& a, double (*Are)[TM + PAD], double (*Aim)[TM + PAD],
                               int t, const double2 r[4]) {
  if (a.opA == OP_N) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int kk = (t >> 6) + 4 * j, mm = t & 63;
      Are[kk][mm] = r[j].x;
      Aim[kk][mm] = r[j].y;
    }
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int kk = t & 15, mm = (t >> 4) + 16 * j;
      Are[kk][mm] = r[j].x;
      Aim[kk][mm] = r[j].y;
    }
  }
}

__device__ inline void load_b(const Args& a, const double2* B, int n0, int k0, int t,
                              double2 r[4]) {
  if (a.opB == OP_N) {
    const int k = k0 + (t & 15);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = n0 + (t >> 4) + 16 * j;
      r[j] = (n < a.N && k < a.K) ? B[(ll)k + (ll)n * a.ldb] : make_double2(0.0, 0.0);
    }
  } else {
    const int n = n0 + (t & 63);
    const bool cj = a.opB == OP_C;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + (t >> 6) + 4 * j;
      r[j] = (n < a.N && k < a.K) ? ld_op(B + (ll)n + (ll)k * a.ldb, cj) : make_double2(0.0, 0.0);
    }
  }
}

__device__ inline void store_b(const Args& a, double (*Bre)[TN + PAD], double (*Bim)[TN + PAD],
                               int t, const double2 r[4]) {
  if (a.opB == OP_N) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int kk = t & 15, nn = (t >> 4) + 16 * j;
      Bre[kk][nn] = r[j].x;
      Bim[kk][nn] = r[j].y;
    }
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int kk = (t >> 6) + 4 * j, nn = t & 63;
      Bre[kk][nn] = r[j].x;
      Bim[kk][nn] = r[j].y;
    }
  }
}

__global__ __launch_bounds__(256) void zgemm_kernel(Args a) {
  __shared__ double Are[TK][TM + PAD], Aim[TK][TM + PAD];
  __shared__ double Bre[TK][TN + PAD], Bim[TK][TN + PAD];

  const int tilesM = (a.M + TM - 1) / TM;
  const int m0 = (blockIdx.x % tilesM) * TM;
  const int n0 = (blockIdx.x / tilesM) * TN;
  const ll b = blockIdx.y;
  const double2* A = a.A + b * a.sA;
  const double2* B = a.B + b * a.sB;
  double2* C = a.C + b * a.sC;

  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int wm = (w & 1) * 32, wn = (w >> 1) * 32;
  const int lr = lane & 15, lk = lane >> 4;

  v4d acc_re[2][2], acc_im[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc_re[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
      acc_im[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    }

  double2 ra[4], rb[4];
  load_a(a, A, m0, 0, t, ra);
  load_b(a, B, n0, 0, t, rb);
  const int nk = (a.K + TK - 1) / TK;
  for (int kt = 0; kt < nk; ++kt) {
    __syncthreads();
    store_a(a, Are, Aim, t, ra);
    store_b(a, Bre, Bim, t, rb);
    __syncthreads();
    if (kt + 1 < nk) {
      load_a(a, A, m0, (kt + 1) * TK, t, ra);
      load_b(a, B, n0, (kt + 1) * TK, t, rb);
    }
#pragma unroll
    for (int ks = 0; ks < TK / 4; ++ks) {
      const int kk = ks * 4 + lk;
      double ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        ar[i] = Are[kk][wm + 16 * i + lr];
        ai[i] = Aim[kk][wm + 16 * i + lr];
        br[i] = Bre[kk][wn + 16 * i + lr];
        bi[i] = Bim[kk][wn + 16 * i + lr];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          acc_re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], acc_re[i][j], 0, 0, 0);
          acc_re[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[i], bi[j], acc_re[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bi[j], acc_im[i][j], 0, 0, 0);
          acc_im[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], br[j], acc_im[i][j], 0, 0, 0);
        }
    }
  }

  // D layout of the 16x16x4 f64 MFMA: item r of a lane is row lane/16 + 4 r,
  // column lane % 16.
  const bool use_beta = (a.beta.x != 0.0 || a.beta.y != 0.0);
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn + 16 * j + lr;
      if (col >= a.N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + 16 * i + lk + 4 * r;
        if (row >= a.M) continue;
        const double xr = acc_re[i][j][r], xi = acc_im[i][j][r];
        double2 v = make_double2(a.alpha.x * xr - a.alpha.y * xi, a.alpha.x * xi + a.alpha.y * xr);
        double2* pc = C + (ll)row + (ll)col * a.ldc;
        if (use_beta) {
          const double2 c = *pc;
          v.x += a.beta.x * c.x - a.beta.y * c.y;
          v.y += a.beta.x * c.y + a.beta.y * c.x;
        }
        *pc = v;
      }
    }
}

}  // namespace

hipError_t zgemm(hipStream_t st, int opA, int opB, int M, int N, int K, double2 alpha,
                 const double2* A, ll lda, ll sA, const double2* B, ll ldb, ll sB, double2 beta,
                 double2* C, ll ldc, ll sC, int batch) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  if (batch > 65535) return hipErrorInvalidValue;
  Args a{M, N, K < 0 ? 0 : K, opA, opB, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, beta};
  const ll tiles = (ll)((M + TM - 1) / TM) * ((N + TN - 1) / TN);
  if (tiles > 0x7fffffffLL) return hipErrorInvalidValue;
  dim3 grid((unsigned)tiles, (unsigned)batch);
  const bool rb = (beta.x != 0.0 || beta.y != 0.0);
  KernelTimer kt(st, K_ZGEMM, 8.0 * M * N * (double)a.K * batch,
                 16.0 * ((double)M * a.K + (double)a.K * N + (rb ? 2.0 : 1.0) * M * N) * batch);
  hipLaunchKernelGGL(zgemm_kernel, grid, dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace hps
