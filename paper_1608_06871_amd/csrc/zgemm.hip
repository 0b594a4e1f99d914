// Batched complex GEMM on CDNA4 matrix cores, in FP64 (zgemm) and FP32
// (cgemm).
//
// Complex products run on the 16x16x4 MFMA of the precision
// (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32) as real products on split
// real/imaginary planes, with the 3M method (Re = ArBr - AiBi,
// Im = (Ar + Ai)(Br + Bi) - ArBr - AiBi: three matrix-core operations per
// complex multiply-add, the sums formed in registers from the LDS planes;
// Higham analyses its accuracy) or the four direct products.
// A 256-thread workgroup (4 wave64s, 2 x 2) owns a (32 WM) x (32 WN) tile of
// C; each wave owns (16 WM) x (16 WN) as WM x WN MFMA blocks of 16 x 16.  The
// K loop steps by TK: the A and B tiles are loaded from HBM with coalesced
// accesses into real/imaginary planes in LDS, and the next tile is
// prefetched into registers while the current one is multiplied.  Operands
// may be used as stored (N), transposed (T) or conjugate-transposed (C); all
// shapes are bounds-checked (zero fill).  The tile shape is chosen per call.
#include <cstdio>
#include <cstdlib>

#include "common.h"

namespace hps {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T>
struct Cx;
template <>
struct Cx<double> {
  typedef double2 T2;
  typedef v4d V4;
};
template <>
struct Cx<float> {
  typedef float2 T2;
  typedef v4f V4;
};

// 16x16x4 MFMA.  Inputs (both precisions): lane l holds A[l % 16][l / 16]
// and B[l / 16][l % 16].  Output item r of lane l: FP64 row l / 16 + 4 r,
// FP32 row 4 (l / 16) + r; column l % 16 (probed on the hardware).
__device__ inline v4d mfma16(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline v4f mfma16(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
template <typename T>
__device__ inline int mfma_row(int lk, int r) {
  return sizeof(T) == 8 ? lk + 4 * r : 4 * lk + r;
}

constexpr int PAD = 1;
constexpr int NT = 256;

template <typename T>
struct ArgsT {
  typedef typename Cx<T>::T2 T2;
  int M, N, K, opA, opB;
  const T2* A;
  ll lda, sA;
  const T2* B;
  ll ldb, sB;
  T2* C;
  ll ldc, sC;
  T2 alpha, beta;
  const int* rpos;  // optional: rows r with plo <= rpos[r] < phi take beta = 0
  ll srp;
  int plo, phi;
  int adiv, bdiv;  // batch index divisors of A and B (operand of batch b: b / div)
};
typedef ArgsT<double> Args;

template <typename T2>
__device__ inline T2 ld_op(const T2* p, bool conj) {
  T2 v = *p;
  if (conj) v.y = -v.y;
  return v;
}

// Loads / stores of a TR x TK tile of a matrix X viewed as rows x K: A as
// op(A) (M x K), B through the transpose of op(B) (N x K).  `contig` means
// consecutive rows are adjacent in memory, so threads run along the rows.
template <int TR, int TK, typename T>
struct TileIO {
  typedef typename Cx<T>::T2 T2;
  static constexpr int PER = TR * TK / NT;
  __device__ static void load(const T2* X, ll ld, int nrow, int ncol, int r0, int k0, bool contig, bool conj,
                              int t, T2* reg) {
    T2 z;
    z.x = 0;
    z.y = 0;
    if (contig) {
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const int idx = t + j * NT;
        const int r = r0 + idx % TR, k = k0 + idx / TR;
        reg[j] = (r < nrow && k < ncol) ? ld_op(X + (ll)r + (ll)k * ld, conj) : z;
      }
    } else {
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const int idx = t + j * NT;
        const int k = k0 + idx % TK, r = r0 + idx / TK;
        reg[j] = (r < nrow && k < ncol) ? ld_op(X + (ll)k + (ll)r * ld, conj) : z;
      }
    }
  }
  __device__ static void store(T (*re)[TR + PAD], T (*im)[TR + PAD], bool contig, int t, const T2* reg) {
#pragma unroll
    for (int j = 0; j < PER; ++j) {
      const int idx = t + j * NT;
      const int r = contig ? idx % TR : idx / TK;
      const int k = contig ? idx / TR : idx % TK;
      re[k][r] = reg[j].x;
      im[k][r] = reg[j].y;
    }
  }
};

template <typename T, int WM, int WN, bool M3, int TK, int WAVES>
__global__ __launch_bounds__(NT, WAVES) void gemm_kernel(ArgsT<T> a) {
  typedef typename Cx<T>::T2 T2;
  typedef typename Cx<T>::V4 V4;
  constexpr int TM = 32 * WM, TN = 32 * WN;
  __shared__ T Are[TK][TM + PAD], Aim[TK][TM + PAD];
  __shared__ T Bre[TK][TN + PAD], Bim[TK][TN + PAD];

  const int tilesM = (a.M + TM - 1) / TM;
  const int m0 = (blockIdx.x % tilesM) * TM;
  const int n0 = (blockIdx.x / tilesM) * TN;
  const ll b = blockIdx.y;
  const T2* A = a.A + (b / a.adiv) * a.sA;
  const T2* B = a.B + (b / a.bdiv) * a.sB;
  T2* C = a.C + b * a.sC;

  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int wm = (w & 1) * 16 * WM, wn = (w >> 1) * 16 * WN;
  const int lr = lane & 15, lk = lane >> 4;
  const bool a_rows = a.opA == OP_N, a_conj = a.opA == OP_C;
  const bool b_rows = a.opB != OP_N, b_conj = a.opB == OP_C;

  // M3: p1 = ArBr, p2 = AiBi, p3 = (Ar+Ai)(Br+Bi); otherwise p1 = Re, p3 = Im
  V4 p1[WM][WN], p2[WM][WN], p3[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      p1[i][j] = V4{0, 0, 0, 0};
      p2[i][j] = V4{0, 0, 0, 0};
      p3[i][j] = V4{0, 0, 0, 0};
    }

  typedef TileIO<TM, TK, T> IOA;
  typedef TileIO<TN, TK, T> IOB;
  T2 ra[IOA::PER], rb[IOB::PER];
  IOA::load(A, a.lda, a.M, a.K, m0, 0, a_rows, a_conj, t, ra);
  IOB::load(B, a.ldb, a.N, a.K, n0, 0, b_rows, b_conj, t, rb);
  const int nk = (a.K + TK - 1) / TK;
  for (int kt = 0; kt < nk; ++kt) {
    __syncthreads();
    IOA::store(Are, Aim, a_rows, t, ra);
    IOB::store(Bre, Bim, b_rows, t, rb);
    __syncthreads();
    if (kt + 1 < nk) {
      IOA::load(A, a.lda, a.M, a.K, m0, (kt + 1) * TK, a_rows, a_conj, t, ra);
      IOB::load(B, a.ldb, a.N, a.K, n0, (kt + 1) * TK, b_rows, b_conj, t, rb);
    }
#pragma unroll
    for (int ks = 0; ks < TK / 4; ++ks) {
      const int kk = ks * 4 + lk;
      T ar[WM], ai[WM], br[WN], bi[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) {
        ar[i] = Are[kk][wm + 16 * i + lr];
        ai[i] = Aim[kk][wm + 16 * i + lr];
      }
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        br[j] = Bre[kk][wn + 16 * j + lr];
        bi[j] = Bim[kk][wn + 16 * j + lr];
      }
      if constexpr (M3) {
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
          for (int j = 0; j < WN; ++j) {
            p1[i][j] = mfma16(ar[i], br[j], p1[i][j]);
            p2[i][j] = mfma16(ai[i], bi[j], p2[i][j]);
            p3[i][j] = mfma16(ar[i] + ai[i], br[j] + bi[j], p3[i][j]);
          }
      } else {
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
          for (int j = 0; j < WN; ++j) {
            p1[i][j] = mfma16(ar[i], br[j], p1[i][j]);
            p1[i][j] = mfma16(-ai[i], bi[j], p1[i][j]);
            p3[i][j] = mfma16(ar[i], bi[j], p3[i][j]);
            p3[i][j] = mfma16(ai[i], br[j], p3[i][j]);
          }
      }
    }
  }

  // output layout: see mfma16
  const bool use_beta = (a.beta.x != 0.0 || a.beta.y != 0.0);
  const int* rp = a.rpos ? a.rpos + (ll)blockIdx.y * a.srp : nullptr;
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      const int col = n0 + wn + 16 * j + lr;
      if (col >= a.N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + 16 * i + mfma_row<T>(lk, r);
        if (row >= a.M) continue;
        const T xr = M3 ? p1[i][j][r] - p2[i][j][r] : p1[i][j][r];
        const T xi = M3 ? p3[i][j][r] - p1[i][j][r] - p2[i][j][r] : p3[i][j][r];
        T2 v;
        v.x = a.alpha.x * xr - a.alpha.y * xi;
        v.y = a.alpha.x * xi + a.alpha.y * xr;
        T2* pc = C + (ll)row + (ll)col * a.ldc;
        if (use_beta && !(rp && rp[row] >= a.plo && rp[row] < a.phi)) {
          const T2 c = *pc;
          v.x += a.beta.x * c.x - a.beta.y * c.y;
          v.y += a.beta.x * c.y + a.beta.y * c.x;
        }
        *pc = v;
      }
    }
}

template <typename T, int WM, int WN, bool M3, int TK, int WAVES>
hipError_t launch_t(hipStream_t st, const ArgsT<T>& a, int batch) {
  constexpr int TM = 32 * WM, TN = 32 * WN;
  const ll tiles = (ll)((a.M + TM - 1) / TM) * ((a.N + TN - 1) / TN);
  if (tiles > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((gemm_kernel<T, WM, WN, M3, TK, WAVES>), dim3((unsigned)tiles, (unsigned)batch), dim3(NT),
                     0, st, a);
  return hipGetLastError();
}
template <int WM, int WN, bool M3, int TK, int WAVES>
hipError_t launch(hipStream_t st, const Args& a, int batch) {
  return launch_t<double, WM, WN, M3, TK, WAVES>(st, a, batch);
}

// Kernel variants (tile WM x WN, 3M or four products, K step, waves per
// SIMD); HPS_ZGEMM_VARIANT=<index> forces one for tuning runs.
typedef hipError_t (*LaunchFn)(hipStream_t, const Args&, int);
const LaunchFn VARIANTS[] = {
    launch<2, 2, false, 16, 2>,  // 0
    launch<2, 2, true, 16, 2>,   // 1
    launch<2, 2, false, 32, 2>,  // 2
    launch<2, 2, true, 32, 2>,   // 3
    launch<2, 2, true, 16, 1>,   // 4
    launch<2, 1, false, 16, 2>,  // 5
    launch<1, 2, false, 16, 2>,  // 6
    launch<2, 2, false, 8, 2>,   // 7
    launch<2, 1, true, 16, 2>,   // 8
    launch<1, 2, true, 16, 2>,   // 9
    launch<2, 2, true, 8, 2>,    // 10
    launch<2, 1, true, 16, 3>,   // 11
    launch<2, 1, true, 8, 3>,    // 12
};
constexpr int NVARIANT = sizeof(VARIANTS) / sizeof(VARIANTS[0]);

// HPS_ZGEMM_TRACE=<file> appends one line per call (M N K batch opA opB
// beta!=0 rowmask) for offline analysis of the call shapes.
void trace_call(const Args& a, int batch) {
  static FILE* f = nullptr;
  static int state = 0;
  if (state == 0) {
    const char* e = std::getenv("HPS_ZGEMM_TRACE");
    f = (e && *e) ? std::fopen(e, "a") : nullptr;
    state = 1;
  }
  if (!f) return;
  const bool rb = (a.beta.x != 0.0 || a.beta.y != 0.0);
  std::fprintf(f, "%d %d %d %d %d %d %d %d\n", a.M, a.N, a.K, batch, a.opA, a.opB, rb ? 1 : 0,
               a.rpos ? 1 : 0);
  std::fflush(f);
}

int forced_variant() {
  static int v = -2;
  if (v == -2) {
    const char* e = std::getenv("HPS_ZGEMM_VARIANT");
    v = -1;
    if (e && *e) {
      const int x = std::atoi(e);
      if (x >= 0 && x < NVARIANT) v = x;
    }
  }
  return v;
}

}  // namespace

hipError_t zgemm(hipStream_t st, int opA, int opB, int M, int N, int K, double2 alpha,
                 const double2* A, ll lda, ll sA, const double2* B, ll ldb, ll sB, double2 beta,
                 double2* C, ll ldc, ll sC, int batch) {
  return zgemm_rowmask(st, opA, opB, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, nullptr, 0, 0,
                       0, batch);
}

hipError_t zgemm_rowmask(hipStream_t st, int opA, int opB, int M, int N, int K, double2 alpha,
                         const double2* A, ll lda, ll sA, const double2* B, ll ldb, ll sB, double2 beta,
                         double2* C, ll ldc, ll sC, const int* rpos, ll srp, int plo, int phi, int batch) {
  return zgemm_full(st, opA, opB, M, N, K, alpha, A, lda, sA, 1, B, ldb, sB, 1, beta, C, ldc, sC, rpos, srp,
                    plo, phi, batch);
}

hipError_t zgemm_div(hipStream_t st, int opA, int opB, int M, int N, int K, double2 alpha,
                     const double2* A, ll lda, ll sA, int adiv, const double2* B, ll ldb, ll sB, int bdiv,
                     double2 beta, double2* C, ll ldc, ll sC, int batch) {
  return zgemm_full(st, opA, opB, M, N, K, alpha, A, lda, sA, adiv, B, ldb, sB, bdiv, beta, C, ldc, sC,
                    nullptr, 0, 0, 0, batch);
}

hipError_t zgemm_full(hipStream_t st, int opA, int opB, int M, int N, int K, double2 alpha,
                      const double2* A, ll lda, ll sA, int adiv, const double2* B, ll ldb, ll sB, int bdiv,
                      double2 beta, double2* C, ll ldc, ll sC, const int* rpos, ll srp, int plo, int phi,
                      int batch) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  if (batch > 65535 || adiv < 1 || bdiv < 1) return hipErrorInvalidValue;
  Args a{M, N, K < 0 ? 0 : K, opA, opB, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, beta, rpos, srp, plo, phi,
         adiv, bdiv};
  const bool rb = (beta.x != 0.0 || beta.y != 0.0);
  KernelTimer kt(st, K_ZGEMM, 8.0 * M * N * (double)a.K * batch,
                 16.0 * ((double)M * a.K + (double)a.K * N + (rb ? 2.0 : 1.0) * M * N) * batch);
  trace_call(a, batch);
  const int fv = forced_variant();
  if (fv >= 0) return VARIANTS[fv](st, a, batch);
  // Tuned on MI355X over the solver's shapes (rank-32 updates of the
  // inverses, leaf sweeps, merge products, top solve): all 3M.
  if (a.K <= 64) return launch<2, 1, true, 8, 3>(st, a, batch);
  if (M >= 1024 && N >= 1024 && a.K >= 512) return launch<2, 2, true, 16, 2>(st, a, batch);
  return launch<2, 1, true, 16, 2>(st, a, batch);
}

hipError_t cgemm(hipStream_t st, int opA, int opB, int M, int N, int K, float2 alpha, const float2* A, ll lda,
                 ll sA, const float2* B, ll ldb, ll sB, float2 beta, float2* C, ll ldc, ll sC, int batch) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  if (batch > 65535) return hipErrorInvalidValue;
  ArgsT<float> a{M, N, K < 0 ? 0 : K, opA, opB, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, beta, nullptr, 0,
                 0, 0, 1, 1};
  const bool rb = (beta.x != 0.0f || beta.y != 0.0f);
  KernelTimer kt(st, K_CGEMM, 8.0 * M * N * (double)a.K * batch,
                 8.0 * ((double)M * a.K + (double)a.K * N + (rb ? 2.0 : 1.0) * M * N) * batch);
  if (a.K <= 64) return launch_t<float, 2, 1, true, 8, 3>(st, a, batch);
  if (M >= 1024 && N >= 1024 && a.K >= 512) return launch_t<float, 2, 2, true, 16, 2>(st, a, batch);
  return launch_t<float, 2, 1, true, 16, 2>(st, a, batch);
}

}  // namespace hps
