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
#include <atomic>
#include <chrono>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

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
  int kchunk;      // split K: slice z of the grid covers [z kchunk, (z + 1) kchunk)
  ll sCz;          // split K: C offset of slice z
  const int* rmap; // optional: row r of C is stored at row rmap[r] (+ rpart if r >= rsplit)
  int rsplit;
  ll rpart;
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

template <typename T, int WM, int WN, bool M3, int TK, int WAVES, bool SK, bool DIV>
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
  // DIV: operands shared by groups of the batch (a separate instantiation:
  // the division changes the register allocation of the whole kernel)
  const T2* A = a.A + (DIV ? (ll)((int)blockIdx.y / a.adiv) : b) * a.sA;
  const T2* B = a.B + (DIV ? (ll)((int)blockIdx.y / a.bdiv) : b) * a.sB;
  // SK (split K): this workgroup covers K range [kb, ke) and writes slice z
  const int kb = SK ? (int)blockIdx.z * a.kchunk : 0;
  const int ke = SK ? ((kb + a.kchunk < a.K) ? kb + a.kchunk : a.K) : a.K;
  T2* C = a.C + b * a.sC + (SK ? (ll)blockIdx.z * a.sCz : 0);

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
  IOA::load(A, a.lda, a.M, ke, m0, kb, a_rows, a_conj, t, ra);
  IOB::load(B, a.ldb, a.N, ke, n0, kb, b_rows, b_conj, t, rb);
  const int nk = (ke - kb + TK - 1) / TK;
  for (int kt = 0; kt < nk; ++kt) {
    __syncthreads();
    IOA::store(Are, Aim, a_rows, t, ra);
    IOB::store(Bre, Bim, b_rows, t, rb);
    __syncthreads();
    if (kt + 1 < nk) {
      IOA::load(A, a.lda, a.M, ke, m0, kb + (kt + 1) * TK, a_rows, a_conj, t, ra);
      IOB::load(B, a.ldb, a.N, ke, n0, kb + (kt + 1) * TK, b_rows, b_conj, t, rb);
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

// Workgroups are dispatched round-robin over the 8 XCDs of the chip (the
// i-th one of a grid in linear order x, then y runs on XCD i % 8), and each
// XCD has its own L2.  The work item of workgroup i is renumbered so that
// every XCD takes a contiguous range of the grid's (tile, batch) items: the
// tiles of one small matrix, or neighbouring tiles of a large one, then share
// their operand panels in one L2 instead of fetching them on several XCDs.
constexpr unsigned NXCD = 8;
constexpr int GROUP_M = 8;  // row tiles per group in the single-matrix tile order
__device__ inline unsigned xcd_order(unsigned i, unsigned n) {
  const unsigned x = i % NXCD, k = i / NXCD, q = n / NXCD, r = n % NXCD;
  return x * q + (x < r ? x : r) + k;
}

// The FP64 kernel used by default.  It is kept as its own (non-template)
// source: the same loop written through the precision template above
// compiles to code that runs about 10% slower on MI355X (measured), so the
// template serves FP32, split-K and shared-operand calls only.
__device__ inline double2 ld_op64(const double2* p, bool conj) {
  double2 v = *p;
  if (conj) v.y = -v.y;
  return v;
}

// Loads / stores of a TR x TK tile of a matrix X viewed as rows x K: A as
// op(A) (M x K), B through the transpose of op(B) (N x K).  `contig` means
// consecutive rows are adjacent in memory, so threads run along the rows.
template <int TR, int TK>
struct TileIO64 {
  static constexpr int PER = TR * TK / NT;
  __device__ static void load(const double2* X, ll ld, int nrow, int ncol, int r0, int k0, bool contig,
                              bool conj, int t, double2* reg) {
    if (contig) {
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const int idx = t + j * NT;
        const int r = r0 + idx % TR, k = k0 + idx / TR;
        reg[j] = (r < nrow && k < ncol) ? ld_op64(X + (ll)r + (ll)k * ld, conj) : make_double2(0.0, 0.0);
      }
    } else {
#pragma unroll
      for (int j = 0; j < PER; ++j) {
        const int idx = t + j * NT;
        const int k = k0 + idx % TK, r = r0 + idx / TK;
        reg[j] = (r < nrow && k < ncol) ? ld_op64(X + (ll)k + (ll)r * ld, conj) : make_double2(0.0, 0.0);
      }
    }
  }
  __device__ static void store(double (*re)[TR + PAD], double (*im)[TR + PAD], bool contig, int t,
                               const double2* reg) {
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

// DB: two LDS buffers, so that the tile of the next K step is stored while
// the current one is multiplied (one barrier per step instead of two).
template <int WM, int WN, bool M3, int TK, int WAVES, bool DB = false>
__global__ __launch_bounds__(NT, WAVES) void zgemm_kernel(Args a) {
  constexpr int TM = 32 * WM, TN = 32 * WN, NB = DB ? 2 : 1;
  __shared__ double Are[NB][TK][TM + PAD], Aim[NB][TK][TM + PAD];
  __shared__ double Bre[NB][TK][TN + PAD], Bim[NB][TK][TN + PAD];

  const int tilesM = (a.M + TM - 1) / TM;
  const unsigned wg = xcd_order(blockIdx.x + blockIdx.y * gridDim.x, gridDim.x * gridDim.y);
  const unsigned tile = wg % gridDim.x;
  int m0, n0;
  const int tilesN = (int)gridDim.x / tilesM;
  if (tilesM > GROUP_M && tilesN >= 2 * GROUP_M) {
    // large matrices with many column tiles (the rank-W updates of the
    // large inverses, the coarse merge levels): groups of GROUP_M row tiles,
    // columns within a group, so that an XCD's contiguous range of tiles is a
    // band of rows (its A rows read once) and the tiles running together
    // share A and B panels
    const int per_group = GROUP_M * tilesN, g = (int)tile / per_group;
    const int first = g * GROUP_M, gsize = min(tilesM - first, GROUP_M), r = (int)tile % per_group;
    m0 = (first + r % gsize) * TM;
    n0 = (r / gsize) * TN;
  } else {
    m0 = (tile % tilesM) * TM;
    n0 = (tile / tilesM) * TN;
  }
  const ll b = wg / gridDim.x;
  const double2* A = a.A + b * a.sA;
  const double2* B = a.B + b * a.sB;
  double2* C = a.C + b * a.sC;

  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int wm = (w & 1) * 16 * WM, wn = (w >> 1) * 16 * WN;
  const int lr = lane & 15, lk = lane >> 4;
  const bool a_rows = a.opA == OP_N, a_conj = a.opA == OP_C;
  const bool b_rows = a.opB != OP_N, b_conj = a.opB == OP_C;

  // M3: p1 = ArBr, p2 = AiBi, p3 = (Ar+Ai)(Br+Bi); otherwise p1 = Re, p3 = Im
  v4d p1[WM][WN], p2[WM][WN], p3[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      p1[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
      p2[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
      p3[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    }

  double2 ra[TileIO64<TM, TK>::PER], rb[TileIO64<TN, TK>::PER];
  TileIO64<TM, TK>::load(A, a.lda, a.M, a.K, m0, 0, a_rows, a_conj, t, ra);
  TileIO64<TN, TK>::load(B, a.ldb, a.N, a.K, n0, 0, b_rows, b_conj, t, rb);
  const int nk = (a.K + TK - 1) / TK;
  if constexpr (DB) {
    TileIO64<TM, TK>::store(Are[0], Aim[0], a_rows, t, ra);
    TileIO64<TN, TK>::store(Bre[0], Bim[0], b_rows, t, rb);
    __syncthreads();
  }
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = DB ? (kt & 1) : 0;
    if constexpr (!DB) {
      __syncthreads();
      TileIO64<TM, TK>::store(Are[0], Aim[0], a_rows, t, ra);
      TileIO64<TN, TK>::store(Bre[0], Bim[0], b_rows, t, rb);
      __syncthreads();
    }
    if (kt + 1 < nk) {
      TileIO64<TM, TK>::load(A, a.lda, a.M, a.K, m0, (kt + 1) * TK, a_rows, a_conj, t, ra);
      TileIO64<TN, TK>::load(B, a.ldb, a.N, a.K, n0, (kt + 1) * TK, b_rows, b_conj, t, rb);
    }
#pragma unroll
    for (int ks = 0; ks < TK / 4; ++ks) {
      const int kk = ks * 4 + lk;
      double ar[WM], ai[WM], br[WN], bi[WN];
#pragma unroll
      for (int i = 0; i < WM; ++i) {
        ar[i] = Are[cur][kk][wm + 16 * i + lr];
        ai[i] = Aim[cur][kk][wm + 16 * i + lr];
      }
#pragma unroll
      for (int j = 0; j < WN; ++j) {
        br[j] = Bre[cur][kk][wn + 16 * j + lr];
        bi[j] = Bim[cur][kk][wn + 16 * j + lr];
      }
      if constexpr (M3) {
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
          for (int j = 0; j < WN; ++j) {
            p1[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], p1[i][j], 0, 0, 0);
            p2[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], bi[j], p2[i][j], 0, 0, 0);
            p3[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i] + ai[i], br[j] + bi[j], p3[i][j], 0,
                                                            0, 0);
          }
      } else {
#pragma unroll
        for (int i = 0; i < WM; ++i)
#pragma unroll
          for (int j = 0; j < WN; ++j) {
            p1[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], br[j], p1[i][j], 0, 0, 0);
            p1[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ai[i], bi[j], p1[i][j], 0, 0, 0);
            p3[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i], bi[j], p3[i][j], 0, 0, 0);
            p3[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ai[i], br[j], p3[i][j], 0, 0, 0);
          }
      }
    }
    if constexpr (DB) {
      // the other buffer was last read in step kt - 1, before the previous
      // barrier
      if (kt + 1 < nk) {
        TileIO64<TM, TK>::store(Are[cur ^ 1], Aim[cur ^ 1], a_rows, t, ra);
        TileIO64<TN, TK>::store(Bre[cur ^ 1], Bim[cur ^ 1], b_rows, t, rb);
      }
      __syncthreads();
    }
  }

  // D layout of the 16x16x4 f64 MFMA: item r of a lane is row lane/16 + 4 r,
  // column lane % 16.
  const bool use_beta = (a.beta.x != 0.0 || a.beta.y != 0.0);
  const int* rp = a.rpos ? a.rpos + b * a.srp : nullptr;
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) {
      const int col = n0 + wn + 16 * j + lr;
      if (col >= a.N) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + 16 * i + lk + 4 * r;
        if (row >= a.M) continue;
        const double xr = M3 ? p1[i][j][r] - p2[i][j][r] : p1[i][j][r];
        const double xi = M3 ? p3[i][j][r] - p1[i][j][r] - p2[i][j][r] : p3[i][j][r];
        double2 v = make_double2(a.alpha.x * xr - a.alpha.y * xi, a.alpha.x * xi + a.alpha.y * xr);
        const ll roff = a.rmap ? (ll)a.rmap[row] + (row >= a.rsplit ? a.rpart : 0) : (ll)row;
        double2* pc = C + roff + (ll)col * a.ldc;
        if (use_beta && !(rp && rp[row] >= a.plo && rp[row] < a.phi)) {
          const double2 c = *pc;
          v.x += a.beta.x * c.x - a.beta.y * c.y;
          v.y += a.beta.x * c.y + a.beta.y * c.x;
        }
        *pc = v;
      }
    }
}

template <typename T, int WM, int WN, bool M3, int TK, int WAVES, bool SK = false, bool DIV = false>
hipError_t launch_t(hipStream_t st, const ArgsT<T>& a, int batch, int splits = 1) {
  constexpr int TM = 32 * WM, TN = 32 * WN;
  const ll tiles = (ll)((a.M + TM - 1) / TM) * ((a.N + TN - 1) / TN);
  if (tiles > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((gemm_kernel<T, WM, WN, M3, TK, WAVES, SK, DIV>),
                     dim3((unsigned)tiles, (unsigned)batch, splits), dim3(NT), 0, st, a);
  return hipGetLastError();
}

// C = alpha sum_z W[z] + beta C (rows in the overwrite range take beta = 0);
// W[z] holds batch consecutive M x N blocks.
__global__ void k_splitk_reduce(const double2* W, int splits, ll sz, int M, int N, double2 alpha, double2 beta,
                                double2* C, ll ldc, ll sC, const int* rpos, ll srp, int plo, int phi,
                                const int* rmap, int rsplit, ll rpart, int batch) {
  const ll per = (ll)M * N, total = per * batch;
  const bool use_beta = (beta.x != 0.0 || beta.y != 0.0);
  for (ll idx = blockIdx.x * (ll)NT + threadIdx.x; idx < total; idx += (ll)gridDim.x * NT) {
    const ll b = idx / per;
    const int e = (int)(idx % per);
    const int i = e % M, j = e / M;
    double2 acc = W[idx];
    for (int z = 1; z < splits; ++z) {
      const double2 w = W[idx + z * sz];
      acc.x += w.x;
      acc.y += w.y;
    }
    double2 v = make_double2(alpha.x * acc.x - alpha.y * acc.y, alpha.x * acc.y + alpha.y * acc.x);
    const ll roff = rmap ? (ll)rmap[i] + (i >= rsplit ? rpart : 0) : (ll)i;
    double2* pc = C + b * sC + roff + (ll)j * ldc;
    const int* rp = rpos ? rpos + b * srp : nullptr;
    if (use_beta && !(rp && rp[i] >= plo && rp[i] < phi)) {
      const double2 c = *pc;
      v.x += beta.x * c.x - beta.y * c.y;
      v.y += beta.x * c.y + beta.y * c.x;
    }
    *pc = v;
  }
}

// Split-K workspace, one per stream (calls on one stream are ordered).
struct SplitWs {
  hipStream_t st;
  void* p;
  size_t bytes;
};
std::mutex g_ws_mu;
std::vector<SplitWs> g_ws;

hipError_t splitk_workspace(hipStream_t st, size_t bytes, void** out) {
  std::lock_guard<std::mutex> lk(g_ws_mu);
  for (auto& w : g_ws)
    if (w.st == st) {
      if (w.bytes < bytes) {
        HPS_HIP_TRY(hipStreamSynchronize(st));
        HPS_HIP_TRY(hipFree(w.p));
        w.p = nullptr;
        w.bytes = 0;
        HPS_HIP_TRY(hipMalloc(&w.p, bytes));
        w.bytes = bytes;
      }
      *out = w.p;
      return hipSuccess;
    }
  void* p = nullptr;
  HPS_HIP_TRY(hipMalloc(&p, bytes));
  g_ws.push_back({st, p, bytes});
  *out = p;
  return hipSuccess;
}

// Number of K slices for a call with fewer output tiles than compute units
// and a long K: about two workgroups per compute unit, slices of at least
// 512 (a split costs a reduction pass, so shapes that already fill the chip
// are left alone).
// Products with at most 32 columns (sweeps with few right-hand sides) are
// bound by streaming A, so they take thinner slices (at least 256) and aim at
// about 2048 workgroups to keep more loads in flight.
int choose_splits(int M, int N, int K, int batch) {
  const ll tiles = (ll)((M + 63) / 64) * ((N + 31) / 32) * batch;
  const bool skinny = N <= 32;
  const ll target = skinny ? 2048 : 512, slice = skinny ? 256 : 512, most = skinny ? 32 : 16;
  if (tiles >= (skinny ? 1024 : 256) || K < 1024) return 1;
  ll s = (target + tiles - 1) / tiles;
  if (s > K / slice) s = K / slice;
  if (s > most) s = most;
  return s < 2 ? 1 : (int)s;
}
template <int WM, int WN, bool M3, int TK, int WAVES, bool DB = false>
hipError_t launch(hipStream_t st, const Args& a, int batch) {
  constexpr int TM = 32 * WM, TN = 32 * WN;
  const ll tiles = (ll)((a.M + TM - 1) / TM) * ((a.N + TN - 1) / TN);
  if (tiles > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((zgemm_kernel<WM, WN, M3, TK, WAVES, DB>), dim3((unsigned)tiles, (unsigned)batch), dim3(NT),
                     0, st, a);
  return hipGetLastError();
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
    launch<2, 1, true, 16, 2, true>,   // 13
    launch<2, 2, true, 16, 2, true>,   // 14
    launch<2, 1, true, 8, 3, true>,    // 15
    launch<2, 2, true, 16, 1, true>,   // 16
    launch<1, 2, true, 8, 3>,          // 17
    launch<1, 1, true, 8, 4>,          // 18
};
constexpr int NVARIANT = sizeof(VARIANTS) / sizeof(VARIANTS[0]);

// HPS_ZGEMM_TRACE=<file> appends one line per call (M N K batch opA opB
// beta!=0 rowmask) for offline analysis of the call shapes.
// HPS_ZGEMM_TRACE=<file>: one line per call (sizes, batch, ops, beta != 0,
// row mask / row map, tile variant; -1 split-K, -2 shared-operand path).
void trace_call(const Args& a, int batch, int variant) {
  static FILE* f = nullptr;
  static int state = 0;
  if (state == 0) {
    const char* e = std::getenv("HPS_ZGEMM_TRACE");
    f = (e && *e) ? std::fopen(e, "a") : nullptr;
    state = 1;
  }
  if (!f) return;
  const bool rb = (a.beta.x != 0.0 || a.beta.y != 0.0);
  std::fprintf(f, "%d %d %d %d %d %d %d %d %d\n", a.M, a.N, a.K, batch, a.opA, a.opB, rb ? 1 : 0,
               (a.rpos ? 1 : 0) + (a.rmap ? 2 : 0), variant);
  std::fflush(f);
}

std::atomic<int> g_force{-2};  // -2: not read from the environment yet

thread_local bool g_noalloc = false;  // NoAllocScope active on this thread

int forced_variant() {
  int v = g_force.load();
  if (v == -2) {
    const char* e = std::getenv("HPS_ZGEMM_VARIANT");
    v = -1;
    if (e && *e) {
      const int x = std::atoi(e);
      if (x >= 0 && x < NVARIANT) v = x;
    }
    int expect = -2;
    g_force.compare_exchange_strong(expect, v);
    v = g_force.load();
  }
  return v;
}

// ---- tile-shape autotuning ----
// Candidates are 3M variants only: they all accumulate the K products of an
// output element in the same order, so the choice never changes a result.
constexpr int TUNE_CAND[] = {12, 8, 11, 1, 10, 9, 17, 18};
constexpr int NCAND = sizeof(TUNE_CAND) / sizeof(TUNE_CAND[0]);

struct TuneKey {
  int M, N, K, batch, opA, opB, beta, mask;
  ll lda, ldb, ldc, sA, sB, sC;
  bool operator<(const TuneKey& o) const {
    return std::tie(M, N, K, batch, opA, opB, beta, mask, lda, ldb, ldc, sA, sB, sC) <
           std::tie(o.M, o.N, o.K, o.batch, o.opA, o.opB, o.beta, o.mask, o.lda, o.ldb, o.ldc, o.sA, o.sB, o.sC);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tuned;
std::atomic<int> g_tune_mode{0};
double g_tune_seconds = 0.0;

// Copies the M x N output block of every batch entry of a strided C to a
// packed buffer (dir 0) or back (dir 1).  Only those elements: other
// columns of the same arrays may be written concurrently by another stream
// (the look-ahead updates of the inverse).
__global__ void k_block_copy(double2* C, ll ldc, ll sC, int M, int N, int batch, double2* buf, int dir) {
  const ll per = (ll)M * N, total = per * batch;
  for (ll e = (ll)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (ll)gridDim.x * blockDim.x) {
    const ll b = e / per, r = e % per, i = r % M, j = r / M;
    double2* c = C + b * sC + j * ldc + i;
    if (dir == 0)
      buf[e] = *c;
    else
      *c = buf[e];
  }
}

hipError_t block_copy(hipStream_t st, const Args& a, int batch, double2* buf, int dir) {
  const ll total = (ll)a.M * a.N * batch;
  ll blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_block_copy, dim3((unsigned)blocks), dim3(256), 0, st, a.C, a.ldc, a.sC, a.M, a.N, batch, buf,
                     dir);
  return hipGetLastError();
}

// Times every candidate on the call's own operands (the output block is saved
// first and restored before each trial and at the end) and returns the index
// of the fastest in VARIANTS.  Synchronises the stream.
hipError_t tune_shape(hipStream_t st, const Args& a, int batch, int* best) {
  const auto t0 = std::chrono::steady_clock::now();
  const bool rb = (a.beta.x != 0.0 || a.beta.y != 0.0);
  const size_t bytes = (size_t)a.M * a.N * batch * sizeof(double2);
  void* save = nullptr;
  hipEvent_t ev[2 * NCAND];
  for (auto& e : ev) e = nullptr;
  hipError_t err = hipSuccess;
  float ms[NCAND];
  for (int i = 0; i < NCAND; ++i) ms[i] = 1e30f;
  do {
    if (rb) {
      if ((err = hipMalloc(&save, bytes)) != hipSuccess) break;
      if ((err = block_copy(st, a, batch, (double2*)save, 0)) != hipSuccess) break;
    }
    for (auto& e : ev)
      if ((err = hipEventCreate(&e)) != hipSuccess) break;
    if (err != hipSuccess) break;
    for (int round = 0; round < 3 && err == hipSuccess; ++round) {
      for (int i = 0; i < NCAND && err == hipSuccess; ++i) {
        if (rb && (err = block_copy(st, a, batch, (double2*)save, 1)) != hipSuccess) break;
        if ((err = hipEventRecord(ev[2 * i], st)) != hipSuccess) break;
        if ((err = VARIANTS[TUNE_CAND[i]](st, a, batch)) != hipSuccess) break;
        err = hipEventRecord(ev[2 * i + 1], st);
      }
      if (err != hipSuccess || round == 0) continue;  // round 0 warms up
      if ((err = hipStreamSynchronize(st)) != hipSuccess) break;
      for (int i = 0; i < NCAND; ++i) {
        float x = 0.0f;
        if ((err = hipEventElapsedTime(&x, ev[2 * i], ev[2 * i + 1])) != hipSuccess) break;
        if (x < ms[i]) ms[i] = x;
      }
    }
    if (err == hipSuccess && rb) err = block_copy(st, a, batch, (double2*)save, 1);
    if (err == hipSuccess) err = hipStreamSynchronize(st);
  } while (0);
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  if (save) {
    (void)hipStreamSynchronize(st);
    (void)hipFree(save);
  }
  int b = 0;
  for (int i = 1; i < NCAND; ++i)
    if (ms[i] < ms[b]) b = i;
  *best = TUNE_CAND[b];
  g_tune_seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return err;
}

// Fixed rules, from the autotuner's choices on MI355X over the solver's
// shapes (with the XCD-contiguous work order): 32 x 64 tiles with K step 8
// and three waves per SIMD, 32 x 32 tiles with four waves per SIMD for
// products of at most 64 columns (the rank-32/64 updates of the inverses).
int rule_variant(int M, int N, int K) {
  (void)M;
  (void)K;
  return N <= 64 ? 18 : 17;
}

}  // namespace

NoAllocScope::NoAllocScope() : prev_(g_noalloc) { g_noalloc = true; }
NoAllocScope::~NoAllocScope() { g_noalloc = prev_; }
bool no_alloc_active() { return g_noalloc; }

void gemm_set_tuning(int mode, int force) {
  g_tune_mode.store(mode);
  forced_variant();
  g_force.store(force >= 0 && force < NVARIANT ? force : -1);
}

void gemm_tuning_info(int* shapes, double* seconds) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (shapes) *shapes = (int)g_tuned.size();
  if (seconds) *seconds = g_tune_seconds;
}

int gemm_variant_count() { return NVARIANT; }

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
                    plo, phi, batch, nullptr, 0, 0);
}

hipError_t zgemm_rowmap(hipStream_t st, int opA, int opB, int M, int N, int K, double2 alpha, const double2* A,
                        ll lda, ll sA, const double2* B, ll ldb, ll sB, double2 beta, double2* C, ll ldc, ll sC,
                        const int* rmap, int rsplit, ll rpart, int batch) {
  return zgemm_full(st, opA, opB, M, N, K, alpha, A, lda, sA, 1, B, ldb, sB, 1, beta, C, ldc, sC, nullptr, 0, 0,
                    0, batch, rmap, rsplit, rpart);
}

hipError_t zgemm_div(hipStream_t st, int opA, int opB, int M, int N, int K, double2 alpha,
                     const double2* A, ll lda, ll sA, int adiv, const double2* B, ll ldb, ll sB, int bdiv,
                     double2 beta, double2* C, ll ldc, ll sC, int batch) {
  return zgemm_full(st, opA, opB, M, N, K, alpha, A, lda, sA, adiv, B, ldb, sB, bdiv, beta, C, ldc, sC,
                    nullptr, 0, 0, 0, batch, nullptr, 0, 0);
}

hipError_t zgemm_full(hipStream_t st, int opA, int opB, int M, int N, int K, double2 alpha,
                      const double2* A, ll lda, ll sA, int adiv, const double2* B, ll ldb, ll sB, int bdiv,
                      double2 beta, double2* C, ll ldc, ll sC, const int* rpos, ll srp, int plo, int phi,
                      int batch, const int* rmap, int rsplit, ll rpart) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  if (batch > 65535 || adiv < 1 || bdiv < 1) return hipErrorInvalidValue;
  // an operand shared by the whole batch is a stride-0 broadcast: the default
  // kernel (tuned, faster than the shared-operand template) serves it
  if (adiv >= batch) {
    adiv = 1;
    sA = 0;
  }
  if (bdiv >= batch) {
    bdiv = 1;
    sB = 0;
  }
  if (rmap && (adiv != 1 || bdiv != 1)) return hipErrorInvalidValue;
  Args a{M, N, K < 0 ? 0 : K, opA, opB, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, beta, rpos, srp, plo, phi,
         adiv, bdiv, K < 0 ? 0 : K, 0, rmap, rsplit, rpart};
  const bool rb = (beta.x != 0.0 || beta.y != 0.0);
  KernelTimer kt(st, K_ZGEMM, 8.0 * M * N * (double)a.K * batch,
                 16.0 * ((double)M * a.K + (double)a.K * N + (rb ? 2.0 : 1.0) * M * N) * batch);
  if (adiv != 1 || bdiv != 1) {
    trace_call(a, batch, -2);
    if (a.K <= 64) return launch_t<double, 2, 1, true, 8, 3, false, true>(st, a, batch);
    return launch_t<double, 2, 1, true, 16, 2, false, true>(st, a, batch);
  }
  const int fv = forced_variant();
  if (fv >= 0) {
    trace_call(a, batch, fv);
    return VARIANTS[fv](st, a, batch);
  }
  const int splits = g_noalloc ? 1 : choose_splits(M, N, a.K, batch);
  if (splits > 1) {
    trace_call(a, batch, -1);
    // partial products of K slices into the workspace, then one reduction
    const ll per = (ll)M * N * batch;
    void* ws = nullptr;
    HPS_HIP_TRY(splitk_workspace(st, (size_t)per * splits * sizeof(double2), &ws));
    Args p = a;
    p.C = (double2*)ws;
    p.ldc = M;
    p.sC = (ll)M * N;
    p.alpha = make_double2(1.0, 0.0);
    p.beta = make_double2(0.0, 0.0);
    p.rpos = nullptr;
    p.rmap = nullptr;
    p.kchunk = ((a.K + splits - 1) / splits + 15) / 16 * 16;
    p.sCz = per;
    const int used = (a.K + p.kchunk - 1) / p.kchunk;
    HPS_HIP_TRY((launch_t<double, 2, 1, true, 16, 2, true>(st, p, batch, used)));
    ll blocks = (per + NT - 1) / NT;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_splitk_reduce, dim3((unsigned)blocks), dim3(NT), 0, st, (const double2*)ws, used, per, M,
                       N, alpha, beta, C, ldc, sC, rpos, srp, plo, phi, a.rmap, a.rsplit, a.rpart, batch);
    return hipGetLastError();
  }
  if (g_tune_mode.load() == 1 && !(rmap && rb) && !g_noalloc) {
    const TuneKey key{M, N, a.K, batch, opA, opB, rb ? 1 : 0, (rpos ? 1 : 0) + (rmap ? 2 : 0), lda, ldb, ldc,
                      sA, sB, sC};
    int v = -1;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tuned.find(key);
      if (it != g_tuned.end()) v = it->second;
    }
    if (v < 0) {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      HPS_HIP_TRY(tune_shape(st, a, batch, &v));
      g_tuned[key] = v;
    }
    trace_call(a, batch, v);
    return VARIANTS[v](st, a, batch);
  }
  const int v = rule_variant(M, N, a.K);
  trace_call(a, batch, v);
  return VARIANTS[v](st, a, batch);
}

hipError_t cgemm(hipStream_t st, int opA, int opB, int M, int N, int K, float2 alpha, const float2* A, ll lda,
                 ll sA, const float2* B, ll ldb, ll sB, float2 beta, float2* C, ll ldc, ll sC, int batch) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  if (batch > 65535) return hipErrorInvalidValue;
  ArgsT<float> a{M, N, K < 0 ? 0 : K, opA, opB, A, lda, sA, B, ldb, sB, C, ldc, sC, alpha, beta, nullptr, 0,
                 0, 0, 1, 1, K < 0 ? 0 : K, 0};
  const bool rb = (beta.x != 0.0f || beta.y != 0.0f);
  KernelTimer kt(st, K_CGEMM, 8.0 * M * N * (double)a.K * batch,
                 8.0 * ((double)M * a.K + (double)a.K * N + (rb ? 2.0 : 1.0) * M * N) * batch);
  if (a.K <= 64) return launch_t<float, 2, 1, true, 8, 3>(st, a, batch);
  if (M >= 1024 && N >= 1024 && a.K >= 512) return launch_t<float, 2, 2, true, 16, 2>(st, a, batch);
  return launch_t<float, 2, 1, true, 16, 2>(st, a, batch);
}

}  // namespace hps
