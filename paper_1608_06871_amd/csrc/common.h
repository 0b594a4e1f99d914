// Internal declarations shared by the HIP translation units of libhps.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

typedef long long ll;

namespace hps {

enum Op { OP_N = 0, OP_T = 1, OP_C = 2 };

// Batched complex FP64 GEMM: C_b = alpha op(A_b) op(B_b) + beta C_b for
// b < batch, column-major operands with leading dimensions ld* and batch
// strides s* (a stride of 0 broadcasts one operand to the whole batch).
// beta == 0 never reads C.
hipError_t zgemm(hipStream_t st, int opA, int opB, int M, int N, int K, double2 alpha,
                 const double2* A, ll lda, ll sA, const double2* B, ll ldb, ll sB,
                 double2 beta, double2* C, ll ldc, ll sC, int batch);

// zgemm in which the rows r of C_b with plo <= rpos[b * srp + r] < phi are
// overwritten (beta taken as 0 there), the others updated with beta.
hipError_t zgemm_rowmask(hipStream_t st, int opA, int opB, int M, int N, int K, double2 alpha,
                         const double2* A, ll lda, ll sA, const double2* B, ll ldb, ll sB,
                         double2 beta, double2* C, ll ldc, ll sC, const int* rpos, ll srp,
                         int plo, int phi, int batch);

// zgemm whose A / B operand for batch entry b is number b / adiv (b / bdiv):
// one operand shared by consecutive groups of the batch.
hipError_t zgemm_div(hipStream_t st, int opA, int opB, int M, int N, int K, double2 alpha,
                     const double2* A, ll lda, ll sA, int adiv, const double2* B, ll ldb, ll sB,
                     int bdiv, double2 beta, double2* C, ll ldc, ll sC, int batch);
// zgemm whose output row r is stored at row rmap[r] of C, plus rpart
// elements for r >= rsplit (a product scattered into two vectors, e.g. the
// children of a merge).
hipError_t zgemm_rowmap(hipStream_t st, int opA, int opB, int M, int N, int K, double2 alpha, const double2* A,
                        ll lda, ll sA, const double2* B, ll ldb, ll sB, double2 beta, double2* C, ll ldc, ll sC,
                        const int* rmap, int rsplit, ll rpart, int batch);
// All of the above.
hipError_t zgemm_full(hipStream_t st, int opA, int opB, int M, int N, int K, double2 alpha,
                      const double2* A, ll lda, ll sA, int adiv, const double2* B, ll ldb, ll sB,
                      int bdiv, double2 beta, double2* C, ll ldc, ll sC, const int* rpos, ll srp,
                      int plo, int phi, int batch, const int* rmap, int rsplit, ll rpart);

// FP32 complex GEMM (same conventions as zgemm; FP32 MFMA, FP32 accumulation).
hipError_t cgemm(hipStream_t st, int opA, int opB, int M, int N, int K, float2 alpha,
                 const float2* A, ll lda, ll sA, const float2* B, ll ldb, ll sB, float2 beta,
                 float2* C, ll ldc, ll sC, int batch);
// Tile-shape selection of the complex FP64 GEMM (process-wide): mode 0 fixed
// rules, 1 autotuning per distinct shape; force >= 0 pins one variant.
void gemm_set_tuning(int mode, int force);
void gemm_tuning_info(int* shapes, double* seconds);
int gemm_variant_count();

// Blocking of zinv for orders above 512 and butterfly-transformed orders
// below (process-wide): -1 by size (look-ahead while the batch fits the
// last-level cache, and below order 512 for at most 32 matrices), 0
// recursive, 1 look-ahead.
void zinv_set_blocking(int mode);

// Pivoting of zinv (process-wide): -1 butterfly transform + pivot-free
// elimination for orders of at least 224 (checked on probe vectors, pivoted
// fallback), 0 always pivoted, 1 butterfly for every order that is a multiple
// of 4; tol >= 0 sets the probe-check tolerance.
void zinv_set_pivoting(int mode, double tol);
void zinv_pivoting_info(long* calls, long* fallbacks, double* max_err);

// While an RbtDeferScope lives on a thread, butterfly inverses (zinv) do not
// synchronise for their probe check: each folds its verdict into *flag_dev
// (|= 1 on a failed check; the failed matrices' zero-pivot flags in info are
// cleared) and its largest probe error into *maxerr_dev (bit pattern of a
// non-negative double, updated by atomicMax); both must start at zero.  The
// caller reads them after its own synchronisation, reports them with
// zinv_note_deferred, and redoes its work inside an RbtOffScope (pivoted
// path only) when the flag is set.
class RbtDeferScope {
 public:
  RbtDeferScope(int* flag_dev, unsigned long long* maxerr_dev);
  ~RbtDeferScope();
  RbtDeferScope(const RbtDeferScope&) = delete;
  RbtDeferScope& operator=(const RbtDeferScope&) = delete;

 private:
  int* prev_flag_;
  unsigned long long* prev_err_;
};
class RbtOffScope {
 public:
  RbtOffScope();
  ~RbtOffScope();
  RbtOffScope(const RbtOffScope&) = delete;
  RbtOffScope& operator=(const RbtOffScope&) = delete;

 private:
  bool prev_;
};
void zinv_note_deferred(double max_err, bool fallback);

// Workspace sizes (bytes) for zinv with matrices of order n in batches of `batch`.
size_t zinv_workspace(int n, int batch);
size_t zinv_perm_workspace(int n, int batch);

// Batched inverse by swap-free Gauss-Jordan elimination with partial
// pivoting (recursive column blocking: panel eliminations and GEMM updates).  `work`
// (order n, lda, stride sA) is destroyed; the inverse is written to `out`.
// info[b] (device, one int per matrix) is set non-zero when a zero pivot was
// met.  `ws` must hold zinv_workspace(n, batch) bytes.
hipError_t zinv(hipStream_t st, int n, double2* work, ll lda, ll sA, double2* out, ll ldo,
                ll sO, int batch, void* ws, int* info);

// zinv_perm never takes the butterfly path.
// zinv without the final permutation: `work` is left holding M with
// inv[c][k] = M[sig[c]][pos[k]] for every matrix of the batch; sig and pos
// (batch x n ints each, in ws) are returned for the caller's own gathers and
// stay valid until ws is reused.
hipError_t zinv_perm(hipStream_t st, int n, double2* work, ll lda, ll sA, int batch, void* ws, int* info,
                     const int** sig, const int** pos);

// While a NoAllocScope lives on a thread, the library calls made from that
// thread allocate no device memory and create no HIP objects: GEMMs take the
// fixed tile rules (no autotuning trials, which save their output in a new
// buffer) and never split K (the split-K workspace is allocated on first use
// per stream), and the launch profiler records nothing (it creates events).
class NoAllocScope {
 public:
  NoAllocScope();
  ~NoAllocScope();
  NoAllocScope(const NoAllocScope&) = delete;
  NoAllocScope& operator=(const NoAllocScope&) = delete;

 private:
  bool prev_;
};
bool no_alloc_active();

// Allocation-free batched inverse for n <= 512 with its workspace in the
// library's static device scratch array (one per GPU, kept until the process
// ends).  Enqueued on st; status_dev (device, one int) receives 1 if a zero
// pivot was met, else 0.  Returns hipErrorInvalidValue when the workspace
// does not fit the array (see zinv_noalloc_bytes).
hipError_t zinv_noalloc(hipStream_t st, int n, double2* A, double2* inv, int batch, int* status_dev);
// Scratch bytes zinv_noalloc needs, and the size of the scratch array.
size_t zinv_noalloc_bytes(int n, int batch);
size_t zinv_noalloc_capacity();
// Device address of this GPU's scratch array's status slot (for the host
// to read a synchronous call's status); resolved once per device.
hipError_t zinv_noalloc_status_slot(int** out);

// Kernel classes of the optional launch profiler.
enum KernelKind {
  K_ZGEMM = 0,
  K_CGEMM,      // FP32 complex GEMM (mixed precision)
  K_GJ_PANEL,   // Gauss-Jordan panel elimination (register / LDS / global panel)
  K_TP_SELECT,  // tournament pivot selection (leaves and reductions)
  K_TP_EXCH,   // panel exchange of the tournament path
  K_GJ_PERM,
  K_MOVE,
  K_LEAF,
  K_POINT,
  KIND_COUNT
};

// Stage tags of the launch profiler (process-wide: the stage of the library
// call that is issuing kernels).
enum Phase { PH_OTHER = 0, PH_LEAF, PH_MERGE, PH_TOP, PH_SOLVE, PH_FAR, PH_JVP, PH_VJP, PHASE_COUNT };
void profile_set_phase(int phase);
// True while the launch profiler records (its events must not be captured).
bool profile_active();

// RAII: when profiling is on, records HIP events around the kernel launched
// inside its scope, with that launch's algorithmic flops and bytes.
class KernelTimer {
 public:
  KernelTimer(hipStream_t st, int kind, double flops, double bytes);
  ~KernelTimer();
  KernelTimer(const KernelTimer&) = delete;
  KernelTimer& operator=(const KernelTimer&) = delete;

 private:
  hipStream_t st_;
  long idx_;
};

}  // namespace hps

#define HPS_HIP_TRY(expr)                            \
  do {                                               \
    hipError_t _e = (expr);                          \
    if (_e != hipSuccess) return _e;                 \
  } while (0)
