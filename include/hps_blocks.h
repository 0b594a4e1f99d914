/*
 * hps_blocks.h - the building blocks of libhps, exposed for testing,
 * measurement and callers that need them on their own: dense batched complex
 * FP64 GEMM and matrix inverses (the kernels every stage of the solver in
 * hps.h is made of), an allocation-free inverse, the host-side boundary
 * operators of the exterior relation, GEMM tile tuning and the launch
 * profiler.  Status codes and hps_opts come from hps.h.
 */
#ifndef HPS_BLOCKS_H_
#define HPS_BLOCKS_H_

#include "hps.h"

#ifdef __cplusplus
extern "C" {
#endif

/* ---- host-side operators of the exterior relation (Remark in Section 2) ---- */

/* Host-only (no device work): the single- and double-layer matrices S and K
 * (row-major complex128 [nb][nb], nb = 4 nleaf (p-2)) of hps_set_wavenumber
 * for the geometry in *opts at wavenumber k, in the library's root order of
 * the outer-boundary nodes, whose coordinates go to xy_host ([nb][2], may be
 * NULL). */
hps_status hps_boundary_operators(const hps_opts* opts, double k, double* xy_host, double* S_host,
                                  double* K_host);

/* Host-only: the operators HPS_EXT_BURTON_MILLER adds, same layout and order
 * as hps_boundary_operators: Kp_host = K' (adjoint double layer,
 * Kp[i][j] = int dG/dn_x(x_i, y) ell_j(y) ds) and T_host = T (hypersingular,
 * the normal derivative at x_i of the double layer of ell_j, by Maue's
 * identity: tangential derivative of the single layer of d ell_j / d sigma,
 * including the interpolant's jumps at panel ends, plus
 * k^2 (n_i . n_j) S[i][j]).  HPS_EINVAL for bad options or k <= 0. */
hps_status hps_combined_field_operators(const hps_opts* opts, double k, double* Kp_host, double* T_host);

/* ---- dense building blocks ---- */

/* Batched complex GEMM C_b = alpha op(A_b) op(B_b) + beta C_b, b < batch,
 * column-major; op: 0 = none, 1 = transpose, 2 = conjugate transpose.
 * alpha/beta are (re, im) pairs on the host; strides are in elements
 * (0 broadcasts).  Enqueued on `stream`. */
hps_status hps_zgemm(void* stream, int opA, int opB, int M, int N, int K, const double* alpha,
                     const double* A, int64_t lda, int64_t strideA, const double* B, int64_t ldb,
                     int64_t strideB, const double* beta, double* C, int64_t ldc, int64_t strideC,
                     int batch);

/* Batched inverse of n x n complex matrices (column-major, leading dimension
 * n, contiguous batch) by Gauss-Jordan elimination with partial pivoting:
 * inv = A^{-1}; A is destroyed.  Synchronous; HPS_ESINGULAR on a zero
 * pivot.  Allocates its own workspace. */
hps_status hps_zinv(void* stream, int n, int batch, double* A, double* inv);

/* hps_zinv without any device allocation, for callers that cannot allocate
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): the workspace lives in the library's static device scratch
 * array of HPS_NOALLOC_SCRATCH_BYTES (one per GPU, held until the process
 * ends); no GEMM autotuning or split-K runs inside the call.
 *   Limits: n <= 512, and the workspace (about batch * (n^2/4 + n) * 16
 *   bytes) must fit the array, else HPS_EINVAL before any launch; e.g.
 *   n = 512: batch <= 63, n = 448: <= 83, n = 252: <= 262, n = 128: <= 1008.
 *   A: destroyed; inv: the inverses (both device, column-major, leading
 *   dimension n, contiguous batch), as hps_zinv.
 *   status_dev == NULL: synchronous, returns HPS_ESINGULAR on a zero pivot;
 *   status_dev != NULL (device, one int): enqueued on `stream` only, the int
 *   receives 1 on a zero pivot, else 0.
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on one GPU (different streams, or host threads) race and must be
 * serialised by the caller.  The array keeps the last call's contents; each
 * call clears what it needs itself. */
#define HPS_NOALLOC_SCRATCH_BYTES (64LL << 20)
hps_status hps_zinv_noalloc(void* stream, int n, int batch, double* A, double* inv, int* status_dev);

/* Column blocking of the inverses of order above 512, and of the
 * butterfly-transformed ones (pivot-free panels, order >= 224) below it
 * (hps_zinv and the factorisation's W and Z inverses), process-wide; a
 * performance choice, both give the inverse to rounding (the merges and the
 * top of the Section 2 direct solver only use the products with W^{-1} and
 * Z^{-1}):
 *   mode 1: right-looking with one panel of look-ahead (the next panel's
 *           pivot search overlaps the update of the other columns on a
 *           second stream);
 *   mode 0: recursive column blocking (fewer, larger GEMM updates);
 *   mode -1 (default): mode 1 while the batch of matrices fits the 256 MB
 *           last-level cache (batch * n * n * 16 bytes) and, below order
 *           512, holds at most 32 matrices; else mode 0.
 * HPS_ZINV_LOOKAHEAD = 0 / 1 in the environment sets the initial mode.
 * HPS_EINVAL for other modes. */
hps_status hps_zinv_blocking(int mode);

/* Pivoting of the explicit inverses of hps_zinv and of the factorisation's
 * W and Z inverses (the merges and the top of the Section 2 direct solver
 * only use the products with W^{-1} and Z^{-1}), process-wide:
 *   mode -1 (default): orders of at least 224 that are multiples of 4 are first
 *           mixed by a depth-2 random butterfly transform (Parker 1995;
 *           Baboulin, Dongarra, Herrmann, Tomov 2013), A~ = U^T A V, then
 *           eliminated without searching the rows for pivots (Gauss-Jordan
 *           with each 32-column panel pivoting on its own rows), and
 *           A^{-1} = V A~^{-1} U^T.  The result is checked on two fixed probe
 *           vectors x: ||A^{-1}(A x) - x|| <= tol ||x||; a failed check or a
 *           zero pivot re-inverts the batch with pivoting.  Other orders:
 *           partial / tournament pivoting.
 *   mode 0: partial / tournament pivoting for every order.
 *   mode 1: the butterfly path for every order that is a multiple of 4.
 * tol >= 0 sets the probe tolerance (default 1e-10; 0 forces the fallback,
 * for testing); tol = -1 keeps it.  HPS_ZINV_PIVOTING = 0 / 1 in the
 * environment sets the initial mode.  HPS_EINVAL for other values. */
hps_status hps_zinv_pivoting(int mode, double tol);

/* Butterfly-path inverse calls so far, how many fell back to pivoting, and
 * the largest probe error seen (host outputs; NULL skips one). */
hps_status hps_zinv_pivoting_info(int64_t* calls, int64_t* fallbacks, double* max_err);

/* Tile shapes of the complex FP64 GEMM behind every call of this library,
 * process-wide (a performance choice; results do not depend on it: every
 * candidate tile shape accumulates the products of an output element in the
 * same order, so the bits of every result are the same).
 *   mode 0: fixed rules (default).
 *   mode 1: autotuning: the first GEMM of each distinct shape (sizes,
 *           operations, strides, batch) times every candidate tile shape on
 *           that call's own operands, saving the output first and restoring it
 *           before each trial and at the end, and keeps the fastest for the
 *           later calls of that shape.  A tuning call synchronises its stream
 *           and allocates a copy of its output, so run one warm-up pass (e.g.
 *           a factor and solve) before timing.
 *   force >= 0 pins tile variant `force` for every call (testing and tuning;
 *   HPS_EINVAL beyond the variant count); -1 clears it.
 * The table of tuned shapes lives until the process ends. */
hps_status hps_gemm_tuning(int mode, int force);

/* Number of GEMM tile variants, shapes tuned so far and the seconds spent
 * tuning them (host outputs; NULL skips one). */
hps_status hps_gemm_tuning_info(int* variants, int* shapes_tuned, double* seconds);

/* ---- launch profiler (measurement support) ---- */

typedef struct hps_kernel_stat {
  char name[32];     /* kernel class: zgemm, cgemm, gj_panel, tp_select, tp_exchange,
                        gj_permute, gather_scatter, leaf_assemble, pointwise */
  int64_t launches;  /* launches timed */
  double total_ms;   /* sum of per-launch durations (HIP events on the launch stream) */
  double flops;      /* sum of algorithmic flops (complex multiply-add = 8) */
  double bytes;      /* sum of algorithmic bytes read + written */
} hps_kernel_stat;

/* Clears the records and times every following kernel launch of the library
 * (process-wide) until hps_profile_stop.  Adds two event records per launch. */
hps_status hps_profile_start(void);

/* Stops timing, synchronises the device and writes up to `max` per-class
 * totals to out (host array), followed by per-phase totals named
 * "phase:leaf", "phase:merge", "phase:top", "phase:solve", "phase:far_field",
 * "phase:jvp", "phase:vjp", "phase:other" (the same launches grouped by the
 * library call and factorisation stage that issued them); returns their
 * number (or a negative hps_status). */
int hps_profile_stop(hps_kernel_stat* out, int max);

#ifdef __cplusplus
}
#endif

#endif /* HPS_BLOCKS_H_ */
