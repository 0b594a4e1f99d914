/*
 * hps.h - C ABI of libhps: variable-coefficient Helmholtz scattering solves by a
 * hierarchical impedance-to-impedance (HPS/ItI) direct solver on an AMD MI355X.
 *
 * The calls follow the statement of the problem in the paper (Borges,
 * Gillman, Greengard, "High resolution inverse scattering in two dimensions
 * using recursive linearization"):
 *   hps_factor      factorisation of the interior problem for a contrast q at
 *                   wavenumber k (Section 2: O(N^{3/2}) factor of the system
 *                   matrix for a given q; eq. origpde);
 *   hps_solve       forward solves for plane waves exp(i k x.d) (Section 1,
 *                   eqs. fscatprob, srad; Section 2: O(N log N) per right-hand
 *                   side given the factorisation);
 *   hps_far_field   the measured data u_far(theta) = u_s(R cos theta,
 *                   R sin theta) (Section 1; operator F of eq. farfielddef);
 *   hps_jvp         the Frechet derivative J dq (Theorem 1, eqs. Jdef, vdef);
 *   hps_vjp         its adjoint Re(J^* r), summed over the directions
 *                   (Theorem 2 and eq. adjfrechetdef, as the exact discrete
 *                   conjugate transpose);
 *   hps_sine_eval / hps_sine_adjoint
 *                   the band-limited sine model E_k and its adjoint
 *                   (Section 3.2, eq. sineseries; square index set).
 *
 * Discretisation (the paper defers it to the HPS solver it cites; the
 * reading used here): Omega = [x0, x1] x [y0, y1] is split into nleaf x nleaf
 * square leaves with p x p Chebyshev-Lobatto points (corner points dropped).
 * The PDE is collocated at the (p-2)^2 interior points of every leaf; leaves
 * are glued by continuity of u and of its normal derivative, through
 * impedance-to-impedance maps merged on a binary tree (alternating x / y
 * merges); the outer boundary is coupled to the radiating exterior through
 * the Calderon relation S t = (K - I/2) s of the single- and double-layer
 * operators (Remark in Section 2), never inverting S.
 *
 * Conventions
 *  - "PDE nodes": the npde = nleaf^2 (p-2)^2 leaf-interior collocation points,
 *    ordered by leaf in Morton order (bit 2b of the leaf index = bit b of the
 *    column, bit 2b+1 = bit b of the row), then row-major inside the leaf
 *    (y slow, x fast).  hps_node_coords returns their coordinates.
 *  - Complex arrays are interleaved (re, im) double pairs (complex128).
 *  - Pointers named *_host are host memory; every other array argument is
 *    device memory on the GPU current when the context was created.
 *  - All work is enqueued on opts.stream (NULL = the default stream) in call
 *    order; calls return after enqueueing unless stated otherwise.  Inputs
 *    are only read during the call's kernels; the caller keeps ownership of
 *    every buffer it passes and must keep it alive until the stream reaches
 *    the call's end.  The context owns all factors, fields and workspaces.
 *  - Every call returns an hps_status; on failure hps_last_error() holds a
 *    message.  A failed call leaves the context usable; the results of a
 *    failed call are unspecified.
 *  - Batches: a context may hold nprob independent problems on the same
 *    leaf grid, each with its own contrast and wavenumber (the
 *    recursive-linearization solves are uncoupled, Section 3).  They are
 *    factored and solved together: every leaf-stage, merge-level and top
 *    kernel runs once for all problems.  Every per-problem array then has a
 *    leading problem index: q_nodes [nprob][npde], ufar [nprob][ndir][ntheta],
 *    u [nprob][ndir][npde], dq and grad [nprob][npde], r [nprob][ndir][ntheta].
 *    All problems use the same number of directions per solve.  The sine
 *    model and the Gauss-Newton step take nprob = 1.
 */
#ifndef HPS_H_
#define HPS_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HPS_OK = 0,
  HPS_EINVAL = -1,     /* invalid argument (sizes, NULL pointers, k <= 0, ...) */
  HPS_ENOMEM = -2,     /* device allocation failed */
  HPS_EDEVICE = -3,    /* a HIP runtime call or kernel launch failed */
  HPS_ESTATE = -4,     /* call order violated (solve before factor, ...) */
  HPS_ESINGULAR = -5,  /* a zero pivot was met in a factorisation */
  HPS_ENOCONV = -6,    /* HPS_MIXED: refinement stopped above refine_tol (results kept) */
  HPS_ENONFINITE = -7  /* a NaN or infinity in the contrast or in the factorisation */
} hps_status;

/* HPS_FP64: everything in complex128.
 * HPS_MIXED: the factorisation is complex128; the forward solves run their
 * level sweeps in complex64 on FP32 matrix cores (copies of the merge
 * operators) and are then refined on the interface (skeleton) system of
 * leaf-edge impedance data: the residual is formed in complex128 with the
 * leaf impedance-to-impedance maps (interface mismatches at every merge and
 * the outer-boundary relation) and corrected with complex64 sweeps, until
 * its norm is at most refine_tol times that of the boundary data or
 * max_refine corrections were made.  hps_jvp / hps_vjp use the complex128
 * operators. */
typedef enum { HPS_FP64 = 0, HPS_MIXED = 1 } hps_precision;

/* Exterior relation on the outer boundary (the E4 rows of the discrete
 * system), with t = d_nu u_s and s = u_s the scattered traces:
 * HPS_EXT_GREEN: S t = (K - I/2) s, the Green relation of the Remark in
 *   Section 2.  It is singular when k^2 is a Dirichlet eigenvalue of the
 *   Laplacian on Omega (for [-1, 1]^2: k = (pi/2) sqrt(m^2 + n^2)), which the
 *   Remark excludes;
 * HPS_EXT_BURTON_MILLER: (S + i beta (K' + I/2)) t = ((K - I/2) + i beta T) s,
 *   beta = 1/k: the Green relation plus i beta times its normal derivative
 *   (K' the adjoint double layer, T the hypersingular operator in Maue's
 *   form), uniquely solvable at every k > 0.  The extra operators cost host
 *   quadrature in hps_set_wavenumber only; factor, solves and derivatives
 *   are unchanged in cost. */
typedef enum { HPS_EXT_GREEN = 0, HPS_EXT_BURTON_MILLER = 1 } hps_exterior;

typedef struct hps_opts {
  double x0, x1, y0, y1; /* square domain Omega; x1 - x0 must equal y1 - y0 */
  int nleaf;             /* leaves per side, a power of two (1 .. 256) */
  int p;                 /* Chebyshev-Lobatto points per leaf side (4 .. 20) */
  double eta_scale;      /* impedance parameter eta = eta_scale * k (<= 0: 1) */
  int keep_derivs;       /* non-zero: keep the operators hps_jvp / hps_vjp need */
  int precision;         /* hps_precision */
  int host_threads;      /* threads for the per-k boundary quadrature (<= 0: auto) */
  void* stream;          /* hipStream_t for all work (NULL = default stream) */
  int nprob;             /* independent problems on this grid (1 .. 4096); see Batches */
  int max_refine;        /* HPS_MIXED: most refinement corrections per solve (0 .. 100) */
  double refine_tol;     /* HPS_MIXED: relative residual target (> 0) */
  int fallback_fp64;     /* HPS_MIXED: non-zero: a solve whose refinement stops above refine_tol
                            redoes its sweep in complex128 (exact FP64 result, refine_fallback = 1
                            in hps_stats) instead of returning HPS_ENOCONV */
  int exterior;          /* hps_exterior */
  int streams;           /* streams of hps_factor: 2 (default) runs half the leaf stage, each merge
                            level's operators for the sweeps (V, U) while the next level proceeds,
                            and on the levels whose W inverse has order >= 224 the level's Q
                            product, on a second stream the context owns (forked from and joined
                            to `stream` with events inside the call); 1 keeps all work on `stream`
                            (for callers that already run several contexts concurrently).  The
                            results are the same bit for bit.  (hps_gn_step captures its CG
                            iterations in a graph on `stream`, or on the second stream when
                            `stream` is the legacy default stream, which cannot be captured.) */
} hps_opts;

typedef struct hps_ctx hps_ctx;

/* Fills *o with the defaults: Omega = [-1, 1]^2, nleaf = 4, p = 16,
 * eta_scale = 1, keep_derivs = 1, HPS_FP64, default stream, nprob = 1,
 * max_refine = 8, fallback_fp64 = 1, refine_tol = 1e-10, HPS_EXT_GREEN,
 * streams = 2 (the far-field error follows the interface residual closely, so
 * 1e-10 leaves two orders of margin under a 1e-8 far-field target; one
 * correction reaches it at k = 80). */
void hps_default_opts(hps_opts* o);

/* Creates a context for the geometry in *opts (host-side set-up only; device
 * memory is allocated by the first hps_factor).  *out receives the handle. */
hps_status hps_create(const hps_opts* opts, hps_ctx** out);

/* Releases the context and all device memory it owns (synchronises its
 * stream first).  NULL is ignored. */
void hps_destroy(hps_ctx* ctx);

/* Message of the last failed call on this context ("" if none). */
const char* hps_last_error(const hps_ctx* ctx);

/* Number of PDE nodes npde = nleaf^2 (p-2)^2 (per problem). */
int64_t hps_num_nodes(const hps_ctx* ctx);

/* Number of outer-boundary nodes 4 nleaf (p-2). */
int64_t hps_num_boundary_nodes(const hps_ctx* ctx);

/* Coordinates of the PDE nodes: xy_host[2 i], xy_host[2 i + 1] for node i
 * (host array of 2 npde doubles). */
hps_status hps_node_coords(const hps_ctx* ctx, double* xy_host);

/* Per-wavenumber set-up: everything of the discrete problem that depends on
 * k but not on q.  The exterior relation's layer operators on the outer
 * boundary (the Remark of Section 2: S, K, and K', T for the combined field)
 * by product quadrature on the host; the leaf blocks of the PDE (eq. origpde)
 * at q = 0 with the edge unknowns folded in; the top blocks scaled by the
 * exterior impedance block (an order-nb inverse and two products on the
 * device).  Synchronous.  hps_factor calls it when k changes; calling it
 * first keeps this work out of the factorisation, as the Newton steps of
 * Section 3.4 at one k share it.  k > 0. */
hps_status hps_set_wavenumber(hps_ctx* ctx, double k);

/* As hps_set_wavenumber with one wavenumber per problem: k_host[nprob]
 * (problems whose wavenumber is unchanged keep their operators). */
hps_status hps_set_wavenumbers(hps_ctx* ctx, const double* k_host);

/* Sets hps_opts.streams (1 or 2, else HPS_EINVAL) for the next hps_factor
 * calls of this context: a scheduling choice only, the results are the same
 * bit for bit. */
hps_status hps_set_streams(hps_ctx* ctx, int streams);

/* Factorises the discrete interior + exterior problem for the real contrast
 * q_nodes (device, npde doubles, PDE-node order) at wavenumber k > 0: leaf
 * impedance maps, the merge tree, and the inverse of the top (boundary)
 * system.  Synchronises the stream once to read the pivot and finiteness
 * flags; returns HPS_ENONFINITE if q holds a NaN or infinity (checked on the
 * device) or the top inverse came out non-finite, HPS_ESINGULAR if a zero
 * pivot occurred.  Invalidates earlier solves. */
hps_status hps_factor(hps_ctx* ctx, const double* q_nodes, double k);

/* hps_factor for a batch: problem b has contrast q_nodes[b][.] and
 * wavenumber k_host[b]. */
hps_status hps_factor_batch(hps_ctx* ctx, const double* q_nodes, const double* k_host);

/* Total-field solves for ndir plane waves exp(i k x.d_m),
 * d_m = (cos a_m, sin a_m), a_m = dir_angle_host[m]; keeps the fields u_0 at
 * the PDE nodes and the boundary data on the device for far-field, jvp and
 * vjp calls.  Requires hps_factor.  1 <= ndir <= 65535. */
hps_status hps_solve(hps_ctx* ctx, int ndir, const double* dir_angle_host);

/* hps_solve for a batch with directions per problem:
 * dir_angle_host[b * ndir + m] is direction m of problem b.  (hps_solve
 * uses the same ndir angles for every problem.) */
hps_status hps_solve_batch(hps_ctx* ctx, int ndir, const double* dir_angle_host);

/* Scattered field at x_p = R (cos theta_p, sin theta_p), p < ntheta, for every
 * solved direction: ufar (device, complex128 [ndir][ntheta]).  The
 * measurement set (theta, R) is remembered for hps_jvp / hps_vjp; its
 * quadrature matrices are rebuilt on the host when it changes.  The points
 * must lie outside Omega.  Requires hps_solve. */
hps_status hps_far_field(hps_ctx* ctx, int ntheta, const double* theta_host, double R,
                         double* ufar);

/* Total field u_0 at the PDE nodes for every solved direction:
 * u (device, complex128 [ndir][npde]).  Requires hps_solve. */
hps_status hps_total_field(hps_ctx* ctx, double* u);

/* Frechet derivative (Theorem 1): dufar = J dq for a real perturbation dq
 * (device, npde doubles) of the factored contrast, at the solved directions
 * and the last measurement set: dufar (device, complex128 [ndir][ntheta]).
 * Requires hps_far_field and keep_derivs. */
hps_status hps_jvp(hps_ctx* ctx, const double* dq, double* dufar);

/* Adjoint (Theorem 2, discrete): grad = Re(J^H r) for r (device, complex128
 * [ndir][ntheta]); grad (device, npde doubles).  Same requirements as
 * hps_jvp. */
hps_status hps_vjp(hps_ctx* ctx, const double* r, double* grad);

/* Sine model on Omega = [x0, x1] x [y0, y1]:
 * q(x, y) = sum_{m,n=1..S} C[(m-1) S + (n-1)] sin(m pi (x - x0)/(x1 - x0))
 *                                             sin(n pi (y - y0)/(y1 - y0))
 * at the PDE nodes.  coef (device, S*S doubles), q_nodes (device, npde). */
hps_status hps_sine_eval(hps_ctx* ctx, int S, const double* coef, double* q_nodes);

/* Transpose of hps_sine_eval: coef = E^T g for g (device, npde doubles). */
hps_status hps_sine_adjoint(hps_ctx* ctx, int S, const double* g, double* coef);

/* One Gauss-Newton step of the Newton iteration of Section 3.3 on the sine
 * model (eq. normaleq; real unknowns, so the normal equations are taken in
 * their real part):
 *   q = E coef;  factor(q, k);  solve(ndir directions);
 *   r = data - F[q]  (data: device complex128 [ndir][ntheta], at R, theta);
 *   solve Re(E^T J^H J E) dc = Re(E^T J^H r) by conjugate gradients from
 *   dc = 0 (each iteration = one hps_jvp + one hps_vjp over all directions),
 *   stopping after max_iter iterations or when the CG residual falls to
 *   tol times its initial norm;
 *   coef_out = coef + dc.
 * band > 0 restricts the unknowns to the modes with m + n <= band (the
 * triangular index set of eq. sineseries, S(k) = floor(2k) in the paper);
 * the other entries of dc are zero (coefficients outside the band keep their
 * values).  band = 0: all S x S modes.
 * coef, coef_out: device, S*S doubles (layout of hps_sine_eval).  Host
 * outputs (may be NULL): CG iterations, final relative CG residual, and the
 * data misfit ||r|| before the step.  Leaves the context factored and solved
 * at q = E coef.  Synchronous.  Requires keep_derivs.  The CG scalars stay on
 * the device; after the first iteration the others replay one captured graph
 * (bit-identical to direct launches; hps_stats.cg_graph_iters). */
hps_status hps_gn_step(hps_ctx* ctx, double k, int ndir, const double* dir_angle_host, int ntheta,
                       const double* theta_host, double R, int S, int band, const double* coef,
                       const double* data, int max_iter, double tol, double* coef_out,
                       int* iters_host, double* cg_rel_res_host, double* misfit_host);

typedef struct hps_stats {
  double t_wavenumber_ms; /* last hps_set_wavenumber (host quadrature + upload) */
  double t_factor_ms;     /* last hps_factor, device time between events */
  double t_solve_ms;      /* last hps_solve */
  double t_far_field_ms;  /* last hps_far_field (device part) */
  double t_jvp_ms;        /* last hps_jvp */
  double t_vjp_ms;        /* last hps_vjp */
  double t_leaf_ms;       /* last hps_factor: leaf stage (collocation, inverses, leaf maps) */
  double t_merge_ms;      /* last hps_factor: merge tree (all levels) */
  double t_top_ms;        /* last hps_factor: top system A2^-1 A1 + R and its inverse */
  int64_t device_bytes;   /* device memory held by the context */
  int ndir;               /* directions of the last solve */
  int singular;           /* 1 if the last factorisation met a zero pivot */
  int nonfinite;          /* last factorisation: bit 0 non-finite contrast, bit 1 non-finite top inverse */
  int refine_iters;       /* HPS_MIXED: corrections made by the last solve */
  double refine_residual; /* HPS_MIXED: its final relative interface residual */
  int refine_fallback;    /* HPS_MIXED: 1 if the last solve redid its sweep in complex128 */
  int cg_graph_iters;     /* last hps_gn_step: CG iterations replayed from a captured graph (the
                             first runs directly; 0 when capture was not possible, e.g. with the
                             launch profiler recording) */
} hps_stats;

/* Timings of the last calls (synchronises the stream) and memory use. */
hps_status hps_get_stats(hps_ctx* ctx, hps_stats* out);

/* The building blocks of the solver (dense complex GEMM and batched inverses,
 * the allocation-free inverse, host-side boundary operators, tile tuning and
 * the launch profiler) are declared in hps_blocks.h. */

#ifdef __cplusplus
}
#endif

#endif /* HPS_H_ */
