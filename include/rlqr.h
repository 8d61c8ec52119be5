/*
 * rlqr.h -- C ABI of the MI355X dual-regularized LQR solver.
 *
 * The library solves batches of dual-regularized LQR problems (Definition in
 * Section "Dual-Regularized LQR" of arXiv 2509.16370): for each instance it
 * returns the unique solution (x, u, y) of the first-order conditions
 *
 *     [[P, C^T], [C, -Delta]] [x; y] = -[s; c]       (eq. primal-dual-linear-system)
 *
 * with the stagewise blocks of eq. optimal-control-specialization and
 * Delta_i = delta * I for i = 0..N, or a positive diagonal Delta_i per stage
 * (rlqr_lhs.delta_diag; the definition allows any SPD Delta_i, and the
 * paper's per-constraint penalties Delta_C, Delta_G give diagonal ones).
 * The call split follows the paper's
 * factorization / solve / residual callbacks (Section "Software
 * Contributions"): one factorization serves any number of right-hand sides.
 *
 * Memory. Every array argument is a DEVICE pointer owned by the caller unless
 * it is marked [host]. Scalars and matrices are float64, row-major. The handle
 * owns its workspace, allocated once by rlqr_create; no other call allocates
 * device memory.
 *
 * Layout of a batch (instances packed one after another; per instance the
 * arrays are stage-stacked):
 *     Q (N+1)*n*n   M N*n*m   R N*m*m   A N*n*n   B N*n*m
 *     q (N+1)*n     r N*m     c (N+1)*n   (c[0] = c_0, c[i+1] offset of step i)
 *     x (N+1)*n     u N*m     y (N+1)*n
 *     delta_diag (N+1)*n  (optional; like x: Delta_i's diagonal at i*n)
 *     residual  N*(n+m) + n + (N+1)*n  (order given at rlqr_residual)
 * Instance b's block of array k starts at the exclusive prefix sum of the
 * per-instance element counts; rlqr_layout_offsets returns those offsets.
 *
 * Streams. Calls are ordered on the given stream (a hipStream_t passed as
 * void*; NULL means the default stream) and return before the GPU finishes.
 * A handle must not be used from two streams at once.
 *
 * Errors. Whole-call failures return a negative rlqr_status and leave outputs
 * untouched; no call aborts or throws. Per-instance outcomes are reported in
 * inst_status (RLQR_INST_*).
 */
#ifndef RLQR_H
#define RLQR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rlqr_handle rlqr_handle;
typedef void *rlqr_stream; /* hipStream_t */

typedef enum {
  RLQR_OK = 0,
  RLQR_E_INVALID = -1,     /* bad argument: NULL pointer, shape out of range, unknown mode */
  RLQR_E_NOMEM = -2,       /* workspace allocation failed */
  RLQR_E_HIP = -3,         /* a HIP runtime call or kernel launch failed */
  RLQR_E_STATE = -4,       /* call order: solve/inertia/residual before factor */
  RLQR_E_UNSUPPORTED = -5  /* mode not available for these shapes */
} rlqr_status;

typedef enum {
  /* Sequential recursion (Section "Sequential Algorithm"), every product and
     pivot in float64. */
  RLQR_SEQ_FP64 = 0,
  /* Sequential recursion with float32 matrix products and float64 pivot
     factorizations; rlqr_solve refines against the float64 residual. */
  RLQR_SEQ_MIXED = 1,
  /* Parallel-in-time (Section "Parallel Algorithm"): the horizon is cut into
     segments of L stages; the reverse associative scan of the interval
     value-function elements (eqs. lqr-gpu-init-running, lqr-gpu-combo), in
     float32, gives the cost-to-go at every segment start, and all segments
     then run the recursion of RLQR_SEQ_MIXED at once. The solve runs the
     segments in parallel as well and joins them through each segment's
     transfer matrix (the product of its closed-loop maps
     F_i = S_hat_{i+1}^{-1}(A_i + B_i K_i)), then refines against the float64
     residual. Instances whose scan or pivots fall outside the float32 guard
     band are factored in float64 by the sequential recursion. */
  RLQR_SCAN_FP32 = 2,
  /* RLQR_SCAN_FP32 with bfloat16 operands (float32 accumulation) in the
     matrix products of the scan combine (eq. lqr-gpu-combo); the inversion of
     I + C P, the segment recursion, the pivots and the refinement are as in
     RLQR_SCAN_FP32. The boundary cost-to-go carries bfloat16 rounding, so
     rlqr_solve typically needs more refinement steps. */
  RLQR_SCAN_BF16 = 3
} rlqr_mode;

/* per-instance outcome written by rlqr_solve */
enum {
  RLQR_INST_OK = 0,             /* solved to rel_tol, pivot certificate holds  */
  RLQR_INST_NOT_PD = 1,         /* solved to rel_tol, certificate fails (wrong inertia) */
  RLQR_INST_SINGULAR = 2,       /* a pivot is zero; x, u, y are NaN             */
  RLQR_INST_NOT_CONVERGED = 3,  /* relative residual above rel_tol after max_refine steps */
  /* A NaN or +-Inf reached the computation: in the data (||[s; c]||_inf is
     not finite, or a pivot of the factorization is), or arising in the
     recursion itself (a non-finite residual with finite pivots). Detected
     from the pivots and the residual, which every non-finite entry of the
     data reaches; no separate pass over the inputs is made. x, u, y hold
     whatever non-finite values arose; the certificate reports the instance
     as failed. */
  RLQR_INST_NONFINITE = 4
};

/* Precision path of each instance (rlqr_precision_path). */
enum {
  RLQR_PATH_FP32 = 0,        /* served from float32 tiles (RLQR_SEQ_MIXED, RLQR_SCAN_*) */
  RLQR_PATH_FP64 = 1,        /* float64 by mode (RLQR_SEQ_FP64) or by rlqr_tuning.inst_fp64 */
  RLQR_PATH_FP64_GUARD = 2,  /* float32 factorization, then refactored in float64 before any
                                solve: a pivot fell inside the guard band (|d| < 1e-4 max|diag|),
                                a pivot was zero, or the scan met a singular I + C P */
  RLQR_PATH_FP64_REDO = 3    /* refinement from float32 tiles did not reach rel_tol; the
                                instance was refactored and solved again in float64 */
};

/* array identifiers for rlqr_layout_offsets */
enum {
  RLQR_ARR_Q = 0, RLQR_ARR_M, RLQR_ARR_R, RLQR_ARR_A, RLQR_ARR_B,
  RLQR_ARR_q, RLQR_ARR_r, RLQR_ARR_c, RLQR_ARR_x, RLQR_ARR_u, RLQR_ARR_y,
  RLQR_ARR_RES, RLQR_ARR_COUNT
};

typedef struct {
  int32_t batch;        /* number of instances B >= 0                          */
  const int32_t *N;     /* [host][B] horizon, N >= 0                            */
  const int32_t *nx;    /* [host][B] state size n, 1 <= n                       */
  const int32_t *nu;    /* [host][B] control size m, 1 <= m; n <= 64, n + m <= 96 */
} rlqr_shape;

typedef struct {        /* left-hand side: stage blocks and regularization       */
  const double *Q, *M, *R, *A, *B;
  const double *delta;  /* [B] delta_b >= 0; Delta_i = delta_b * I, i = 0..N    */
  /* Optional per-stage diagonal regularization (NULL: Delta_i = delta_b I).
   * Laid out like x: instance b's Delta_i = diag(delta_diag[off_x(b) + i n_b
   * .. + n_b - 1]), i = 0..N_b. Every entry must be > 0 and finite (Delta_i
   * SPD, Definition "dual-regularized LQR"); other values give undefined
   * (non-finite) results. When set, delta is not read and may be NULL. The
   * state pivots are then those of the symmetric representative S_hat_i =
   * I + Delta_i^{1/2} P_i Delta_i^{1/2} (Section "Inertia Certification"),
   * which is similar to I + Delta_i P_i. All modes (in the scan modes the
   * interval elements' C carries Delta_{i+1}). */
  const double *delta_diag;
} rlqr_lhs;

typedef struct { const double *q, *r, *c; } rlqr_rhs;   /* s = (q_0, r_0, ..., q_N), c */
typedef struct { double *x, *u, *y; } rlqr_sol;

/* Largest n and n + m the kernels accept. */
#define RLQR_MAX_NX 64
#define RLQR_MAX_NXU 96

/* Launch tuning fixed at create (an autotuner fills the per-instance arrays
   bucket by bucket). */
typedef struct {
  int32_t scan_chunk;          /* RLQR_SCAN_*: stages per segment L >= 1; 0 picks L
                                  from the batch (about one segment per compute unit).
                                  An instance with N <= L is one segment and skips the
                                  scan. Ignored by the sequential modes. */
  const int32_t *inst_chunk;   /* [host][B] or NULL. RLQR_SCAN_*: per-instance L
                                  (>= 1), or 0 for one segment (the sequential float32
                                  recursion of RLQR_SEQ_MIXED); overrides scan_chunk. */
  const int32_t *inst_fp64;    /* [host][B] or NULL. RLQR_SEQ_MIXED and RLQR_SCAN_*:
                                  1 = factor and solve this instance in float64 only
                                  (no float32 attempt). */
  int32_t max_rhs;             /* sequential modes: solve state for up to max_rhs
                                  right-hand sides at once (rlqr_solve_multi); 0 or 1:
                                  none. Costs max_rhs times the solve workspace
                                  (right-hand-side-sized vectors, per-instance flags). */
  int32_t scan_carry_pc;       /* RLQR_SCAN_*: nonzero = rlqr_factor_rhs also carries
                                  p and c through the reverse scan (eq. lqr-gpu-combo,
                                  the alternative the paper sets beside the
                                  p-recurrence), and the next rlqr_solve with the same
                                  rhs pointers takes every segment's boundary p from
                                  the scan instead of a backward pass over the
                                  segments and the sequential boundary chain; its
                                  refinement passes use the p-recurrence. Float32
                                  vectors, 2 n_pad floats per element. Ignored by the
                                  sequential modes and by rlqr_factor. */
  int32_t mw_waves;            /* wavefronts per instance (one workgroup) in the kernels
                                  of instances with 16 < n + m <= 48 and n <= 32: 0 or 4
                                  (default), 1, 2 or 8 (instances with n > 16 take at
                                  least 2). More wavefronts shorten each stage's
                                  dependent chain of block products; fewer make its
                                  workgroup barriers cheaper. Certificates are identical
                                  and solutions agree to rounding. Larger stages keep
                                  their fixed counts. Other values: RLQR_E_INVALID. */
} rlqr_tuning;

/*
 * Create a handle for a fixed batch of shapes and one mode; allocates the
 * factor workspace (the only allocation the library makes). The shape arrays
 * are copied. *workspace_bytes (may be NULL) receives the device bytes held.
 * Errors: RLQR_E_INVALID (NULL h/s, batch < 0, a shape out of range, unknown
 * mode), RLQR_E_NOMEM, RLQR_E_HIP. On error *h is set to NULL.
 */
rlqr_status rlqr_create(rlqr_handle **h, const rlqr_shape *s, rlqr_mode mode,
                        size_t *workspace_bytes);

/* rlqr_create with explicit tuning (t may be NULL: defaults). Errors as
 * rlqr_create, plus RLQR_E_INVALID for scan_chunk < 0. */
rlqr_status rlqr_create_tuned(rlqr_handle **h, const rlqr_shape *s, rlqr_mode mode,
                              const rlqr_tuning *t, size_t *workspace_bytes);

/* The tuning in effect (scan_chunk resolved when it was 0; the per-instance
 * pointers are returned NULL) [host]. Errors: RLQR_E_INVALID. */
rlqr_status rlqr_get_tuning(const rlqr_handle *h, rlqr_tuning *t);

/* Write the B+1 exclusive prefix offsets (in float64 elements) of array `array`
 * (RLQR_ARR_*) to off [host]. Errors: RLQR_E_INVALID. */
rlqr_status rlqr_layout_offsets(const rlqr_handle *h, int32_t array, int64_t *off);

/*
 * Factor the left-hand side: the backward Riccati recursion of Section
 * "Sequential Algorithm" (S_hat_{k+1} = I + delta P_{k+1}, W_{k+1} =
 * P_{k+1} S_hat_{k+1}^{-1}, G_k = R_k + B_k^T W B_k, H_k = B_k^T W A_k + M_k^T,
 * K_k = -G_k^{-1} H_k, P_k = A_k^T W A_k + Q_k + H_k^T K_k, P_N = Q_N) for every
 * instance, recording the pivots of S_hat_i (i = 0..N) and G_i (i = 0..N-1)
 * for the certificate. With lhs->delta_diag (Delta_i = D_i^2 diagonal) the
 * swept matrix is S_hat_{k+1} = I + D P_{k+1} D and W_{k+1} = P_{k+1} D
 * S_hat_{k+1}^{-1} D^{-1} = P_{k+1} (I + Delta_{k+1} P_{k+1})^{-1}. The lhs
 * arrays must stay valid and unchanged until the last rlqr_solve/rlqr_residual
 * on this factorization, which re-read them.
 * Errors: RLQR_E_INVALID (NULL pointer), RLQR_E_HIP.
 */
rlqr_status rlqr_factor(rlqr_handle *h, const rlqr_lhs *lhs, rlqr_stream st);

/*
 * rlqr_factor for a caller who already knows the right-hand side it will
 * solve next: in the sequential modes the backward vector pass of the solve
 * (p_k, k_k of Theorem "main-seq-theorem") runs inside the factorization's
 * stage loop for the instances with n + m <= 16, so the next rlqr_solve with
 * the same rhs pointers starts those instances at the forward rollout.
 * Results are identical to rlqr_factor followed by rlqr_solve. The rhs arrays
 * must keep their contents until that rlqr_solve; any other rlqr_solve (other
 * pointers, or a second call) runs the full passes. In the scan modes this is
 * rlqr_factor. Errors: as rlqr_factor, and RLQR_E_INVALID for a NULL rhs
 * array when the batch is not empty.
 */
rlqr_status rlqr_factor_rhs(rlqr_handle *h, const rlqr_lhs *lhs, const rlqr_rhs *rhs, rlqr_stream st);

/*
 * Solve for one right-hand side with the current factorization: backward
 * vector pass (g, h, k_k, p_k), forward rollout x_0 = S_hat_0^{-1}(c_0 -
 * delta p_0), u_k = K_k x_k + k_k, x_{k+1} = S_hat_{k+1}^{-1}(A_k x_k + B_k u_k
 * + c_{k+1} - delta p_{k+1}), y_k = P_k x_k + p_k (Theorem "main-seq-theorem").
 * Then up to max_refine steps of iterative refinement against the float64
 * residual of Section "Residual Computation": z <- z + solve(residual),
 * per instance until ||residual||_inf <= rel_tol * ||[s; c]||_inf.
 * inst_status [B] (RLQR_INST_*) and inst_relres [B] (final relative residual)
 * may be NULL. Errors: RLQR_E_INVALID, RLQR_E_STATE (no factorization),
 * RLQR_E_HIP.
 */
rlqr_status rlqr_solve(rlqr_handle *h, const rlqr_rhs *rhs, rlqr_sol *out,
                       double rel_tol, int32_t max_refine,
                       int32_t *inst_status, double *inst_relres, rlqr_stream st);

/*
 * rlqr_solve for nrhs right-hand sides with the same factorization (the
 * reuse of one factorization for many right-hand sides that Corollary
 * "p-recurrence" allows). The arrays of rhs and out each hold nrhs vectors
 * one after another: right-hand side j is (q + j*Lq, r + j*Lr, c + j*Lc) and
 * its solution (x + j*Lq, u + j*Lr, y + j*Lq), where Lq, Lr, Lc are the batch
 * lengths of the q, r and c arrays (rlqr_layout_offsets; x and y have the
 * length of q and c, u that of r). inst_status and inst_relres, when not
 * NULL, hold [nrhs][B] entries. Each right-hand side is solved and refined
 * exactly as by rlqr_solve, with identical results. In the sequential modes,
 * when the handle was created with max_rhs >= nrhs, all right-hand sides run
 * in the same launches (one wavefront or workgroup per instance and
 * right-hand side, those of one instance placed on one XCD so that its tiles
 * are read from HBM once and from L2 by the others); otherwise they run one
 * after another. nrhs = 0 is a no-op. Errors: as rlqr_solve, and
 * RLQR_E_INVALID for nrhs < 0.
 */
rlqr_status rlqr_solve_multi(rlqr_handle *h, int32_t nrhs, const rlqr_rhs *rhs, rlqr_sol *out,
                             double rel_tol, int32_t max_refine,
                             int32_t *inst_status, double *inst_relres, rlqr_stream st);

/*
 * Leave the instances with skip[b] != 0 out of the following rlqr_factor,
 * rlqr_factor_rhs and rlqr_solve calls (sequential modes): their tiles,
 * certificate, solution, status and relative residual keep their previous
 * values, and they cost nothing but a flag test. skip is a DEVICE array [B]
 * owned by the caller, read by each of those calls when it runs (so a
 * captured graph reads its contents at replay); NULL clears the mask.
 * rlqr_solve_multi and rlqr_residual ignore it. For drivers whose instances
 * finish at different iterations (an interior-point batch, where converged
 * problems drop out and only those whose certificate failed are refactored
 * with a larger inertia correction). Errors: RLQR_E_INVALID (NULL h),
 * RLQR_E_UNSUPPORTED (scan modes, when skip is not NULL).
 */
rlqr_status rlqr_set_skip(rlqr_handle *h, const int32_t *skip);

/*
 * Pivot certificate of Theorem "riccati-inertia-certification-theorem":
 * pd_verdict[b] = 1 iff every pivot of every S_hat_i and G_i is positive, i.e.
 * iff the KKT matrix has inertia (N(n+m)+n, (N+1)n, 0). first_bad[b] is the
 * first failing pivot in elimination order (S_hat_N, G_{N-1}, S_hat_{N-1},
 * ..., G_0, S_hat_0), coded 2i for S_hat_i and 2i+1 for G_i, or -1.
 * inertia[3b..3b+2] = (0, (N+1)n, 0) + the sign counts of all pivots; a pivot
 * with |d| <= 1e3 * dim * eps64 * max|diag| of its matrix counts as zero.
 * Any output pointer may be NULL. Errors: RLQR_E_STATE, RLQR_E_HIP.
 */
rlqr_status rlqr_pivot_inertia(rlqr_handle *h, int32_t *pd_verdict, int32_t *first_bad,
                               int64_t *inertia, rlqr_stream st);

/*
 * Which precision served each instance in the last rlqr_factor /
 * rlqr_factor_rhs and the rlqr_solve calls after it: path[b] = RLQR_PATH_*
 * (DEVICE array [B], written on stream st). In RLQR_SEQ_FP64 every instance
 * is RLQR_PATH_FP64. The mixed and scan modes decide per instance: a
 * float32 attempt that a pivot, the scan or refinement rejects is finished
 * in float64, and this call reports which instances that was (so a float32
 * result is not float64 work in disguise). Instances left out by
 * rlqr_set_skip keep their previous path. Errors: RLQR_E_INVALID (NULL h,
 * or NULL path for a non-empty batch), RLQR_E_STATE (no factorization),
 * RLQR_E_HIP.
 */
rlqr_status rlqr_precision_path(rlqr_handle *h, int32_t *path, rlqr_stream st);

/*
 * Float64 residual of the first-order conditions at z = (x, u, y) (Section
 * "Residual Computation"), written per instance in this order:
 *   for i < N: Q_i x_i + M_i u_i + A_i^T y_{i+1} + q_i - y_i      (n)
 *              M_i^T x_i + R_i u_i + B_i^T y_{i+1} + r_i          (m)
 *   Q_N x_N + q_N - y_N                                            (n)
 *   c_0 - delta y_0 - x_0                                          (n)
 *   for i < N: A_i x_i + B_i u_i + c_{i+1} - delta y_{i+1} - x_{i+1} (n)
 * res may be NULL (then only inst_relres); inst_relres [B] receives
 * ||res||_inf / ||[s; c]||_inf and may be NULL. Uses the lhs of the last
 * rlqr_factor. Errors: RLQR_E_INVALID, RLQR_E_STATE, RLQR_E_HIP.
 */
rlqr_status rlqr_residual(rlqr_handle *h, const rlqr_rhs *rhs, const rlqr_sol *z,
                          double *res, double *inst_relres, rlqr_stream st);

/* Size of the device array rlqr_residual_noalloc works in (per GPU). */
#define RLQR_NOALLOC_SCRATCH_BYTES (16u << 20)

/*
 * For callers that cannot allocate device memory (serving loops that must
 * not call hipMalloc, harnesses that forbid it): rlqr_residual without a
 * handle. Same residual, same order of rows and same inst_relres as
 * rlqr_residual on a handle created with the same shape (bit-identical: the
 * same kernels run), for z at the lhs given here. Allocates nothing: the
 * per-instance metadata, the stage-chunk list and the per-instance maxima
 * live in one device array of RLQR_NOALLOC_SCRATCH_BYTES that the library
 * holds on every GPU it runs on until the process ends. The batch must fit:
 * 160 B per instance + 16 B per stage chunk (ceil((N_b + 1) / 16) chunks for
 * n + m <= 16, ceil((N_b + 1) / 2) otherwise) + 2 x 8 B per instance, each
 * part rounded up to 256 B, at most RLQR_NOALLOC_SCRATCH_BYTES (e.g. 4096
 * instances of N = 128 with n + m <= 16 take 1.2 MB); a larger batch returns
 * RLQR_E_INVALID and touches nothing. Runs on the current device; st must
 * belong to it. The metadata are uploaded by a copy from pageable host memory,
 * which HIP performs synchronously with respect to the host, so the call
 * cannot be captured into a graph. Calls on one stream are ordered; calls
 * that overlap on one GPU (other streams, other host threads) share the
 * array and race. The array keeps the last call's contents; the maxima are
 * cleared at every call. Errors: RLQR_E_INVALID (NULL pointer, a shape out
 * of range, batch too large), RLQR_E_HIP.
 */
rlqr_status rlqr_residual_noalloc(const rlqr_shape *s, const rlqr_lhs *lhs, const rlqr_rhs *rhs,
                                  const rlqr_sol *z, double *res, double *inst_relres, rlqr_stream st);

/*
 * Capture rlqr_factor followed by rlqr_solve (same arguments as those calls)
 * on stream st into a HIP graph owned by the handle, for callers that repeat
 * the same solve on new values in the same buffers (a Newton iteration, a
 * serving loop): one graph launch then replaces the whole launch sequence of
 * the batch. Nothing executes during capture. A replay reads the arrays
 * behind the captured pointers as they are at replay time; every pointer must
 * stay valid while the graph may be launched. A new capture replaces the
 * previous graph. st must be a created stream (not NULL: the legacy default
 * stream cannot be captured). Errors: RLQR_E_INVALID, RLQR_E_HIP (capture or
 * instantiation failed; the handle keeps no graph).
 */
rlqr_status rlqr_graph_capture(rlqr_handle *h, const rlqr_lhs *lhs, const rlqr_rhs *rhs,
                               rlqr_sol *out, double rel_tol, int32_t max_refine,
                               int32_t *inst_status, double *inst_relres, rlqr_stream st);

/* Launch the captured graph on st (any stream). Errors: RLQR_E_INVALID,
 * RLQR_E_STATE (nothing captured), RLQR_E_HIP. */
rlqr_status rlqr_graph_launch(rlqr_handle *h, rlqr_stream st);

/* Release the handle and its workspace (waits for the device). NULL is a no-op. */
void rlqr_destroy(rlqr_handle *h);

/* Static description of a status code. */
const char *rlqr_status_string(rlqr_status s);

#ifdef __cplusplus
}
#endif
#endif /* RLQR_H */
