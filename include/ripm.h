/*
 * ripm.h -- C ABI of the batched regularized interior-point driver for
 * constrained trajectory problems.
 *
 * The method is the regularized primal-dual interior-point method of Section
 * "The Regularized Interior Point Method" of arXiv 2509.16370: barrier-
 * Lagrangian L = f - mu sum log s + y^T c + z^T (g + s), augmented
 * barrier-Lagrangian merit L + 1/2 eta (|c|^2 + |g + s|^2) (Delta_C =
 * Delta_G = eta I), Newton-KKT system eq. ipm-4x4-newton-kkt reduced by
 * eliminating ds and then dz (Section "Applying the regularized IPM to
 * optimal control"). The reduced system of every Newton step is one batched
 * dual-regularized LQR with delta = 1/eta, solved by rlqr_factor /
 * rlqr_solve (rlqr.h); its pivot certificate (Theorem
 * inertia-al-descent-theorem) decides the inertia correction rho I.
 *
 * Problem b of a batch (all share the model):
 *   min  sum_{i<N} 1/2 wx |x_i - goal_b|^2 + 1/2 wu |u_i|^2 + 1/2 wN |x_N - goal_b|^2
 *   s.t. x_0 = x0_b,  x_{i+1} = x_i + dt tanh(A x_i + B u_i)            (i < N)
 *        a_j^T x_i <= xmax (j = 1, 2; i = 0..N),  |u_i| <= umax componentwise
 * Inequalities per stage i < N: [a_1^T x - xmax, a_2^T x - xmax, u - umax,
 * -u - umax] (ng = 2 + 2m rows); stage N: the two state rows.
 * Optional stagewise equality rows E_u u_i = b_i (i < N; ne rows per stage,
 * E_u shared, b per problem and stage) with multipliers y_e: like the
 * dynamics rows they carry the -1/eta dual-regularization block, and they are
 * eliminated into the Newton LQR (Section "Applying the regularized IPM to
 * optimal control": the other equality rows go "in the same fashion"):
 * R_i += eta E_u^T E_u, r_i += E_u^T (y_e + eta e_i) with e_i = E_u u_i - b_i,
 * then dy_e = eta (E_u du_i + e_i) and the full step y_e <- y_e + dy_e; the
 * merit gains y_e^T e + eta/2 |e|^2 and the convergence test |e|.
 *
 * Iteration rules (where the paper leaves them open): exact Lagrangian
 * Hessian; rho = 0 at start, rho <- max(1e-8, 10 rho) while the certificate
 * fails, rho <- rho / 3 after each iteration; fraction to the boundary
 * tau = max(0.99, 1 - mu); Armijo (1e-4) on the merit over the step ladder
 * alpha_max 2^-k, k = 0..11 (the last if none passes); y <- y + dy,
 * z <- z + alpha_z dz; mu <- max(mu / 10, 1e-9) when the barrier error is
 * <= 10 mu; converged when |grad_x L|, |c|, |g + s| and |s z| (inf-norms)
 * are all <= tol.
 *
 * Memory: pointers are DEVICE pointers unless marked [host]; float64,
 * row-major, instance-major. The handle owns all iterates and workspace.
 * Errors: negative rlqr_status codes as in rlqr.h.
 */
#ifndef RIPM_H
#define RIPM_H

#include "rlqr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ripm_handle ripm_handle;

typedef struct {
  int32_t batch, N, n, m;      /* n + m <= 32 */
  double dt, wx, wu, wN, xmax, umax;
  const double *A, *B, *a;     /* [host] model: A (n x n), B (n x m), a (2 x n) */
  double eta;                  /* Delta_C = Delta_G = eta I; LQR delta = 1 / eta */
  double tol;                  /* convergence tolerance (inf-norms) */
  int32_t lqr_mode;            /* RLQR_SEQ_FP64 or RLQR_SEQ_MIXED for the Newton LQR */
  int32_t ne;                  /* stagewise equality rows per stage, 0 <= ne <= min(m, 8) */
  const double *Eu;            /* [host] E_u (ne x m), full row rank; NULL when ne = 0 */
} ripm_problem;

/* Allocate the driver (iterates, Newton-LQR handle and workspace).
 * Errors: RLQR_E_INVALID, RLQR_E_NOMEM, RLQR_E_HIP. */
rlqr_status ripm_create(ripm_handle **h, const ripm_problem *p, size_t *workspace_bytes);

/*
 * Set the problems and the starting point. x0, goal: [batch][n]; eb: the
 * equality rows' right-hand sides [batch][N][ne] (NULL when ne = 0; their
 * multipliers start at 0).
 * warm == NULL: cold start x_i = x0, u_i = 0, y = 0, s = max(-g, 1e-2),
 * z = mu0 / s, mu0 = 0.1. Otherwise warm = [batch][(N+1)n + Nm + (N+1)n +
 * (N+1)ng] holding x, u, y and log z per problem (rows of stage N beyond its
 * two state rows are ignored): s = max(-g(x), 1e-2), z = exp(log z),
 * mu0 = mean(s z) clipped to [1e-9, 0.1].
 */
rlqr_status ripm_start(ripm_handle *h, const double *x0, const double *goal, const double *warm,
                       const double *eb, rlqr_stream st);

/* One iteration for every problem not yet converged. *active [host] receives
 * the number of problems still running afterwards (this call synchronizes
 * the stream). */
rlqr_status ripm_iterate(ripm_handle *h, int32_t *active, rlqr_stream st);

/* Iterate until every problem converged or max_iter iterations. iters and
 * converged [host][batch] (may be NULL) receive per-problem counts and flags. */
rlqr_status ripm_solve(ripm_handle *h, int32_t max_iter, int32_t *iters, int32_t *converged,
                       rlqr_stream st);

/* Copy the current iterate: x [batch][(N+1)n], u [batch][Nm], y [batch][(N+1)n],
 * z [batch][(N+1)ng], ye [batch][N][ne] (any may be NULL; ye is not written
 * when ne = 0). */
rlqr_status ripm_solution(ripm_handle *h, double *x, double *u, double *y, double *z, double *ye,
                          rlqr_stream st);

void ripm_destroy(ripm_handle *h);

#ifdef __cplusplus
}
#endif
#endif /* RIPM_H */
