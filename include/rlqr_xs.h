/*
 * rlqr_xs.h -- cross-stage variables: the arrowhead Newton step of Section
 * "Cross-Stage Variables" of arXiv 2509.16370.
 *
 * With p variables theta shared by every stage the Newton system of each
 * instance is (eq. cross-stage-kkt)
 *
 *     [[K, J], [J^T, H]] [dw; dtheta] = -[r_w; r_theta],
 *
 * K the dual-regularized LQR matrix of rlqr.h, J the p columns of
 * derivatives with respect to theta, H symmetric p x p. It is solved through
 * the Schur complement S = H - J^T K^{-1} J (eq. cross-stage-schur): the
 * factorization step computes K^{-1} J with p solves that reuse the LQR
 * factorization and factors S; each solve then needs one more LQR solve,
 * dtheta = -S^{-1}(r_theta - J^T K^{-1} r_w) and dw = -K^{-1} r_w - K^{-1}J
 * dtheta (a combination of solves already made), followed by iterative
 * refinement against the float64 residual of the whole arrowhead system.
 *
 * Layout. A column of J and r_w are in the row space of K and use the
 * layout of an LQR right-hand side (rlqr_rhs: x-rows in q, u-rows in r, dual
 * rows in c); column j of J is (Jq + j*Lq, Jr + j*Lr, Jc + j*Lc) with Lq, Lr,
 * Lc the batch lengths of q, r, c. dw uses the solution layout (rlqr_sol).
 * H is [B][p][p] row-major (symmetrized on use), r_theta and dtheta [B][p].
 * Every pointer is a DEVICE pointer owned by the caller; float64.
 *
 * Statuses (inst_status, RLQR_INST_*): SINGULAR when K or S has a zero pivot
 * (S: |d| <= 1e3 * p * eps64 * max|diag S|); NOT_CONVERGED when the relative
 * residual max(|res_w|, |res_theta|) / max(|r_w|, |r_theta|) (inf-norms) is
 * above rel_tol after the refinement; NOT_PD when the arrowhead matrix lacks
 * the inertia of K's target plus p positive values (K's certificate fails
 * or S is not positive definite; Haynsworth: In = In(K) + In(S)); else OK.
 *
 * Threading. An rlqr_xs drives the LQR handle it was created on: neither may
 * be used from another stream while an rlqr_xs call is in flight.
 */
#ifndef RLQR_XS_H
#define RLQR_XS_H

#include "rlqr.h"

#ifdef __cplusplus
extern "C" {
#endif

#define RLQR_XS_MAX_P 8

typedef struct rlqr_xs rlqr_xs;

typedef struct {
  const double *Jq, *Jr, *Jc;  /* p stacked columns of J in the rhs layout     */
  const double *H;             /* [B][p][p]                                    */
} rlqr_xs_lhs;

/*
 * Create the cross-stage context for p variables on LQR handle h (which it
 * uses but does not own; h must outlive it). Allocates the p + 3 solution-
 * and right-hand-side-sized vectors and the per-instance blocks (the only
 * allocation; *workspace_bytes may be NULL). Errors: RLQR_E_INVALID (NULL,
 * p < 1 or p > RLQR_XS_MAX_P), RLQR_E_NOMEM, RLQR_E_HIP.
 */
rlqr_status rlqr_xs_create(rlqr_xs **x, rlqr_handle *h, int32_t p, size_t *workspace_bytes);

/*
 * Factor: rlqr_factor(h, lhs), the p solves K^{-1} J_j (rlqr_solve with
 * rel_tol, max_refine), S = H - J^T K^{-1} J (float64 dot products over each
 * instance's rows), and the unpivoted LDL^T of S in float64 with its pivot
 * signs. The lhs and xl arrays must stay valid until the last rlqr_xs_solve.
 * Errors: RLQR_E_INVALID, RLQR_E_HIP and those of rlqr_factor/rlqr_solve.
 */
rlqr_status rlqr_xs_factor(rlqr_xs *x, const rlqr_lhs *lhs, const rlqr_xs_lhs *xl,
                           double rel_tol, int32_t max_refine, rlqr_stream st);

/*
 * Solve the arrowhead system for (r_w, r_theta), then refine: up to
 * max_refine times, while an instance's relative residual exceeds rel_tol,
 * (dw, dtheta) += the Schur-route solution for the float64 residual. Each
 * LQR solve inside uses rlqr_solve with the same rel_tol and max_refine.
 * Instances that have converged are left unchanged by later passes. When
 * max_refine > 0 the call waits on st once per pass for the count of
 * unconverged instances (it stops early when there are none), so unlike
 * the rlqr.h calls it may return after the GPU work. inst_status and
 * inst_relres [B] may be NULL. Errors: RLQR_E_INVALID, RLQR_E_STATE (no
 * rlqr_xs_factor), RLQR_E_HIP.
 */
rlqr_status rlqr_xs_solve(rlqr_xs *x, const rlqr_rhs *rw, const double *rtheta,
                          rlqr_sol *dw, double *dtheta, double rel_tol, int32_t max_refine,
                          int32_t *inst_status, double *inst_relres, rlqr_stream st);

/*
 * Inertia of the arrowhead matrix from the pivots: pd_verdict[b] = 1 iff
 * K's certificate holds and S is positive definite; inertia[3b..3b+2] =
 * In(K) (rlqr_pivot_inertia) + the sign counts of S's pivots. Either output
 * may be NULL. Errors: RLQR_E_STATE, RLQR_E_HIP.
 */
rlqr_status rlqr_xs_inertia(rlqr_xs *x, int32_t *pd_verdict, int64_t *inertia, rlqr_stream st);

/* Release the context (waits for the device). NULL is a no-op. */
void rlqr_xs_destroy(rlqr_xs *x);

#ifdef __cplusplus
}
#endif

#endif /* RLQR_XS_H */
