/*
 * rlqr_spd.h -- general SPD per-stage regularization Delta_i for the
 * dual-regularized LQR solver of rlqr.h (Definition in Section
 * "Dual-Regularized LQR" of arXiv 2509.16370: every Delta_i may be any
 * symmetric positive definite matrix; the regularized interior-point method
 * of the paper produces such blocks from its penalties Delta_C, Delta_G).
 *
 * Method. Each Delta_i is factored Delta_i = L_i D_i L_i^T (L_i unit lower
 * triangular, D_i positive diagonal). The congruence
 *     x_i = L_i x~_i,   u_i = u~_i,   y_i = L_i^{-T} y~_i
 * maps the problem to one with the diagonal regularization D_i and data
 *     Q~_i = L_i^T Q_i L_i,  M~_i = L_i^T M_i,  R~_i = R_i,
 *     A~_i = L_{i+1}^{-1} A_i L_i,  B~_i = L_{i+1}^{-1} B_i,
 *     q~_i = L_i^T q_i,  r~_i = r_i,  c~_i = L_i^{-1} c_i,
 * whose KKT matrix is T^T K T for T = blockdiag(L_i on x_i, I on u_i,
 * L_i^{-T} on y_i), so its inertia is that of K (Sylvester) and its solution
 * is T^{-1} times K's. The transformed problem is solved by the per-stage
 * diagonal path of rlqr.h (rlqr_lhs.delta_diag = D_i), in the handle's mode.
 * Its state pivots are those of I + D_i^{1/2} P~_i D_i^{1/2} =
 * I + C_i^T P_i C_i with C_i = L_i D_i^{1/2} the Cholesky factor of Delta_i:
 * a symmetric matrix congruent to the state pivot S_i = P_i + Delta_i^{-1}
 * (C_i^T S_i C_i) and similar to I + Delta_i P_i, as Section "Inertia
 * Certification" allows. rlqr_pivot_inertia on the handle therefore
 * certifies the SPD problem.
 *
 * Refinement. rlqr_spd_solve refines the transformed problem with the
 * handle's refinement, maps the solution back, then computes the float64
 * residual of the original system (Section "Residual Computation" with
 * Delta_i y_i a matrix-vector product) and, while an instance is above the
 * tolerance, corrects z <- z + T solve(T^T residual) (the same congruence
 * applied to the residual as a right-hand side). The outer loop reads one
 * flag from the device per pass (a stream synchronization), so this call
 * cannot be captured into a graph.
 *
 * Layout. Delta: float64, instance after instance, (N+1) n x n row-major
 * blocks per instance (the layout of Q in rlqr.h); each block symmetric
 * positive definite (only the lower triangle is read). A block that is not
 * positive definite gives non-finite results for its instance, reported as
 * RLQR_INST_NONFINITE.
 */
#ifndef RLQR_SPD_H
#define RLQR_SPD_H

#include "rlqr.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rlqr_spd rlqr_spd;

/* Context over the batch of handle h (its shapes, layout and mode).
 * Allocates once: the factors L_i, L_i^{-1}, D_i, the transformed Q, M, A, B
 * and right-hand sides, and residual vectors (about 4x the left-hand side of
 * the batch in float64); *workspace_bytes (may be NULL) receives the device
 * bytes it holds. h must outlive the context.
 * Errors: RLQR_E_INVALID (NULL), RLQR_E_NOMEM, RLQR_E_HIP. */
rlqr_status rlqr_spd_create(rlqr_spd **ctx, rlqr_handle *h, size_t *workspace_bytes);

/* Factor D_i, L_i of every Delta_i, transform the left-hand side and run
 * rlqr_factor on the handle with the transformed data and delta_diag = D.
 * lhs->delta and lhs->delta_diag are not read. lhs and Delta must stay valid
 * and unchanged until the last rlqr_spd_solve / rlqr_spd_residual on this
 * factorization. Errors: RLQR_E_INVALID (NULL pointer for a non-empty batch),
 * RLQR_E_HIP, and the errors of rlqr_factor. */
rlqr_status rlqr_spd_factor(rlqr_spd *ctx, const rlqr_lhs *lhs, const double *Delta, rlqr_stream st);

/* Solve for one right-hand side of the original system: transform it,
 * rlqr_solve on the handle (refined to rel_tol against the transformed
 * problem's residual, up to max_refine steps), map back, then up to
 * max_refine outer correction steps against the original float64 residual
 * (above). inst_status [B] (RLQR_INST_*: SINGULAR, NONFINITE and NOT_PD from
 * the handle's factorization, NOT_CONVERGED when the original relative
 * residual stays above rel_tol) and inst_relres [B] (original relative
 * residual ||res||_inf / ||[s; c]||_inf) may be NULL. Synchronizes the
 * stream once per outer step. Errors: RLQR_E_INVALID, RLQR_E_STATE (no
 * rlqr_spd_factor), RLQR_E_HIP, and those of rlqr_solve. */
rlqr_status rlqr_spd_solve(rlqr_spd *ctx, const rlqr_rhs *rhs, rlqr_sol *out, double rel_tol,
                           int32_t max_refine, int32_t *inst_status, double *inst_relres, rlqr_stream st);

/* Float64 residual of the original system at z (row order of rlqr_residual;
 * dual rows c_0 - Delta_0 y_0 - x_0 and A_i x_i + B_i u_i + c_{i+1} -
 * Delta_{i+1} y_{i+1} - x_{i+1}) with the lhs and Delta of the last
 * rlqr_spd_factor. res (may be NULL) and inst_relres [B] (may be NULL).
 * Errors: RLQR_E_INVALID, RLQR_E_STATE, RLQR_E_HIP. */
rlqr_status rlqr_spd_residual(rlqr_spd *ctx, const rlqr_rhs *rhs, const rlqr_sol *z, double *res,
                              double *inst_relres, rlqr_stream st);

void rlqr_spd_destroy(rlqr_spd *ctx);

#ifdef __cplusplus
}
#endif

#endif /* RLQR_SPD_H */
