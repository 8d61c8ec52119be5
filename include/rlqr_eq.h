/*
 * rlqr_eq.h -- stagewise equality constraints eliminated into the
 * dual-regularized LQR of rlqr.h (Section "Applying the regularized IPM to
 * optimal control" of arXiv 2509.16370).
 *
 * In the Newton-KKT system of the regularized interior-point method every
 * equality constraint other than the dynamics carries the diagonal -1/eta of
 * the dual regularization. For ne_b rows per stage of instance b, with
 * Jacobian E_i = [E_x | E_u] (stage N: E_x only), residual r_e and penalties
 * D = diag(eta), the system in the sign convention of rlqr.h is
 *
 *     [[P, C^T, E^T], [C, -Delta, 0], [E, 0, -D^{-1}]] [z; y; w] = -[s; c; r_e].
 *
 * Its last row gives w = D (E z + r_e); substituted into the first, it
 * leaves a dual-regularized LQR whose stage Hessian and gradient are
 *
 *     [[Q, M], [M^T, R]] + E^T D E,    (q, r) + E^T D r_e,
 *
 * (A, B, c, Delta unchanged). The elimination keeps the problem stagewise
 * because E is stagewise and D diagonal. A Newton step is then
 *     rlqr_eq_reduce -> rlqr_factor / rlqr_solve on the reduced data ->
 *     rlqr_eq_recover (w).
 * The reduced matrix has the inertia of the full one minus the ne(N+1)
 * negative values of -D^{-1} (Haynsworth), so rlqr_pivot_inertia of the
 * reduced factorization certifies the full step.
 *
 * Layout (float64, DEVICE pointers owned by the caller, instances packed one
 * after another; offsets from rlqr_eq_offsets):
 *     E    per instance: stage i < N an ne x (n + m) row-major block
 *          [E_x | E_u], then stage N an ne x n block (E_x).
 *     r, eta, w   (N + 1) * ne per instance (stage-stacked rows);
 *          every eta entry must be > 0 and finite.
 * The reduced Q, M, R, q, r use the layout of rlqr.h and may be the input
 * arrays themselves (in place).
 */
#ifndef RLQR_EQ_H
#define RLQR_EQ_H

#include "rlqr.h"

#ifdef __cplusplus
extern "C" {
#endif

#define RLQR_EQ_MAX_NE 16 /* equality rows per stage */

typedef struct rlqr_eq rlqr_eq;

typedef struct {
  const double *E, *r, *eta;
} rlqr_eq_data;

enum { RLQR_EQ_ARR_E = 0, RLQR_EQ_ARR_V = 1 }; /* E; r, eta, w */

/* Context over the batch of handle h (its shapes and layout) with ne[b]
 * equality rows per stage of instance b ([host][B], 0 <= ne[b] <=
 * RLQR_EQ_MAX_NE). Allocates its small metadata once; *workspace_bytes
 * (may be NULL) receives the device bytes it holds. h must outlive it.
 * Errors: RLQR_E_INVALID (NULL, ne out of range, batch above 65535),
 * RLQR_E_NOMEM, RLQR_E_HIP. */
rlqr_status rlqr_eq_create(rlqr_eq **ctx, const rlqr_handle *h, const int32_t *ne, size_t *workspace_bytes);

/* The B + 1 exclusive prefix offsets (float64 elements) of RLQR_EQ_ARR_E or
 * RLQR_EQ_ARR_V into off [host]. Errors: RLQR_E_INVALID. */
rlqr_status rlqr_eq_offsets(const rlqr_eq *ctx, int32_t array, int64_t *off);

/* Write the reduced stage Hessian blocks (Qo, Mo, Ro) and gradient (qo, ro)
 * for lhs / rhs and the equality rows eq. The outputs may alias lhs->Q,
 * lhs->M, lhs->R, rhs->q, rhs->r (each element is read before it is
 * written by the same thread). Stream-ordered; allocates nothing.
 * Errors: RLQR_E_INVALID (NULL pointer when the batch is not empty),
 * RLQR_E_HIP. */
rlqr_status rlqr_eq_reduce(rlqr_eq *ctx, const rlqr_lhs *lhs, const rlqr_rhs *rhs, const rlqr_eq_data *eq,
                           double *Qo, double *Mo, double *Ro, double *qo, double *ro, rlqr_stream st);

/* w = D (E z + r_e) for a solution z = (x, u) of the reduced problem.
 * Errors: RLQR_E_INVALID, RLQR_E_HIP. */
rlqr_status rlqr_eq_recover(rlqr_eq *ctx, const rlqr_eq_data *eq, const rlqr_sol *z, double *w, rlqr_stream st);

void rlqr_eq_destroy(rlqr_eq *ctx);

#ifdef __cplusplus
}
#endif

#endif /* RLQR_EQ_H */
