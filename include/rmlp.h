/*
 * rmlp.h -- C ABI of the hand-written kernels that train and run the
 * warm-start network of the interior-point driver (a multilayer perceptron:
 * dense layers Y = X W + b with tanh between them, trained on a scaled mean
 * squared error with Adam).
 *
 * Matrices are row-major with explicit leading dimensions (in elements).
 * Operand arrays are float32 (RMLP_F32) or bfloat16 (RMLP_BF16, stored as
 * uint16 bit patterns, round-to-nearest-even); every product accumulates in
 * float32 on the matrix cores. Pointers are DEVICE pointers. Calls are
 * ordered on the stream and return before the GPU finishes. Errors:
 * RLQR_E_INVALID (bad sizes, NULL required pointers, unknown dtype),
 * RLQR_E_HIP (launch failure).
 */
#ifndef RMLP_H
#define RMLP_H

#include "rlqr.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { RMLP_F32 = 0, RMLP_BF16 = 1 };
enum { RMLP_ACT_NONE = 0, RMLP_ACT_TANH = 1 };

/*
 * C (M x N, float32) = alpha * op(A) * op(B) + beta * C + bias (broadcast
 * over rows, may be NULL), then the activation act; Cq (may be NULL)
 * receives the result in dtype as well. op(A) is M x K: A (M x K, lda) or,
 * with transA, the transpose of A (K x M, lda); likewise op(B) is K x N.
 * beta == 0 does not read C.
 */
rlqr_status rmlp_gemm(int32_t dtype, int32_t transA, int32_t transB, int32_t M, int32_t N, int32_t K,
                      const void *A, int32_t lda, const void *B, int32_t ldb, float alpha, float beta,
                      float *C, int32_t ldc, const float *bias, int32_t act, void *Cq, rlqr_stream st);

/* dpre[i] = dh[i] * (1 - h[i]^2) (tanh backward, count elements); dpreq (may
 * be NULL) receives it in dtype. */
rlqr_status rmlp_tanh_backward(int32_t dtype, int64_t count, const float *dh, const float *h, float *dpre,
                               void *dpreq, rlqr_stream st);

/* out[j] = sum_i X[i][j] (M x N, ldx): bias gradients. Fixed summation order. */
rlqr_status rmlp_colsum(int32_t M, int32_t N, const float *X, int32_t ldx, float *out, rlqr_stream st);

/* Mean squared error over an M x N batch: loss[0] = 1/(2M) sum (pred - target)^2
 * (float64, fixed summation order; loss holds M + 1 doubles, loss[1..M] are
 * per-row scratch), dpred = (pred - target) / M in float32 and, if dpredq is
 * not NULL, in dtype. */
rlqr_status rmlp_mse(int32_t dtype, int32_t M, int32_t N, const float *pred, const float *target, float *dpred,
                     void *dpredq, double *loss, rlqr_stream st);

/* Adam step t >= 1 on count float32 weights w with moments m, v; wq (may be
 * NULL) receives the updated weights in dtype. */
rlqr_status rmlp_adam(int32_t dtype, int64_t count, float *w, void *wq, const float *g, float *m, float *v,
                      float lr, float beta1, float beta2, float eps, int32_t t, rlqr_stream st);

/* Y = X * scale + shift per column (M x N, ld = N; scale, shift [N]); Y may be X. */
rlqr_status rmlp_affine_cols(int32_t M, int32_t N, const float *X, const float *scale, const float *shift, float *Y,
                             rlqr_stream st);

/* y = x converted to dtype (count elements). */
rlqr_status rmlp_cast(int32_t dtype, int64_t count, const float *x, void *y, rlqr_stream st);

#ifdef __cplusplus
}
#endif
#endif /* RMLP_H */
