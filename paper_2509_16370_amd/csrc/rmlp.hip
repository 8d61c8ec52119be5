// rmlp.hip -- kernels of the warm-start network (include/rmlp.h).
//
// GEMM: one 256-thread workgroup per 64 x 64 tile of C, four wavefronts of
// 32 x 32 (2 x 2 blocks of 16 x 16). op(A) and op(B) tiles of depth 16 are
// staged in LDS in the operand type (zero-filled outside the matrices), 32
// deep. The products use gfx950's v_mfma_f32_16x16x32_bf16 for bfloat16
// operands (lane l holds A[l & 15][8 (l >> 4) .. +7] and
// B[8 (l >> 4) .. +7][l & 15]) and v_mfma_f32_16x16x4_f32 for float32
// operands; both accumulate in float32 with the result of lane l in rows
// 4 (l >> 4) + v, column l & 15.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rmlp.h"

namespace {

typedef short s8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

// float32 -> bfloat16 bits, round to nearest even (NaN kept quiet)
__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x0040u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

template <typename T> struct Op;
template <> struct Op<float> {
  static __device__ __forceinline__ float load(const void* p, int64_t i) { return reinterpret_cast<const float*>(p)[i]; }
  static __device__ __forceinline__ void store(void* p, int64_t i, float v) { reinterpret_cast<float*>(p)[i] = v; }
};
template <> struct Op<uint16_t> {
  static __device__ __forceinline__ uint16_t load(const void* p, int64_t i) {
    return reinterpret_cast<const uint16_t*>(p)[i];
  }
  static __device__ __forceinline__ void store(void* p, int64_t i, float v) {
    reinterpret_cast<uint16_t*>(p)[i] = to_bf16(v);
  }
};

constexpr int TM = 64, TN = 64, TK = 32;

template <typename T, bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const void* __restrict__ A, int lda,
                                              const void* __restrict__ B, int ldb, float alpha, float beta,
                                              float* __restrict__ C, int ldc, const float* __restrict__ bias,
                                              int act, void* __restrict__ Cq) {
  __shared__ T As[TM][TK + 4];
  __shared__ T Bs[TK][TN + 4];
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int row0 = blockIdx.y * TM, col0 = blockIdx.x * TN;
  const int wr = 32 * (w >> 1), wc = 32 * (w & 1);
  f4 acc[2][2];
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = f4{0, 0, 0, 0};
  for (int k0 = 0; k0 < K; k0 += TK) {
    // stage op(A) (TM x TK) and op(B) (TK x TN), 8 elements per thread each
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int idx = tid + 256 * e;
      const int ai = idx / TK, ak = idx % TK;
      const int gi = row0 + ai, gk = k0 + ak;
      T va = T(0);
      if (gi < M && gk < K) va = Op<T>::load(A, TA ? (int64_t)gk * lda + gi : (int64_t)gi * lda + gk);
      As[ai][ak] = va;
      const int bk = idx / TN, bj = idx % TN;
      const int gk2 = k0 + bk, gj = col0 + bj;
      T vb = T(0);
      if (gk2 < K && gj < N) vb = Op<T>::load(B, TB ? (int64_t)gj * ldb + gk2 : (int64_t)gk2 * ldb + gj);
      Bs[bk][bj] = vb;
    }
    __syncthreads();
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
      for (int bj = 0; bj < 2; ++bj) {
        const int r = wr + 16 * bi + (lane & 15), c = wc + 16 * bj + (lane & 15), kq = lane >> 4;
        if constexpr (sizeof(T) == 2) {
          s8 a, b;
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            a[j] = (short)As[r][8 * kq + j];
            b[j] = (short)Bs[8 * kq + j][c];
          }
          acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b),
                                                                 acc[bi][bj], 0, 0, 0);
        } else {
#pragma unroll
          for (int kk = 0; kk < 8; ++kk)
            acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)As[r][4 * kk + kq], (float)Bs[4 * kk + kq][c],
                                                                acc[bi][bj], 0, 0, 0);
        }
      }
    __syncthreads();
  }
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int gi = row0 + wr + 16 * bi + 4 * (lane >> 4) + v;
        const int gj = col0 + wc + 16 * bj + (lane & 15);
        if (gi >= M || gj >= N) continue;
        float val = alpha * acc[bi][bj][v];
        if (beta != 0.0f) val += beta * C[(int64_t)gi * ldc + gj];
        if (bias) val += bias[gj];
        if (act == RMLP_ACT_TANH) val = tanhf(val);
        C[(int64_t)gi * ldc + gj] = val;
        if (Cq) Op<T>::store(Cq, (int64_t)gi * ldc + gj, val);
      }
}

template <typename T>
static hipError_t gemm_t(int ta, int tb, int M, int N, int K, const void* A, int lda, const void* B, int ldb,
                         float alpha, float beta, float* C, int ldc, const float* bias, int act, void* Cq,
                         hipStream_t st) {
  const dim3 grid((N + TN - 1) / TN, (M + TM - 1) / TM);
  if (!ta && !tb)
    hipLaunchKernelGGL((k_gemm<T, false, false>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, alpha, beta, C,
                       ldc, bias, act, Cq);
  else if (ta && !tb)
    hipLaunchKernelGGL((k_gemm<T, true, false>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, alpha, beta, C,
                       ldc, bias, act, Cq);
  else if (!ta && tb)
    hipLaunchKernelGGL((k_gemm<T, false, true>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, alpha, beta, C,
                       ldc, bias, act, Cq);
  else
    hipLaunchKernelGGL((k_gemm<T, true, true>), grid, dim3(256), 0, st, M, N, K, A, lda, B, ldb, alpha, beta, C,
                       ldc, bias, act, Cq);
  return hipGetLastError();
}

template <typename T>
__global__ void k_tanh_bwd(int64_t n, const float* dh, const float* h, float* dpre, void* dpreq) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float v = dh[i] * (1.0f - h[i] * h[i]);
  dpre[i] = v;
  if (dpreq) Op<T>::store(dpreq, i, v);
}

// one thread per column, rows summed in order
__global__ void k_colsum(int M, int N, const float* X, int ldx, float* out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  float s = 0.0f;
  for (int i = 0; i < M; ++i) s += X[(int64_t)i * ldx + j];
  out[j] = s;
}

// per-row partial sums (one block per row, fixed-order tree), then rows in order
template <typename T>
__global__ __launch_bounds__(256) void k_mse_rows(int M, int N, const float* pred, const float* target,
                                                  float* dpred, void* dpredq, double* rowsum) {
  __shared__ double red[256];
  const int i = blockIdx.x, t = threadIdx.x;
  double s = 0.0;
  const float inv = 1.0f / (float)M;
  for (int j = t; j < N; j += 256) {
    const int64_t k = (int64_t)i * N + j;
    const float d = pred[k] - target[k];
    s += (double)d * (double)d;
    dpred[k] = d * inv;
    if (dpredq) Op<T>::store(dpredq, k, d * inv);
  }
  red[t] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  if (t == 0) rowsum[i] = red[0];
}
__global__ void k_mse_total(int M, const double* rowsum, double* loss) {
  double s = 0.0;
  for (int i = 0; i < M; ++i) s += rowsum[i];
  *loss = s / (2.0 * M);
}

template <typename T>
__global__ void k_adam(int64_t n, float* w, void* wq, const float* g, float* m, float* v, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  if (wq) Op<T>::store(wq, i, wi);
}

template <typename T>
__global__ void k_cast(int64_t n, const float* x, void* y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) Op<T>::store(y, i, x[i]);
}

__global__ void k_affine_cols(int64_t total, int N, const float* X, const float* scale, const float* shift, float* Y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const int j = (int)(i % N);
  Y[i] = X[i] * scale[j] + shift[j];
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

#define RMLP_TRY(x)                            \
  do {                                         \
    if ((x) != hipSuccess) return RLQR_E_HIP; \
  } while (0)

extern "C" {

rlqr_status rmlp_gemm(int32_t dtype, int32_t transA, int32_t transB, int32_t M, int32_t N, int32_t K, const void* A,
                      int32_t lda, const void* B, int32_t ldb, float alpha, float beta, float* C, int32_t ldc,
                      const float* bias, int32_t act, void* Cq, rlqr_stream stv) {
  if (M < 0 || N < 0 || K < 0 || (dtype != RMLP_F32 && dtype != RMLP_BF16)) return RLQR_E_INVALID;
  if (act != RMLP_ACT_NONE && act != RMLP_ACT_TANH) return RLQR_E_INVALID;
  if (M == 0 || N == 0) return RLQR_OK;
  if (!A || !B || !C) return RLQR_E_INVALID;
  if (ldc < N || lda < (transA ? M : K) || ldb < (transB ? K : N)) return RLQR_E_INVALID;
  hipStream_t st = (hipStream_t)stv;
  RMLP_TRY(dtype == RMLP_F32 ? gemm_t<float>(transA, transB, M, N, K, A, lda, B, ldb, alpha, beta, C, ldc, bias, act,
                                             Cq, st)
                             : gemm_t<uint16_t>(transA, transB, M, N, K, A, lda, B, ldb, alpha, beta, C, ldc, bias,
                                                act, Cq, st));
  return RLQR_OK;
}

rlqr_status rmlp_tanh_backward(int32_t dtype, int64_t count, const float* dh, const float* h, float* dpre,
                               void* dpreq, rlqr_stream stv) {
  if (count < 0 || (dtype != RMLP_F32 && dtype != RMLP_BF16)) return RLQR_E_INVALID;
  if (count == 0) return RLQR_OK;
  if (!dh || !h || !dpre) return RLQR_E_INVALID;
  hipStream_t st = (hipStream_t)stv;
  if (dtype == RMLP_F32) hipLaunchKernelGGL(k_tanh_bwd<float>, dim3(blocks(count)), dim3(256), 0, st, count, dh, h, dpre, dpreq);
  else hipLaunchKernelGGL(k_tanh_bwd<uint16_t>, dim3(blocks(count)), dim3(256), 0, st, count, dh, h, dpre, dpreq);
  RMLP_TRY(hipGetLastError());
  return RLQR_OK;
}

rlqr_status rmlp_colsum(int32_t M, int32_t N, const float* X, int32_t ldx, float* out, rlqr_stream stv) {
  if (M < 0 || N < 0 || ldx < N) return RLQR_E_INVALID;
  if (N == 0) return RLQR_OK;
  if (!X || !out) return RLQR_E_INVALID;
  hipLaunchKernelGGL(k_colsum, dim3(blocks(N)), dim3(256), 0, (hipStream_t)stv, M, N, X, ldx, out);
  RMLP_TRY(hipGetLastError());
  return RLQR_OK;
}

rlqr_status rmlp_mse(int32_t dtype, int32_t M, int32_t N, const float* pred, const float* target, float* dpred,
                     void* dpredq, double* loss, rlqr_stream stv) {
  if (M < 1 || N < 1 || (dtype != RMLP_F32 && dtype != RMLP_BF16)) return RLQR_E_INVALID;
  if (!pred || !target || !dpred || !loss) return RLQR_E_INVALID;
  hipStream_t st = (hipStream_t)stv;
  // row sums land in loss[1 .. M] (the caller provides M + 1 doubles)
  if (dtype == RMLP_F32)
    hipLaunchKernelGGL(k_mse_rows<float>, dim3(M), dim3(256), 0, st, M, N, pred, target, dpred, dpredq, loss + 1);
  else
    hipLaunchKernelGGL(k_mse_rows<uint16_t>, dim3(M), dim3(256), 0, st, M, N, pred, target, dpred, dpredq, loss + 1);
  hipLaunchKernelGGL(k_mse_total, dim3(1), dim3(1), 0, st, M, (const double*)(loss + 1), loss);
  RMLP_TRY(hipGetLastError());
  return RLQR_OK;
}

rlqr_status rmlp_adam(int32_t dtype, int64_t count, float* w, void* wq, const float* g, float* m, float* v, float lr,
                      float beta1, float beta2, float eps, int32_t t, rlqr_stream stv) {
  if (count < 0 || t < 1 || (dtype != RMLP_F32 && dtype != RMLP_BF16)) return RLQR_E_INVALID;
  if (count == 0) return RLQR_OK;
  if (!w || !g || !m || !v) return RLQR_E_INVALID;
  const float c1 = 1.0f - powf(beta1, (float)t), c2 = 1.0f - powf(beta2, (float)t);
  hipStream_t st = (hipStream_t)stv;
  if (dtype == RMLP_F32)
    hipLaunchKernelGGL(k_adam<float>, dim3(blocks(count)), dim3(256), 0, st, count, w, wq, g, m, v, lr, beta1, beta2,
                       eps, c1, c2);
  else
    hipLaunchKernelGGL(k_adam<uint16_t>, dim3(blocks(count)), dim3(256), 0, st, count, w, wq, g, m, v, lr, beta1,
                       beta2, eps, c1, c2);
  RMLP_TRY(hipGetLastError());
  return RLQR_OK;
}

rlqr_status rmlp_affine_cols(int32_t M, int32_t N, const float* X, const float* scale, const float* shift, float* Y,
                             rlqr_stream stv) {
  if (M < 0 || N < 0) return RLQR_E_INVALID;
  if (M == 0 || N == 0) return RLQR_OK;
  if (!X || !scale || !shift || !Y) return RLQR_E_INVALID;
  const int64_t total = (int64_t)M * N;
  hipLaunchKernelGGL(k_affine_cols, dim3(blocks(total)), dim3(256), 0, (hipStream_t)stv, total, N, X, scale, shift, Y);
  RMLP_TRY(hipGetLastError());
  return RLQR_OK;
}

rlqr_status rmlp_cast(int32_t dtype, int64_t count, const float* x, void* y, rlqr_stream stv) {
  if (count < 0 || (dtype != RMLP_F32 && dtype != RMLP_BF16)) return RLQR_E_INVALID;
  if (count == 0) return RLQR_OK;
  if (!x || !y) return RLQR_E_INVALID;
  hipStream_t st = (hipStream_t)stv;
  if (dtype == RMLP_F32) hipLaunchKernelGGL(k_cast<float>, dim3(blocks(count)), dim3(256), 0, st, count, x, y);
  else hipLaunchKernelGGL(k_cast<uint16_t>, dim3(blocks(count)), dim3(256), 0, st, count, x, y);
  RMLP_TRY(hipGetLastError());
  return RLQR_OK;
}

}  // extern "C"
