// rlqr_device.h -- device-side building blocks shared by the rlqr kernels.
//
// One wavefront (64 lanes) owns one 16 x 16 tile. Tiles live in registers in
// the accumulator layout of the 16x16x4 MFMA instructions: lane l holds four
// entries (v = 0..3) of column l & 15. The rows differ by instruction:
// v_mfma_f32_16x16x4f32 puts row 4*(l>>4) + v in register v, while
// v_mfma_f64_16x16x4f64 puts row (l>>4) + 4*v there (measured on gfx950).
// trow<T>(grp, v) gives that row; every register tile of a kernel working with
// products in T uses it. The A/B operand layouts are the same for both:
// lane l supplies A[l & 15][k0 + (l>>4)] and B[k0 + (l>>4)][l & 15].
// Matrices smaller than 16 are zero-padded (identity-padded where a pivot
// sweep runs over them).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rlqr {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int NT = 16;   // tile edge
constexpr int LD = 17;   // LDS row stride (odd, avoids bank conflicts on column reads)

template <typename T> __device__ __forceinline__ constexpr int trow(int grp, int v);
template <> __device__ __forceinline__ constexpr int trow<float>(int grp, int v) { return 4 * grp + v; }
template <> __device__ __forceinline__ constexpr int trow<double>(int grp, int v) { return grp + 4 * v; }

template <typename T> struct AccT;
template <> struct AccT<double> { typedef d4 type; };
template <> struct AccT<float> { typedef f4 type; };

__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma16(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// C = op(A) * B for 16 x 16 tiles in LDS (row stride LD); op(A) = A or A^T.
// Returns the accumulator tile (row trow<T>(lane>>4, v), column lane&15).
template <typename T, bool TRANS_A>
__device__ __forceinline__ typename AccT<T>::type gemm16(const T* sa, const T* sb, int lane) {
  typename AccT<T>::type acc = {0, 0, 0, 0};
  const int i = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int k = 4 * kk + kq;
    const T av = TRANS_A ? sa[k * LD + i] : sa[i * LD + k];
    const T bv = sb[k * LD + i];
    acc = mfma16(av, bv, acc);
  }
  return acc;
}

// Per-instance pivot bookkeeping for the certificate.
struct PivStats {
  int npos, nneg, nzero, first_bad;
  double minrel;
  __device__ void init() { npos = nneg = nzero = 0; first_bad = -1; minrel = 1.0e300; }
};

// A value every lane holds identically, moved to scalar registers.
__device__ __forceinline__ double uniform(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the four 16-lane groups (lanes l, l^16, l^32, l^48).
__device__ __forceinline__ double group_sum(double v) {
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

// Symmetric pivot sweep (Gauss-Jordan on a symmetric tile) over pivots
// j0 .. j1-1 of the tile X held in registers (accumulator layout, float64).
// Sweeping a block S of a symmetric matrix [[X_SS, X_ST], [X_TS, X_TT]] turns
// it into [[-X_SS^{-1}, X_SS^{-1} X_ST], [X_TS X_SS^{-1}, X_TT - X_TS X_SS^{-1} X_ST]].
// The pivots met are the D entries of the unpivoted LDL^T of X_SS.
// Every update is written so that exact symmetry is preserved bit for bit.
// colbuf: 2 x 16 doubles of LDS (double-buffered pivot column).
// code: certificate code shared by all pivots of the block. TL selects the row map.
// LDS ordering inside a one-wavefront workgroup: the LDS unit executes one
// wavefront's instructions in order, so a compiler-level barrier suffices.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename TL>
__device__ __forceinline__ void sweep16(double (&X)[4], int j0, int j1, int lane,
                                        double* colbuf, PivStats& ps, int code,
                                        double tol, double scale) {
  const int col = lane & 15, grp = lane >> 4;
  for (int j = j0; j < j1; ++j) {
    double* cb = colbuf + 16 * (j & 1);
    if (col == j) {
#pragma unroll
      for (int v = 0; v < 4; ++v) cb[trow<TL>(grp, v)] = X[v];
    }
    wave_sync();
    const double d = uniform(cb[j]);
    const double cc = cb[col];
    double ci[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) ci[v] = cb[trow<TL>(grp, v)];
    const bool zero = !(fabs(d) > tol);
    ps.nzero += zero ? 1 : 0;
    ps.npos += (!zero && d > 0) ? 1 : 0;
    ps.nneg += (!zero && d < 0) ? 1 : 0;
    ps.first_bad = ((zero || d < 0) && ps.first_bad < 0) ? code : ps.first_bad;
    ps.minrel = fmin(ps.minrel, fabs(d) / scale);
    const double rd = zero ? 0.0 : 1.0 / d;
    const double ccr = cc * rd;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = trow<TL>(grp, v);
      const double gen = __fma_rn(-(ci[v] * cc), rd, X[v]);
      const double onrow = (col == j) ? -rd : ccr;
      const double offrow = (col == j) ? ci[v] * rd : gen;
      X[v] = (r == j) ? onrow : offrow;
    }
  }
}

// Block numbering of a stage tile Z (NZ = 16 TZ) in the multi-wavefront
// kernels: the TX x TX state blocks first (row-major, numbered like the blocks
// of the state tiles), then the (x, u) blocks, then the u block-rows.
template <int TX, int TZ>
__device__ __forceinline__ void zmap(int z, int& I, int& J) {
  if (z < TX * TX) {
    I = z / TX;
    J = z % TX;
    return;
  }
  int e = z - TX * TX;
  if (TZ > TX && e < TX * (TZ - TX)) {
    I = e / (TZ - TX);
    J = TX + e % (TZ - TX);
    return;
  }
  e -= TX * (TZ - TX);
  I = TX + e / TZ;
  J = e % TZ;
}

}  // namespace rlqr
