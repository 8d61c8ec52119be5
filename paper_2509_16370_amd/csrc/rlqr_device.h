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
  int nonfinite;  // a pivot was NaN or +-Inf (it also counts as zero)
  double minrel;
  __device__ void init() { npos = nneg = nzero = nonfinite = 0; first_bad = -1; minrel = 1.0e300; }
};

// A value every lane holds identically, moved to scalar registers.
__device__ __forceinline__ double uniform(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// gfx950's lane-permute swaps, each 32-bit half separately (old = src = x):
// permlane16_swap gives [0] = rows (0, 0, 2, 2) and [1] = rows (1, 1, 3, 3)
// of x (rows = 16-lane groups, same lane within the row), permlane32_swap
// [0] = rows (0, 1, 0, 1) and [1] = rows (2, 3, 2, 3). VALU operations: no
// LDS round trip as with ds_bpermute.
__device__ __forceinline__ double mk_double(unsigned lo, unsigned hi) {
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ void pl16(double x, double& a, double& b) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  const auto l = __builtin_amdgcn_permlane16_swap((unsigned)u, (unsigned)u, true, false);
  const auto h = __builtin_amdgcn_permlane16_swap((unsigned)(u >> 32), (unsigned)(u >> 32), true, false);
  a = mk_double(l[0], h[0]);
  b = mk_double(l[1], h[1]);
}
__device__ __forceinline__ void pl32(double x, double& a, double& b) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  const auto l = __builtin_amdgcn_permlane32_swap((unsigned)u, (unsigned)u, true, false);
  const auto h = __builtin_amdgcn_permlane32_swap((unsigned)(u >> 32), (unsigned)(u >> 32), true, false);
  a = mk_double(l[0], h[0]);
  b = mk_double(l[1], h[1]);
}

// Sum over the four 16-lane groups (lanes l, l^16, l^32, l^48): (r0 + r1) +
// (r2 + r3) in every lane, the same value a butterfly over lane xor 16, 32
// gives (the additions commute exactly).
__device__ __forceinline__ double group_sum(double v) {
  double a, b;
  pl16(v, a, b);
  const double s = a + b;  // rows 0, 1: r0 + r1; rows 2, 3: r2 + r3
  pl32(s, a, b);
  return a + b;
}

// x of row group G (lane 16 G + (lane & 15)), in every row group
template <int G>
__device__ __forceinline__ double group_bcast(double x) {
  double a, b;
  pl16(x, a, b);
  pl32((G & 1) ? b : a, a, b);
  return (G & 2) ? b : a;
}
template <int G>
__device__ __forceinline__ float group_bcast_f(float x) {
  const unsigned u = __float_as_uint(x);
  const auto a = __builtin_amdgcn_permlane16_swap(u, u, true, false);
  const unsigned y = (G & 1) ? a[1] : a[0];
  const auto b = __builtin_amdgcn_permlane32_swap(y, y, true, false);
  return __uint_as_float((G & 2) ? b[1] : b[0]);
}

// max that keeps a NaN (fmax drops it): residual maxima must not hide a
// non-finite residual entry
__device__ __forceinline__ double maxnan(double a, double b) { return (b > a || b != b) ? b : a; }

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = maxnan(v, __shfl_xor(v, o));
  return v;
}

// LDS ordering inside a one-wavefront workgroup: the LDS unit executes one
// wavefront's instructions in order, so a compiler-level barrier suffices.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 1 / d by Newton-Raphson from the hardware estimate: each step
// r <- r + r (1 - d r) squares the relative error, so two steps from the
// estimate reach float64 unit roundoff (within one ulp of the rounded quotient).
__device__ __forceinline__ double recip(double d) {
  double r = __builtin_amdgcn_rcp(d);
  double e = __fma_rn(-d, r, 1.0);
  r = __fma_rn(r, e, r);
  e = __fma_rn(-d, r, 1.0);
  return __fma_rn(r, e, r);
}

// value of lane J of each 16-lane row, for every lane of that row (DPP row broadcast)
template <int J>
__device__ __forceinline__ double row_bcast(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), 0x150 + J, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x150 + J, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// x of lane `src` (a wave-uniform lane index), moved to scalar registers
__device__ __forceinline__ double lane_value(double x, int src) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// max over the 16 lanes of each row (DPP row rotations), then over the rows
__device__ __forceinline__ double wave_max_rows(double s) {
#pragma unroll
  for (int k = 1; k < 16; k <<= 1) {
    const long long b = __double_as_longlong(s);
    int lo, hi;
    switch (k) {
      case 1: lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), 0x121, 0xf, 0xf, false);
              hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x121, 0xf, 0xf, false); break;
      case 2: lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), 0x122, 0xf, 0xf, false);
              hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x122, 0xf, 0xf, false); break;
      case 4: lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), 0x124, 0xf, 0xf, false);
              hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x124, 0xf, 0xf, false); break;
      default: lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), 0x128, 0xf, 0xf, false);
               hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x128, 0xf, 0xf, false); break;
    }
    s = fmax(s, __longlong_as_double(((long long)hi << 32) | (unsigned int)lo));
  }
  return fmax(fmax(lane_value(s, 0), lane_value(s, 16)), fmax(lane_value(s, 32), lane_value(s, 48)));
}

// One pivot J of the symmetric sweep (see sweep16). Row J of the tile sits in
// row group GJ, register VJ; column J of row group g sits in lane 16 g + J.
template <typename TL, int J>
__device__ __forceinline__ void sweep_pivot(double (&X)[4], int lane, double tol, double& dsave) {
  constexpr bool F32 = trow<TL>(1, 0) == 4;
  constexpr int GJ = F32 ? (J >> 2) : (J & 3);
  constexpr int VJ = F32 ? (J & 3) : (J >> 2);
  const int col = lane & 15, grp = lane >> 4;
  const double d = lane_value(X[VJ], 16 * GJ + J);        // X[J][J]
  const double cc = group_bcast<GJ>(X[VJ]);                // X[J][col] = X[col][J]
  double ci[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) ci[v] = row_bcast<J>(X[v]);  // X[row(v)][J]
  const bool nz = fabs(d) > tol;
  dsave = (lane == J) ? d : dsave;
  const double rd = nz ? recip(d) : 0.0;
  // One formula for every element but row J: X - ci cc' / d with X zeroed in
  // column J and cc' = -1 there, so column J becomes ci / d (the same
  // rounding as ci * rd); row J is cc' / d (cc / d, and -1/d at (J, J)).
  const bool cj = col == J;
  const double ccs = cj ? -1.0 : cc;
  const double keep = cj ? 0.0 : 1.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double gen = __fma_rn(-(ci[v] * ccs), rd, X[v] * keep);
    if (v == VJ) X[v] = (grp == GJ) ? ccs * rd : gen;
    else X[v] = gen;
  }
}

// Symmetric pivot sweep (Gauss-Jordan on a symmetric tile) over pivots
// j0 .. j1-1 of the tile X held in registers (accumulator layout, float64).
// Sweeping a block S of a symmetric matrix [[X_SS, X_ST], [X_TS, X_TT]] turns
// it into [[-X_SS^{-1}, X_SS^{-1} X_ST], [X_TS X_SS^{-1}, X_TT - X_TS X_SS^{-1} X_ST]].
// The pivots met are the D entries of the unpivoted LDL^T of X_SS.
// Every update is written so that exact symmetry is preserved bit for bit
// (the product ci * cc is formed before the scaling). The pivot column moves
// between lanes by DPP row broadcasts, the pivot row by two lane-permute swaps; the
// pivots are counted once per sweep from a ballot.
// code: certificate code shared by all pivots of the block. TL selects the row map.
template <typename TL>
__device__ __forceinline__ void sweep16(double (&X)[4], int j0, int j1, int lane, PivStats& ps, int code,
                                        double tol, double scale) {
  double dsave = 1.0;
#define RLQR_PIVOT(J) \
  if (J >= j0 && J < j1) sweep_pivot<TL, J>(X, lane, tol, dsave);
  RLQR_PIVOT(0) RLQR_PIVOT(1) RLQR_PIVOT(2) RLQR_PIVOT(3) RLQR_PIVOT(4) RLQR_PIVOT(5) RLQR_PIVOT(6)
  RLQR_PIVOT(7) RLQR_PIVOT(8) RLQR_PIVOT(9) RLQR_PIVOT(10) RLQR_PIVOT(11) RLQR_PIVOT(12) RLQR_PIVOT(13)
  RLQR_PIVOT(14) RLQR_PIVOT(15)
#undef RLQR_PIVOT
  const bool mine = lane >= j0 && lane < j1;
  const bool zero = mine && !(fabs(dsave) > tol);
  const bool pos = mine && !zero && dsave > 0;
  const bool neg = mine && !zero && dsave < 0;
  const int nz = __popcll(__ballot(zero)), np = __popcll(__ballot(pos)), nn = __popcll(__ballot(neg));
  if (__ballot(mine && !__builtin_isfinite(dsave))) ps.nonfinite = 1;
  ps.nzero += nz;
  ps.npos += np;
  ps.nneg += nn;
  ps.first_bad = ((nz + nn) > 0 && ps.first_bad < 0) ? code : ps.first_bad;
  // smallest |pivot| of the sweep (lanes 0..15 hold the pivots)
  const double dmin = -wave_max_rows(mine ? -fabs(dsave) : -1.0e300);
  if (j1 > j0) ps.minrel = fmin(ps.minrel, dmin / scale);
}

// sum over the 16 lanes of each row (DPP row rotations), then over the rows
__device__ __forceinline__ double wave_sum_rows(double s) {
#pragma unroll
  for (int k = 1; k < 16; k <<= 1) {
    const long long b = __double_as_longlong(s);
    int lo, hi;
    switch (k) {
      case 1: lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), 0x121, 0xf, 0xf, false);
              hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x121, 0xf, 0xf, false); break;
      case 2: lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), 0x122, 0xf, 0xf, false);
              hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x122, 0xf, 0xf, false); break;
      case 4: lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), 0x124, 0xf, 0xf, false);
              hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x124, 0xf, 0xf, false); break;
      default: lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), 0x128, 0xf, 0xf, false);
               hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x128, 0xf, 0xf, false); break;
    }
    s += __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
  }
  return (lane_value(s, 0) + lane_value(s, 16)) + (lane_value(s, 32) + lane_value(s, 48));
}

// Inverse of a state pivot S_hat = I + E close to the identity, without its
// pivot sweep. E (= delta P, or D P D with a per-stage diagonal) is symmetric,
// so ||E||_2 <= ||E||_F = e. When e < 1, every eigenvalue of S_hat lies in
// [1 - e, 1 + e]: S_hat is positive definite, every pivot of its LDL^T lies
// in the same interval (a pivot is a Schur complement of a leading block,
// bounded by that block's extreme eigenvalues), and
//     S_hat^{-1} = I - E + E^2 - ... = Y_k + O(e^{k+1} / (1 - e)),
// Y_1 = I - E, Y_j = I - E Y_{j-1}. neumann_terms returns the number of
// terms k (<= 13) for which e^{k+1} stays below the unit roundoff of the
// precision TG the tile is stored and multiplied in (a quarter of it), or 0
// when e is too large (or not finite) and the sweep must run.
template <typename TG>
__device__ __forceinline__ int neumann_terms(double e) {
  constexpr double tau = sizeof(TG) == 8 ? 0x1p-55 : 0x1p-26;
  if (!(e <= 0.0625)) return 0;
  int k = 1;
  double t = e * e;
  while (t > tau && k < 13) {
    t *= e;
    ++k;
  }
  return t <= tau ? k : 0;
}

// ||X - I||_F of a register tile X (wave-uniform), rows trow<TL>.
template <typename TL>
__device__ __forceinline__ double dist_identity(const double (&X)[4], int lane) {
  const int col = lane & 15, grp = lane >> 4;
  double s = 0.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double d = X[v] - (trow<TL>(grp, v) == col ? 1.0 : 0.0);
    s = __fma_rn(d, d, s);
  }
  return sqrt(wave_sum_rows(s));
}

// Certificate bookkeeping of a state pivot certified by the norm bound
// (pivots j0..j1-1, all in [1 - e, 1 + e], hence positive and nonzero):
// the counts the pivot sweep would give, and the bound (1 - e) / (1 + e) on
// min |pivot| / max |diag|.
__device__ __forceinline__ void neumann_stats(PivStats& ps, int j0, int j1, double e) {
  ps.npos += j1 - j0;
  if (j1 > j0) ps.minrel = fmin(ps.minrel, (1.0 - e) / (1.0 + e));
}

// X[J][J] of a register tile (wave-uniform)
template <typename TL, int J>
__device__ __forceinline__ double tile_diag(const double (&X)[4]) {
  constexpr bool F32 = trow<TL>(1, 0) == 4;
  constexpr int GJ = F32 ? (J >> 2) : (J & 3);
  constexpr int VJ = F32 ? (J & 3) : (J >> 2);
  return lane_value(X[VJ], 16 * GJ + J);
}

}  // namespace rlqr
