// rlqr_device_mw.h -- device-side building blocks of the multi-wavefront
// kernels (one workgroup of NW wavefronts per instance or segment, tiles of
// 16 x 16 blocks distributed over the wavefronts): block numbering, workgroup
// reductions and the pivot sweeps over distributed tiles.
#pragma once
#include "rlqr_device.h"

namespace rlqr {

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

// max over the workgroup of a per-lane value (all threads get the result)
template <int NW>
__device__ __forceinline__ double wg_max(double v, double* red, int w, int lane) {
  v = wave_max(v);
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double s = red[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) s = fmax(s, red[i]);
  return s;
}

// Symmetric sweep of pivots j0..j1-1 over a tile whose owned blocks are
// X[t] at block coordinates (bi[t], bj[t]) (valid if ok[t]). colbuf holds
// 2 x 16*TT doubles. Same update rules (and exact symmetry) as sweep16.
template <typename TL, int C, int TT>
__device__ __forceinline__ void sweep_mw(double (&X)[C][4], const int (&bi)[C], const int (&bj)[C],
                                         const bool (&ok)[C], int j0, int j1, int lane, double* colbuf,
                                         PivStats& ps, int code, double tol, double scale) {
  const int col = lane & 15, grp = lane >> 4;
  double dmin = 1.0e300;
  for (int j = j0; j < j1; ++j) {
    double* cb = colbuf + 16 * TT * (j & 1);
    const int jb = j >> 4, jj = j & 15;
#pragma unroll
    for (int t = 0; t < C; ++t)
      if (ok[t] && bj[t] == jb && col == jj) {
#pragma unroll
        for (int v = 0; v < 4; ++v) cb[16 * bi[t] + trow<TL>(grp, v)] = X[t][v];
      }
    __syncthreads();
    const double d = cb[j];
    const bool zero = !(fabs(d) > tol);
    if (!__builtin_isfinite(d)) ps.nonfinite = 1;
    if (zero) ps.nzero++;
    else if (d > 0) ps.npos++;
    else ps.nneg++;
    if ((zero || d < 0) && ps.first_bad < 0) ps.first_bad = code;
    dmin = fmin(dmin, fabs(d));
    const double rd = zero ? 0.0 : recip(d);
#pragma unroll
    for (int t = 0; t < C; ++t) {
      if (!ok[t]) continue;
      const int c = 16 * bj[t] + col;
      const double cc = cb[c];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * bi[t] + trow<TL>(grp, v);
        const double ci = cb[r];
        double x;
        if (r == j && c == j) x = -rd;
        else if (r == j) x = cc * rd;
        else if (c == j) x = ci * rd;
        else x = __fma_rn(-(ci * cc), rd, X[t][v]);
        X[t][v] = x;
      }
    }
  }
  if (j1 > j0) ps.minrel = fmin(ps.minrel, dmin / scale);
}

// Blocked form of sweep_mw: the pivots j0..j1-1 are swept 16 at a time.
// For the pivots S of block column K (U = the block column before the sweep,
// one LDS panel of 16 x 16 blocks), every wavefront sweeps the diagonal block
// with sweep16 (the same pivots, counts and float64 arithmetic as the
// element-wise sweep) and takes M = -X_SS^{-1} from it; then each owned block
// (I, J) is updated with float64 MFMA products:
//   I, J != K:  X_IJ + U_I M U_J^T            (= X_TT - X_TS X_SS^{-1} X_ST)
//   J == K:     columns in S: -(U_I M), others: X + U_I M U_K^T
//   I == K:     rows in S: -(M U_J^T), others: X + U_K M U_J^T
//   I == J == K: the swept diagonal block.
// Three workgroup barriers per 16 pivots instead of one per pivot. The A
// operands are read with their rows permuted so that the float64 MFMA
// accumulator comes out in the register layout TL of the blocks.
// panel: 16 TT x 17 doubles, mbuf: 2 x 16 x 17 doubles (LDS, free during the call).
// Only wavefront 0's PivStats receive the pivots.
// pscale: the pivots j0..j1-1 lie in one block column and the caller passes
// the tolerance as a multiple of the scale (tol = coefficient, scale unused):
// wavefront 0 takes the scale, max |X_jj| over the pivots, from the panel's
// diagonal block (the same values a workgroup reduction over the tile would
// find), which saves that reduction's barriers.
// TAIL = false: no barrier after the last update; the caller's next barrier
// must come before anything is written to the panel's LDS region.
// LEAD = false: no barrier before the first block's panel stores; every
// earlier reader of the panel region must be behind a barrier already.
template <typename TL>
__device__ __forceinline__ int blk_row(int i) { return trow<TL>(i & 3, i >> 2); }

template <typename TL, int C, int TT, bool TAIL = true, bool LEAD = true>
__device__ __forceinline__ void sweep_blk(double (&X)[C][4], const int (&bi)[C], const int (&bj)[C],
                                          const bool (&ok)[C], int j0, int j1, int w, int lane, double* panel,
                                          double* mbuf, PivStats& ps, int code, double tol, double scale,
                                          bool pscale = false) {
  constexpr int LP = 17;
  const int col = lane & 15, grp = lane >> 4;
  const int ia = lane & 15, kq = lane >> 4;  // MFMA operand coordinates
  for (int K = j0 >> 4; 16 * K < j1; ++K) {
    const int s0 = j0 > 16 * K ? j0 - 16 * K : 0;
    const int s1 = j1 < 16 * K + 16 ? j1 - 16 * K : 16;
    if (LEAD || K != (j0 >> 4)) __syncthreads();  // earlier readers of the panel / LDS region are done
#pragma unroll
    for (int t = 0; t < C; ++t)
      if (ok[t] && bj[t] == K) {
#pragma unroll
        for (int v = 0; v < 4; ++v) panel[(16 * bi[t] + trow<TL>(grp, v)) * LP + col] = X[t][v];
      }
    __syncthreads();
    // the diagonal block, swept by wavefront 0 alone: the others wait at the
    // barrier, so the serial sweep has its SIMD to itself (run by every
    // wavefront it is issue-bound, several copies per SIMD). mbuf receives
    // M (zero outside S), dbuf the whole swept block. The pivot counts land
    // in wavefront 0's PivStats, the ones the kernels report.
    double* dbuf = mbuf + 16 * LP;
    if (w == 0) {
      double D[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) D[v] = panel[(16 * K + trow<TL>(grp, v)) * LP + col];
      int lane_s = lane;  // opaque: the per-pivot lane masks stay inside the loop
      asm volatile("" : "+v"(lane_s));
      double t = tol, sc = scale;
      if (pscale) {
        double dm = 0.0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = trow<TL>(grp, v);
          if (r == col && r >= s0 && r < s1) dm = fmax(dm, fabs(D[v]));
        }
        sc = wave_max(dm);
        t = tol * sc;
      }
      sweep16<TL>(D, s0, s1, lane_s, ps, code, t, sc);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = trow<TL>(grp, v);
        mbuf[r * LP + col] = (r >= s0 && r < s1 && col >= s0 && col < s1) ? D[v] : 0.0;
        dbuf[r * LP + col] = D[v];
      }
    }
    __syncthreads();
    // M is zero outside the pivots s0..s1-1 (rows and columns): the products'
    // inner dimension runs over the 4-wide chunks that hold pivots only (the
    // skipped chunks would add exact zeros)
    const int kb0 = s0 >> 2, kb1 = (s1 + 3) >> 2;
#pragma unroll
    for (int t = 0; t < C; ++t) {
      if (!ok[t]) continue;
      const int I = bi[t], J = bj[t];
      if (I == K && J == K) {
#pragma unroll
        for (int v = 0; v < 4; ++v) X[t][v] = dbuf[trow<TL>(grp, v) * LP + col];
        continue;
      }
      // F = M U_J^T (accumulator rows grp + 4v feed the next product as its B operand)
      d4 F = {0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        if (kk < kb0 || kk >= kb1) continue;  // uniform
        const int k = 4 * kk + kq;
        F = mfma16(mbuf[ia * LP + k], panel[(16 * J + ia) * LP + k], F);
      }
      // E = U_I M U_J^T, rows permuted into the layout TL
      d4 E = {0, 0, 0, 0};
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        if (kk < kb0 || kk >= kb1) continue;
        E = mfma16(panel[(16 * I + blk_row<TL>(ia)) * LP + 4 * kk + kq], F[kk], E);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) X[t][v] += E[v];
      if (J == K) {
        d4 V = {0, 0, 0, 0};  // U_I M
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          if (kk < kb0 || kk >= kb1) continue;
          const int k = 4 * kk + kq;
          V = mfma16(panel[(16 * I + blk_row<TL>(ia)) * LP + k], mbuf[k * LP + ia], V);
        }
        const bool cs = col >= s0 && col < s1;
#pragma unroll
        for (int v = 0; v < 4; ++v) X[t][v] = cs ? -V[v] : X[t][v];
      } else if (I == K) {
        d4 F2 = {0, 0, 0, 0};  // M U_J^T, rows permuted into the layout TL
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          if (kk < kb0 || kk >= kb1) continue;
          const int k = 4 * kk + kq;
          F2 = mfma16(mbuf[blk_row<TL>(ia) * LP + k], panel[(16 * J + ia) * LP + k], F2);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = trow<TL>(grp, v);
          X[t][v] = (r >= s0 && r < s1) ? -F2[v] : X[t][v];
        }
      }
      __builtin_amdgcn_sched_barrier(0);  // one block at a time: bounds the live accumulators
    }
  }
  if constexpr (TAIL) __syncthreads();  // the panel is read until here; the caller may reuse the region
}

template <int C, typename TL>
__device__ __forceinline__ double diag_max(const double (&X)[C][4], const int (&bi)[C], const int (&bj)[C],
                                           const bool (&ok)[C], int lo, int hi, int lane) {
  const int col = lane & 15, grp = lane >> 4;
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < C; ++t) {
    if (!ok[t]) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * bi[t] + trow<TL>(grp, v), c = 16 * bj[t] + col;
      if (r == c && r >= lo && r < hi) s = fmax(s, fabs(X[t][v]));
    }
  }
  return s;
}

}  // namespace rlqr
