// rlqr_kernels_mw.hip -- the sequential dual-regularized Riccati recursion for
// larger stages (n + m > 16): one workgroup of NW wavefronts per instance.
//
// Same per-stage algebra as the one-wavefront kernels (Section "Sequential
// Algorithm" of arXiv 2509.16370): sweep S_hat = I + delta P, W = -P X,
// T = W [A B], Z = [A B]^T T + Hessian, sweep the control pivots of Z. The
// state tiles (P, X = -S_hat^{-1}, W) are NX x NX with NX = 16 TX >= n; the
// stage tiles (Z) are NZ x NZ with NZ = 16 TZ >= n + m. Every tile is split in
// 16 x 16 blocks dealt round-robin to the wavefronts; Z blocks are numbered so
// that the state block (I, J), I, J < TX, of Z has the index of block (I, J)
// of the state tiles -- the wavefront that owns a block of Z_xx therefore
// also owns the same block of P for the next stage.
//
// Pivot sweeps broadcast each pivot column through LDS with one workgroup
// barrier per pivot. Workspace per stage: TZ^2 + TX^2 blocks (Z, then X).
#include "rlqr_device_mw.h"
#include "rlqr_internal.h"

namespace rlqr {

// C block (I, J) = op(A) * B over KB 16-blocks of the inner dimension.
template <typename T, bool TRANS_A, int KB>
__device__ __forceinline__ typename AccT<T>::type gemm_blk(const T* sa, int lda, const T* sb, int ldb,
                                                           int I, int J, int lane) {
  typename AccT<T>::type acc = {0, 0, 0, 0};
  const int i = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int k = 16 * kb + 4 * kk + kq;
      const T av = TRANS_A ? sa[k * lda + 16 * I + i] : sa[(16 * I + i) * lda + k];
      const T bv = sb[k * ldb + 16 * J + i];
      acc = mfma16(av, bv, acc);
    }
  }
  return acc;
}

template <typename TL, typename T>
__device__ __forceinline__ void blk_to_lds(T* s, int ld, int I, int J, const double (&X)[4], int lane) {
  const int col = lane & 15, grp = lane >> 4;
#pragma unroll
  for (int v = 0; v < 4; ++v) s[(16 * I + trow<TL>(grp, v)) * ld + 16 * J + col] = (T)X[v];
}

template <typename TG, int TX, int TZ, int NW>
struct MwCfg {
  static constexpr int NX = 16 * TX, NZ = 16 * TZ;
  static constexpr int LDX = NX + 1, LDZ = NZ + 1;
  static constexpr int CX = (TX * TX + NW - 1) / NW;
  static constexpr int CZ = (TZ * TZ + NW - 1) / NW;
  static constexpr int CT = (TX * TZ + NW - 1) / NW;
  static constexpr int NAB = (NX * NZ + 64 * NW - 1) / (64 * NW);
  static constexpr int BYTES_P = (int)sizeof(TG) * NX * LDX;
  static constexpr int BYTES_X = (int)sizeof(TG) * NX * LDZ;
  static constexpr int BYTES_D = 8 * NZ * LDZ;
  static constexpr int BYTES_SW = 8 * (NZ * 17 + 2 * 16 * 17);  // blocked sweep: panel, M and the swept block
  static constexpr int BYTES_Q = 4 * (int)sizeof(TG) * NX * LDX;  // Neumann by squaring: four state tiles
  static constexpr int BYTES_U1 = BYTES_P + BYTES_X > BYTES_D ? BYTES_P + BYTES_X : BYTES_D;
  static constexpr int BYTES_U2 = BYTES_U1 > BYTES_SW ? BYTES_U1 : BYTES_SW;
  // the squaring form of the Neumann series needs four state tiles; it is
  // built for states up to 32 wide (where many terms occur and the registers
  // are there) if the tiles fit in 160 KB of LDS with [A B] beside them
  static constexpr bool SQ =
      TX <= 2 && (BYTES_Q > BYTES_U2 ? BYTES_Q : BYTES_U2) + (int)sizeof(TG) * NX * LDZ <= 160 * 1024;
  static constexpr int BYTES_U0 = SQ && BYTES_Q > BYTES_U2 ? BYTES_Q : BYTES_U2;
  // up to 48-wide states the control sweep's panel and pivot block sit after
  // Z's symmetrization tile (the sweep's first panel stores need no barrier
  // after its reads); the 64-wide classes keep them at the start of the work
  // region (a second panel address costs them registers)
  static constexpr bool CSEP = TX <= 3;
  static constexpr int BYTES_U3 = !CSEP || BYTES_U0 > BYTES_D + BYTES_SW ? BYTES_U0 : BYTES_D + BYTES_SW;
  static constexpr int BYTES_U = (BYTES_U3 + 15) / 16 * 16;
  // W in a tile of its own after the X tile, where the work region has room
  static constexpr bool WSEP = 2 * BYTES_P + BYTES_X <= BYTES_U;
  static constexpr int BYTES_AB = (int)sizeof(TG) * NX * LDZ;
  static constexpr int BLOCKS_PER_STAGE = TZ * TZ + TX * TX;
};

// State pivot S_hat over a distributed NX x NX tile (owned blocks X[t] at
// (xi[t], xj[t])) -> X = -S_hat^{-1}, certificate bookkeeping in ps. As in the
// one-wavefront kernels: when ||S_hat - I||_F is small (neumann_terms), the
// truncated Neumann series Y_1 = I - E, Y_j = I - E Y_{j-1} (one blocked MFMA
// product and two workgroup barriers per further term, E and Y through the
// LDS tiles sE and sY, stride LDX) replaces the pivot sweep and the norm bound
// certifies every pivot positive. The series is a polynomial in the symmetric
// E, symmetric up to the rounding of its products, and is not symmetrized:
// the tiles built from it (W, then Z) are symmetrized where the symmetric
// sweep needs it. With SQ (four state tiles from sE on) four or more terms
// are summed by squaring instead. Otherwise the blocked sweep runs.
// rnorm: NW doubles of LDS used by nothing else (its previous readers, the
// call before, are behind the caller's barriers, so no barrier precedes its
// stores); red: NW doubles for the sweep's scale.
template <typename TG, int TX, int CX, int NW, bool SQ>
__device__ __forceinline__ void shat_inverse_mw(double (&X)[CX][4], const int (&xi)[CX], const int (&xj)[CX],
                                                const bool (&xo)[CX], int n, int w, int lane, double* red,
                                                double* rnorm, double* panel, double* mbuf, PivStats& ps,
                                                int code, TG* sE) {
  constexpr int NX = 16 * TX, LDX = NX + 1;
  const int col = lane & 15, grp = lane >> 4;
  double s2 = 0.0;
#pragma unroll
  for (int t = 0; t < CX; ++t)
    if (xo[t])
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double d = X[t][v] - (16 * xi[t] + trow<TG>(grp, v) == 16 * xj[t] + col ? 1.0 : 0.0);
        s2 = __fma_rn(d, d, s2);
      }
  s2 = wave_sum_rows(s2);
  if (lane == 0) rnorm[w] = s2;
  __syncthreads();
  double tot = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) tot += rnorm[i];  // same order in every thread: uniform
  const double e = sqrt(tot);
  const int terms = neumann_terms<TG>(e);
  if (terms == 0) {
    const double sc = wg_max<NW>(diag_max<CX, TG>(X, xi, xj, xo, 0, n, lane), red, w, lane);
    sweep_blk<TG, CX, TX>(X, xi, xj, xo, 0, n, w, lane, panel, mbuf, ps, code,
                          1.0e3 * n * 2.220446049250313e-16 * sc, sc);
    return;
  }
  if (terms > 1) {
#pragma unroll
    for (int t = 0; t < CX; ++t)
      if (xo[t]) {
        double E[4];
#pragma unroll
        for (int v = 0; v < 4; ++v)
          E[v] = X[t][v] - (16 * xi[t] + trow<TG>(grp, v) == 16 * xj[t] + col ? 1.0 : 0.0);
        blk_to_lds<TG>(sE, LDX, xi[t], xj[t], E, lane);
      }
  }
  // X holds Y from here on
#pragma unroll
  for (int t = 0; t < CX; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const double id = (16 * xi[t] + trow<TG>(grp, v) == 16 * xj[t] + col) ? 1.0 : 0.0;
      X[t][v] = xo[t] ? id - (X[t][v] - id) : 0.0;
    }
  if (SQ && terms >= 4) {
    // the same series by squaring: with F = -E, (I + F)(I + F^2)(I + F^4)...
    // over L factors sums F^0 .. F^(2^L - 1), 2^L - 1 >= terms; products
    // that do not depend on each other share a phase (two barriers), so
    // terms <= 7 take 3 phases and terms <= 15 take 4 (Horner: terms - 1).
    // Tiles (stride LDX): 0 = E, then E^8; 1 = E^2; 2 = E^4; 3 = partial sum S.
    constexpr int NXX = 16 * TX * (16 * TX + 1);
    TG* t0 = sE;
    TG* t1 = sE + NXX;
    TG* t2 = sE + 2 * NXX;
    TG* t3 = sE + 3 * NXX;
    __syncthreads();  // E in t0
    double E2[CX][4];
#pragma unroll
    for (int t = 0; t < CX; ++t) {
      if (!xo[t]) continue;
      auto acc = gemm_blk<TG, false, TX>(t0, LDX, t0, LDX, xi[t], xj[t], lane);
#pragma unroll
      for (int v = 0; v < 4; ++v) E2[t][v] = (double)acc[v];
      blk_to_lds<TG>(t1, LDX, xi[t], xj[t], E2[t], lane);
    }
    __syncthreads();  // E^2 in t1
    // S = I - E + E^2 - E^3 (X holds I - E), E^4 = E^2 E^2
#pragma unroll
    for (int t = 0; t < CX; ++t) {
      if (!xo[t]) continue;
      auto e3 = gemm_blk<TG, false, TX>(t0, LDX, t1, LDX, xi[t], xj[t], lane);
      auto e4 = gemm_blk<TG, false, TX>(t1, LDX, t1, LDX, xi[t], xj[t], lane);
      double E4[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        X[t][v] = X[t][v] + E2[t][v] - (double)e3[v];
        E4[v] = (double)e4[v];
      }
      blk_to_lds<TG>(t2, LDX, xi[t], xj[t], E4, lane);
      blk_to_lds<TG>(t3, LDX, xi[t], xj[t], X[t], lane);
    }
    __syncthreads();  // E^4 in t2, S in t3
    // S <- S + S E^4 (8 terms); with more terms also E^8 = E^4 E^4 into t0
#pragma unroll
    for (int t = 0; t < CX; ++t) {
      if (!xo[t]) continue;
      auto se = gemm_blk<TG, false, TX>(t3, LDX, t2, LDX, xi[t], xj[t], lane);
#pragma unroll
      for (int v = 0; v < 4; ++v) X[t][v] += (double)se[v];
      if (terms > 7) {
        auto e8 = gemm_blk<TG, false, TX>(t2, LDX, t2, LDX, xi[t], xj[t], lane);
        double E8[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) E8[v] = (double)e8[v];
        blk_to_lds<TG>(t0, LDX, xi[t], xj[t], E8, lane);
      }
    }
    __syncthreads();  // every read of t3 done (and E^8 in t0)
    if (terms > 7) {
      // S <- S + S E^8 (16 terms)
#pragma unroll
      for (int t = 0; t < CX; ++t)
        if (xo[t]) blk_to_lds<TG>(t3, LDX, xi[t], xj[t], X[t], lane);
      __syncthreads();
#pragma unroll
      for (int t = 0; t < CX; ++t) {
        if (!xo[t]) continue;
        auto se = gemm_blk<TG, false, TX>(t3, LDX, t0, LDX, xi[t], xj[t], lane);
#pragma unroll
        for (int v = 0; v < 4; ++v) X[t][v] += (double)se[v];
      }
      __syncthreads();
    }
  } else if (terms > 1) {
    TG* sY = sE + NX * LDX;
    for (int j = 2; j <= terms; ++j) {
#pragma unroll
      for (int t = 0; t < CX; ++t)
        if (xo[t]) blk_to_lds<TG>(sY, LDX, xi[t], xj[t], X[t], lane);
      __syncthreads();
#pragma unroll
      for (int t = 0; t < CX; ++t) {
        if (!xo[t]) continue;
        auto acc = gemm_blk<TG, false, TX>(sE, LDX, sY, LDX, xi[t], xj[t], lane);
#pragma unroll
        for (int v = 0; v < 4; ++v)
          X[t][v] = (16 * xi[t] + trow<TG>(grp, v) == 16 * xj[t] + col ? 1.0 : 0.0) - (double)acc[v];
      }
      __syncthreads();
    }
  }
  // (both forms end with a barrier: the caller may overwrite sE onwards)
#pragma unroll
  for (int t = 0; t < CX; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) X[t][v] = -X[t][v];
  neumann_stats(ps, 0, n, e);
}

// One zero in global memory (never written): the padding elements of the
// branch-free stage loads read it. Not const: a constant-address-space
// operand would turn the selected pointers into generic ones (flat loads).
__device__ double kZeroPad[1];

// Makes the lane coordinates opaque at this point of a stage loop, so that
// the compiler re-derives the lane-dependent addresses after it instead of
// hoisting all of them out of the loop: hoisted, they stay live across every
// stage and the large tile classes spill them.
__device__ __forceinline__ void lane_fence(int& tid, int& lane, int& col, int& grp) {
  asm volatile("" : "+v"(tid), "+v"(lane), "+v"(col), "+v"(grp));
}

// DG: per-stage diagonal Delta_i (a.dd); the instantiations without it carry none of its code
template <typename TG, int TX, int TZ, int NW, bool DG>
__global__ __launch_bounds__(64 * NW) void k_factor_mw(FactorArgs a) {
  using C = MwCfg<TG, TX, TZ, NW>;
  constexpr int NX = C::NX, NZ = C::NZ, LDX = C::LDX, LDZ = C::LDZ;
  constexpr int CX = C::CX, CZ = C::CZ, CT = C::CT, NAB = C::NAB;
  const SegDesc sd = a.segs[blockIdx.x];
  const int b = sd.inst;
  if (a.run && !a.run[b]) return;
  const InstMeta mt = a.meta[b];
  const int N = mt.N, n = mt.n, m = mt.m;
  const int klo = sd.lo, khi = sd.hi;
  const double delta = DG ? 0.0 : a.delta[b];
  const double* __restrict__ Qg = a.Q + mt.oQ;
  const double* __restrict__ Mg = a.M + mt.oM;
  const double* __restrict__ Rg = a.R + mt.oR;
  const double* __restrict__ Ag = a.A + mt.oA;
  const double* __restrict__ Bg = a.B + mt.oB;
  TG* __restrict__ ws = reinterpret_cast<TG*>(a.ws) + mt.ows;
  constexpr int64_t STAGE = (int64_t)C::BLOCKS_PER_STAGE * 256;
  auto ztile = [&](int i) { return ws + (int64_t)i * STAGE; };
  auto xtile = [&](int i) { return ws + (int64_t)i * STAGE + (int64_t)TZ * TZ * 256; };

  __shared__ __align__(16) unsigned char smem[C::BYTES_U + C::BYTES_AB];
  __shared__ double red[NW], rnorm[NW];
  TG* sP = reinterpret_cast<TG*>(smem);
  TG* sX = reinterpret_cast<TG*>(smem + C::BYTES_P);
  TG* sW = C::WSEP ? reinterpret_cast<TG*>(smem + C::BYTES_P + C::BYTES_X) : sP;
  double* sD = reinterpret_cast<double*>(smem);
  TG* sAB = reinterpret_cast<TG*>(smem + C::BYTES_U);
  // the blocked sweeps' panel and pivot block overlay the work region, which
  // is free while a sweep runs
  double* panel = reinterpret_cast<double*>(smem);
  double* mbuf = panel + NZ * 17;
  static_assert((NZ * 17 + 2 * 16 * 17) * 8 <= C::BYTES_U, "sweep panel exceeds the work region");
  static_assert(C::BYTES_U + C::BYTES_AB + 8 * (2 * NW + 2 * NX) <= 160 * 1024, "LDS exceeds 160 KB");
  double* cpanel = C::CSEP ? reinterpret_cast<double*>(smem + C::BYTES_D) : panel;  // the control sweep's
  double* cmbuf = cpanel + NZ * 17;

  int tid = threadIdx.x, lane = tid & 63, col = lane & 15, grp = lane >> 4;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  int xi[CX], xj[CX], zi[CZ], zj[CZ], ti[CT], tj[CT];
  bool xo[CX], zo[CZ], to[CT];
#pragma unroll
  for (int t = 0; t < CX; ++t) {
    const int bx = w + NW * t;
    xo[t] = bx < TX * TX;
    xi[t] = bx / TX;
    xj[t] = bx % TX;
  }
#pragma unroll
  for (int t = 0; t < CZ; ++t) {
    const int bz = w + NW * t;
    zo[t] = bz < TZ * TZ;
    zmap<TX, TZ>(zo[t] ? bz : 0, zi[t], zj[t]);
  }
#pragma unroll
  for (int t = 0; t < CT; ++t) {
    const int bt = w + NW * t;
    to[t] = bt < TX * TZ;
    ti[t] = bt / TZ;
    tj[t] = bt % TZ;
  }

  PivStats ps;
  ps.init();
  const double eps = 2.220446049250313e-16;

  // per-stage diagonal Delta_{k+1} = D^2 (a.dd): the swept matrix is
  // S_hat = I + D P D, the stored tile X~ = D X D (symmetric) and the product
  // takes X~ Delta^{-1} (W = P (I + Delta P)^{-1} = -P X~ Delta^{-1}); D and
  // Delta^{-1} of the stage sit in LDS (0 outside the state block), the
  // thread's entry of the next stage is loaded one stage ahead
  const double* __restrict__ ddg = DG ? a.dd + mt.od : nullptr;
  __shared__ double sdl[DG ? NX : 1], idl[DG ? NX : 1];
  double dpre = (DG && tid < n) ? ddg[(int64_t)khi * n + tid] : 0.0;
  auto put_diag = [&](double d) {
    if (tid < NX) {
      sdl[tid] = tid < n ? sqrt(d) : 0.0;
      idl[tid] = tid < n ? 1.0 / d : 0.0;
    }
  };
  auto scale_x = [&](double (&X)[CX][4]) {
#pragma unroll
    for (int t = 0; t < CX; ++t)
      if (xo[t])
#pragma unroll
        for (int v = 0; v < 4; ++v) X[t][v] *= sdl[16 * xi[t] + trow<TG>(grp, v)] * sdl[16 * xj[t] + col];
  };

  // The stage loads below are branch-free: a padding element reads the zero
  // kZeroPad. Loads issued under divergent branches, or masked right after
  // they are issued, make the compiler wait for every outstanding load.
  auto load_ab = [&](double (&o)[NAB], int k) {
    const double* A = Ag + (int64_t)k * n * n;
    const double* B = Bg + (int64_t)k * n * m;
#pragma unroll
    for (int t = 0; t < NAB; ++t) {
      const int e = tid + 64 * NW * t, r = e / NZ, c = e % NZ;
      const bool inA = e < NX * NZ && r < n && c < n, inB = e < NX * NZ && r < n && c >= n && c < n + m;
      o[t] = *(inA ? A + r * n + c : (inB ? B + r * m + (c - n) : kZeroPad));
    }
  };
  auto load_h = [&](double (&o)[CZ][4], int k) {
    const double* Q = Qg + (int64_t)k * n * n;
    const double* M = Mg + (int64_t)k * n * m;
    const double* R = Rg + (int64_t)k * m * m;
#pragma unroll
    for (int t = 0; t < CZ; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * zi[t] + trow<TG>(grp, v), c = 16 * zj[t] + col;
        const bool rx = zo[t] && r < n, ru = zo[t] && r >= n && r < n + m;
        const bool cx = c < n, cu = c >= n && c < n + m;
        const double* src = (rx && cx) ? Q + r * n + c
                          : (rx && cu) ? M + r * m + (c - n)
                          : (ru && cx) ? M + c * m + (r - n)
                          : (ru && cu) ? R + (r - n) * m + (c - n) : kZeroPad;
        o[t][v] = *src;
      }
  };
  auto store_ab = [&](const double (&o)[NAB]) {
#pragma unroll
    for (int t = 0; t < NAB; ++t) {
      const int e = tid + 64 * NW * t;
      if (e < NX * NZ) sAB[(e / NZ) * LDZ + (e % NZ)] = (TG)o[t];
    }
  };

  // P_hi: Q_N at the top of the horizon, else the boundary tile of the scan
  double P[CX][4];
  {
    const double* QN = Qg + (int64_t)N * n * n;
#pragma unroll
    for (int t = 0; t < CX; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * xi[t] + trow<TG>(grp, v), c = 16 * xj[t] + col;
        const bool in = xo[t] && r < n && c < n;
        P[t][v] = !in ? 0.0 : (sd.P0 ? (double)sd.P0[r * sd.p0_ld + c] : QN[r * n + c]);
      }
  }
  if (khi == N) {
    TG* zt = ztile(N);
#pragma unroll
    for (int t = 0; t < CZ; ++t) {
      if (!zo[t]) continue;
      const int bz = w + NW * t;
#pragma unroll
      for (int v = 0; v < 4; ++v)
        zt[(int64_t)bz * 256 + v * 64 + lane] = (TG)((t < CX && bz < TX * TX) ? P[t < CX ? t : 0][v] : 0.0);
    }
  }

  // [A B] of stage k is staged in sAB after the Z product of stage k + 1
  // (sAB is free once that product has read it), from registers loaded at
  // the end of stage k + 2: the loads have the state pivot and three
  // products to arrive, their registers are not live across a control
  // sweep, and no wait at the top of a stage covers the tile stores of the
  // stage before it. Stage khi - 1 is staged before the loop.
  double ab[NAB], H[CZ][4];
  if (khi > klo) {
    load_ab(ab, khi - 1);
    store_ab(ab);
    if (khi - 2 >= klo) load_ab(ab, khi - 2);
  }
  // every load so far has been consumed: say so before the stage loop, or the
  // compiler's wait analysis, merging the loop entry with its back edge,
  // waits for all outstanding memory operations inside every stage
  __builtin_amdgcn_s_waitcnt(0);

  for (int k = khi - 1; k >= klo; --k) {
    lane_fence(tid, lane, col, grp);
    // (the previous stage's reads of sdl / idl are behind its barriers)
    // Without a per-stage diagonal no barrier is needed here: nothing is
    // stored to LDS before the state pivot's norm barrier, which also orders
    // the previous stage's sweep reads before the stores after it.
    if constexpr (DG) {
      put_diag(dpre);
      dpre = tid < n ? ddg[(int64_t)k * n + tid] : 0.0;
      __syncthreads();
    }
    load_h(H, k);  // consumed by the Z product, after the state pivot and two products
    // X = I + delta P_{k+1} (per-stage diagonal: I + D P D), swept -> -S_hat^{-1}
    double X[CX][4];
#pragma unroll
    for (int t = 0; t < CX; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * xi[t] + trow<TG>(grp, v), c = 16 * xj[t] + col;
        const double sc = DG ? (xo[t] ? sdl[r] * sdl[c] : 0.0) : delta;
        X[t][v] = (xo[t] && r == c ? 1.0 : 0.0) + sc * P[t][v];
      }
    shat_inverse_mw<TG, TX, CX, NW, C::SQ>(X, xi, xj, xo, n, w, lane, red, rnorm, panel, mbuf, ps, 2 * (k + 1), sP);
    if constexpr (DG) scale_x(X);  // X~ = D X D
    {
      TG* xt = xtile(k + 1);
#pragma unroll
      for (int t = 0; t < CX; ++t)
        if (xo[t])
#pragma unroll
          for (int v = 0; v < 4; ++v) xt[(int64_t)(w + NW * t) * 256 + v * 64 + lane] = (TG)X[t][v];
    }
#pragma unroll
    for (int t = 0; t < CX; ++t)
      if (xo[t]) {
        blk_to_lds<TG>(sP, LDX, xi[t], xj[t], P[t], lane);
        if constexpr (DG) {  // the product takes X~ Delta^{-1}
          double Xs[4];
#pragma unroll
          for (int v = 0; v < 4; ++v) Xs[v] = X[t][v] * idl[16 * xj[t] + col];
          blk_to_lds<TG>(sX, LDX, xi[t], xj[t], Xs, lane);
        } else {
          blk_to_lds<TG>(sX, LDX, xi[t], xj[t], X[t], lane);
        }
      }
    __syncthreads();
    lane_fence(tid, lane, col, grp);
    // W = -P X, symmetric only up to rounding and left so: Z = [A B]^T W [A B]
    // + Hessian is symmetrized below, which symmetrizes W's share of it as
    // well. W goes to its own tile sW where the work region has room for one
    // (no barrier before its stores), else over P once every product has read it.
    double W[CX][4];
#pragma unroll
    for (int t = 0; t < CX; ++t) {
#pragma unroll
      for (int v = 0; v < 4; ++v) W[t][v] = 0.0;
      if (!xo[t]) continue;
      auto acc = gemm_blk<TG, false, TX>(sP, LDX, sX, LDX, xi[t], xj[t], lane);
#pragma unroll
      for (int v = 0; v < 4; ++v) W[t][v] = -(double)acc[v];
    }
    if constexpr (!C::WSEP) __syncthreads();
#pragma unroll
    for (int t = 0; t < CX; ++t)
      if (xo[t]) blk_to_lds<TG>(sW, LDX, xi[t], xj[t], W[t], lane);
    __syncthreads();
    lane_fence(tid, lane, col, grp);
    // T = W [A B]  (NX x NZ)
#pragma unroll
    for (int t = 0; t < CT; ++t) {
      if (!to[t]) continue;
      auto acc = gemm_blk<TG, false, TX>(sW, LDX, sAB, LDZ, ti[t], tj[t], lane);
      double Tb[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) Tb[v] = (double)acc[v];
      blk_to_lds<TG>(sX, LDZ, ti[t], tj[t], Tb, lane);
    }
    __syncthreads();
    lane_fence(tid, lane, col, grp);
    // Z = [A B]^T T + Hessian, symmetrized
    double Z[CZ][4];
#pragma unroll
    for (int t = 0; t < CZ; ++t) {
#pragma unroll
      for (int v = 0; v < 4; ++v) Z[t][v] = 0.0;
      if (!zo[t]) continue;
      auto acc = gemm_blk<TG, true, TX>(sAB, LDZ, sX, LDZ, zi[t], zj[t], lane);
#pragma unroll
      for (int v = 0; v < 4; ++v) Z[t][v] = (double)acc[v] + H[t][v];
    }
    __syncthreads();
    if (k > klo) store_ab(ab);  // stage k - 1; every wavefront is past its last read of sAB for stage k
#pragma unroll
    for (int t = 0; t < CZ; ++t)
      if (zo[t]) blk_to_lds<TG>(sD, LDZ, zi[t], zj[t], Z[t], lane);
    __syncthreads();
#pragma unroll
    for (int t = 0; t < CZ; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * zi[t] + trow<TG>(grp, v), c = 16 * zj[t] + col;
        if (zo[t]) Z[t][v] = 0.5 * (Z[t][v] + sD[c * LDZ + r]);
      }
    lane_fence(tid, lane, col, grp);
    {
      // control pivots within one block column: wavefront 0 takes their scale
      // from the sweep's panel; else a workgroup reduction over the tile. Up
      // to 48-wide states the panel lies outside Z's symmetrization tile (no
      // barrier before its first stores), and no barrier follows the sweep:
      // the next one (the state pivot's norm, or the top of the stage with a
      // per-stage diagonal) comes before any store to its region.
      const bool one = m > 0 && (n >> 4) == ((n + m - 1) >> 4);
      const double sc = one ? 0.0 : wg_max<NW>(diag_max<CZ, TG>(Z, zi, zj, zo, n, n + m, lane), red, w, lane);
      const double coef = 1.0e3 * m * eps;
      sweep_blk<TG, CZ, TZ, false, !C::CSEP>(Z, zi, zj, zo, n, n + m, w, lane, cpanel, cmbuf, ps, 2 * k + 1,
                                             one ? coef : coef * sc, sc, one);
    }
    {
      TG* zt = ztile(k);
#pragma unroll
      for (int t = 0; t < CZ; ++t)
        if (zo[t])
#pragma unroll
          for (int v = 0; v < 4; ++v) zt[(int64_t)(w + NW * t) * 256 + v * 64 + lane] = (TG)Z[t][v];
    }
    // P_k = Z_xx (same owner, same slot)
#pragma unroll
    for (int t = 0; t < CX; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * xi[t] + trow<TG>(grp, v), c = 16 * xj[t] + col;
        P[t][v] = (xo[t] && r < n && c < n) ? Z[t < CZ ? t : 0][v] : 0.0;
      }
    if (k - 2 >= klo) load_ab(ab, k - 2);  // staged after the next stage's Z product
  }
  // S_hat_0
  if (klo == 0) {
    if constexpr (DG) {
      __syncthreads();
      put_diag(dpre);
      __syncthreads();
    }
    double X[CX][4];
#pragma unroll
    for (int t = 0; t < CX; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * xi[t] + trow<TG>(grp, v), c = 16 * xj[t] + col;
        const double sc = DG ? (xo[t] ? sdl[r] * sdl[c] : 0.0) : delta;
        X[t][v] = (xo[t] && r == c ? 1.0 : 0.0) + sc * P[t][v];
      }
    shat_inverse_mw<TG, TX, CX, NW, C::SQ>(X, xi, xj, xo, n, w, lane, red, rnorm, panel, mbuf, ps, 0, sP);
    if constexpr (DG) scale_x(X);  // X~_0 = D_0 X_0 D_0
    TG* xt = xtile(0);
#pragma unroll
    for (int t = 0; t < CX; ++t)
      if (xo[t])
#pragma unroll
        for (int v = 0; v < 4; ++v) xt[(int64_t)(w + NW * t) * 256 + v * 64 + lane] = (TG)X[t][v];
  }
  if (tid == 0) {
    SegStats st;
    st.first_bad = ps.first_bad;
    st.nzero = ps.nzero;
    st.npos = ps.npos;
    st.nneg = ps.nneg;
    st.minrel = ps.minrel;
    st.nonfinite = ps.nonfinite;
    st.pad = 0;
    a.stats[sd.gidx] = st;
  }
}

// ------------------------------------------------------------------ solve

// y[c] = sum_r Tile[r][c] vec[r] over a tile of TR x TC blocks owned
// round-robin (blocks at (bi[t], bj[t])); vec and out in LDS; red is
// TR x 16 TC doubles. Deterministic: block-row partials are summed in order.
template <typename TL, int Cn, int TR, int TC>
__device__ __forceinline__ void tmatvec_mw(const double (&X)[Cn][4], const int (&bi)[Cn], const int (&bj)[Cn],
                                           const bool (&ok)[Cn], const double* vec, double* out, double* red,
                                           int tid, int lane) {
  const int col = lane & 15, grp = lane >> 4;
#pragma unroll
  for (int t = 0; t < Cn; ++t) {
    if (!ok[t]) continue;  // wave-uniform
    double s = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) s += X[t][v] * vec[16 * bi[t] + trow<TL>(grp, v)];
    s = group_sum(s);
    if (grp == 0) red[bi[t] * 16 * TC + 16 * bj[t] + col] = s;
  }
  __syncthreads();
  if (tid < 16 * TC) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < TR; ++i) s += red[i * 16 * TC + tid];
    out[tid] = s;
  }
  __syncthreads();
}

// Solve pass over the stages [lo, hi) of one instance. SEG == false: the whole
// horizon (lo = 0, hi = N): backward vector pass from p_N = q_N, forward
// rollout from x_0 = S_hat_0^{-1}(c_0 - delta p_0), x, u, y written.
// SEG == true (scan mode; p_k and x_k are affine in the segment's boundary
// values through the transfer matrix Psi of the segment):
//   phase 1: backward from p_hi = 0 (q_N on the last segment); p_lo -> plo
//   phase 2: backward from the true p_hi (the next segment's plo), p_k and
//            k_k written; forward from x_lo = 0 (x_0 on the first segment);
//            x_hi -> xhi
//   phase 3: forward from the true x_lo (the previous segment's xhi), x, u, y
//            written (x_N, y_N by the last segment)
template <typename TG, int TX, int TZ, int NW, bool SEG, bool DG = false>
__global__ __launch_bounds__(64 * NW) void k_solve_mw(SolveArgs a) {
  using C = MwCfg<TG, TX, TZ, NW>;
  constexpr int NZ = C::NZ, CX = C::CX, CZ = C::CZ, CT = C::CT;
  constexpr bool PF = NW <= 9;  // operands of the next step loaded one step ahead
  SegDesc sd{};
  if (SEG) sd = a.segs[blockIdx.x];
  const int b = SEG ? sd.inst : (a.list ? a.list[blockIdx.x] : (int)blockIdx.x);
  int tid = threadIdx.x, lane = tid & 63, col = lane & 15, grp = lane >> 4;
  const int w = tid >> 6;
  if (a.run && !a.run[b]) return;
  const InstMeta mt = a.meta[b];
  const int N = mt.N, n = mt.n, m = mt.m;
  const int lo = SEG ? sd.lo : 0, hi = SEG ? sd.hi : N;
  const int phase = SEG ? a.phase : 0;
  const bool do_bwd = !SEG || phase <= 2, do_fwd = !SEG || phase >= 2;
  const bool write_pk = !SEG || phase == 2, write_z = !SEG || phase == 3;
  const double delta = DG ? 0.0 : a.delta[b];
  // DG: per-stage diagonal Delta_i (a.dd, laid out like x); with the stored
  // X~ = -D S_hat^{-1} D: (I + P Delta)^{-1} = -Delta^{-1} X~, (I + Delta P)^{-1} = -X~ Delta^{-1}
  const double* __restrict__ ddg = DG ? a.dd + mt.od : nullptr;
  const double* __restrict__ Ag = a.A + mt.oA;
  const double* __restrict__ Bg = a.B + mt.oB;
  const TG* __restrict__ ws = reinterpret_cast<const TG*>(a.ws) + mt.ows;
  constexpr int64_t STAGE = (int64_t)C::BLOCKS_PER_STAGE * 256;
  auto ztile = [&](int i) { return ws + (int64_t)i * STAGE; };
  auto xtile = [&](int i) { return ws + (int64_t)i * STAGE + (int64_t)TZ * TZ * 256; };
  double* __restrict__ pg = a.pk + mt.opk;
  double* __restrict__ kg = a.pk + mt.opk + (int64_t)(N + 1) * n;
  const double *qb, *rb, *cb;
  int64_t qs, rs;
  const bool accum = a.corr != nullptr;
  if (accum) {
    const double* res = a.corr + mt.ores;
    qb = res; qs = n + m;
    rb = res + n; rs = n + m;
    cb = res + (int64_t)N * (n + m) + n;
  } else {
    qb = a.q + mt.oq; qs = n;
    rb = a.r + mt.or_; rs = m;
    cb = a.c + mt.oc;
  }
  double* __restrict__ xg = a.x + mt.ox;
  double* __restrict__ ug = a.u + mt.ou;
  double* __restrict__ yg = a.y + mt.oy;
  if (a.info[b].singular) {
    if (!accum && write_z) {
      const double nanv = __builtin_nan("");
      const int x1 = hi == N ? N + 1 : hi;
      for (int i = lo * n + tid; i < x1 * n; i += 64 * NW) { xg[i] = nanv; yg[i] = nanv; }
      for (int i = lo * m + tid; i < hi * m; i += 64 * NW) ug[i] = nanv;
    }
    return;
  }

  __shared__ double s0[NZ], s1[NZ], s2[NZ];
  __shared__ double red[TZ * NZ];

  int xi[CX], xj[CX], zi[CZ], zj[CZ], ai[CT], aj[CT], ati[CT], atj[CT];
  bool xo[CX], zo[CZ], ao[CT];
#pragma unroll
  for (int t = 0; t < CX; ++t) {
    const int bx = w + NW * t;
    xo[t] = bx < TX * TX; xi[t] = bx / TX; xj[t] = bx % TX;
  }
#pragma unroll
  for (int t = 0; t < CZ; ++t) {
    const int bz = w + NW * t;
    zo[t] = bz < TZ * TZ;
    zmap<TX, TZ>(zo[t] ? bz : 0, zi[t], zj[t]);
  }
#pragma unroll
  for (int t = 0; t < CT; ++t) {
    const int bt = w + NW * t;
    ao[t] = bt < TX * TZ;
    ai[t] = bt / TZ; aj[t] = bt % TZ;      // block of [A B]   (TX x TZ)
    ati[t] = bt % TZ; atj[t] = bt / TZ;    // block of [A B]^T (TZ x TX)
  }
  auto load_tile = [&](auto& R, const TG* g, auto& ok, int cnt) {
    for (int t = 0; t < cnt; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        R[t][v] = ok[t] ? (double)g[(int64_t)(w + NW * t) * 256 + v * 64 + lane] : 0.0;
  };
  // [A B] block (rows state, cols n+m) in tile layout, or its transpose
  auto load_ab = [&](double (&R)[CT][4], int k, bool trans) {
    const double* A = Ag + (int64_t)k * n * n;
    const double* B = Bg + (int64_t)k * n * m;
#pragma unroll
    for (int t = 0; t < CT; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int rr = trans ? 16 * ati[t] + trow<TG>(grp, v) : 16 * ai[t] + trow<TG>(grp, v);
        const int cc = trans ? 16 * atj[t] + col : 16 * aj[t] + col;
        const int r = trans ? cc : rr, c = trans ? rr : cc;  // element [A B][r][c]
        double x = 0.0;
        if (ao[t] && r < n) {
          if (c < n) x = A[r * n + c];
          else if (c < n + m) x = B[r * m + (c - n)];
        }
        R[t][v] = x;
      }
  };
  const bool xr = tid < n, ur = tid >= n && tid < n + m;

  // ---- backward vector pass over k = hi-1 .. lo; threads tid < NZ carry vector entries
  if (do_bwd) {
    double p;
    if (hi == N) p = xr ? qb[(int64_t)N * qs + tid] : 0.0;
    else if (phase == 1) p = 0.0;
    else p = xr ? a.plo[mt.ovec + (int64_t)(sd.s + 1) * n + tid] : 0.0;
    // p_hi belongs to the next segment (hi < N): only the last segment writes p_N
    if (write_pk && xr && hi == N) pg[(int64_t)hi * n + tid] = p;
    double Zp[CZ][4];
    load_tile(Zp, ztile(hi), zo, CZ);
    // step k's operands, loaded one step ahead
    double Zk[CZ][4], Xn[CX][4], AB[CT][4];
    double ck = 0.0, qk = 0.0, rk = 0.0, dk = 0.0;
    if (PF && hi > lo) {
      load_tile(Zk, ztile(hi - 1), zo, CZ);
      load_tile(Xn, xtile(hi), xo, CX);
      load_ab(AB, hi - 1, false);
      ck = xr ? cb[(int64_t)hi * n + tid] : 0.0;
      dk = (DG && xr) ? ddg[(int64_t)hi * n + tid] : 0.0;
      qk = xr ? qb[(int64_t)(hi - 1) * qs + tid] : 0.0;
      rk = ur ? rb[(int64_t)(hi - 1) * rs + (tid - n)] : 0.0;
    }
    for (int k = hi - 1; k >= lo; --k) {
      lane_fence(tid, lane, col, grp);
      // PF: the next step's operands are loaded now; otherwise (the 16-wavefront
      // classes, whose register budget the second set would exceed) this step's
      const int k1 = k > lo ? k - 1 : k;
      // the tiles of the next step stay in their stored precision until they are
      // used (a conversion at the load would wait for it)
      TG Zk1[CZ][4], Xn1[CX][4];
      double AB1[CT][4];
      double ck1 = 0.0, qk1 = 0.0, rk1 = 0.0, dk1 = 0.0;
      if constexpr (PF) {
        load_tile(Zk1, ztile(k1), zo, CZ);
        load_tile(Xn1, xtile(k1 + 1), xo, CX);
        load_ab(AB1, k1, false);
        ck1 = xr ? cb[(int64_t)(k1 + 1) * n + tid] : 0.0;
        dk1 = (DG && xr) ? ddg[(int64_t)(k1 + 1) * n + tid] : 0.0;
        qk1 = xr ? qb[(int64_t)k1 * qs + tid] : 0.0;
        rk1 = ur ? rb[(int64_t)k1 * rs + (tid - n)] : 0.0;
      } else {
        load_tile(Zk, ztile(k), zo, CZ);
        load_tile(Xn, xtile(k + 1), xo, CX);
        load_ab(AB, k, false);
        ck = xr ? cb[(int64_t)(k + 1) * n + tid] : 0.0;
        dk = (DG && xr) ? ddg[(int64_t)(k + 1) * n + tid] : 0.0;
        qk = xr ? qb[(int64_t)k * qs + tid] : 0.0;
        rk = ur ? rb[(int64_t)k * rs + (tid - n)] : 0.0;
      }
      __syncthreads();
      if (tid < NZ) s0[tid] = xr ? ck : 0.0;
      __syncthreads();
      tmatvec_mw<TG, CZ, TZ, TZ>(Zp, zi, zj, zo, s0, s1, red, tid, lane);   // s1 = Z_{k+1} c (x rows = P c)
      const double idk = (DG && xr) ? 1.0 / dk : 1.0;
      if (tid < NZ) s2[tid] = xr ? p + s1[tid] : 0.0;                      // v
      __syncthreads();
      tmatvec_mw<TG, CX, TX, TX>(Xn, xi, xj, xo, s2, s1, red, tid, lane);   // s1 = -S_hat^{-1} v (DG: X~ v)
      if (tid < NZ) s0[tid] = xr ? (DG ? -idk * s1[tid] : -s1[tid]) : 0.0;  // g
      __syncthreads();
      tmatvec_mw<TG, CT, TX, TZ>(AB, ai, aj, ao, s0, s1, red, tid, lane);   // s1 = [A^T g; B^T g]
      const double abg = tid < NZ ? s1[tid] : 0.0;
      if (tid < NZ) s2[tid] = ur ? rk + abg : 0.0;                          // h
      __syncthreads();
      tmatvec_mw<TG, CZ, TZ, TZ>(Zk, zi, zj, zo, s2, s1, red, tid, lane);   // s1 = [-K^T h; -G^{-1} h]
      if (xr) {
        p = qk + abg - s1[tid];
        if (write_pk) pg[(int64_t)k * n + tid] = p;
      }
      if (ur && write_pk) kg[(int64_t)k * m + (tid - n)] = s1[tid];
#pragma unroll
      for (int t = 0; t < CZ; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) Zp[t][v] = Zk[t][v];
      if constexpr (PF) {
#pragma unroll
        for (int t = 0; t < CZ; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) Zk[t][v] = Zk1[t][v];
#pragma unroll
        for (int t = 0; t < CX; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) Xn[t][v] = Xn1[t][v];
#pragma unroll
        for (int t = 0; t < CT; ++t)
#pragma unroll
          for (int v = 0; v < 4; ++v) AB[t][v] = AB1[t][v];
        ck = ck1; qk = qk1; rk = rk1; dk = dk1;
      }
    }
    if (SEG && phase == 1 && xr) a.plo[mt.ovec + (int64_t)sd.s * n + tid] = p;
    __syncthreads();
  }
  if (!do_fwd) return;

  // ---- forward rollout over k = lo .. hi-1
  double x;
  if (lo == 0) {
    double X0[CX][4];
    load_tile(X0, xtile(0), xo, CX);
    const double p0 = xr ? pg[tid] : 0.0;
    const double d0 = (DG && xr) ? ddg[tid] : delta;
    if (tid < NZ) s0[tid] = xr ? (DG ? (cb[tid] - d0 * p0) / d0 : cb[tid] - delta * p0) : 0.0;
    __syncthreads();
    tmatvec_mw<TG, CX, TX, TX>(X0, xi, xj, xo, s0, s1, red, tid, lane);
    x = xr ? -s1[tid] : 0.0;
  } else if (phase == 2) {
    x = 0.0;
  } else {
    x = xr ? a.xhi[mt.ovec + (int64_t)(sd.s - 1) * n + tid] : 0.0;
  }
  // p_{k+1}; at a segment end (k + 1 == hi < N) the boundary value of the chain
  auto pnext = [&](int k) {
    const bool pbound = SEG && k + 1 == hi && hi < N;
    const double* pnp = pbound ? a.plo + mt.ovec + (int64_t)(sd.s + 1) * n : pg + (int64_t)(k + 1) * n;
    return xr ? pnp[tid] : 0.0;
  };
  // step k's operands, loaded one step ahead
  double Zk[CZ][4], Xn[CX][4], ABt[CT][4];
  double pk = 0.0, kk = 0.0, pn = 0.0, cn = 0.0, dn = delta;
  if (PF && hi > lo) {
    if constexpr (DG) dn = xr ? ddg[(int64_t)(lo + 1) * n + tid] : 0.0;
    load_tile(Zk, ztile(lo), zo, CZ);
    load_tile(Xn, xtile(lo + 1), xo, CX);
    load_ab(ABt, lo, true);
    pk = xr ? pg[(int64_t)lo * n + tid] : 0.0;
    kk = ur ? kg[(int64_t)lo * m + (tid - n)] : 0.0;
    pn = pnext(lo);
    cn = xr ? cb[(int64_t)(lo + 1) * n + tid] : 0.0;
  }
  for (int k = lo; k < hi; ++k) {
    lane_fence(tid, lane, col, grp);
    const int k1 = k + 1 < hi ? k + 1 : k;
    TG Zk1[CZ][4], Xn1[CX][4];  // stored precision until used
    double ABt1[CT][4];
    double pk1 = 0.0, kk1 = 0.0, pn1 = 0.0, cn1 = 0.0, dn1 = delta;
    if constexpr (PF) {
      if constexpr (DG) dn1 = xr ? ddg[(int64_t)(k1 + 1) * n + tid] : 0.0;
      load_tile(Zk1, ztile(k1), zo, CZ);
      load_tile(Xn1, xtile(k1 + 1), xo, CX);
      load_ab(ABt1, k1, true);
      pk1 = xr ? pg[(int64_t)k1 * n + tid] : 0.0;
      kk1 = ur ? kg[(int64_t)k1 * m + (tid - n)] : 0.0;
      pn1 = pnext(k1);
      cn1 = xr ? cb[(int64_t)(k1 + 1) * n + tid] : 0.0;
    } else {
      load_tile(Zk, ztile(k), zo, CZ);
      load_tile(Xn, xtile(k + 1), xo, CX);
      load_ab(ABt, k, true);
      pk = xr ? pg[(int64_t)k * n + tid] : 0.0;
      kk = ur ? kg[(int64_t)k * m + (tid - n)] : 0.0;
      pn = pnext(k);
      cn = xr ? cb[(int64_t)(k + 1) * n + tid] : 0.0;
      if constexpr (DG) dn = xr ? ddg[(int64_t)(k + 1) * n + tid] : 0.0;
    }
    __syncthreads();
    if (tid < NZ) s0[tid] = xr ? x : 0.0;
    __syncthreads();
    tmatvec_mw<TG, CZ, TZ, TZ>(Zk, zi, zj, zo, s0, s1, red, tid, lane);  // [P x; -K x]
    double uk = 0.0;
    if (xr && write_z) {
      const double yk = s1[tid] + pk;
      const int64_t i = (int64_t)k * n + tid;
      yg[i] = accum ? yg[i] + yk : yk;
      xg[i] = accum ? xg[i] + x : x;
    }
    if (ur) {
      uk = kk - s1[tid];
      const int64_t i = (int64_t)k * m + (tid - n);
      if (write_z) ug[i] = accum ? ug[i] + uk : uk;
    }
    if (tid < NZ) s2[tid] = xr ? x : (ur ? uk : 0.0);
    __syncthreads();
    tmatvec_mw<TG, CT, TZ, TX>(ABt, ati, atj, ao, s2, s1, red, tid, lane); // [A B] z
    const double idn = (DG && xr) ? 1.0 / dn : 1.0;
    if (tid < NZ) s0[tid] = xr ? (DG ? (s1[tid] + cn - dn * pn) * idn : s1[tid] + cn - delta * pn) : 0.0;
    __syncthreads();
    tmatvec_mw<TG, CX, TX, TX>(Xn, xi, xj, xo, s0, s1, red, tid, lane);
    x = xr ? -s1[tid] : 0.0;
    if constexpr (PF) {
#pragma unroll
      for (int t = 0; t < CZ; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) Zk[t][v] = Zk1[t][v];
#pragma unroll
      for (int t = 0; t < CX; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) Xn[t][v] = Xn1[t][v];
#pragma unroll
      for (int t = 0; t < CT; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) ABt[t][v] = ABt1[t][v];
      pk = pk1; kk = kk1; pn = pn1; cn = cn1; dn = dn1;
    }
  }
  if (SEG && phase == 2) {
    if (xr) a.xhi[mt.ovec + (int64_t)sd.s * n + tid] = x;
    return;
  }
  if (hi == N) {
    double ZN[CZ][4];
    load_tile(ZN, ztile(N), zo, CZ);
    const double pN = xr ? pg[(int64_t)N * n + tid] : 0.0;
    __syncthreads();
    if (tid < NZ) s0[tid] = xr ? x : 0.0;
    __syncthreads();
    tmatvec_mw<TG, CZ, TZ, TZ>(ZN, zi, zj, zo, s0, s1, red, tid, lane);
    if (xr) {
      const int64_t i = (int64_t)N * n + tid;
      const double yN = s1[tid] + pN;
      yg[i] = accum ? yg[i] + yN : yN;
      xg[i] = accum ? xg[i] + x : x;
    }
  }
}

// Column-owned whole-instance solve for the stage tiles up to 48 wide (TZ <= 3):
// the passes of k_solve_mw (SEG = false; Theorem "main-seq-theorem") with one
// wavefront per block column, TZ in all. Wavefront J holds block column J of
// every tile it multiplies, so a product y = T^T v is a sum over the block
// rows in registers and over the four lane groups (group_sum), and entry
// y_i lands in the thread that owns index i (wavefront i / 16, the lanes of
// column i % 16), the thread that holds every other per-index quantity of
// the step as well. Each product costs one workgroup barrier (its operand
// vector goes through LDS): three per step in each direction. The backward
// pass forms P_k c_k for the next step from the same tile Z_k, in the same
// phase as [-K_k^T h; -G_k^{-1} h].
template <int TX, int TZ>
__device__ __forceinline__ int zblock(int I, int J) {
  if (I < TX && J < TX) return I * TX + J;
  if (I < TX) return TX * TX + I * (TZ - TX) + (J - TX);
  return TX * TX + TX * (TZ - TX) + (I - TX) * TZ + J;
}

// sum over the rows of R blocks of one block column: sum_r T[r][c] vec[r]
template <typename TL, typename T, int R>
__device__ __forceinline__ double col_dot(const T (&X)[R][4], const double* vec, int grp) {
  double s0 = 0.0, s1 = 0.0;
#pragma unroll
  for (int I = 0; I < R; ++I) {
    s0 = __fma_rn((double)X[I][0], vec[16 * I + trow<TL>(grp, 0)], s0);
    s1 = __fma_rn((double)X[I][1], vec[16 * I + trow<TL>(grp, 1)], s1);
    s0 = __fma_rn((double)X[I][2], vec[16 * I + trow<TL>(grp, 2)], s0);
    s1 = __fma_rn((double)X[I][3], vec[16 * I + trow<TL>(grp, 3)], s1);
  }
  return group_sum(s0 + s1);
}

template <typename TG, int TX, int TZ, bool DG>
__global__ __launch_bounds__(64 * TZ) void k_solve_col(SolveArgs a) {
  using C = MwCfg<TG, TX, TZ, TZ>;
  constexpr int NX = C::NX, NZ = C::NZ;
  const int b = a.list ? a.list[blockIdx.x] : (int)blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, col = lane & 15, grp = lane >> 4;
  const int J = __builtin_amdgcn_readfirstlane(tid >> 6);  // the wavefront's block column (uniform)
  if (a.run && !a.run[b]) return;
  const InstMeta mt = a.meta[b];
  const int N = mt.N, n = mt.n, m = mt.m;
  const double delta = DG ? 0.0 : a.delta[b];
  const double* __restrict__ ddg = DG ? a.dd + mt.od : nullptr;
  const double* __restrict__ Ag = a.A + mt.oA;
  const double* __restrict__ Bg = a.B + mt.oB;
  const TG* __restrict__ ws = reinterpret_cast<const TG*>(a.ws) + mt.ows;
  constexpr int64_t STAGE = (int64_t)C::BLOCKS_PER_STAGE * 256;
  auto ztile = [&](int i) { return ws + (int64_t)i * STAGE; };
  auto xtile = [&](int i) { return ws + (int64_t)i * STAGE + (int64_t)TZ * TZ * 256; };
  double* __restrict__ pg = a.pk + mt.opk;
  double* __restrict__ kg = a.pk + mt.opk + (int64_t)(N + 1) * n;
  const double *qb, *rb, *cb;
  int64_t qs, rs;
  const bool accum = a.corr != nullptr;
  if (accum) {
    const double* res = a.corr + mt.ores;
    qb = res; qs = n + m;
    rb = res + n; rs = n + m;
    cb = res + (int64_t)N * (n + m) + n;
  } else {
    qb = a.q + mt.oq; qs = n;
    rb = a.r + mt.or_; rs = m;
    cb = a.c + mt.oc;
  }
  double* __restrict__ xg = a.x + mt.ox;
  double* __restrict__ ug = a.u + mt.ou;
  double* __restrict__ yg = a.y + mt.oy;
  if (a.info[b].singular) {
    if (!accum) {
      const double nanv = __builtin_nan("");
      for (int i = tid; i < (N + 1) * n; i += 64 * TZ) { xg[i] = nanv; yg[i] = nanv; }
      for (int i = tid; i < N * m; i += 64 * TZ) ug[i] = nanv;
    }
    return;
  }

  // operand vectors, one per product of a step (a buffer is rewritten only
  // after a barrier that every reader of its previous contents has passed)
  __shared__ double bv[NZ], bg[NZ], bh[NZ], bc[NZ], bx[NZ], bz[NZ], bw[NZ];
  const int vi = 16 * J + col;  // the vector index this thread owns
  const bool xr = vi < n, ur = vi >= n && vi < n + m, own = grp == 0;
  const bool wx = J < TX;  // the wavefront holds state indices (and X, [A B]^T columns)

  // tile loads in the stored precision (converted where used); padding
  // elements of [A B] read the zero kZeroPad (branch-free)
  auto load_z = [&](TG (&R)[TZ][4], const TG* zt) {
#pragma unroll
    for (int I = 0; I < TZ; ++I)
#pragma unroll
      for (int v = 0; v < 4; ++v) R[I][v] = zt[(int64_t)zblock<TX, TZ>(I, J) * 256 + v * 64 + lane];
  };
  const int Jx = wx ? J : 0;  // the other wavefronts load a state column too (unused): no masked loads
  auto load_x = [&](TG (&R)[TX][4], const TG* xt) {
#pragma unroll
    for (int I = 0; I < TX; ++I)
#pragma unroll
      for (int v = 0; v < 4; ++v) R[I][v] = xt[(int64_t)(I * TX + Jx) * 256 + v * 64 + lane];
  };
  // &[A_k B_k][r][c]; outside the n x (n+m) block the first element of A_k
  // (any finite value does: the products below multiply such entries only by
  // zero vector entries or write only outputs that are discarded). Integer
  // choices only: a choice between address computations becomes a branch.
  auto ab_ptr = [&](int k, int r, int c) {
    const uint64_t ua = reinterpret_cast<uint64_t>(Ag + (int64_t)k * n * n);
    const uint64_t ub = reinterpret_cast<uint64_t>(Bg + (int64_t)k * n * m);
    const bool inA = r < n && c < n, inB = r < n && c >= n && c < n + m;
    const int o1 = r * n + c, o2 = r * m + (c - n);
    const int off = inA ? o1 : (inB ? o2 : 0);
    return reinterpret_cast<const double*>(inB ? ub : ua) + off;
  };
  auto load_ab = [&](double (&R)[TX][4], int k) {  // column J of [A B]
#pragma unroll
    for (int I = 0; I < TX; ++I)
#pragma unroll
      for (int v = 0; v < 4; ++v) R[I][v] = *ab_ptr(k, 16 * I + trow<TG>(grp, v), 16 * J + col);
  };
  auto load_abt = [&](double (&R)[TZ][4], int k) {  // column J of [A B]^T (J < TX)
#pragma unroll
    for (int I = 0; I < TZ; ++I)
#pragma unroll
      for (int v = 0; v < 4; ++v) R[I][v] = *ab_ptr(k, wx ? 16 * J + col : NX, 16 * I + trow<TG>(grp, v));
  };
  auto ldv = [&](const double* p, int64_t i, bool ok) { return *(ok ? p + i : kZeroPad); };

  // ---- backward vector pass, k = N-1 .. 0. p_k and k_k go to pk from every
  // lane group (the same value): each thread reads back only its own stores.
  double p = ldv(qb, (int64_t)N * qs + vi, xr);  // p_{k+1}
  if (xr) pg[(int64_t)N * n + vi] = p;
  double pc;  // (P_{k+1} c_{k+1})_vi
  {
    TG ZN[TZ][4];
    load_z(ZN, ztile(N));
    const double cN = ldv(cb, (int64_t)N * n + vi, xr);
    if (own) bc[vi] = cN;
    __syncthreads();
    pc = col_dot<TG, TG, TX>(reinterpret_cast<const TG(&)[TX][4]>(ZN), bc, grp);
  }
  // A step's operands are loaded two steps ahead (the loads are in flight for
  // two steps of products and barriers): three operand sets in rotation,
  // the loop unrolled by three so that no set is copied.
  struct BwdOps {
    TG Z[TZ][4];      // column J of Z_k (state rows only in the state columns)
    TG X[TX][4];      // column J of X_{k+1}
    double AB[TX][4]; // column J of [A_k B_k]
    double q, r, c, d;
  };
  // the backward products take Z_k's state block (P_k c_k) and its control
  // rows (h only has control entries, rows n .. n+m-1): in the control
  // columns the block rows above row n are not read, and their registers are
  // zero
  const int hrow0 = n >> 4;  // first block row holding a control row
  auto load_bwd = [&](BwdOps& o, int k) {
    k = k > 0 ? k : 0;
#pragma unroll
    for (int I = 0; I < TZ; ++I) {
      if (wx || I >= hrow0) {  // uniform branch
#pragma unroll
        for (int v = 0; v < 4; ++v) o.Z[I][v] = ztile(k)[(int64_t)zblock<TX, TZ>(I, J) * 256 + v * 64 + lane];
      } else {
#pragma unroll
        for (int v = 0; v < 4; ++v) o.Z[I][v] = (TG)0;
      }
    }
    load_x(o.X, xtile(k + 1));
    load_ab(o.AB, k);
    o.q = ldv(qb, (int64_t)k * qs + vi, xr);
    o.r = ldv(rb, (int64_t)k * rs + (vi - n), ur);
    o.c = ldv(cb, (int64_t)k * n + vi, xr);
    o.d = DG ? ldv(ddg, (int64_t)(k + 1) * n + vi, xr) : 0.0;
  };
  auto bwd_step = [&](const BwdOps& o, int k) {
    // g = S_hat_{k+1}^{-1} (p_{k+1} + P_{k+1} c_{k+1})  (DG: -Delta^{-1} X~ v)
    if (own && wx) bv[vi] = xr ? p + pc : 0.0;
    __syncthreads();
    double g = 0.0;
    if (wx) {
      const double t = col_dot<TG, TG, TX>(o.X, bv, grp);
      g = xr ? (DG ? -t / o.d : -t) : 0.0;
    }
    // [A^T g; B^T g]
    if (own && wx) bg[vi] = g;
    __syncthreads();
    const double abg = col_dot<TG, double, TX>(o.AB, bg, grp);
    // h = r_k + B^T g; [-K^T h; -G^{-1} h] and P_k c_k, both from Z_k
    if (own) {
      bh[vi] = ur ? o.r + abg : 0.0;
      bc[vi] = xr ? o.c : 0.0;
    }
    __syncthreads();
    const double zh = col_dot<TG, TG, TZ>(o.Z, bh, grp);
    pc = wx ? col_dot<TG, TG, TX>(reinterpret_cast<const TG(&)[TX][4]>(o.Z), bc, grp) : 0.0;
    if (xr) {
      p = o.q + abg - zh;
      pg[(int64_t)k * n + vi] = p;
    }
    if (ur) kg[(int64_t)k * m + (vi - n)] = zh;
  };
  if (N > 0) {
    BwdOps S0, S1, S2;
    load_bwd(S0, N - 1);
    load_bwd(S1, N - 2);
    int k = N - 1;
    for (;;) {
      load_bwd(S2, k - 2);
      bwd_step(S0, k);
      if (--k < 0) break;
      load_bwd(S0, k - 2);
      bwd_step(S1, k);
      if (--k < 0) break;
      load_bwd(S1, k - 2);
      bwd_step(S2, k);
      if (--k < 0) break;
    }
  }

  // ---- forward rollout, k = 0 .. N-1
  double x;
  {
    TG X0[TX][4];
    load_x(X0, xtile(0));
    const double p0 = ldv(pg, vi, xr);
    const double c0 = ldv(cb, vi, xr);
    const double d0 = DG ? ldv(ddg, vi, xr) : delta;
    if (own && wx) bw[vi] = xr ? (DG ? (c0 - d0 * p0) / d0 : c0 - delta * p0) : 0.0;
    __syncthreads();
    x = (wx && xr) ? -col_dot<TG, TG, TX>(X0, bw, grp) : 0.0;
  }
  struct FwdOps {
    TG Z[TX][4];       // column J of Z_k, state rows
    TG X[TX][4];       // column J of X_{k+1}
    double ABt[TZ][4]; // column J of [A_k B_k]^T
    double pk, kk, pn, cn, dn;
  };
  auto load_fwd = [&](FwdOps& o, int k) {
    k = k < N - 1 ? k : N - 1;
#pragma unroll
    for (int I = 0; I < TX; ++I)
#pragma unroll
      for (int v = 0; v < 4; ++v) o.Z[I][v] = ztile(k)[(int64_t)zblock<TX, TZ>(I, J) * 256 + v * 64 + lane];
    load_x(o.X, xtile(k + 1));
    load_abt(o.ABt, k);
    o.pk = ldv(pg, (int64_t)k * n + vi, xr);
    o.kk = ldv(kg, (int64_t)k * m + (vi - n), ur);
    o.pn = ldv(pg, (int64_t)(k + 1) * n + vi, xr);
    o.cn = ldv(cb, (int64_t)(k + 1) * n + vi, xr);
    o.dn = DG ? ldv(ddg, (int64_t)(k + 1) * n + vi, xr) : delta;
  };
  auto fwd_step = [&](const FwdOps& o, int k) {
    // [P_k x_k; -K_k x_k]: y_k and u_k
    if (own && wx) bx[vi] = x;
    __syncthreads();
    const double zx = col_dot<TG, TG, TX>(o.Z, bx, grp);
    double uk = 0.0;
    if (own && xr) {
      const int64_t i = (int64_t)k * n + vi;
      const double yk = zx + o.pk;
      yg[i] = accum ? yg[i] + yk : yk;
      xg[i] = accum ? xg[i] + x : x;
    }
    if (ur) {
      uk = o.kk - zx;
      const int64_t i = (int64_t)k * m + (vi - n);
      if (own) ug[i] = accum ? ug[i] + uk : uk;
    }
    // [A_k B_k] z_k
    if (own) bz[vi] = xr ? x : uk;
    __syncthreads();
    double wv = 0.0;
    if (wx) {
      const double t = col_dot<TG, double, TZ>(o.ABt, bz, grp);
      wv = xr ? (DG ? (t + o.cn - o.dn * o.pn) / o.dn : t + o.cn - delta * o.pn) : 0.0;
    }
    // x_{k+1} = S_hat_{k+1}^{-1} (...)  (DG: -X~ Delta^{-1} (...))
    if (own && wx) bw[vi] = wv;
    __syncthreads();
    x = (wx && xr) ? -col_dot<TG, TG, TX>(o.X, bw, grp) : 0.0;
  };
  if (N > 0) {
    FwdOps S0, S1, S2;
    load_fwd(S0, 0);
    load_fwd(S1, 1);
    int k = 0;
    for (;;) {
      load_fwd(S2, k + 2);
      fwd_step(S0, k);
      if (++k >= N) break;
      load_fwd(S0, k + 2);
      fwd_step(S1, k);
      if (++k >= N) break;
      load_fwd(S1, k + 2);
      fwd_step(S2, k);
      if (++k >= N) break;
    }
  }
  // x_N, y_N = P_N x_N + p_N
  {
    TG ZN[TZ][4];
    load_z(ZN, ztile(N));
    const double pN = ldv(pg, (int64_t)N * n + vi, xr);
    if (own && wx) bx[vi] = x;
    __syncthreads();
    const double zx = col_dot<TG, TG, TX>(reinterpret_cast<const TG(&)[TX][4]>(ZN), bx, grp);
    if (own && xr) {
      const int64_t i = (int64_t)N * n + vi;
      const double yN = zx + pN;
      yg[i] = accum ? yg[i] + yN : yN;
      xg[i] = accum ? xg[i] + x : x;
    }
  }
}

// ------------------------------------------------------------------ dispatch

template <typename TG, int TX, int TZ, int NW>
static hipError_t launch_mw_pair(bool factor, const void* args, int nblocks, hipStream_t st) {
  if (factor) {
    const FactorArgs& a = *reinterpret_cast<const FactorArgs*>(args);
    if (a.dd)
      hipLaunchKernelGGL((k_factor_mw<TG, TX, TZ, NW, true>), dim3(nblocks), dim3(64 * NW), 0, st, a);
    else
      hipLaunchKernelGGL((k_factor_mw<TG, TX, TZ, NW, false>), dim3(nblocks), dim3(64 * NW), 0, st, a);
  } else {
    // whole-instance solves: one wavefront per block column up to 48-wide tiles
    const SolveArgs& a = *reinterpret_cast<const SolveArgs*>(args);
    if constexpr (TZ <= 3) {
      if (a.dd)
        hipLaunchKernelGGL((k_solve_col<TG, TX, TZ, true>), dim3(nblocks), dim3(64 * TZ), 0, st, a);
      else
        hipLaunchKernelGGL((k_solve_col<TG, TX, TZ, false>), dim3(nblocks), dim3(64 * TZ), 0, st, a);
    } else {
      if (a.dd)
        hipLaunchKernelGGL((k_solve_mw<TG, TX, TZ, NW, false, true>), dim3(nblocks), dim3(64 * NW), 0, st, a);
      else
        hipLaunchKernelGGL((k_solve_mw<TG, TX, TZ, NW, false, false>), dim3(nblocks), dim3(64 * NW), 0, st, a);
    }
  }
  return hipGetLastError();
}

// waves: wavefronts per instance of the classes up to 32 x 48 (1, 2, 4 or 8;
// the 32-wide classes take at least 2). With fewer wavefronts each owns more
// blocks and the stage's workgroup barriers get cheaper (one wavefront:
// none to wait for).
template <typename TG>
static hipError_t launch_mw_t(int cls, bool factor, const void* args, int nblocks, hipStream_t st, int waves) {
  switch (cls) {
    case TILE_X1_Z2:
      switch (waves) {
        case 1: return launch_mw_pair<TG, 1, 2, 1>(factor, args, nblocks, st);
        case 2: return launch_mw_pair<TG, 1, 2, 2>(factor, args, nblocks, st);
        case 8: return launch_mw_pair<TG, 1, 2, 8>(factor, args, nblocks, st);
        default: return launch_mw_pair<TG, 1, 2, 4>(factor, args, nblocks, st);
      }
    case TILE_X2_Z2:
      switch (waves) {
        case 1: case 2: return launch_mw_pair<TG, 2, 2, 2>(factor, args, nblocks, st);
        case 8: return launch_mw_pair<TG, 2, 2, 8>(factor, args, nblocks, st);
        default: return launch_mw_pair<TG, 2, 2, 4>(factor, args, nblocks, st);
      }
    case TILE_X2_Z3:
      switch (waves) {
        case 1: case 2: return launch_mw_pair<TG, 2, 3, 2>(factor, args, nblocks, st);
        case 8: return launch_mw_pair<TG, 2, 3, 8>(factor, args, nblocks, st);
        default: return launch_mw_pair<TG, 2, 3, 4>(factor, args, nblocks, st);
      }
    case TILE_X3_Z3: return launch_mw_pair<TG, 3, 3, 9>(factor, args, nblocks, st);
    case TILE_X4_Z4: return launch_mw_pair<TG, 4, 4, 16>(factor, args, nblocks, st);
    case TILE_X4_Z6: return launch_mw_pair<TG, 4, 6, 16>(factor, args, nblocks, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_factor_mw(int cls, const FactorArgs& a, int nblocks, bool fp32, hipStream_t st, int waves) {
  if (nblocks <= 0) return hipSuccess;
  return fp32 ? launch_mw_t<float>(cls, true, &a, nblocks, st, waves)
              : launch_mw_t<double>(cls, true, &a, nblocks, st, waves);
}

hipError_t launch_solve_mw(int cls, const SolveArgs& a, int nblocks, bool fp32, hipStream_t st, int waves) {
  if (nblocks <= 0) return hipSuccess;
  return fp32 ? launch_mw_t<float>(cls, false, &a, nblocks, st, waves)
              : launch_mw_t<double>(cls, false, &a, nblocks, st, waves);
}

// Segment solves (scan mode, float32 tiles); the one-wavefront class uses the
// same kernel with a single 16 x 16 block (its workspace layout is identical).
template <int TX, int TZ, int NW>
static hipError_t launch_seg_t(const SolveArgs& a, int nblocks, hipStream_t st) {
  if (a.dd)
    hipLaunchKernelGGL((k_solve_mw<float, TX, TZ, NW, true, true>), dim3(nblocks), dim3(64 * NW), 0, st, a);
  else
    hipLaunchKernelGGL((k_solve_mw<float, TX, TZ, NW, true, false>), dim3(nblocks), dim3(64 * NW), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_seg_solve(int cls, const SolveArgs& a, int nblocks, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  switch (cls) {
    case TILE_16: return launch_seg_t<1, 1, 1>(a, nblocks, st);
    case TILE_X1_Z2: return launch_seg_t<1, 2, 4>(a, nblocks, st);
    case TILE_X2_Z2: return launch_seg_t<2, 2, 4>(a, nblocks, st);
    case TILE_X2_Z3: return launch_seg_t<2, 3, 4>(a, nblocks, st);
    case TILE_X3_Z3: return launch_seg_t<3, 3, 9>(a, nblocks, st);
    case TILE_X4_Z4: return launch_seg_t<4, 4, 16>(a, nblocks, st);
    case TILE_X4_Z6: return launch_seg_t<4, 6, 16>(a, nblocks, st);
  }
  return hipErrorInvalidValue;
}

int tile_blocks_per_stage(int cls) {
  switch (cls) {
    case TILE_16: return 2;
    case TILE_X1_Z2: return 4 + 1;
    case TILE_X2_Z2: return 4 + 4;
    case TILE_X2_Z3: return 9 + 4;
    case TILE_X3_Z3: return 9 + 9;
    case TILE_X4_Z4: return 16 + 16;
    case TILE_X4_Z6: return 36 + 16;
  }
  return 0;
}

}  // namespace rlqr
