// rlqr_scan.hip -- parallel-in-time pieces of the dual-regularized Riccati
// solver (Section "Parallel Algorithm" of arXiv 2509.16370), float32 products;
// the combine's products optionally take bfloat16 operands (float32
// accumulation, RLQR_SCAN_BF16).
//
// Interval value-function elements e = (P, A, C) (eqs. lqr-gpu-init-running,
// lqr-gpu-init-terminal) are stored per element as three NX x NX float32
// tiles, row-major with stride NX, zero outside n x n:
//     P at 0, A at NX^2, C at 2 NX^2.
// The combine (i->j) (+) (j->k) is the single-inversion form of eq.
// lqr-gpu-combo with X = I + C_ij P_jk inverted by Gauss-Jordan elimination
// with partial pivoting. By default p and c are not carried (the p-recurrence
// recovers p, as the paper recommends); with ScanArgs::pc they are carried as
// float32 vectors beside the elements (the paper's alternative), built from
// one right-hand side.
#include "rlqr_device_mw.h"
#include "rlqr_internal.h"

namespace rlqr {

// ------------------------------------------------------------ block helpers

// C block (I, J) = op(A) * B, KB 16-blocks of inner dimension, float32 LDS operands.
template <bool TRANS_A, int KB>
__device__ __forceinline__ f4 sgemm_blk(const float* sa, int lda, const float* sb, int ldb, int I, int J, int lane) {
  f4 acc = {0, 0, 0, 0};
  const int i = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int kb = 0; kb < KB; ++kb)
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int k = 16 * kb + 4 * kk + kq;
      const float av = TRANS_A ? sa[k * lda + 16 * I + i] : sa[(16 * I + i) * lda + k];
      const float bv = sb[k * ldb + 16 * J + i];
      acc = mfma16(av, bv, acc);
    }
  return acc;
}
// same with op(B) = B^T
template <int KB>
__device__ __forceinline__ f4 sgemm_blk_bt(const float* sa, int lda, const float* sb, int ldb, int I, int J, int lane) {
  f4 acc = {0, 0, 0, 0};
  const int i = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int kb = 0; kb < KB; ++kb)
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      const int k = 16 * kb + 4 * kk + kq;
      const float av = sa[(16 * I + i) * lda + k];
      const float bv = sb[(16 * J + i) * ldb + k];
      acc = mfma16(av, bv, acc);
    }
  return acc;
}

typedef short s4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf4 __attribute__((ext_vector_type(4)));

// The same block products with bfloat16 operands (float32 -> bfloat16 by the
// hardware conversion, round to nearest even) and float32 accumulation, on
// gfx950's 16x16x32 MFMA: lane l supplies op(A)[i][32 kb + 8 kq + j] and
// B[32 kb + 8 kq + j][i] (i = l & 15, kq = l >> 4, j = 0..7), the accumulator
// layout being that of the float32 instruction. An odd last 16-block of the
// inner dimension takes the 16x16x16 instruction (4 per lane).
template <bool TRANS_A, int KB>
__device__ __forceinline__ f4 bgemm_blk(const float* sa, int lda, const float* sb, int ldb, int I, int J, int lane) {
  f4 acc = {0, 0, 0, 0};
  const int i = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int kb = 0; kb + 1 < KB; kb += 2) {
    bf8 av, bv;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = 16 * kb + 8 * kq + j;
      av[j] = (__bf16)(TRANS_A ? sa[k * lda + 16 * I + i] : sa[(16 * I + i) * lda + k]);
      bv[j] = (__bf16)sb[k * ldb + 16 * J + i];
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
  }
  if constexpr (KB % 2) {
    bf4 av, bv;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = 16 * (KB - 1) + 4 * kq + j;
      av[j] = (__bf16)(TRANS_A ? sa[k * lda + 16 * I + i] : sa[(16 * I + i) * lda + k]);
      bv[j] = (__bf16)sb[k * ldb + 16 * J + i];
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4, av), __builtin_bit_cast(s4, bv), acc, 0, 0, 0);
  }
  return acc;
}
template <int KB>
__device__ __forceinline__ f4 bgemm_blk_bt(const float* sa, int lda, const float* sb, int ldb, int I, int J, int lane) {
  f4 acc = {0, 0, 0, 0};
  const int i = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int kb = 0; kb + 1 < KB; kb += 2) {
    bf8 av, bv;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = 16 * kb + 8 * kq + j;
      av[j] = (__bf16)sa[(16 * I + i) * lda + k];
      bv[j] = (__bf16)sb[(16 * J + i) * ldb + k];
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
  }
  if constexpr (KB % 2) {
    bf4 av, bv;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = 16 * (KB - 1) + 4 * kq + j;
      av[j] = (__bf16)sa[(16 * I + i) * lda + k];
      bv[j] = (__bf16)sb[(16 * J + i) * ldb + k];
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4, av), __builtin_bit_cast(s4, bv), acc, 0, 0, 0);
  }
  return acc;
}

// operand precision of the combine's products: float32 or bfloat16
template <bool BF, bool TRANS_A, int KB>
__device__ __forceinline__ f4 cgemm(const float* sa, int lda, const float* sb, int ldb, int I, int J, int lane) {
  if constexpr (BF) return bgemm_blk<TRANS_A, KB>(sa, lda, sb, ldb, I, J, lane);
  else return sgemm_blk<TRANS_A, KB>(sa, lda, sb, ldb, I, J, lane);
}
template <bool BF, int KB>
__device__ __forceinline__ f4 cgemm_bt(const float* sa, int lda, const float* sb, int ldb, int I, int J, int lane) {
  if constexpr (BF) return bgemm_blk_bt<KB>(sa, lda, sb, ldb, I, J, lane);
  else return sgemm_blk_bt<KB>(sa, lda, sb, ldb, I, J, lane);
}

// max over the 64 lanes (every lane gets it): DPP row rotations, then the
// four row maxima
__device__ __forceinline__ float wave_max_f32(float x) {
  x = fmaxf(x, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x121, 0xf, 0xf, false)));
  x = fmaxf(x, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x122, 0xf, 0xf, false)));
  x = fmaxf(x, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x124, 0xf, 0xf, false)));
  x = fmaxf(x, __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x128, 0xf, 0xf, false)));
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 0));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 16));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 32));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 48));
  return fmaxf(fmaxf(r0, r1), fmaxf(r2, r3));
}

// accumulator element (v) of block (I, J): row 16 I + 4 grp + v, column 16 J + col
__device__ __forceinline__ int arow(int I, int grp, int v) { return 16 * I + 4 * grp + v; }

// ------------------------------------------------------------ combine

template <int TX, int NW>
struct ScanCfg {
  static constexpr int NX = 16 * TX, LDX = NX + 1, LDW = 2 * NX + 1;
  static constexpr int NB = TX * TX;                   // blocks of a state tile
  static constexpr int CB = (NB + NW - 1) / NW;        // blocks per wavefront
  static constexpr int TILE = NX * LDX;                // floats of an LDS tile
  static constexpr int ELEM = 3 * NX * NX;             // floats of a stored element
  static constexpr int KE = (NX * NX + 64 * NW - 1) / (64 * NW);  // tile floats per thread
};

// LDS working set of one combine
template <int TX, int NW>
struct ScanLds {
  using C = ScanCfg<TX, NW>;
  float P1[C::TILE], A1[C::TILE], C1[C::TILE];  // accumulated (i -> j)
  float P2[C::TILE], A2[C::TILE];               // next (j -> k)
  float W[C::NX * C::LDW];                      // [X | X^{-1}], later temporaries
  float YA[C::TILE], YC[C::TILE];
  int xrow[C::NX];  // Gauss-Jordan: row r of X^{-1} ends as right-half row xrow[r]
  int pv[2][16];                // Gauss-Jordan: pivot rows of a block of columns (by its parity)
  float G[2][C::NX * 17];       // Gauss-Jordan: a block's row coefficients (row stride 17, by its parity)
  unsigned long long pm[2];     // Gauss-Jordan: the pivot rows of a block as a row mask (by its parity)
  float pv1[C::NX], cv1[C::NX], pv2[C::NX], cv2[C::NX], tv[C::NX], tw[C::NX];  // carried p, c
  int piv;
};

// carried vectors of an element / aggregate (2 NX floats: p, then c)
template <int TX, int NW>
__device__ __forceinline__ void load_pc(float* p, float* c, const float* __restrict__ g, int tid) {
  constexpr int NX = 16 * TX;
  if (tid < NX) {
    p[tid] = g[tid];
    c[tid] = g[NX + tid];
  }
}
template <int TX, int NW>
__device__ __forceinline__ void store_pc(float* __restrict__ g, const float* p, const float* c, int tid) {
  constexpr int NX = 16 * TX;
  if (tid < NX) {
    g[tid] = p[tid];
    g[NX + tid] = c[tid];
  }
}

// copy an element's P, A (and C if withC) from global into LDS tiles
template <int TX, int NW>
__device__ __forceinline__ void load_elem(float* P, float* A, float* Cc, const float* __restrict__ e, int tid) {
  using C = ScanCfg<TX, NW>;
  for (int x = tid; x < C::NX * C::NX; x += 64 * NW) {
    const int r = x / C::NX, c = x % C::NX;
    P[r * C::LDX + c] = e[x];
    A[r * C::LDX + c] = e[C::NX * C::NX + x];
    if (Cc) Cc[r * C::LDX + c] = e[2 * C::NX * C::NX + x];
  }
}
template <int TX, int NW>
__device__ __forceinline__ void store_elem(float* __restrict__ e, const float* P, const float* A, const float* Cc, int tid) {
  using C = ScanCfg<TX, NW>;
  for (int x = tid; x < C::NX * C::NX; x += 64 * NW) {
    const int r = x / C::NX, c = x % C::NX;
    e[x] = P[r * C::LDX + c];
    e[C::NX * C::NX + x] = A[r * C::LDX + c];
    e[2 * C::NX * C::NX + x] = Cc[r * C::LDX + c];
  }
}

// Gauss-Jordan elimination with partial pivoting of one 16-column panel held
// one row per lane (v; rows past the matrix are zero and never candidates),
// first kn columns: for column j the largest unused |entry| (to a relative
// 2^-17, lowest row among those) is the pivot row p_j, and every other row
// subtracts its multiple of row p_j (pivot rows are not scaled on the way).
// g carries each row as a combination of the pivot rows' original rows: on
// return row l of the eliminated panel matrix is (l not a pivot row of this
// panel ? M[l] : 0) + sum_j g[j] M[p_j], which is the update every other
// column block takes. used gains the pivot rows, lane j gets p_j in pl, and
// sing is set if a column has no nonzero candidate. FULL: kn == 16 (no
// run-time test per column).
template <bool FULL>
__device__ __forceinline__ void panel_gj(float (&v)[16], float (&g)[16], int kn, int lane, unsigned long long rows,
                                         unsigned long long& used, bool& sing, int& pl) {
  // opaque lane index: the lane tests below are made in place, not kept as
  // loop-invariant scalar masks for the whole panel loop
  int ln = lane;
  asm volatile("" : "+v"(ln));
  const unsigned long long u0 = used;
  float dme = 1.0f;  // a pivot row's own pivot
#pragma unroll
  for (int c = 0; c < 16; ++c) g[c] = 0.0f;
#pragma unroll
  for (int jj = 0; jj < 16; ++jj) {
    if (FULL || jj < kn) {
      // |entry| of a candidate as its bit pattern (ordered like the values for
      // non-negative floats) with the 6 low mantissa bits replaced by 63 - lane,
      // -1 for non-candidates and NaN: the wavefront maximum (a DPP row reduction
      // and a scalar max of the four rows) names the pivot row itself, the
      // largest |entry| to a relative 2^-17, the lowest row among those. With no
      // valid candidate the lowest unused row is taken.
      const bool cand = ((rows & ~used) >> lane) & 1ull;
      const float a = fabsf(v[jj]);
      const int key = (cand && !__builtin_isnan(a)) ? ((__float_as_int(a) & ~63) | (63 - lane)) : -1;
      int k = key;
      k = max(k, __builtin_amdgcn_mov_dpp(k, 0x121, 0xf, 0xf, false));
      k = max(k, __builtin_amdgcn_mov_dpp(k, 0x122, 0xf, 0xf, false));
      k = max(k, __builtin_amdgcn_mov_dpp(k, 0x124, 0xf, 0xf, false));
      k = max(k, __builtin_amdgcn_mov_dpp(k, 0x128, 0xf, 0xf, false));
      const int best = max(max(__builtin_amdgcn_readlane(k, 0), __builtin_amdgcn_readlane(k, 16)),
                           max(__builtin_amdgcn_readlane(k, 32), __builtin_amdgcn_readlane(k, 48)));
      const bool piv = best >= 64;  // a nonzero pivot (|entry| above 64 times the smallest subnormal)
      const int p = best >= 0 ? 63 - (best & 63) : __builtin_ctzll(~used & rows);
      used |= 1ull << p;
      sing = sing || !piv;
      if (ln == jj) pl = p;
      const float d = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v[jj]), p));
      // 1 / d: hardware estimate and one Newton step, r + r (1 - d r); no
      // elimination without a nonzero pivot
      const float r0 = __builtin_amdgcn_rcpf(d);
      const float rd = piv ? fmaf(r0, fmaf(-d, r0, 1.0f), r0) : 0.0f;
      const bool me = ln == p;
      if (me) dme = d;
      const float f = me ? 0.0f : v[jj] * rd;
#pragma unroll
      for (int c = jj + 1; c < 16; ++c)
        v[c] = fmaf(-f, __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v[c]), p)), v[c]);
#pragma unroll
      for (int c = 0; c < jj; ++c)
        g[c] = fmaf(-f, __int_as_float(__builtin_amdgcn_readlane(__float_as_int(g[c]), p)), g[c]);
      g[jj] = me ? 1.0f : -f;
    }
  }
  // scale this panel's pivot rows by their pivots
  const float r0 = __builtin_amdgcn_rcpf(dme);
  const float rs = dme != 0.0f ? fmaf(r0, fmaf(-dme, r0, 1.0f), r0) : 0.0f;
  if (((used & ~u0) >> lane) & 1ull) {
#pragma unroll
    for (int c = 0; c < 16; ++c) g[c] *= rs;
  }
}

// acc (P1, A1, C1 in LDS) <- acc (+) next (P2, A2 in LDS, C2 in global).
// pc: also the carried vectors (p1, c1) <- (+) (p2, c2), all in LDS.
// nxt (or null): the element after next, whose P and A are read into pf
// (the thread's share, as load_elem lays it out) while the products run.
// Returns false if X = I + C1 P2 is singular (no pivot above tol).
template <int TX, int NW, bool BF>
__device__ __forceinline__ bool combine(ScanLds<TX, NW>& s, const float* __restrict__ C2g, int n, int tid, bool pc,
                                        const float* __restrict__ nxt, float (&pf)[2 * ScanCfg<TX, NW>::KE]) {
  // opaque thread index: in the chunk fold's loop the lane-dependent offsets
  // are re-derived in every combine instead of being hoisted out of the loop
  asm volatile("" : "+v"(tid));
  using C = ScanCfg<TX, NW>;
  constexpr int NX = C::NX, LDX = C::LDX, LDW = C::LDW, CB = C::CB;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63, col = lane & 15, grp = lane >> 4;
  bool ok = true;
  // X = I + C1 P2 into the left half of W
#pragma unroll
  for (int t = 0; t < CB; ++t) {
    const int bx = w + NW * t;
    if (bx >= C::NB) break;
    const int I = bx / TX, J = bx % TX;
    f4 acc = cgemm<BF, false, TX>(s.C1, LDX, s.P2, LDX, I, J, lane);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = arow(I, grp, v), c = 16 * J + col;
      s.W[r * LDW + c] = acc[v] + (r == c ? 1.0f : 0.0f);  // the identity half is written below
    }
  }
  __syncthreads();
  // Blocked Gauss-Jordan with partial pivoting on the first n pivots of
  // M = [X | I] (W; rows are never swapped), 16 pivot columns C_K per block K:
  //  * wavefront 0 eliminates the panel M[:, C_K] in registers (one row per
  //    lane) with partial pivoting, which picks the pivot rows P_K in order, and
  //    carries every row as a combination G of the rows P_K; P_K and G go to
  //    LDS (two buffers, by the parity of K);
  //  * each live column block J is then updated by one wavefront, which reads
  //    all it needs (its own column block, P_K, G) before it writes:
  //    M[i, J] <- (i in P_K ? 0 : M[i, J]) + G[i, :] M[P_K, J] (MFMA).
  // This is the same elimination as 16 single pivot steps. A left-half column
  // block is dead once it has been a panel (only the right half is read
  // afterwards) and is not updated. Wavefront 0 updates the next panel's
  // column block itself and factors it in the same phase (one block of
  // lookahead), so a block takes one workgroup barrier and the serial panel
  // overlaps the other column updates. At the end row j of X^{-1} is the right
  // half's row p_j (xrow), which the products read in place.
  {
    constexpr int NJ = 2 * TX;  // column blocks of M
    // column block J >= 1 goes to the J-th wavefront w with w % 4 != 0, so no
    // other update shares wavefront 0's SIMD (wavefronts are dealt round-robin)
    static_assert(NJ - 1 <= (NW - 1) - (NW - 1) / 4, "one wavefront per column block");
    const int i = lane & 15, kq = lane >> 4;
    const int nk = (n + 15) >> 4;  // blocks of pivot columns
    for (int x = tid; x < NX * NX; x += 64 * NW) {
      const int r = x / NX, c = x % NX;
      s.W[r * LDW + NX + c] = (r == c) ? 1.0f : 0.0f;
    }
    if (tid < NX) s.xrow[tid] = tid;
    const unsigned long long rows = NX >= 64 ? ~0ull : ((1ull << (NX & 63)) - 1ull);
    unsigned long long used = 0ull;  // pivot rows so far (wavefront 0)
    bool sing = false;
    for (int K = -1; K < nk; ++K) {
      // this wavefront's column block after the pivots of block K: wavefront 0
      // takes the next panel's, the others the later left-half ones and the
      // right half
      int J = -1;
      if (K >= 0) {
        const int Jw = w - (w >> 2);
        if (w == 0) J = K + 1 < nk ? K + 1 : -1;
        else if ((w & 3) && ((Jw < TX && Jw > K + 1 && Jw < nk) || (Jw >= TX && Jw < NJ))) J = Jw;
      }
      if (J >= 0) {
        const int kn = min(16, n - 16 * K), b = K & 1;
        // B operand M[P_K, J] (k = 4 kk + kq, rows past kn zero), the owned
        // blocks M[I, J] and the A operands G[I, :]
        float Bv[4];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          const int k = 4 * kk + kq;
          Bv[kk] = k < kn ? s.W[s.pv[b][k] * LDW + 16 * J + i] : 0.0f;
        }
        float Mo[TX][4], Ga[TX][4];
#pragma unroll
        for (int I = 0; I < TX; ++I) {
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            Mo[I][e] = s.W[(16 * I + 4 * kq + e) * LDW + 16 * J + i];
            Ga[I][e] = s.G[b][(16 * I + i) * 17 + 4 * e + kq];
          }
        }
        const unsigned long long cur = s.pm[b];
#pragma unroll
        for (int I = 0; I < TX; ++I) {
          f4 acc = {0, 0, 0, 0};
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) acc = mfma16(Ga[I][kk], Bv[kk], acc);
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int r = 16 * I + 4 * kq + e;
            s.W[r * LDW + 16 * J + i] = ((cur >> r) & 1ull) ? acc[e] : Mo[I][e] + acc[e];
          }
        }
      }
      if (w == 0 && K + 1 < nk) {
        // the panel of block K + 1 (its column block was just updated by this
        // wavefront); rows >= NX are padding
        const int Kp = K + 1, kn = min(16, n - 16 * Kp), b = Kp & 1;
        float v[16], g[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) v[c] = lane < NX ? s.W[lane * LDW + 16 * Kp + c] : 0.0f;
        int pl = 0;  // lane j holds the pivot row of column 16 Kp + j
        const unsigned long long u0 = used;
        if (kn == 16) panel_gj<true>(v, g, kn, lane, rows, used, sing, pl);
        else panel_gj<false>(v, g, kn, lane, rows, used, sing, pl);
        if (lane < NX) {
#pragma unroll
          for (int c = 0; c < 16; ++c) s.G[b][lane * 17 + c] = g[c];
        }
        if (lane < 16) s.pv[b][lane] = pl;
        if (lane == 0) s.pm[b] = used & ~u0;
        if (lane < kn) s.xrow[16 * Kp + lane] = pl;
        if (lane == 0 && sing) s.piv = -1;
      }
      __syncthreads();  // block K's columns, P_{K+1} and its G published
    }
  }
  if (s.piv < 0) ok = false;
  if (nxt) {
#pragma unroll
    for (int q = 0; q < C::KE; ++q) {
      const int x = tid + 64 * NW * q;
      if (x < NX * NX) {
        pf[q] = nxt[x];
        pf[C::KE + q] = nxt[NX * NX + x];
      }
    }
  }
  // Y_A = X^{-1} A1, Y_C = X^{-1} C1; a lane reads one row of the A operand,
  // X^{-1} row r = right-half row xrow[r], so its row base is shifted there
#pragma unroll
  for (int t = 0; t < CB; ++t) {
    const int bx = w + NW * t;
    if (bx >= C::NB) break;
    const int I = bx / TX, J = bx % TX, ra = 16 * I + col;
    const float* xa = s.W + NX + (s.xrow[ra] - ra) * LDW;
    f4 ya = cgemm<BF, false, TX>(xa, LDW, s.A1, LDX, I, J, lane);
    f4 yc = cgemm<BF, false, TX>(xa, LDW, s.C1, LDX, I, J, lane);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = arow(I, grp, v), c = 16 * J + col;
      s.YA[r * LDX + c] = ya[v];
      s.YC[r * LDX + c] = yc[v];
    }
  }
  __syncthreads();
  if (pc) {
    // while W still holds X^{-1} (eq. lqr-gpu-combo; X^{-T} = (I + P2 C1)^{-1}):
    //   p = (X^{-1} A1)^T (p2 + P2 c1) + p1,   c = A2 X^{-1} (c1 - C1 p2) + c2
    // one thread per row; rows >= n stay zero (the tiles are zero there and
    // X^{-1} is the identity)
    if (tid < NX) {
      float v1 = s.pv2[tid], v2 = s.cv1[tid];
      for (int j = 0; j < n; ++j) {
        v1 = fmaf(s.P2[tid * LDX + j], s.cv1[j], v1);
        v2 = fmaf(-s.C1[tid * LDX + j], s.pv2[j], v2);
      }
      s.tv[tid] = v1;
      s.tw[tid] = v2;
    }
    __syncthreads();
    float pn = 0.0f, wn = 0.0f;
    if (tid < NX) {
      pn = s.pv1[tid];
      for (int j = 0; j < n; ++j) {
        pn = fmaf(s.YA[j * LDX + tid], s.tv[j], pn);
        wn = fmaf(s.W[s.xrow[tid] * LDW + NX + j], s.tw[j], wn);
      }
    }
    __syncthreads();
    if (tid < NX) {
      s.pv1[tid] = pn;
      s.tv[tid] = wn;  // X^{-1} (c1 - C1 p2)
    }
    __syncthreads();
    float cn = 0.0f;
    if (tid < NX) {
      cn = s.cv2[tid];
      for (int j = 0; j < n; ++j) cn = fmaf(s.A2[tid * LDX + j], s.tv[j], cn);
    }
    __syncthreads();
    if (tid < NX) s.cv1[tid] = cn;
    __syncthreads();
  }
  // T1 = P2 Y_A (into W left half), T2 = Y_C A2^T (into W right half)
#pragma unroll
  for (int t = 0; t < CB; ++t) {
    const int bx = w + NW * t;
    if (bx >= C::NB) break;
    const int I = bx / TX, J = bx % TX;
    f4 t1 = cgemm<BF, false, TX>(s.P2, LDX, s.YA, LDX, I, J, lane);
    f4 t2 = cgemm_bt<BF, TX>(s.YC, LDX, s.A2, LDX, I, J, lane);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = arow(I, grp, v), c = 16 * J + col;
      s.W[r * LDW + c] = t1[v];
      s.W[r * LDW + NX + c] = t2[v];
    }
  }
  __syncthreads();
  // P = A1^T T1 + P1,  A = A2 Y_A,  C = A2 T2 + C2. The new P and C go to the
  // tiles YC and P2, which no product of this phase reads (no barrier before
  // the stores); after one barrier every wavefront symmetrizes its blocks from
  // them (the products keep P and C symmetric only up to rounding) and writes
  // the accumulated element.
  float An[CB][4];
#pragma unroll
  for (int t = 0; t < CB; ++t) {
    const int bx = w + NW * t;
    if (bx >= C::NB) break;
    const int I = bx / TX, J = bx % TX;
    f4 pa = cgemm<BF, true, TX>(s.A1, LDX, s.W, LDW, I, J, lane);
    f4 aa = cgemm<BF, false, TX>(s.A2, LDX, s.YA, LDX, I, J, lane);
    f4 ca = cgemm<BF, false, TX>(s.A2, LDX, s.W + NX, LDW, I, J, lane);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = arow(I, grp, v), c = 16 * J + col;
      s.YC[r * LDX + c] = pa[v] + s.P1[r * LDX + c];
      An[t][v] = aa[v];
      s.P2[r * LDX + c] = ca[v] + C2g[r * NX + c];
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < CB; ++t) {
    const int bx = w + NW * t;
    if (bx >= C::NB) break;
    const int I = bx / TX, J = bx % TX;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = arow(I, grp, v), c = 16 * J + col;
      s.P1[r * LDX + c] = 0.5f * (s.YC[r * LDX + c] + s.YC[c * LDX + r]);
      s.C1[r * LDX + c] = 0.5f * (s.P2[r * LDX + c] + s.P2[c * LDX + r]);
      s.A1[r * LDX + c] = An[t][v];
    }
  }
  __syncthreads();
  return ok;
}

// ------------------------------------------------------------ kernels

// u-elimination (eq. lqr-gpu-init-running) for stage i = blockIdx.x of
// instance insts[blockIdx.y]. With S = [M^T | B^T] (m x 2n) the element is
//     P = Q - M R^{-1} M^T,   A = A - B R^{-1} M^T,   C = delta I + B R^{-1} B^T,
// i.e. the blocks of T - S^T R^{-1} S for T = [[Q, 0], [0, -delta I]]. R is
// swept in float64 (its pivots decide whether the scan can be used: a zero
// pivot marks the instance bad); Y = (-R^{-1}) S and S^T Y are float32 MFMA
// products. Block N holds the terminal element (Q_N, 0, 0).
template <int TX, int TM, int NW>
__global__ __launch_bounds__(64 * NW) void k_scan_init(ScanArgs a) {
  constexpr int NX = 16 * TX, NM = 16 * TM, LDM = NM + 1, LDS2 = 2 * NX + 1;
  constexpr int CR = (TM * TM + NW - 1) / NW;            // R blocks per wavefront
  constexpr int CY = (TM * 2 * TX + NW - 1) / NW;        // Y blocks per wavefront
  constexpr int CW = (3 * TX * TX + NW - 1) / NW;        // output blocks per wavefront
  const int b = a.insts[blockIdx.y];
  const InstMeta mt = a.meta[b];
  const int N = mt.N, n = mt.n, m = mt.m;
  const int i = blockIdx.x;
  if (i > N) return;
  const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63, col = lane & 15,
            grp = lane >> 4;
  float* __restrict__ e = a.elems + (a.eoff[blockIdx.y] + i) * 3 * NX * NX;
  float* __restrict__ epc = a.pc ? a.pce + (a.eoff[blockIdx.y] + i) * 2 * NX : nullptr;
  if (i == N) {  // terminal element (eq. lqr-gpu-init-terminal): (Q_N, q_N, 0, 0, 0)
    const double* QN = a.Q + mt.oQ + (int64_t)N * n * n;
    for (int x = tid; x < NX * NX; x += 64 * NW) {
      const int r = x / NX, c = x % NX;
      e[x] = (r < n && c < n) ? (float)QN[r * n + c] : 0.0f;
      e[NX * NX + x] = 0.0f;
      e[2 * NX * NX + x] = 0.0f;
    }
    if (epc && tid < NX) {
      epc[tid] = tid < n ? (float)a.q[mt.oq + (int64_t)N * n + tid] : 0.0f;
      epc[NX + tid] = 0.0f;
    }
    return;
  }
  const double delta = a.dd ? 0.0 : a.delta[b];
  // per-stage diagonal: C takes Delta_{i+1} (the regularization of the row defining x_{i+1})
  const double* ddn = a.dd ? a.dd + mt.od + (int64_t)(i + 1) * n : nullptr;
  const double* Q = a.Q + mt.oQ + (int64_t)i * n * n;
  const double* M = a.M + mt.oM + (int64_t)i * n * m;
  const double* R = a.R + mt.oR + (int64_t)i * m * m;
  const double* A = a.A + mt.oA + (int64_t)i * n * n;
  const double* B = a.B + mt.oB + (int64_t)i * n * m;
  __shared__ float sRi[NM * LDM];     // -R^{-1}
  __shared__ float sS[NM * LDS2];     // S = [M^T | B^T], columns x at 0.., z at NX..
  __shared__ float sY[NM * LDS2];     // Y = -R^{-1} S
  __shared__ double swbuf[NM * 17 + 2 * 16 * 17];  // blocked sweep: panel, M, swept block
  __shared__ double red[NW];
  // S, zero-padded
  for (int x = tid; x < NM * 2 * NX; x += 64 * NW) {
    const int k = x / (2 * NX), j = x % (2 * NX);
    float v = 0.0f;
    if (k < m) {
      if (j < n) v = (float)M[j * m + k];
      else if (j >= NX && j < NX + n) v = (float)B[(j - NX) * m + k];
    }
    sS[k * LDS2 + j] = v;
  }
  // R in register blocks (rows 16 bi + 4 grp + v), identity-padded, swept in float64
  int ri[CR], rj[CR];
  bool ro[CR];
  double X[CR][4];
#pragma unroll
  for (int t = 0; t < CR; ++t) {
    const int bz = w + NW * t;
    ro[t] = bz < TM * TM;
    ri[t] = ro[t] ? bz / TM : 0;
    rj[t] = ro[t] ? bz % TM : 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * ri[t] + trow<float>(grp, v), c = 16 * rj[t] + col;
      X[t][v] = !ro[t] ? 0.0 : ((r < m && c < m) ? R[r * m + c] : (r == c ? 1.0 : 0.0));
    }
  }
  PivStats ps;
  ps.init();
  {
    const double sc = wg_max<NW>(diag_max<CR, float>(X, ri, rj, ro, 0, m, lane), red, w, lane);
    sweep_blk<float, CR, TM>(X, ri, rj, ro, 0, m, w, lane, swbuf, swbuf + NM * 17, ps, 0,
                             1.0e3 * m * 2.220446049250313e-16 * sc, sc);
  }
  if (ps.nzero && tid == 0) a.bad[b] = 1;
#pragma unroll
  for (int t = 0; t < CR; ++t)
    if (ro[t])
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * ri[t] + trow<float>(grp, v), c = 16 * rj[t] + col;
        sRi[r * LDM + c] = (r < m && c < m) ? (float)X[t][v] : 0.0f;
      }
  __syncthreads();
  if (epc) {
    // carried vectors of the running element: with t = -R^{-1} r_i,
    // p = q_i + M t, c = c_{i+1} + B t
    __shared__ float tvec[NM];
    const double* ri = a.r + mt.or_ + (int64_t)i * m;
    if (tid < NM) {
      float acc = 0.0f;
      for (int k = 0; k < m; ++k) acc = fmaf(sRi[tid * LDM + k], (float)ri[k], acc);
      tvec[tid] = tid < m ? acc : 0.0f;
    }
    __syncthreads();
    if (tid < NX) {
      float pv = 0.0f, cv = 0.0f;
      if (tid < n) {
        double ps = a.q[mt.oq + (int64_t)i * n + tid], cs = a.c[mt.oc + (int64_t)(i + 1) * n + tid];
        for (int k = 0; k < m; ++k) {
          ps += M[tid * m + k] * (double)tvec[k];
          cs += B[tid * m + k] * (double)tvec[k];
        }
        pv = (float)ps;
        cv = (float)cs;
      }
      epc[tid] = pv;
      epc[NX + tid] = cv;
    }
  }
  // Y = (-R^{-1}) S  (TM x 2TX blocks, inner TM)
#pragma unroll
  for (int t = 0; t < CY; ++t) {
    const int by = w + NW * t;
    if (by >= TM * 2 * TX) break;
    const int I = by / (2 * TX), J = by % (2 * TX);
    f4 acc = sgemm_blk<false, TM>(sRi, LDM, sS, LDS2, I, J, lane);
#pragma unroll
    for (int v = 0; v < 4; ++v) sY[arow(I, grp, v) * LDS2 + 16 * J + col] = acc[v];
  }
  __syncthreads();
  // S^T Y = -S^T R^{-1} S: blocks xx (P), zx (A), zz (C)
#pragma unroll
  for (int t = 0; t < CW; ++t) {
    const int bo = w + NW * t;
    if (bo >= 3 * TX * TX) break;
    const int part = bo / (TX * TX), I = (bo % (TX * TX)) / TX, J = bo % TX;
    const int rowblk = part == 0 ? I : TX + I;          // rows of S^T: x (0..) or z (NX..)
    const int colblk = part == 2 ? TX + J : J;          // columns of Y: x or z
    f4 acc = sgemm_blk<true, TM>(sS, LDS2, sY, LDS2, rowblk, colblk, lane);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * I + 4 * grp + v, c = 16 * J + col;
      const bool in = r < n && c < n;
      float val = 0.0f;
      if (part == 0) val = in ? (float)(Q[r * n + c] + (double)acc[v]) : 0.0f;             // P
      else if (part == 1) val = in ? (float)(A[r * n + c] + (double)acc[v]) : 0.0f;        // A
      else val = in ? (float)((r == c ? (ddn ? ddn[r] : delta) : 0.0) - (double)acc[v]) : 0.0f;  // C
      e[part * NX * NX + r * NX + c] = val;
    }
  }
}

// Fold the elements of chunk c = blockIdx.x (elements [c L, min(c L + L, N + 1)))
// into one aggregate, left to right: acc = acc (+) e_next.
template <int TX, int NW, bool BF>
__global__ __launch_bounds__(64 * NW) void k_scan_reduce(ScanArgs a) {
  using C = ScanCfg<TX, NW>;
  extern __shared__ __align__(16) unsigned char smem[];
  ScanLds<TX, NW>& s = *reinterpret_cast<ScanLds<TX, NW>*>(smem);
  const int b = a.insts[blockIdx.y];
  const InstMeta mt = a.meta[b];
  const int N = mt.N, n = mt.n;
  const int c = blockIdx.x, L = mt.chunk;
  const int e0 = c * L, e1 = min(e0 + L, N + 1);
  if (e0 > N) return;
  const float* elems = a.elems + a.eoff[blockIdx.y] * C::ELEM;
  const int tid = threadIdx.x;
  if (tid == 0) s.piv = 0;
  const bool pc = a.pc != 0;
  const float* pce = pc ? a.pce + a.eoff[blockIdx.y] * 2 * C::NX : nullptr;
  load_elem<TX, NW>(s.P1, s.A1, s.C1, elems + (int64_t)e0 * C::ELEM, tid);
  if (pc) load_pc<TX, NW>(s.pv1, s.cv1, pce + (int64_t)e0 * 2 * C::NX, tid);
  if (e0 + 1 < e1) load_elem<TX, NW>(s.P2, s.A2, nullptr, elems + (int64_t)(e0 + 1) * C::ELEM, tid);
  __syncthreads();
  bool ok = true;
  float pf[2 * C::KE];  // P and A of the element after next, read during a combine
  for (int k = e0 + 1; k < e1; ++k) {
    const float* en = elems + (int64_t)k * C::ELEM;
    if (pc) load_pc<TX, NW>(s.pv2, s.cv2, pce + (int64_t)k * 2 * C::NX, tid);
    __syncthreads();
    const bool more = k + 1 < e1;
    ok &= combine<TX, NW, BF>(s, en + 2 * C::NX * C::NX, n, tid, pc, more ? en + C::ELEM : nullptr, pf);
    if (more) {
      // the combine has ended with a barrier: P2 and A2 are free
#pragma unroll
      for (int q = 0; q < C::KE; ++q) {
        const int x = tid + 64 * NW * q;
        if (x < C::NX * C::NX) {
          const int r = x / C::NX, c = x % C::NX;
          s.P2[r * C::LDX + c] = pf[q];
          s.A2[r * C::LDX + c] = pf[C::KE + q];
        }
      }
    }
  }
  store_elem<TX, NW>(a.aggr_out + (a.aoff[blockIdx.y] + c) * C::ELEM, s.P1, s.A1, s.C1, tid);
  if (pc) store_pc<TX, NW>(a.pca_out + (a.aoff[blockIdx.y] + c) * 2 * C::NX, s.pv1, s.cv1, tid);
  if (!ok && tid == 0) a.bad[b] = 1;
}

// One Hillis-Steele level of the reverse scan over chunk aggregates:
// out[c] = in[c] (+) in[c + d] for c + d < NC, else out[c] = in[c].
template <int TX, int NW, bool BF>
__global__ __launch_bounds__(64 * NW) void k_scan_level(ScanArgs a) {
  using C = ScanCfg<TX, NW>;
  extern __shared__ __align__(16) unsigned char smem[];
  ScanLds<TX, NW>& s = *reinterpret_cast<ScanLds<TX, NW>*>(smem);
  const int b = a.insts[blockIdx.y];
  const InstMeta mt = a.meta[b];
  const int n = mt.n;
  const int nch = (mt.N + 1 + mt.chunk - 1) / mt.chunk;
  const int c = blockIdx.x, d = a.dist;
  if (c >= nch) return;
  const float* in = a.aggr_in + a.aoff[blockIdx.y] * C::ELEM;
  float* out = a.aggr_out + a.aoff[blockIdx.y] * C::ELEM;
  const int tid = threadIdx.x;
  if (tid == 0) s.piv = 0;
  const bool pc = a.pc != 0;
  const float* pin = pc ? a.pca_in + a.aoff[blockIdx.y] * 2 * C::NX : nullptr;
  load_elem<TX, NW>(s.P1, s.A1, s.C1, in + (int64_t)c * C::ELEM, tid);
  if (pc) load_pc<TX, NW>(s.pv1, s.cv1, pin + (int64_t)c * 2 * C::NX, tid);
  __syncthreads();
  if (c + d < nch) {
    const float* en = in + (int64_t)(c + d) * C::ELEM;
    load_elem<TX, NW>(s.P2, s.A2, nullptr, en, tid);
    if (pc) load_pc<TX, NW>(s.pv2, s.cv2, pin + (int64_t)(c + d) * 2 * C::NX, tid);
    __syncthreads();
    float pf[2 * C::KE];
    if (!combine<TX, NW, BF>(s, en + 2 * C::NX * C::NX, n, tid, pc, nullptr, pf) && tid == 0) a.bad[b] = 1;
  }
  store_elem<TX, NW>(out + (int64_t)c * C::ELEM, s.P1, s.A1, s.C1, tid);
  if (pc) store_pc<TX, NW>(a.pca_out + a.aoff[blockIdx.y] * 2 * C::NX + (int64_t)c * 2 * C::NX, s.pv1, s.cv1, tid);
}

// Carried p: the suffix aggregate of chunk s is e_{lo(s) -> N+1}, whose p is
// p_{lo(s)}; write it (float64) into segment s's boundary vector for s >= 1.
template <int TX>
__global__ __launch_bounds__(256) void k_scan_pc_boundary(ScanArgs a, double* __restrict__ plo) {
  constexpr int NX = 16 * TX;
  const int b = a.insts[blockIdx.x];
  const InstMeta mt = a.meta[b];
  if (mt.nseg <= 1) return;
  const float* __restrict__ res = a.pca_in + a.aoff[blockIdx.x] * 2 * NX;
  const int64_t cnt = (int64_t)(mt.nseg - 1) * mt.n;  // segments 1 .. nseg-1, n entries each
  for (int64_t x = threadIdx.x; x < cnt; x += 256) {
    const int64_t s = 1 + x / mt.n, j = x % mt.n;
    plo[mt.ovec + s * mt.n + j] = (double)res[s * 2 * NX + j];
  }
}

template <int TX, int NW>
static size_t scan_lds_bytes() { return sizeof(ScanLds<TX, NW>); }

template <int TX, int TM, int NW>
static hipError_t launch_scan_init_t(const ScanArgs& a, int ninst, hipStream_t st) {
  hipLaunchKernelGGL((k_scan_init<TX, TM, NW>), dim3(a.maxN + 1, ninst), dim3(64 * NW), 0, st, a);
  return hipGetLastError();
}

// The tree kernels use more than 64 KB of dynamic LDS; the limit is raised
// once (scan_prepare, at handle creation) so that no launch path makes a
// non-stream call (a launch sequence may be captured into a graph).
template <int TX, int NW, bool BF>
static hipError_t scan_prepare_t() {
  const size_t lds = scan_lds_bytes<TX, NW>();
  hipError_t e = hipFuncSetAttribute((const void*)k_scan_reduce<TX, NW, BF>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)k_scan_level<TX, NW, BF>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lds);
}

hipError_t scan_prepare() {
  hipError_t e = scan_prepare_t<1, 4, false>();
  if (e == hipSuccess) e = scan_prepare_t<2, 4, false>();
  if (e == hipSuccess) e = scan_prepare_t<4, 16, false>();
  if (e == hipSuccess) e = scan_prepare_t<1, 4, true>();
  if (e == hipSuccess) e = scan_prepare_t<2, 4, true>();
  if (e == hipSuccess) e = scan_prepare_t<4, 16, true>();
  return e;
}

template <int TX, int NW, bool BF>
static hipError_t launch_scan_tree_t(ScanArgs a, int ninst, hipStream_t st) {
  const size_t lds = scan_lds_bytes<TX, NW>();
  hipError_t e;
  a.aggr_out = a.aggr[0];
  a.pca_out = a.pca[0];
  hipLaunchKernelGGL((k_scan_reduce<TX, NW, BF>), dim3(a.maxchunks, ninst), dim3(64 * NW), lds, st, a);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  int cur = 0;
  for (int d = 1; d < a.maxchunks; d *= 2) {
    a.aggr_in = a.aggr[cur];
    a.aggr_out = a.aggr[cur ^ 1];
    a.pca_in = a.pca[cur];
    a.pca_out = a.pca[cur ^ 1];
    a.dist = d;
    hipLaunchKernelGGL((k_scan_level<TX, NW, BF>), dim3(a.maxchunks, ninst), dim3(64 * NW), lds, st, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    cur ^= 1;
  }
  return hipSuccess;
}

// Dispatch on the state tile size (tx = NX / 16) and the control tile count
// tm = ceil(m / 16): n <= 16 allows m <= 95, n <= 32 allows m <= 79, n <= 64 allows m <= 63.
hipError_t launch_scan_elements(const ScanArgs& a, int ninst, int tx, int tm, hipStream_t st) {
  if (ninst <= 0) return hipSuccess;
  if (ninst > 65535) return hipErrorInvalidValue;  // grid y limit
  if (tx == 1) {
    if (tm <= 1) return launch_scan_init_t<1, 1, 4>(a, ninst, st);
    if (tm <= 2) return launch_scan_init_t<1, 2, 4>(a, ninst, st);
    if (tm <= 6) return launch_scan_init_t<1, 6, 8>(a, ninst, st);
  } else if (tx == 2) {
    if (tm <= 1) return launch_scan_init_t<2, 1, 8>(a, ninst, st);
    if (tm <= 2) return launch_scan_init_t<2, 2, 8>(a, ninst, st);
    if (tm <= 5) return launch_scan_init_t<2, 5, 8>(a, ninst, st);
  } else if (tx == 4) {
    if (tm <= 1) return launch_scan_init_t<4, 1, 8>(a, ninst, st);
    if (tm <= 2) return launch_scan_init_t<4, 2, 8>(a, ninst, st);
    if (tm <= 4) return launch_scan_init_t<4, 4, 16>(a, ninst, st);
  }
  return hipErrorInvalidValue;
}

// the ping-pong buffer holding the finished suffix scan
int scan_result_buffer(int maxchunks) {
  int cur = 0;
  for (int d = 1; d < maxchunks; d *= 2) cur ^= 1;
  return cur;
}

hipError_t launch_scan_tree(const ScanArgs& a, int ninst, int tx, bool bf16, hipStream_t st) {
  if (ninst <= 0) return hipSuccess;
  if (ninst > 65535) return hipErrorInvalidValue;  // grid y limit
  if (bf16) {
    if (tx == 1) return launch_scan_tree_t<1, 4, true>(a, ninst, st);
    if (tx == 2) return launch_scan_tree_t<2, 4, true>(a, ninst, st);
    if (tx == 4) return launch_scan_tree_t<4, 16, true>(a, ninst, st);
  } else {
    if (tx == 1) return launch_scan_tree_t<1, 4, false>(a, ninst, st);
    if (tx == 2) return launch_scan_tree_t<2, 4, false>(a, ninst, st);
    if (tx == 4) return launch_scan_tree_t<4, 16, false>(a, ninst, st);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_scan_pc_boundary(const ScanArgs& a, int ninst, int tx, double* plo, hipStream_t st) {
  if (ninst <= 0) return hipSuccess;
  if (!plo || !a.pca_in) return hipErrorInvalidValue;
  if (tx == 1) hipLaunchKernelGGL(k_scan_pc_boundary<1>, dim3(ninst), dim3(256), 0, st, a, plo);
  else if (tx == 2) hipLaunchKernelGGL(k_scan_pc_boundary<2>, dim3(ninst), dim3(256), 0, st, a, plo);
  else if (tx == 4) hipLaunchKernelGGL(k_scan_pc_boundary<4>, dim3(ninst), dim3(256), 0, st, a, plo);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

// ------------------------------------------------------------ segment transfer

// Psi = F_{hi-1} ... F_lo for the segment [lo, hi) of blockIdx.x, with
// F_k = S_hat_{k+1}^{-1} (A_k + B_k K_k) taken from the float32 factor tiles
// (Z_k holds -K_k in its (u, x) block, X_{k+1} holds -S_hat_{k+1}^{-1}; with a
// per-stage diagonal X~ = D X D, and F_k = (I + Delta P)^{-1}(A + B K) takes
// X~ Delta^{-1} in place of X).
// Per stage: V = [Psi; K Psi], T = [A B] V, Psi <- -X T, float32 MFMA.
// The last segment of an instance is skipped: no boundary chain uses it.
template <int TX, int TZ, int NW>
__global__ __launch_bounds__(64 * NW) void k_transfer(TransferArgs a) {
  constexpr int NX = 16 * TX, NZ = 16 * TZ, LX = NX + 1, LZ = NZ + 1;
  constexpr int CB = (TX * TX + NW - 1) / NW, CV = (TZ * TX + NW - 1) / NW;
  constexpr int STAGE = (TZ * TZ + TX * TX) * 256;
  const SegDesc sd = a.segs[blockIdx.x];
  const InstMeta mt = a.meta[sd.inst];
  const int N = mt.N, n = mt.n, m = mt.m;
  if (sd.hi >= N) return;
  const float* __restrict__ ws = reinterpret_cast<const float*>(a.ws) + mt.ows;
  const double* __restrict__ Ag = a.A + mt.oA;
  const double* __restrict__ Bg = a.B + mt.oB;
  __shared__ float sPsi[NX * LX], sX[NX * LX], sT[NX * LX];
  __shared__ float sK[NZ * LX], sV[NZ * LX];
  __shared__ float sAB[NX * LZ];
  const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63, col = lane & 15,
            grp = lane >> 4;
  for (int x = tid; x < NX * LX; x += 64 * NW) {
    const int r = x / LX, c = x % LX;
    sPsi[x] = (r == c && r < n) ? 1.0f : 0.0f;
  }
  for (int x = tid; x < NZ * LX; x += 64 * NW) sK[x] = 0.0f;
  for (int x = tid; x < NX * LZ; x += 64 * NW) sAB[x] = 0.0f;
  // A stage's operands are read into registers (this thread's share) while
  // the previous stage's products run, and written to LDS after them:
  // K_k = -(Z_k)_ux from the (u, x) entries of the stage tile, X_{k+1}
  // (scaled by the stage diagonal when there is one), [A_k B_k].
  constexpr int KZ = (TZ * TZ * 256 + 64 * NW - 1) / (64 * NW);
  constexpr int KX = (TX * TX * 256 + 64 * NW - 1) / (64 * NW);
  constexpr int KAB = (NX * NZ + 64 * NW - 1) / (64 * NW);
  float rz[KZ], rx[KX];
  double rd[KX], rab[KAB];
  auto fetch = [&](int k) {
    const float* zt = ws + (int64_t)k * STAGE;
#pragma unroll
    for (int q = 0; q < KZ; ++q) {
      const int x = tid + 64 * NW * q, bz = x >> 8, e = x & 255, v = e >> 6, l = e & 63;
      int I = 0, J = 0;
      if (x < TZ * TZ * 256) zmap<TX, TZ>(bz, I, J);
      const int r = 16 * I + 4 * (l >> 4) + v, c = 16 * J + (l & 15);
      rz[q] = (x < TZ * TZ * 256 && r >= n && r < n + m && c < n) ? zt[x] : 0.0f;
    }
    const float* xt = ws + (int64_t)(k + 1) * STAGE + TZ * TZ * 256;
    const double* dn = a.dd ? a.dd + mt.od + (int64_t)(k + 1) * n : nullptr;
#pragma unroll
    for (int q = 0; q < KX; ++q) {
      const int x = tid + 64 * NW * q, bx = x >> 8, e = x & 255, v = e >> 6, l = e & 63;
      const int r = 16 * (bx / TX) + 4 * (l >> 4) + v, c = 16 * (bx % TX) + (l & 15);
      const bool in = x < TX * TX * 256 && r < n && c < n;
      rx[q] = in ? xt[x] : 0.0f;
      rd[q] = in && dn ? dn[c] : 1.0;
    }
    const double* A = Ag + (int64_t)k * n * n;
    const double* B = Bg + (int64_t)k * n * m;
#pragma unroll
    for (int q = 0; q < KAB; ++q) {
      const int x = tid + 64 * NW * q, r = x / (n + m), c = x % (n + m);
      rab[q] = x < n * (n + m) ? (c < n ? A[r * n + c] : B[r * m + (c - n)]) : 0.0;
    }
  };
  auto store = [&]() {
#pragma unroll
    for (int q = 0; q < KZ; ++q) {
      const int x = tid + 64 * NW * q, bz = x >> 8, e = x & 255, v = e >> 6, l = e & 63;
      int I = 0, J = 0;
      if (x < TZ * TZ * 256) zmap<TX, TZ>(bz, I, J);
      const int r = 16 * I + 4 * (l >> 4) + v, c = 16 * J + (l & 15);
      if (x < TZ * TZ * 256 && r >= n && r < n + m && c < n) sK[r * LX + c] = -rz[q];
    }
#pragma unroll
    for (int q = 0; q < KX; ++q) {
      const int x = tid + 64 * NW * q, bx = x >> 8, e = x & 255, v = e >> 6, l = e & 63;
      const int r = 16 * (bx / TX) + 4 * (l >> 4) + v, c = 16 * (bx % TX) + (l & 15);
      if (x < TX * TX * 256) sX[r * LX + c] = a.dd ? (float)((double)rx[q] / rd[q]) : rx[q];
    }
#pragma unroll
    for (int q = 0; q < KAB; ++q) {
      const int x = tid + 64 * NW * q, r = x / (n + m), c = x % (n + m);
      if (x < n * (n + m)) sAB[r * LZ + c] = (float)rab[q];
    }
  };
  __syncthreads();  // the zero fills are done before any operand lands
  fetch(sd.lo);
  store();
  for (int k = sd.lo; k < sd.hi; ++k) {
    __syncthreads();  // stage k's operands in LDS
    if (k + 1 < sd.hi) fetch(k + 1);
    // V = K Psi (rows n .. n+m-1) + Psi (rows < n)
#pragma unroll
    for (int t = 0; t < CV; ++t) {
      const int bv = w + NW * t;
      if (bv >= TZ * TX) break;
      const int I = bv / TX, J = bv % TX;
      f4 acc = sgemm_blk<false, TX>(sK, LX, sPsi, LX, I, J, lane);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = arow(I, grp, v), c = 16 * J + col;
        sV[r * LX + c] = acc[v] + (r < NX ? sPsi[r * LX + c] : 0.0f);
      }
    }
    __syncthreads();
    // T = [A B] V
#pragma unroll
    for (int t = 0; t < CB; ++t) {
      const int bx = w + NW * t;
      if (bx >= TX * TX) break;
      const int I = bx / TX, J = bx % TX;
      f4 acc = sgemm_blk<false, TZ>(sAB, LZ, sV, LX, I, J, lane);
#pragma unroll
      for (int v = 0; v < 4; ++v) sT[arow(I, grp, v) * LX + 16 * J + col] = acc[v];
    }
    __syncthreads();
    // Psi = -X T
#pragma unroll
    for (int t = 0; t < CB; ++t) {
      const int bx = w + NW * t;
      if (bx >= TX * TX) break;
      const int I = bx / TX, J = bx % TX;
      f4 acc = sgemm_blk<false, TX>(sX, LX, sT, LX, I, J, lane);
#pragma unroll
      for (int v = 0; v < 4; ++v) sPsi[arow(I, grp, v) * LX + 16 * J + col] = -acc[v];
    }
    __syncthreads();
    if (k + 1 < sd.hi) store();  // every reader of sK, sX, sAB has passed the barrier
  }
  double* out = a.psi + mt.opsi + (int64_t)sd.s * 2 * n * n;
  for (int x = tid; x < n * n; x += 64 * NW) {
    const int r = x / n, c = x % n;
    out[x] = (double)sPsi[r * LX + c];
    out[n * n + c * n + r] = (double)sPsi[r * LX + c];
  }
}

template <int TX, int TZ, int NW>
static hipError_t launch_transfer_t(const TransferArgs& a, int nblocks, hipStream_t st) {
  hipLaunchKernelGGL((k_transfer<TX, TZ, NW>), dim3(nblocks), dim3(64 * NW), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_transfer(int cls, const TransferArgs& a, int nblocks, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  switch (cls) {
    case TILE_16: return launch_transfer_t<1, 1, 1>(a, nblocks, st);
    case TILE_X1_Z2: return launch_transfer_t<1, 2, 2>(a, nblocks, st);
    case TILE_X2_Z2: return launch_transfer_t<2, 2, 4>(a, nblocks, st);
    case TILE_X2_Z3: return launch_transfer_t<2, 3, 4>(a, nblocks, st);
    case TILE_X3_Z3: return launch_transfer_t<3, 3, 9>(a, nblocks, st);
    case TILE_X4_Z4: return launch_transfer_t<4, 4, 16>(a, nblocks, st);
    case TILE_X4_Z6: return launch_transfer_t<4, 6, 16>(a, nblocks, st);
  }
  return hipErrorInvalidValue;
}

// Boundary chain of one instance (blockIdx.x indexes the list). Backward:
// p_lo(s) += Psi_s^T p_lo(s+1) for s = S-2 .. 0 (p_lo(S-1) is exact: it starts
// from q_N). Forward: xhi(s) += Psi_s xhi(s-1) for s = 1 .. S-2 (xhi(0) is
// exact: it starts from x_0). Thread (i, q) = (t & 63, t >> 6) forms the
// partial sum of entry i over columns 16q .. 16q+15; the four partials are
// added in order (deterministic). The matrix entries of the next step are
// loaded into registers while the current step is reduced, so the dependent
// chain does not wait on memory.
__global__ __launch_bounds__(256) void k_chain(ChainArgs a) {
  const int b = a.insts[blockIdx.x];
  if (a.run && !a.run[b]) return;
  const InstMeta mt = a.meta[b];
  const int n = mt.n, S = mt.nseg;
  if (S < (a.forward ? 3 : 2)) return;  // forward: s = 1 .. S-2; backward: s = S-2 .. 0
  __shared__ double sv[64], part[4][64];
  const int t = threadIdx.x, i = t & 63, q = t >> 6;
  double* vec = a.vec + mt.ovec;
  const int64_t n2 = (int64_t)n * n;
  // column block of this thread: j = 16 q + jj < n
  const int j0 = 16 * q;
  const bool row_ok = i < n;
  const int fwd = a.forward;
  // matrix of step s: backward uses Psi_s (entry [j][i] at j n + i), forward Psi_s^T (same index)
  auto mat = [&](int s2) { return a.psi + mt.opsi + (int64_t)s2 * 2 * n2 + (fwd ? n2 : 0); };
  const int s_first = fwd ? 1 : S - 2, s_last = fwd ? S - 2 : 0, ds = fwd ? 1 : -1;
  if (t < 64) sv[t] = (t < n) ? vec[(int64_t)(fwd ? 0 : S - 1) * n + t] : 0.0;
  double pv[16];
  {
    const double* P = mat(s_first);
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) {
      const int j = j0 + jj;
      pv[jj] = (row_ok && j < n) ? P[(int64_t)j * n + i] : 0.0;
    }
  }
  __syncthreads();
  for (int s2 = s_first;; s2 += ds) {
    double acc = 0.0;
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) acc = fma(pv[jj], sv[j0 + jj], acc);
    const bool more = s2 != s_last;
    const double own = (q == 0 && row_ok) ? vec[(int64_t)s2 * n + i] : 0.0;
    if (more) {
      const double* P = mat(s2 + ds);
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        const int j = j0 + jj;
        pv[jj] = (row_ok && j < n) ? P[(int64_t)j * n + i] : 0.0;
      }
    }
    part[q][i] = acc;
    __syncthreads();
    if (q == 0) {
      const double v = own + ((part[0][i] + part[1][i]) + (part[2][i] + part[3][i]));
      if (row_ok) vec[(int64_t)s2 * n + i] = v;
      sv[i] = row_ok ? v : 0.0;
    }
    __syncthreads();
    if (!more) break;
  }
}

hipError_t launch_chain(const ChainArgs& a, int ninst, hipStream_t st) {
  if (ninst <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_chain, dim3(ninst), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace rlqr
