// rlqr_kernels.hip -- gfx950 kernels of the dual-regularized Riccati solver.
//
// Factor: the backward recursion of Section "Sequential Algorithm"
// (arXiv 2509.16370), one wavefront per instance, 16 x 16 tiles. Per stage k:
//   X   = I + delta P_{k+1}                 sweep all n pivots -> X = -S_hat^{-1}
//   W   = -P_{k+1} X = P S_hat^{-1}         MFMA (symmetric to rounding; Z's
//                                           symmetrization below covers it)
//   T   = W [A_k B_k]                       MFMA
//   Z   = [A_k B_k]^T T + [[Q_k, M_k], [M_k^T, R_k]]   MFMA, symmetrized
//       = [[A^T W A + Q, H^T], [H, G]]      (G = R + B^T W B, H = B^T W A + M^T)
//   sweep the u-block pivots of Z -> Z = [[P_k, -K_k^T], [-K_k, -G_k^{-1}]]
// The two swept tiles per stage are the whole factorization handed to the
// solve. Pivot signs feed the certificate of Theorem
// "riccati-inertia-certification-theorem".
//
// Solve: backward vector pass and forward rollout of Theorem
// "main-seq-theorem" using only the swept tiles and [A_k B_k]:
//   v = p_{k+1} + P_{k+1} c_{k+1};  g = S_hat_{k+1}^{-1} v  (= the paper's g_{k+1})
//   h = r_k + B_k^T g;  k_k = -G_k^{-1} h;  p_k = q_k + A_k^T g + K_k^T h
//   x_0 = S_hat_0^{-1}(c_0 - delta p_0);  u_k = K_k x_k + k_k;  y_k = P_k x_k + p_k
//   x_{k+1} = S_hat_{k+1}^{-1}(A_k x_k + B_k u_k + c_{k+1} - delta p_{k+1})
// (g = p + W(c - delta p) equals S_hat^{-1}(p + P c) because
//  I - delta W = S_hat^{-1} and W = P S_hat^{-1}; K^T h = H^T k.)
//
// Residual: float64 residual blocks of Section "Residual Computation".
#include "rlqr_device.h"
#include "rlqr_internal.h"

namespace rlqr {

// ------------------------------------------------------------------ helpers

template <typename TL, typename T>
__device__ __forceinline__ void tile_to_lds(T* s, const double (&X)[4], int lane) {
  const int col = lane & 15, grp = lane >> 4;
#pragma unroll
  for (int v = 0; v < 4; ++v) s[trow<TL>(grp, v) * LD + col] = (T)X[v];
}

template <typename T, typename A>
__device__ __forceinline__ void acc_to_regs(double (&X)[4], const A& acc, double scale) {
#pragma unroll
  for (int v = 0; v < 4; ++v) X[v] = scale * (double)acc[v];
}

// Global tile storage: element v of lane l at index v * 64 + l (coalesced).
template <typename T>
__device__ __forceinline__ void tile_store(T* __restrict__ g, const double (&X)[4], int lane) {
#pragma unroll
  for (int v = 0; v < 4; ++v) g[v * 64 + lane] = (T)X[v];
}
template <typename T>
__device__ __forceinline__ void tile_load(double (&X)[4], const T* __restrict__ g, int lane) {
#pragma unroll
  for (int v = 0; v < 4; ++v) X[v] = (double)g[v * 64 + lane];
}

// Tile layout of the one-wavefront class. Full (float32 tiles): two
// 256-element tiles per stage (Z_i at 2i, X_i at 2i+1), element v of lane l
// at v * 64 + l. Compact (float64 tiles): Z_i and X_i are exactly symmetric
// (the sweep and the symmetrization keep them so), so only the upper
// triangle of the leading s x s block of Z_i (s = n + m) and of the leading
// n x n block of X_i (= -S_hat_i^{-1}) is stored, row by row; stage i
// occupies cs = s(s+1)/2 + n(n+1)/2 elements from i * cs. Entries outside
// those blocks read as zero (the solve never uses them): 1,712 bytes per
// stage at n = 12, m = 4 instead of 4,096, and the float64 solve pass runs
// 18 % faster. Float32 tiles keep the full layout: there the element gathers
// of the compact layout cost more in the correction pass than the bytes they
// save. The scan's segment kernels read float32 tiles only.
template <bool CP>
struct TileLayout {
  int s, n, zs, cs;
  __device__ __forceinline__ TileLayout(int n_, int m_)
      : s(n_ + m_), n(n_), zs((n_ + m_) * (n_ + m_ + 1) / 2), cs((n_ + m_) * (n_ + m_ + 1) / 2 + n_ * (n_ + 1) / 2) {}
  __device__ __forceinline__ int64_t z(int i) const { return CP ? (int64_t)i * cs : (int64_t)(2 * i) * 256; }
  __device__ __forceinline__ int64_t x(int i) const { return CP ? (int64_t)i * cs + zs : (int64_t)(2 * i + 1) * 256; }
};

// index of (r, c), r <= c < d, in the row-by-row upper triangle of a d x d block
__device__ __forceinline__ int tri_index(int r, int c, int d) { return r * d - ((r * (r - 1)) >> 1) + (c - r); }

template <typename TG, bool CP, typename T>
__device__ __forceinline__ void tile_store_as(T* __restrict__ g, const double (&X)[4], int lane, int d) {
  if constexpr (!CP) {
    tile_store(g, X, lane);
  } else {
  const int col = lane & 15, grp = lane >> 4;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = trow<TG>(grp, v);
    if (r <= col && col < d) g[tri_index(r, col, d)] = (T)X[v];
  }
  }
}
// The lane's four element indices in the compact triangle of a d x d block,
// 8 bits each; 255 marks an element outside the block. Index 255 from any
// tile start stays inside the instance's workspace (sized for the full
// layout), so the load is issued unconditionally and its value dropped.
template <typename TG>
__device__ __forceinline__ uint32_t tri_pack(int lane, int d) {
  const int col = lane & 15, grp = lane >> 4;
  uint32_t p = 0;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = trow<TG>(grp, v);
    const uint32_t i = (r < d && col < d) ? (uint32_t)tri_index(min(r, col), max(r, col), d) : 255u;
    p |= i << (8 * v);
  }
  return p;
}
template <bool CP, typename T>
__device__ __forceinline__ void tile_load_pk(double (&X)[4], const T* __restrict__ g, int lane, uint32_t pk) {
  if constexpr (!CP) {
    tile_load(X, g, lane);
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const uint32_t i = (pk >> (8 * v)) & 255u;
      const T x = g[i];
      X[v] = i != 255u ? (double)x : 0.0;
    }
  }
}
template <typename TG, bool CP, typename T>
__device__ __forceinline__ void tile_load_as(double (&X)[4], const T* __restrict__ g, int lane, int d) {
  if constexpr (!CP) {
    tile_load(X, g, lane);
  } else {
  const int col = lane & 15, grp = lane >> 4;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = trow<TG>(grp, v);
    const bool in = r < d && col < d;
    const T x = g[in ? tri_index(min(r, col), max(r, col), d) : 0];
    X[v] = in ? (double)x : 0.0;
  }
  }
}

// Stage blocks. Loads are branch-free: every lane loads through a pointer
// that is always valid (the block base when the element is padding) and then
// selects, so the compiler issues all loads back to back and waits only at
// the first use.
//
// [A B] tile element (i, j) of the n x (n+m) block, zero outside.
__device__ __forceinline__ double ab_elem(const double* __restrict__ A, const double* __restrict__ B,
                                          int n, int m, int i, int j) {
  const bool inA = i < n && j < n, inB = i < n && j >= n && j < n + m;
  const double* pa = A + (inA ? i * n + j : 0);
  const double* pb = B + (inB ? i * m + (j - n) : 0);
  const double* p = inB ? pb : pa;
  const double v = *p;
  return (inA || inB) ? v : 0.0;
}

// [A B] tile element e = lane + 64 t (row e>>4, column e&15).
__device__ __forceinline__ void load_ab_rowmajor(double (&o)[4], const double* __restrict__ A,
                                                 const double* __restrict__ B, int n, int m, int lane) {
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int e = lane + 64 * t;
    o[t] = ab_elem(A, B, n, m, e >> 4, e & 15);
  }
}

// Hessian block [[Q, M], [M^T, R]] element (r, c), zero outside (n+m) x (n+m).
__device__ __forceinline__ double hess_elem(const double* __restrict__ Q, const double* __restrict__ M,
                                            const double* __restrict__ R, int n, int m, int r, int c) {
  const bool rx = r < n, ru = r >= n && r < n + m, cx = c < n, cu = c >= n && c < n + m;
  // one offset per array, then a select between the three arrays
  const int oq = (rx && cx) ? r * n + c : 0;
  const int om = (rx && cu) ? r * m + (c - n) : ((ru && cx) ? c * m + (r - n) : 0);
  const int orr = (ru && cu) ? (r - n) * m + (c - n) : 0;
  const bool useM = (rx && cu) || (ru && cx), useR = ru && cu;
  const double* p = useR ? R + orr : (useM ? M + om : Q + oq);
  const double v = *p;
  return ((rx || ru) && (cx || cu)) ? v : 0.0;
}

// Hessian block in the accumulator layout.
template <typename TL>
__device__ __forceinline__ void load_hess(double (&o)[4], const double* __restrict__ Q,
                                          const double* __restrict__ M, const double* __restrict__ R,
                                          int n, int m, int lane) {
  const int c = lane & 15, grp = lane >> 4;
#pragma unroll
  for (int v = 0; v < 4; ++v) o[v] = hess_elem(Q, M, R, n, m, trow<TL>(grp, v), c);
}

// max |diag| over pivots lo..hi-1 of a register tile (wave-uniform result).
template <typename TL>
__device__ __forceinline__ double diag_scale(const double (&X)[4], int lo, int hi, int lane) {
  (void)lane;
  double s = 0.0;
#define RLQR_DIAG(J) \
  if (J >= lo && J < hi) s = fmax(s, fabs(tile_diag<TL, J>(X)));
  RLQR_DIAG(0) RLQR_DIAG(1) RLQR_DIAG(2) RLQR_DIAG(3) RLQR_DIAG(4) RLQR_DIAG(5) RLQR_DIAG(6) RLQR_DIAG(7)
  RLQR_DIAG(8) RLQR_DIAG(9) RLQR_DIAG(10) RLQR_DIAG(11) RLQR_DIAG(12) RLQR_DIAG(13) RLQR_DIAG(14) RLQR_DIAG(15)
#undef RLQR_DIAG
  return s;
}

// ------------------------------------------------------------------ tile-vector helpers

// y[c] = sum_r Tile[r][c] * vec[r] for the register tile (rows trow<TL>),
// vec in LDS; result replicated over the four lane groups.
template <typename TL>
__device__ __forceinline__ double tmatvec(const double (&X)[4], const double* vec, int lane) {
  const int grp = lane >> 4;
  double s = 0.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) s += X[v] * vec[trow<TL>(grp, v)];
  return group_sum(s);
}

// tmatvec of the tile as stored (each element rounded to TL first)
template <typename TL>
__device__ __forceinline__ double tmatvec_r(const double (&X)[4], const double* vec, int lane) {
  const int grp = lane >> 4;
  double s = 0.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) s += (double)(TL)X[v] * vec[trow<TL>(grp, v)];
  return group_sum(s);
}

// masked vector element load: v[i] if ok else 0. A masked-off lane reads the
// zero below instead (an empty block may sit at the end of an array); no
// select follows the load, so the compiler waits for it only at its first use.
__device__ double g_zero = 0.0;
__device__ __forceinline__ double ld_or0(const double* __restrict__ v, int64_t i, bool ok) {
  const double* p = ok ? v + i : &g_zero;
  return *p;
}

// ------------------------------------------------------------------ factor

// One step k of the backward vector pass (Theorem "main-seq-theorem"):
//   g = S_hat_{k+1}^{-1} (p_{k+1} + P_{k+1} c_{k+1}),  h = r_k + B_k^T g,
//   k_k = -G_k^{-1} h,  p_k = q_k + A_k^T g + K_k^T h
// from the tiles Zp = Z_{k+1} (P_{k+1}), Xn = X_{k+1} = -S_hat_{k+1}^{-1},
// Zk = Z_k and ab = [A_k B_k] (all in the register layout trow<TG>); p holds
// p_{k+1} on entry and p_k on exit (x lanes), the return value is k_k (u lanes).
// DG (diagonal Delta_{k+1}): the stored tile is X~ = -D S_hat^{-1} D (S_hat = I +
// D P D, D = Delta^{1/2}), so g = (I + P Delta)^{-1} v = -Delta^{-1} X~ v; id is
// 1 / Delta's entry of the lane's column.
template <typename TG, bool DG = false>
__device__ __forceinline__ double bwd_vec_step(const double (&Zp)[4], const double (&Xn)[4], const double (&ab)[4],
                                               const double (&Zk)[4], double& p, double ck, double qk, double rk,
                                               double (*sv)[16], bool xr, bool ur, bool own, int col, int lane,
                                               double id = 1.0) {
  wave_sync();
  if (own) sv[0][col] = ck;
  wave_sync();
  const double vv = xr ? p + tmatvec<TG>(Zp, sv[0], lane) : 0.0;  // p + P_{k+1} c_{k+1}
  if (own) sv[1][col] = vv;
  wave_sync();
  const double g = DG ? -id * tmatvec<TG>(Xn, sv[1], lane)         // -Delta^{-1} X~ v
                      : -tmatvec<TG>(Xn, sv[1], lane);             // S_hat^{-1} v
  if (own) sv[0][col] = xr ? g : 0.0;
  wave_sync();
  const double abg = tmatvec<TG>(ab, sv[0], lane);                 // [A^T g; B^T g]
  const double h = ur ? rk + abg : 0.0;
  if (own) sv[1][col] = h;
  wave_sync();
  const double zh = tmatvec<TG>(Zk, sv[1], lane);                  // [-K^T h; -G^{-1} h]
  p = xr ? qk + abg - zh : 0.0;
  return zh;
}

// Raw stage blocks [Q_k | M_k | R_k | A_k | B_k | 0] staged in LDS by direct
// global-to-LDS copies (no registers hold the data in flight). STG_MAX covers
// n + m <= 16 (2n^2 + 2nm + m^2 <= 512) plus the zero cell.
constexpr int STG_MAX = 520;
typedef __attribute__((address_space(1))) const void gvoid_t;
typedef __attribute__((address_space(3))) void lvoid_t;

// Copy L doubles from global src to LDS dst, 64 dwords per instruction.
__device__ __forceinline__ void dma_block(const double* src, double* dst, int L, int lane) {
  const int dw = 2 * L;
  for (int j = 0; j < dw; j += 64)
    if (j + lane < dw)
      __builtin_amdgcn_global_load_lds((gvoid_t*)(reinterpret_cast<const char*>(src) + 4 * (j + lane)),
                                       (lvoid_t*)(reinterpret_cast<char*>(dst) + 4 * j), 4, 0, 0);
}

__device__ __forceinline__ void dma_stage(double* stg, const double* Q, const double* M, const double* R,
                                          const double* A, const double* B, int n, int m, int lane) {
  const int nn = n * n, nm = n * m, mm = m * m;
  dma_block(Q, stg, nn, lane);
  dma_block(M, stg + nn, nm, lane);
  dma_block(R, stg + nn + nm, mm, lane);
  dma_block(A, stg + nn + nm + mm, nn, lane);
  dma_block(B, stg + 2 * nn + nm + mm, nm, lane);
}

__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0f70); }  // vmcnt(0)

// staging index of [A B][i][j] (zero cell outside the n x (n+m) block)
__device__ __forceinline__ int stg_ab(int i, int j, int n, int m) {
  const int oA = n * n + n * m + m * m, oB = oA + n * n, oZ = oB + n * m;
  return (i < n && j < n) ? oA + i * n + j : ((i < n && j < n + m) ? oB + i * m + (j - n) : oZ);
}
// staging index of the Hessian [[Q, M], [M^T, R]][r][c]
__device__ __forceinline__ int stg_hess(int r, int c, int n, int m) {
  const int nn = n * n, nm = n * m, oZ = 2 * nn + 2 * nm + m * m;
  const bool rx = r < n, ru = r >= n && r < n + m, cx = c < n, cu = c >= n && c < n + m;
  return (rx && cx) ? r * n + c
       : (rx && cu) ? nn + r * m + (c - n)
       : (ru && cx) ? nn + c * m + (r - n)
       : (ru && cu) ? nn + nm + (r - n) * m + (c - n) : oZ;
}

// T = W [A B] (op A from LDS tile, op B from the staged blocks) and
// Z = [A B]^T T (op A from the staged blocks, op B from LDS tile).
template <typename T>
__device__ __forceinline__ typename AccT<T>::type gemm_w_ab(const T* sw, const double* stg, int n, int m, int lane) {
  typename AccT<T>::type acc = {0, 0, 0, 0};
  const int i = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int k = 4 * kk + kq;
    acc = mfma16(sw[i * LD + k], (T)stg[stg_ab(k, i, n, m)], acc);
  }
  return acc;
}
template <typename T>
__device__ __forceinline__ typename AccT<T>::type gemm_abt_t(const double* stg, const T* st, int n, int m, int lane) {
  typename AccT<T>::type acc = {0, 0, 0, 0};
  const int i = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) {
    const int k = 4 * kk + kq;
    acc = mfma16((T)stg[stg_ab(k, i, n, m)], st[k * LD + i], acc);
  }
  return acc;
}

// State pivot S_hat (register tile X, rows trow<TG>) -> X = -S_hat^{-1}, with
// its certificate bookkeeping in ps (code: the pivot's certificate code).
// When ||S_hat - I||_F is small enough (neumann_terms: always the case for a
// small delta, where the Riccati recursion spends most of its time) the
// inverse is the truncated Neumann series in the tile's precision TG -- Y_1 =
// I - E elementwise, each further term one 16 x 16 MFMA product through LDS
// (sE, sY: free TG tiles; sD: a float64 tile that may overlay them) -- and
// the norm bound certifies every pivot positive; otherwise the pivot sweep
// runs. Either way X is exactly symmetric on return (the compact float64
// tiles keep one triangle). PROD = false (the kernels with a per-stage
// diagonal, short of registers): only the one-term series (no product) is
// taken, anything longer goes to the sweep.
template <typename TG, bool PROD = true>
__device__ __forceinline__ void shat_inverse(double (&X)[4], int n, int lane, PivStats& ps, int code, TG* sE,
                                             TG* sY, double* sD) {
  const double e = dist_identity<TG>(X, lane);
  int terms = neumann_terms<TG>(e);
  if (!PROD && terms > 1) terms = 0;
  if (terms == 0) {
    const double sc = diag_scale<TG>(X, 0, n, lane);
    sweep16<TG>(X, 0, n, lane, ps, code, 1.0e3 * n * 2.220446049250313e-16 * sc, sc);
    return;
  }
  const int col = lane & 15, grp = lane >> 4;
  // X holds Y (the partial sums) from here on: no extra register tiles
  if (PROD && terms > 1) {
    double E[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) E[v] = X[v] - (trow<TG>(grp, v) == col ? 1.0 : 0.0);
    wave_sync();
    tile_to_lds<TG>(sE, E, lane);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double id = trow<TG>(grp, v) == col ? 1.0 : 0.0;
    X[v] = id - (X[v] - id);  // Y_1 = I - E
  }
  if (PROD && terms > 1) {
    for (int j = 2; j <= terms; ++j) {
      wave_sync();
      tile_to_lds<TG>(sY, X, lane);
      wave_sync();
      auto acc = gemm16<TG, false>(sE, sY, lane);
#pragma unroll
      for (int v = 0; v < 4; ++v) X[v] = (trow<TG>(grp, v) == col ? 1.0 : 0.0) - (double)acc[v];
    }
    // E Y is symmetric only up to rounding: Y <- (Y + Y^T) / 2
    wave_sync();
    tile_to_lds<TG>(sD, X, lane);
    wave_sync();
#pragma unroll
    for (int v = 0; v < 4; ++v) X[v] = 0.5 * (X[v] + sD[col * LD + trow<TG>(grp, v)]);
    wave_sync();
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) X[v] = -X[v];
  neumann_stats(ps, 0, n, e);
}

// SN, SM > 0: stage shape fixed at compile time (every instance of the launch
// has n = SN, m = SM); 0: taken from the instance.
// DG: per-stage diagonal Delta_i = D_i^2 (a.dd): the swept matrix is the
// symmetric representative S_hat = I + D P D of Section "Inertia
// Certification". Since I + Delta P = D S_hat D^{-1}, the tile stored is the
// symmetric X~ = D X D (X = -S_hat^{-1}), with (I + Delta P)^{-1} = -X~ Delta^{-1}
// and W = P (I + Delta P)^{-1} = -P X~ Delta^{-1}.
template <typename TG, int SN, int SM, bool DG>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_factor16(FactorArgs a) {
  constexpr bool CP = sizeof(TG) == 8;  // compact tiles in float64 (TileLayout)
  const SegDesc sd = a.segs[blockIdx.x];
  const int b = sd.inst;
  if (a.run && !a.run[b]) return;
  const InstMeta mt = a.meta[b];
  const int N = mt.N, n = SN > 0 ? SN : mt.n, m = SN > 0 ? SM : mt.m;
  const int klo = sd.lo, khi = sd.hi;
  const double delta = DG ? 0.0 : a.delta[b];
  const double* __restrict__ Qg = a.Q + mt.oQ;
  const double* __restrict__ Mg = a.M + mt.oM;
  const double* __restrict__ Rg = a.R + mt.oR;
  const double* __restrict__ Ag = a.A + mt.oA;
  const double* __restrict__ Bg = a.B + mt.oB;
  TG* __restrict__ ws = reinterpret_cast<TG*>(a.ws) + mt.ows;  // tiles Z_i, X_i (TileLayout)
  const TileLayout<CP> tl(n, m);

  const int lane = threadIdx.x, col = lane & 15, grp = lane >> 4;
  // work region: sP (P, then W) and sX (X, then T); the float64
  // symmetrization scratch sD overlays the start of the region. Safe inside
  // one wavefront: LDS accesses complete in program order.
  constexpr int TILE_T = NT * LD;
  constexpr int REGION = (2 * TILE_T * (int)sizeof(TG) > TILE_T * 8) ? 2 * TILE_T * (int)sizeof(TG) : TILE_T * 8;
  __shared__ __align__(16) unsigned char work[REGION];
  __shared__ __align__(16) double stg[STG_MAX];
  TG* sP = reinterpret_cast<TG*>(work);
  TG* sX = sP + TILE_T;
  double* sD = reinterpret_cast<double*>(work);

  PivStats ps;
  ps.init();
  const double eps = 2.220446049250313e-16;
  const int oZ = 2 * n * n + 2 * n * m + m * m;

  // with a right-hand side (whole instances only): the backward vector pass
  // of the solve rides along, on the stage's tiles rounded as stored, so p_k
  // and k_k are those the solve's own backward pass would compute
  const bool vec = a.q != nullptr;
  const bool xr = col < n, ur = col >= n && col < n + m, own = grp == 0;
  __shared__ double sv[2][16];
  const double* __restrict__ qg = a.q + mt.oq;
  const double* __restrict__ rg = a.r + mt.or_;
  const double* __restrict__ cg = a.c + mt.oc;
  double* __restrict__ pg = a.pk + mt.opk;
  double* __restrict__ kg = a.pk + mt.opk + (int64_t)(N + 1) * n;
  double pv = 0.0;
  if (vec) {
    pv = ld_or0(qg, (int64_t)N * n + col, xr);
    if (own && xr) pg[(int64_t)N * n + col] = pv;
  }
  // DG: the lane's diagonal entry of Delta_{k+1}, loaded one stage ahead, and
  // D of every row of the stage in LDS (0 outside the state block)
  const double* __restrict__ ddg = DG ? a.dd + mt.od : nullptr;
  __shared__ double sdl[16];
  double dnx = DG ? ld_or0(ddg, (int64_t)khi * n + col, xr) : 0.0;
  auto diag_scales = [&](double dcur, double& sdc, double& isdc, double (&sdr)[4]) {
    sdc = xr ? sqrt(dcur) : 0.0;
    isdc = xr ? 1.0 / sdc : 0.0;
    wave_sync();
    if (own) sdl[col] = sdc;
    wave_sync();
#pragma unroll
    for (int v = 0; v < 4; ++v) sdr[v] = sdl[trow<TG>(grp, v)];
  };

  // P_hi: Q_N at the top of the horizon, else the boundary tile of the scan
  double P[4];
  if (sd.P0 == nullptr) {
    const double* QN = Qg + (int64_t)N * n * n;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = trow<TG>(grp, v);
      const bool in = r < n && col < n;
      const double x = QN[in ? r * n + col : 0];
      P[v] = in ? x : 0.0;
    }
  } else {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = trow<TG>(grp, v);
      const bool in = r < n && col < n;
      const float x = sd.P0[in ? r * sd.p0_ld + col : 0];
      P[v] = in ? (double)x : 0.0;
    }
  }
  if (khi == N) tile_store_as<TG, CP>(ws + tl.z(N), P, lane, tl.s);
  if (khi > klo) {
    const int k = khi - 1;
    dma_stage(stg, Qg + (int64_t)k * n * n, Mg + (int64_t)k * n * m, Rg + (int64_t)k * m * m,
              Ag + (int64_t)k * n * n, Bg + (int64_t)k * n * m, n, m, lane);
  }

  for (int k = khi - 1; k >= klo; --k) {
    // the lane index, opaque to the compiler once per stage: the per-pivot
    // lane masks of the sweeps are then recomputed inside the stage (one
    // compare each) instead of being hoisted out of the loop, where sixteen
    // of them per sweep exhaust the scalar registers
    int lane_s = lane;
    asm volatile("" : "+v"(lane_s));
    double ck = 0.0, qk = 0.0, rk = 0.0;
    if (vec) {
      ck = ld_or0(cg, (int64_t)(k + 1) * n + col, xr);
      qk = ld_or0(qg, (int64_t)k * n + col, xr);
      rk = ld_or0(rg, (int64_t)k * m + (col - n), ur);
    }
    // X = I + delta P_{k+1} (DG: I + D P D); sweep -> -S_hat_{k+1}^{-1}  (no stage data needed)
    double sdc = 1.0, isdc = 1.0, sdr[4] = {1.0, 1.0, 1.0, 1.0};  // DG: D of the column, of the rows
    if constexpr (DG) {
      const double dcur = dnx;
      dnx = ld_or0(ddg, (int64_t)k * n + col, xr);
      diag_scales(dcur, sdc, isdc, sdr);
    }
    double X[4];
#pragma unroll
    for (int v = 0; v < 4; ++v)
      X[v] = (trow<TG>(grp, v) == col ? 1.0 : 0.0) + (DG ? sdr[v] * sdc * P[v] : delta * P[v]);
    shat_inverse<TG, !DG>(X, n, lane_s, ps, 2 * (k + 1), sP, sX, sD);
    const double idc = isdc * isdc;  // DG: 1 / Delta's entry of the column
    if constexpr (DG) {
#pragma unroll
      for (int v = 0; v < 4; ++v) X[v] = sdr[v] * X[v] * sdc;  // X~ = D X D
    }
    tile_store_as<TG, CP>(ws + tl.x(k + 1), X, lane, n);
    if (vec) {  // vector pass, first part: g = S_hat_{k+1}^{-1} (p_{k+1} + P_{k+1} c_{k+1})
      wave_sync();
      if (own) sv[0][col] = ck;
      wave_sync();
      const double vv = xr ? pv + tmatvec_r<TG>(P, sv[0], lane) : 0.0;
      if (own) sv[1][col] = vv;
      wave_sync();
      const double g = DG ? -idc * tmatvec_r<TG>(X, sv[1], lane) : -tmatvec_r<TG>(X, sv[1], lane);
      if (own) sv[0][col] = xr ? g : 0.0;
    }
    tile_to_lds<TG>(sP, P, lane);
    if constexpr (DG) {  // the product takes X~ Delta^{-1}
      double Xs[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) Xs[v] = X[v] * idc;
      tile_to_lds<TG>(sX, Xs, lane);
    } else {
      tile_to_lds<TG>(sX, X, lane);
    }
    wave_sync();
    // W = -P X. Symmetric only up to rounding, and left so: Z = [A B]^T W [A B]
    // + Hess is symmetrized below, which symmetrizes W's share of it as well
    double W[4];
    {
      auto acc = gemm16<TG, false>(sP, sX, lane);
      acc_to_regs<TG>(W, acc, -1.0);
    }
    wave_sync();
    tile_to_lds<TG>(sP, W, lane);
    // the stage blocks of step k must have landed
    wait_vmem();
    if (k == khi - 1 && lane == 0) stg[oZ] = 0.0;
    wave_sync();
    double H[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) H[v] = stg[stg_hess(trow<TG>(grp, v), col, n, m)];
    // T = W [A B]
    double T[4];
    {
      auto acc = gemm_w_ab<TG>(sP, stg, n, m, lane);
      acc_to_regs<TG>(T, acc, 1.0);
    }
    tile_to_lds<TG>(sX, T, lane);
    wave_sync();
    // Z = [A B]^T T + Hess, symmetrized
    double Z[4];
    {
      auto acc = gemm_abt_t<TG>(stg, sX, n, m, lane);
#pragma unroll
      for (int v = 0; v < 4; ++v) Z[v] = (double)acc[v] + H[v];
    }
    double abg = 0.0;
    if (vec) {  // second part: [A^T g; B^T g] from the staged blocks, h = r_k + B^T g
      wave_sync();
#pragma unroll
      for (int v = 0; v < 4; ++v) abg += stg[stg_ab(trow<TG>(grp, v), col, n, m)] * sv[0][trow<TG>(grp, v)];
      abg = group_sum(abg);
      if (own) sv[1][col] = ur ? rk + abg : 0.0;
    }
    // the staged blocks are no longer read: fetch step k-1's
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): reads of stg returned
    wave_sync();
    if (k > klo)
      dma_stage(stg, Qg + (int64_t)(k - 1) * n * n, Mg + (int64_t)(k - 1) * n * m, Rg + (int64_t)(k - 1) * m * m,
                Ag + (int64_t)(k - 1) * n * n, Bg + (int64_t)(k - 1) * n * m, n, m, lane);
    tile_to_lds<TG>(sD, Z, lane);
    wave_sync();
#pragma unroll
    for (int v = 0; v < 4; ++v) Z[v] = 0.5 * (Z[v] + sD[col * LD + trow<TG>(grp, v)]);
    // sweep the control block: G_k pivots
    {
      const double sc = diag_scale<TG>(Z, n, n + m, lane_s);
      sweep16<TG>(Z, n, n + m, lane_s, ps, 2 * k + 1, 1.0e3 * m * eps * sc, sc);
    }
    tile_store_as<TG, CP>(ws + tl.z(k), Z, lane, tl.s);
    if (vec) {  // third part: k_k = -G_k^{-1} h, p_k = q_k + A^T g + K_k^T h
      wave_sync();
      const double zh = tmatvec_r<TG>(Z, sv[1], lane);
      pv = xr ? qk + abg - zh : 0.0;
      if (own) {
        if (xr) pg[(int64_t)k * n + col] = pv;
        if (ur) kg[(int64_t)k * m + (col - n)] = zh;
      }
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) P[v] = (trow<TG>(grp, v) < n && col < n) ? Z[v] : 0.0;
    wave_sync();
  }
  // S_hat_0
  if (klo == 0) {
    double sdc = 1.0, isdc = 1.0, sdr[4] = {1.0, 1.0, 1.0, 1.0};
    if constexpr (DG) diag_scales(dnx, sdc, isdc, sdr);
    double X[4];
#pragma unroll
    for (int v = 0; v < 4; ++v)
      X[v] = (trow<TG>(grp, v) == col ? 1.0 : 0.0) + (DG ? sdr[v] * sdc * P[v] : delta * P[v]);
    shat_inverse<TG, !DG>(X, n, lane, ps, 0, sP, sX, sD);
    if constexpr (DG) {
#pragma unroll
      for (int v = 0; v < 4; ++v) X[v] = sdr[v] * X[v] * sdc;  // X~_0 = D_0 X_0 D_0
    }
    tile_store_as<TG, CP>(ws + tl.x(0), X, lane, n);
  }
  if (lane == 0) {
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

// Solve pass: backward vector pass and forward rollout (see the file header).
// corr == NULL: solve K z = -b and write z.  corr != NULL: solve for the
// correction with right-hand side corr (the previous residual) and add it to
// z. The tiles and stage blocks of the next step are loaded one step ahead
// so that the dependent chain does not wait on memory.
// ACC: correction pass (right-hand side = a.corr, z += dz); otherwise a.corr is NULL
// DG: per-stage diagonal Delta_i (a.dd); with the stored X~ = -D S_hat^{-1} D,
// (I + Delta P)^{-1} = -X~ Delta^{-1} and (I + P Delta)^{-1} = -Delta^{-1} X~.
// WPE: wavefronts per SIMD the register budget is sized for: 4 for full
// batches (occupancy hides the memory latency), 1 for small launches (the
// longest instance's step chain is the launch: no spills, registers to spare).
template <typename TG, int SN, int SM, bool ACC, bool DG, int WPE = 4>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WPE, 8))) void k_solve16(SolveArgs a) {
  constexpr bool CP = sizeof(TG) == 8;  // compact tiles in float64 (TileLayout)
  const int b = a.list ? a.list[blockIdx.x] : (int)blockIdx.x;
  const int lane = threadIdx.x, col = lane & 15, grp = lane >> 4;
  if (a.run && !a.run[b]) return;
  const InstMeta mt = a.meta[b];
  const int N = mt.N, n = SN > 0 ? SN : mt.n, m = SN > 0 ? SM : mt.m;
  const double delta = DG ? 0.0 : a.delta[b];
  const double* __restrict__ ddg = DG ? a.dd + mt.od : nullptr;
  const double* __restrict__ Ag = a.A + mt.oA;
  const double* __restrict__ Bg = a.B + mt.oB;
  const TG* __restrict__ ws = reinterpret_cast<const TG*>(a.ws) + mt.ows;
  const TileLayout<CP> tl(n, m);
  // compact element indices of the lane (Z: s x s block, X: n x n block);
  // made opaque once per step below so that their byte extraction is not
  // hoisted out of the stage loops into live registers
  uint32_t pz = CP ? tri_pack<TG>(lane, n + m) : 0u, px = CP ? tri_pack<TG>(lane, n) : 0u;
  double* __restrict__ pg = a.pk + mt.opk;                        // p_i at i*n
  double* __restrict__ kg = a.pk + mt.opk + (int64_t)(N + 1) * n;  // k_i at i*m
  const double *qb, *rb, *cb;
  int64_t qs, rs;
  constexpr bool acc = ACC;
  if (acc) {
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
    if (!acc) {
      const double nanv = __builtin_nan("");
      for (int i = lane; i < (N + 1) * n; i += 64) { xg[i] = nanv; yg[i] = nanv; }
      for (int i = lane; i < N * m; i += 64) ug[i] = nanv;
    }
    return;
  }

  __shared__ double sv[2][16];
  const bool xr = col < n, ur = (col >= n) && (col < n + m);
  const bool own = grp == 0;  // lanes 0..15 write outputs

  // ---- backward vector pass (k = N-1 .. 0), one step of lookahead
  // (already done by the factorization when fwd_only is set)
  double Zk[4], Xn[4];
  if (!a.fwd_only) {
    double p = ld_or0(qb, (int64_t)N * qs + col, xr);
    if (own && xr) pg[(int64_t)N * n + col] = p;
    double Zp[4], ab[4];
    tile_load_pk<CP>(Zp, ws + tl.z(N), lane, pz);
    if (N > 0) {
      tile_load_pk<CP>(Zk, ws + tl.z(N - 1), lane, pz);
      tile_load_pk<CP>(Xn, ws + tl.x(N), lane, px);
#pragma unroll
      for (int v = 0; v < 4; ++v)
        ab[v] = ab_elem(Ag + (int64_t)(N - 1) * n * n, Bg + (int64_t)(N - 1) * n * m, n, m, trow<TG>(grp, v), col);
    }
    double ck = 0.0, qk = 0.0, rk = 0.0, dk = 0.0;
    if (N > 0) {
      ck = ld_or0(cb, (int64_t)N * n + col, xr);
      qk = ld_or0(qb, (int64_t)(N - 1) * qs + col, xr);
      rk = ld_or0(rb, (int64_t)(N - 1) * rs + (col - n), ur);
      if (DG) dk = ld_or0(ddg, (int64_t)N * n + col, xr);
    }
    for (int k = N - 1; k >= 0; --k) {
      if constexpr (CP) asm volatile("" : "+v"(pz), "+v"(px));
      // next step's operands
      double Zk1[4], Xn1[4], ab1[4];
      const int k1 = k > 0 ? k - 1 : 0;
      tile_load_pk<CP>(Zk1, ws + tl.z(k1), lane, pz);
      tile_load_pk<CP>(Xn1, ws + tl.x(k1 + 1), lane, px);
#pragma unroll
      for (int v = 0; v < 4; ++v)
        ab1[v] = ab_elem(Ag + (int64_t)k1 * n * n, Bg + (int64_t)k1 * n * m, n, m, trow<TG>(grp, v), col);
      const double ck1 = ld_or0(cb, (int64_t)(k1 + 1) * n + col, xr);
      const double qk1 = ld_or0(qb, (int64_t)k1 * qs + col, xr);
      const double rk1 = ld_or0(rb, (int64_t)k1 * rs + (col - n), ur);
      const double dk1 = DG ? ld_or0(ddg, (int64_t)(k1 + 1) * n + col, xr) : 0.0;
      const double idk = (DG && xr) ? 1.0 / dk : 0.0;
      const double zh = bwd_vec_step<TG, DG>(Zp, Xn, ab, Zk, p, ck, qk, rk, sv, xr, ur, own, col, lane, idk);
      if (own) {
        if (xr) pg[(int64_t)k * n + col] = p;
        if (ur) kg[(int64_t)k * m + (col - n)] = zh;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        Zp[v] = Zk[v];
        Zk[v] = Zk1[v];
        Xn[v] = Xn1[v];
        ab[v] = ab1[v];
      }
      ck = ck1;
      qk = qk1;
      rk = rk1;
      dk = dk1;
    }
  }
  __syncthreads();  // p/k written by lanes 0..15 are read by all lanes below

  // ---- forward rollout (k = 0 .. N-1) with the float64 residual of the
  // updated solution (Section "Residual Computation") when res is set.
  // Per step the stage blocks Q, M, R, A, B of step k+1 are copied to LDS
  // while step k runs (two staging buffers); the tiles and vectors of step
  // k+1 are loaded into registers one step ahead. The chain of a step is
  // w = [A_k B_k] z_k -> x_{k+1} -> Z_{k+1} x_{k+1} (which already gives u_{k+1}
  // and y_{k+1}); the residual rows of stage k hang off it:
  //   x rows: Q x + M u + A^T y_{k+1} + q - y_k,  u rows: M^T x + R u + B^T y_{k+1} + r,
  //   dynamics: A x + B u + c_{k+1} - delta y_{k+1} - x_{k+1}   (totals, original rhs)
  // plus the initial row c_0 - delta y_0 - x_0 and the terminal row
  // Q_N x_N + q_N - y_N. The instance's maxima go to resmax / bmax directly
  // (one wavefront per instance).
  const bool fuse = a.res != nullptr && a.resfuse != nullptr && a.resfuse[b] != 0;
  double* __restrict__ resg = fuse ? a.res + mt.ores : nullptr;
  const double* __restrict__ qo = a.q + mt.oq;
  const double* __restrict__ ro = a.r + mt.or_;
  const double* __restrict__ co = a.c + mt.oc;
  __shared__ __align__(16) double stgA[STG_MAX];
  __shared__ __align__(16) double stgB[STG_MAX];
  __shared__ double sz[2][16];  // z_k totals (x | u) and y_{k+1} totals
  // staging indices of the lane's Hessian, [A B] and [A B]^T elements, packed
  // 10 bits each (STG_MAX < 1024) to keep them in one register per element
  int ipk[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int j = 4 * grp + v;
    ipk[v] = stg_hess(j, col, n, m) | (stg_ab(j, col, n, m) << 10) | (stg_ab(col, j, n, m) << 20);
  }
  const int oZ = 2 * n * n + 2 * n * m + m * m;
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
  wave_sync();
  if (lane == 0) {
    stgA[oZ] = 0.0;
    stgB[oZ] = 0.0;
  }
  // DG: Delta_{k+1}'s diagonal rides with step k's staged blocks (after the zero cell)
  const int oD = oZ + 1;
  if (N > 0) {
    dma_stage(stgA, a.Q + mt.oQ, a.M + mt.oM, a.R + mt.oR, Ag, Bg, n, m, lane);
    if constexpr (DG) dma_block(ddg + n, stgA + oD, n, lane);
  }
  double rmax = 0.0, bmax = 0.0;

  // x_0, then z_0 = Z_0 x_0 (u_0 and y_0)
  // DG: Delta_0's entry of the lane (d0); Delta_{k+1}'s (dn) is staged with step k's blocks
  const double d0 = DG ? ld_or0(ddg, col, xr) : delta;
  double x;
  {
    double X0[4];
    tile_load_pk<CP>(X0, ws + tl.x(0), lane, px);
    const double p0 = ld_or0(pg, col, xr);
    const double c00 = ld_or0(cb, col, xr);
    wave_sync();
    if constexpr (DG) {  // x_0 = -X~_0 Delta_0^{-1} (c_0 - Delta_0 p_0)
      if (own) sv[0][col] = xr ? (c00 - d0 * p0) / d0 : 0.0;
      wave_sync();
      x = xr ? -tmatvec<TG>(X0, sv[0], lane) : 0.0;
    } else {
      if (own) sv[0][col] = xr ? c00 - delta * p0 : 0.0;
      wave_sync();
      x = xr ? -tmatvec<TG>(X0, sv[0], lane) : 0.0;
    }
  }
  tile_load_pk<CP>(Zk, ws + tl.z(0), lane, pz);
  double zx;  // Z_k x_k: [P_k x_k; -K_k x_k]
  {
    wave_sync();
    if (own) sv[0][col] = xr ? x : 0.0;
    wave_sync();
    zx = tmatvec<TG>(Zk, sv[0], lane);
  }
  // step k's vectors (loaded one step ahead)
  double pk = ld_or0(pg, col, xr);
  double kk = N > 0 ? ld_or0(kg, col - n, ur) : 0.0;
  double xold = acc ? ld_or0(xg, col, xr) : 0.0;
  double yold = acc ? ld_or0(yg, col, xr) : 0.0;
  double uold = (acc && N > 0) ? ld_or0(ug, col - n, ur) : 0.0;
  {
    // initial row c_0 - delta y_0 - x_0 (totals, original c_0)
    const double c0 = ld_or0(co, col, xr);
    const double xt = x + xold, yt = zx + pk + yold;
    if (fuse && own && xr) {
      const double r0 = c0 - d0 * yt - xt;
      resg[(int64_t)N * (n + m) + n + col] = r0;
      rmax = maxnan(rmax, fabs(r0));
      bmax = maxnan(bmax, fabs(c0));
    }
  }
  if (N > 0) tile_load_pk<CP>(Xn, ws + tl.x(1), lane, px);
  double pn = N > 0 ? ld_or0(pg, (int64_t)n + col, xr) : 0.0;
  double cn = N > 0 ? ld_or0(cb, (int64_t)n + col, xr) : 0.0;
  double xoldn = (acc && N > 0) ? ld_or0(xg, (int64_t)n + col, xr) : 0.0;
  double yoldn = (acc && N > 0) ? ld_or0(yg, (int64_t)n + col, xr) : 0.0;
  double qok = N > 0 ? ld_or0(qo, col, xr) : 0.0;
  double rok = N > 0 ? ld_or0(ro, col - n, ur) : 0.0;
  double con = N > 0 ? ld_or0(co, (int64_t)n + col, xr) : 0.0;
  double dn = delta;

  for (int k = 0; k < N; ++k) {
    if constexpr (CP) asm volatile("" : "+v"(pz), "+v"(px));
    double* stgc = (k & 1) ? stgB : stgA;
    double* stgn = (k & 1) ? stgA : stgB;
    wait_vmem();  // step k's blocks, tiles and vectors have landed
    wave_sync();
    // DG: Delta_{k+1}'s entry from the staging buffer and its reciprocal, off
    // the step's dependent chain
    if constexpr (DG) dn = xr ? stgc[oD + col] : 0.0;
    const double idn = (DG && xr) ? 1.0 / dn : 0.0;
    const bool more = k + 1 < N;
    if (more) {
      const int k1 = k + 1;
      dma_stage(stgn, a.Q + mt.oQ + (int64_t)k1 * n * n, a.M + mt.oM + (int64_t)k1 * n * m,
                a.R + mt.oR + (int64_t)k1 * m * m, Ag + (int64_t)k1 * n * n, Bg + (int64_t)k1 * n * m, n, m, lane);
      if constexpr (DG) dma_block(ddg + (int64_t)(k1 + 1) * n, stgn + oD, n, lane);
    }
    // step k+1's tiles and vectors
    double Zk1[4], Xn1[4];
    const int k1 = more ? k + 1 : k;
    tile_load_pk<CP>(Zk1, ws + tl.z(k + 1), lane, pz);  // Z_N exists (P_N)
    tile_load_pk<CP>(Xn1, ws + tl.x(k1 + 1), lane, px);
    const double kk1 = ld_or0(kg, (int64_t)k1 * m + (col - n), ur);
    const double uold1 = acc ? ld_or0(ug, (int64_t)k1 * m + (col - n), ur) : 0.0;
    const double pn1 = ld_or0(pg, (int64_t)(k1 + 1) * n + col, xr);
    const double cn1 = ld_or0(cb, (int64_t)(k1 + 1) * n + col, xr);
    const double xoldn1 = acc ? ld_or0(xg, (int64_t)(k1 + 1) * n + col, xr) : 0.0;
    const double yoldn1 = acc ? ld_or0(yg, (int64_t)(k1 + 1) * n + col, xr) : 0.0;
    const double qok1 = ld_or0(qo, (int64_t)k1 * n + col, xr);
    const double rok1 = ld_or0(ro, (int64_t)k1 * m + (col - n), ur);
    const double con1 = ld_or0(co, (int64_t)(k1 + 1) * n + col, xr);

    // u_k, y_k from z_k; write the totals
    const double uk = ur ? kk - zx : 0.0;
    const double xt = x + xold, ut = uk + uold, yt = zx + pk + yold;
    if (own) {
      if (xr) {
        yg[(int64_t)k * n + col] = yt;
        xg[(int64_t)k * n + col] = xt;
      }
      if (ur) ug[(int64_t)k * m + (col - n)] = ut;
      sv[1][col] = xr ? x : (ur ? uk : 0.0);
      sz[0][col] = xr ? xt : (ur ? ut : 0.0);
    }
    wave_sync();
    // w = A x + B u of this pass's z (the chain) and of the totals (residual)
    double w = 0.0, wt = 0.0, hz = 0.0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int j = 4 * grp + v;
      const double abt = stgc[ipk[v] >> 20];
      w += abt * sv[1][j];
      wt += abt * sz[0][j];
      hz += stgc[ipk[v] & 1023] * sz[0][j];
    }
    w = group_sum(w);
    if constexpr (DG) {  // x_{k+1} = -X~ Delta^{-1} (w + c - Delta p)
      if (own) sv[0][col] = xr ? (w + cn - dn * pn) * idn : 0.0;
      wave_sync();
      x = xr ? -tmatvec<TG>(Xn, sv[0], lane) : 0.0;
    } else {
      if (own) sv[0][col] = xr ? w + cn - delta * pn : 0.0;
      wave_sync();
      x = xr ? -tmatvec<TG>(Xn, sv[0], lane) : 0.0;  // x_{k+1} of this pass
    }
    wave_sync();
    if (own) sv[1][col] = xr ? x : 0.0;
    wave_sync();
    zx = tmatvec<TG>(Zk1, sv[1], lane);           // Z_{k+1} x_{k+1}
    if (fuse) {
      wt = group_sum(wt);
      hz = group_sum(hz);
      const double x1t = x + xoldn, y1t = zx + pn + yoldn;
      if (own) sz[1][col] = xr ? y1t : 0.0;
      wave_sync();
      double g = 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) g += stgc[(ipk[v] >> 10) & 1023] * sz[1][4 * grp + v];
      g = group_sum(g);
      if (own) {
        const int64_t base = (int64_t)k * (n + m);
        if (xr) {
          const double rx = hz + g + qok - yt;
          const double rd = wt + con - dn * y1t - x1t;
          resg[base + col] = rx;
          resg[(int64_t)N * (n + m) + n + (int64_t)(k + 1) * n + col] = rd;
          rmax = maxnan(rmax, maxnan(fabs(rx), fabs(rd)));
          bmax = maxnan(bmax, maxnan(fabs(qok), fabs(con)));
        }
        if (ur) {
          const double ru = hz + g + rok;
          resg[base + col] = ru;
          rmax = maxnan(rmax, fabs(ru));
          bmax = maxnan(bmax, fabs(rok));
        }
      }
    }
    __builtin_amdgcn_s_waitcnt(0xc07f);  // reads of this step's staging buffer returned before it is refilled
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Zk[v] = Zk1[v];
      Xn[v] = Xn1[v];
    }
    pk = pn; kk = kk1; pn = pn1; cn = cn1;
    xold = xoldn; yold = yoldn; uold = uold1; xoldn = xoldn1; yoldn = yoldn1;
    qok = qok1; rok = rok1; con = con1;
  }
  {
    // x_N, y_N (zx holds P_N x_N) and the terminal row Q_N x_N + q_N - y_N
    const double xt = x + xold, yt = zx + pk + yold;
    if (own && xr) {
      yg[(int64_t)N * n + col] = yt;
      xg[(int64_t)N * n + col] = xt;
    }
    if (fuse) {
      const double* QN = a.Q + mt.oQ + (int64_t)N * n * n;
      double Hq[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = 4 * grp + v;
        Hq[v] = ld_or0(QN, j * n + col, j < n && xr);
      }
      const double qN = ld_or0(qo, (int64_t)N * n + col, xr);
      wave_sync();
      if (own) sz[0][col] = xr ? xt : 0.0;
      wave_sync();
      double h = 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) h += Hq[v] * sz[0][4 * grp + v];
      h = group_sum(h);
      if (own && xr) {
        const double rt = h + qN - yt;
        resg[(int64_t)N * (n + m) + col] = rt;
        rmax = maxnan(rmax, fabs(rt));
        bmax = maxnan(bmax, fabs(qN));
      }
      rmax = wave_max(rmax);
      bmax = wave_max(bmax);
      if (lane == 0) {
        a.resmax[b] = (unsigned long long)__double_as_longlong(rmax);
        a.bmax[b] = (unsigned long long)__double_as_longlong(bmax);
      }
    }
  }
}

// ------------------------------------------------------------------ residual

__device__ __forceinline__ void atomic_max_nonneg(unsigned long long* p, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax(p, (unsigned long long)__double_as_longlong(v));
}

// Residual of Section "Residual Computation", float64, parallel over
// (instance, chunk of stages): one wavefront walks a chunk of consecutive
// stage slots i of one instance (RES_CHUNK slots for n + m <= 16, 64 / n for
// larger stages; slot N carries the terminal row and the c_0 row) and keeps
// the instance's maxima in registers, so each chunk issues one pair of 64-bit
// atomic max operations (order-independent). For n + m <= 16 a slot is three
// tile-vector products on staged blocks (Hessian [[Q, M], [M^T, R]], [A B] and
// its transpose), with the blocks of the next slot copied to LDS while the
// current one is reduced; larger stages use one lane per (stage, row) of
// each kind of row (residual_chunk_rows).
struct ResVec {
  double xi, ui, yi, yn, xn, qi, ri, cn;
  double dn;  // the lane's entry of the per-stage diagonal Delta_{i+1} (unused with delta I)
};

// dd: the per-stage diagonals (a.dd) or NULL (delta I); likewise below
__device__ __forceinline__ void res_load_vec(const ResidualArgs& a, const InstMeta& mt, int n, int m, int i, int lane,
                                             double delta, const double* dd, ResVec& o) {
  const int col = lane & 15;
  const bool xr = col < n, ur = col >= n && col < n + m;
  o.xi = ld_or0(a.x + mt.ox, (int64_t)i * n + col, xr);
  o.ui = ld_or0(a.u + mt.ou, (int64_t)i * m + (col - n), ur);
  o.yi = ld_or0(a.y + mt.oy, (int64_t)i * n + col, xr);
  o.yn = ld_or0(a.y + mt.oy, (int64_t)(i + 1) * n + col, xr);
  o.xn = ld_or0(a.x + mt.ox, (int64_t)(i + 1) * n + col, xr);
  o.qi = ld_or0(a.q + mt.oq, (int64_t)i * n + col, xr);
  o.ri = ld_or0(a.r + mt.or_, (int64_t)i * m + (col - n), ur);
  o.cn = ld_or0(a.c + mt.oc, (int64_t)(i + 1) * n + col, xr);
  o.dn = dd ? ld_or0(dd + mt.od, (int64_t)(i + 1) * n + col, xr) : 0.0;
}

__device__ __forceinline__ void res_stage_dma(const ResidualArgs& a, const InstMeta& mt, int n, int m, int i,
                                              double* stg, int lane) {
  dma_stage(stg, a.Q + mt.oQ + (int64_t)i * n * n, a.M + mt.oM + (int64_t)i * n * m,
            a.R + mt.oR + (int64_t)i * m * m, a.A + mt.oA + (int64_t)i * n * n,
            a.B + mt.oB + (int64_t)i * n * m, n, m, lane);
}

// Residual rows of stage i < N from the staged blocks (Hessian, [A B], [A B]^T
// read at the per-lane staging indices) and the stage vectors.
__device__ __forceinline__ void res_compute(const ResidualArgs& a, const InstMeta& mt, int n, int m, double delta,
                                            const double* dd, int i, const double* stg, const int (&iH)[4], const int (&iAB)[4],
                                            const int (&iABT)[4], const ResVec& o, double* sv, double& rmax,
                                            double& bmax, int lane) {
  const int N = mt.N;
  const int col = lane & 15, grp = lane >> 4;
  const bool xr = col < n, ur = col >= n && col < n + m, own = grp == 0;
  double* res = a.res ? a.res + mt.ores : nullptr;
  wave_sync();
  if (own) {
    sv[col] = xr ? o.xi : (ur ? o.ui : 0.0);
    sv[16 + col] = xr ? o.yn : 0.0;
  }
  wave_sync();
  double h = 0.0, g = 0.0, w = 0.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int j = 4 * grp + v;
    h += stg[iH[v]] * sv[j];          // Hess z
    g += stg[iAB[v]] * sv[16 + j];    // [A B]^T y_{i+1}
    w += stg[iABT[v]] * sv[j];        // [A B] z
  }
  h = group_sum(h);
  g = group_sum(g);
  w = group_sum(w);
  if (own) {
    const int64_t base = (int64_t)i * (n + m);
    if (xr) {
      const double rx = h + g + o.qi - o.yi;
      const double rd = w + o.cn - (dd ? o.dn : delta) * o.yn - o.xn;
      if (res) {
        res[base + col] = rx;
        res[(int64_t)N * (n + m) + 2 * n + (int64_t)i * n + col] = rd;
      }
      rmax = maxnan(rmax, maxnan(fabs(rx), fabs(rd)));
      bmax = maxnan(bmax, maxnan(fabs(o.qi), fabs(o.cn)));
    }
    if (ur) {
      const double ru = h + g + o.ri;
      if (res) res[base + col] = ru;
      rmax = maxnan(rmax, fabs(ru));
      bmax = maxnan(bmax, fabs(o.ri));
    }
  }
}

// slot N of an instance with n + m <= 16: terminal row and c_0 row
__device__ __forceinline__ void res_terminal(const ResidualArgs& a, const InstMeta& mt, int n, int m, double delta,
                                             const double* dd, double* sv, double& rmax, double& bmax, int lane) {
  const int N = mt.N;
  const int col = lane & 15, grp = lane >> 4;
  const bool xr = col < n, own = grp == 0;
  const double* q = a.q + mt.oq; const double* c = a.c + mt.oc;
  const double* x = a.x + mt.ox; const double* y = a.y + mt.oy;
  double* res = a.res ? a.res + mt.ores : nullptr;
  const double* QN = a.Q + mt.oQ + (int64_t)N * n * n;
  double Hq[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int j = 4 * grp + v;
    Hq[v] = ld_or0(QN, j * n + col, j < n && xr);
  }
  const double xN = ld_or0(x, (int64_t)N * n + col, xr);
  const double yN = ld_or0(y, (int64_t)N * n + col, xr);
  const double qN = ld_or0(q, (int64_t)N * n + col, xr);
  const double c0 = ld_or0(c, col, xr);
  const double x0 = ld_or0(x, col, xr);
  const double y0 = ld_or0(y, col, xr);
  const double d0 = dd ? ld_or0(dd + mt.od, col, xr) : delta;
  wave_sync();
  if (own) sv[col] = xr ? xN : 0.0;
  wave_sync();
  double h = 0.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) h += Hq[v] * sv[4 * grp + v];
  h = group_sum(h);
  if (own && xr) {
    const double rt = h + qN - yN;
    const double ri = c0 - d0 * y0 - x0;
    if (res) {
      res[(int64_t)N * (n + m) + col] = rt;
      res[(int64_t)N * (n + m) + n + col] = ri;
    }
    rmax = maxnan(rmax, maxnan(fabs(rt), fabs(ri)));
    bmax = maxnan(bmax, maxnan(fabs(qN), fabs(c0)));
  }
}

__device__ __forceinline__ void residual_slot_rows(const ResidualArgs& a, const InstMeta& mt, int b, int i,
                                                   const double* ddall, double& rmax, double& bmax, int lane) {
  const int N = mt.N, n = mt.n, m = mt.m;
  const int nn = n * n, nm = n * m, mm = m * m;
  const double delta = ddall ? 0.0 : a.delta[b];
  const double* dd = ddall ? ddall + mt.od : nullptr;  // per-stage diagonal Delta_i, laid out like x
  const double* q = a.q + mt.oq; const double* r = a.r + mt.or_; const double* c = a.c + mt.oc;
  const double* x = a.x + mt.ox; const double* u = a.u + mt.ou; const double* y = a.y + mt.oy;
  double* res = a.res ? a.res + mt.ores : nullptr;
  if (i < N) {
    const double* Q = a.Q + mt.oQ + (int64_t)i * nn; const double* M = a.M + mt.oM + (int64_t)i * nm;
    const double* R = a.R + mt.oR + (int64_t)i * mm; const double* A = a.A + mt.oA + (int64_t)i * nn;
    const double* B = a.B + mt.oB + (int64_t)i * nm;
    const double* xi = x + (int64_t)i * n; const double* ui = u + (int64_t)i * m;
    const double* yn = y + (int64_t)(i + 1) * n;
    // the inner products are unrolled by 8: eight loads in flight per lane
    // instead of one memory round trip per term
    for (int row = lane; row < 2 * n + m; row += 64) {
      double s = 0.0, bv;
      int64_t out;
      if (row < n) {
        const int a0 = row;
#pragma unroll 8
        for (int j = 0; j < n; ++j) s = fma(Q[j * n + a0], xi[j], s);  // Q symmetric: lanes read a row
#pragma unroll 8
        for (int j = 0; j < m; ++j) s = fma(M[a0 * m + j], ui[j], s);
#pragma unroll 8
        for (int j = 0; j < n; ++j) s = fma(A[j * n + a0], yn[j], s);
        bv = q[(int64_t)i * n + a0];
        s += bv - y[(int64_t)i * n + a0];
        out = (int64_t)i * (n + m) + a0;
      } else if (row < n + m) {
        const int a0 = row - n;
#pragma unroll 8
        for (int j = 0; j < n; ++j) s = fma(M[j * m + a0], xi[j], s);
#pragma unroll 8
        for (int j = 0; j < m; ++j) s = fma(R[j * m + a0], ui[j], s);  // R symmetric
#pragma unroll 8
        for (int j = 0; j < n; ++j) s = fma(B[j * m + a0], yn[j], s);
        bv = r[(int64_t)i * m + a0];
        s += bv;
        out = (int64_t)i * (n + m) + n + a0;
      } else {
        const int a0 = row - n - m;
#pragma unroll 8
        for (int j = 0; j < n; ++j) s = fma(A[a0 * n + j], xi[j], s);
#pragma unroll 8
        for (int j = 0; j < m; ++j) s = fma(B[a0 * m + j], ui[j], s);
        bv = c[(int64_t)(i + 1) * n + a0];
        s += bv - (dd ? dd[(int64_t)(i + 1) * n + a0] : delta) * yn[a0] - x[(int64_t)(i + 1) * n + a0];
        out = (int64_t)N * (n + m) + 2 * n + (int64_t)i * n + a0;
      }
      if (res) res[out] = s;
      rmax = maxnan(rmax, fabs(s));
      bmax = maxnan(bmax, fabs(bv));
    }
  } else {
    const double* QN = a.Q + mt.oQ + (int64_t)N * nn;
    const double* xN = x + (int64_t)N * n;
    for (int row = lane; row < 2 * n; row += 64) {
      double s = 0.0, bv;
      int64_t out;
      if (row < n) {
#pragma unroll 8
        for (int j = 0; j < n; ++j) s = fma(QN[j * n + row], xN[j], s);
        bv = q[(int64_t)N * n + row];
        s += bv - y[(int64_t)N * n + row];
        out = (int64_t)N * (n + m) + row;
      } else {
        const int a0 = row - n;
        bv = c[a0];
        s = bv - (dd ? dd[a0] : delta) * y[a0] - x[a0];
        out = (int64_t)N * (n + m) + n + a0;
      }
      if (res) res[out] = s;
      rmax = maxnan(rmax, fabs(s));
      bmax = maxnan(bmax, fabs(bv));
    }
  }
}

// The stage slots [i0, min(i1, N)) of one instance with n + m > 16: the rows
// are taken by kind (primal x rows, primal u rows, dual rows), each kind over
// all the chunk's stages at once with one lane per (stage, row), so that the
// lanes of a wavefront run the same products (no divergence between kinds)
// and a chunk of 64 / n stages fills the wavefront. The inner products are
// unrolled by 8: eight loads in flight per lane.
__device__ __forceinline__ void residual_chunk_rows(const ResidualArgs& a, const InstMeta& mt, int b, int i0, int i1,
                                                    const double* ddall, double& rmax, double& bmax, int lane) {
  const int N = mt.N, n = mt.n, m = mt.m;
  const int64_t nn = (int64_t)n * n, nm = (int64_t)n * m, mm = (int64_t)m * m;
  const double delta = ddall ? 0.0 : a.delta[b];
  const double* dd = ddall ? ddall + mt.od : nullptr;
  const double* q = a.q + mt.oq; const double* r = a.r + mt.or_; const double* c = a.c + mt.oc;
  const double* x = a.x + mt.ox; const double* u = a.u + mt.ou; const double* y = a.y + mt.oy;
  double* res = a.res ? a.res + mt.ores : nullptr;
  const int nst = min(i1, N) - i0;
  for (int t = lane; t < nst * n; t += 64) {  // Q x + M u + A^T y_{i+1} + q - y_i
    const int i = i0 + t / n, a0 = t % n;
    const double* Q = a.Q + mt.oQ + i * nn; const double* M = a.M + mt.oM + i * nm;
    const double* A = a.A + mt.oA + i * nn;
    const double* xi = x + (int64_t)i * n; const double* ui = u + (int64_t)i * m;
    const double* yn = y + (int64_t)(i + 1) * n;
    double s = 0.0;
#pragma unroll 8
    for (int j = 0; j < n; ++j) s = fma(Q[j * n + a0], xi[j], s);  // Q symmetric: lanes read a row
#pragma unroll 8
    for (int j = 0; j < m; ++j) s = fma(M[a0 * m + j], ui[j], s);
#pragma unroll 8
    for (int j = 0; j < n; ++j) s = fma(A[j * n + a0], yn[j], s);
    const double bv = q[(int64_t)i * n + a0];
    s += bv - y[(int64_t)i * n + a0];
    if (res) res[(int64_t)i * (n + m) + a0] = s;
    rmax = maxnan(rmax, fabs(s));
    bmax = maxnan(bmax, fabs(bv));
  }
  for (int t = lane; t < nst * m; t += 64) {  // M^T x + R u + B^T y_{i+1} + r
    const int i = i0 + t / m, a0 = t % m;
    const double* M = a.M + mt.oM + i * nm; const double* R = a.R + mt.oR + i * mm;
    const double* B = a.B + mt.oB + i * nm;
    const double* xi = x + (int64_t)i * n; const double* ui = u + (int64_t)i * m;
    const double* yn = y + (int64_t)(i + 1) * n;
    double s = 0.0;
#pragma unroll 8
    for (int j = 0; j < n; ++j) s = fma(M[j * m + a0], xi[j], s);
#pragma unroll 8
    for (int j = 0; j < m; ++j) s = fma(R[j * m + a0], ui[j], s);  // R symmetric
#pragma unroll 8
    for (int j = 0; j < n; ++j) s = fma(B[j * m + a0], yn[j], s);
    const double bv = r[(int64_t)i * m + a0];
    s += bv;
    if (res) res[(int64_t)i * (n + m) + n + a0] = s;
    rmax = maxnan(rmax, fabs(s));
    bmax = maxnan(bmax, fabs(bv));
  }
  for (int t = lane; t < nst * n; t += 64) {  // A x + B u + c_{i+1} - Delta y_{i+1} - x_{i+1}
    const int i = i0 + t / n, a0 = t % n;
    const double* A = a.A + mt.oA + i * nn; const double* B = a.B + mt.oB + i * nm;
    const double* xi = x + (int64_t)i * n; const double* ui = u + (int64_t)i * m;
    const double* yn = y + (int64_t)(i + 1) * n;
    double s = 0.0;
#pragma unroll 8
    for (int j = 0; j < n; ++j) s = fma(A[a0 * n + j], xi[j], s);
#pragma unroll 8
    for (int j = 0; j < m; ++j) s = fma(B[a0 * m + j], ui[j], s);
    const double bv = c[(int64_t)(i + 1) * n + a0];
    s += bv - (dd ? dd[(int64_t)(i + 1) * n + a0] : delta) * yn[a0] - x[(int64_t)(i + 1) * n + a0];
    if (res) res[(int64_t)N * (n + m) + 2 * n + (int64_t)i * n + a0] = s;
    rmax = maxnan(rmax, fabs(s));
    bmax = maxnan(bmax, fabs(bv));
  }
}

// SN, SM > 0: every instance of the batch has n = SN, m = SM (n + m <= 16).
// DG: per-stage diagonal Delta_i (a.dd) in the dual rows.
// PART 1: only the chunks of stages with n + m <= 16, PART 2: only the
// others (the general launch runs both: the large-stage path's unrolled
// products need registers the small-stage path would pay for in occupancy).
template <int SN, int SM, bool DG, int PART>
__global__ __launch_bounds__(64) void k_residual(ResidualArgs a) {
  const double* dd = DG ? a.dd : nullptr;
  __shared__ double sv[32];
  // two distinct staging arrays: a direct global-to-LDS copy into one never
  // aliases the reads of the other, so no wait is inserted before the reads
  __shared__ __align__(16) double stgA[STG_MAX];
  __shared__ __align__(16) double stgB[STG_MAX];
  const int lane = threadIdx.x, col = lane & 15, grp = lane >> 4;
  for (int64_t g = blockIdx.x; g < a.nchunks; g += gridDim.x) {
    const ResChunk ch = a.chunks[g];
    const int b = ch.inst;
    if (a.run && !a.run[b]) continue;
    if (a.skip && a.skip[b]) continue;
    if (a.info && a.info[b].singular) continue;
    const InstMeta mt = a.meta[b];
    const int n = SN > 0 ? SN : mt.n, m = SN > 0 ? SM : mt.m;
    if ((PART == 1 && n + m > 16) || (PART == 2 && n + m <= 16)) continue;
    const double delta = DG ? 0.0 : a.delta[b];
    double rmax = 0.0, bmax = 0.0;
    if (PART != 2 && n + m <= 16) {
      int iH[4], iAB[4], iABT[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = 4 * grp + v;
        iH[v] = stg_hess(j, col, n, m);
        iAB[v] = stg_ab(j, col, n, m);
        iABT[v] = stg_ab(col, j, n, m);
      }
      const int oZ = 2 * n * n + 2 * n * m + m * m;
      const int iend = min(ch.i1, mt.N);  // stage slots i < N
      __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): earlier reads of the staging arrays returned
      wave_sync();
      if (lane == 0) {
        stgA[oZ] = 0.0;
        stgB[oZ] = 0.0;
      }
      ResVec v0, v1;
      if (ch.i0 < iend) {
        res_stage_dma(a, mt, n, m, ch.i0, stgA, lane);
        res_load_vec(a, mt, n, m, ch.i0, lane, delta, dd, v0);
      }
      for (int i = ch.i0; i < iend; i += 2) {
        wait_vmem();
        wave_sync();
        if (i + 1 < iend) {
          res_stage_dma(a, mt, n, m, i + 1, stgB, lane);
          res_load_vec(a, mt, n, m, i + 1, lane, delta, dd, v1);
        }
        res_compute(a, mt, n, m, delta, dd, i, stgA, iH, iAB, iABT, v0, sv, rmax, bmax, lane);
        if (i + 1 >= iend) break;
        __builtin_amdgcn_s_waitcnt(0xc07f);  // reads of stgA returned before it is refilled
        wait_vmem();
        wave_sync();
        if (i + 2 < iend) {
          res_stage_dma(a, mt, n, m, i + 2, stgA, lane);
          res_load_vec(a, mt, n, m, i + 2, lane, delta, dd, v0);
        }
        res_compute(a, mt, n, m, delta, dd, i + 1, stgB, iH, iAB, iABT, v1, sv, rmax, bmax, lane);
        __builtin_amdgcn_s_waitcnt(0xc07f);  // reads of stgB returned before it is refilled
      }
      if (ch.i1 > mt.N) res_terminal(a, mt, n, m, delta, dd, sv, rmax, bmax, lane);
    } else if (PART != 1) {
      residual_chunk_rows(a, mt, b, ch.i0, ch.i1, dd, rmax, bmax, lane);
      if (ch.i1 > mt.N) residual_slot_rows(a, mt, b, mt.N, dd, rmax, bmax, lane);  // terminal rows
    }
    rmax = wave_max(rmax);
    bmax = wave_max(bmax);
    if (lane == 0) {
      atomic_max_nonneg(a.resmax + b, rmax);
      atomic_max_nonneg(a.bmax + b, bmax);
    }
  }
}

// Per-instance relative residual, convergence flag and status.
// Non-final pass: conv = (rel <= tol), lastrel = rel, resmax cleared for the
// next accumulation. Final pass: status from lastrel in priority SINGULAR,
// NOT_CONVERGED, NOT_PD. Plain: relres = resmax / bmax only.
__global__ void k_check(CheckArgs a) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.batch) return;
  if (a.run && !a.run[b]) return;
  const double rm = __longlong_as_double((long long)a.resmax[b]);
  const double bm = __longlong_as_double((long long)a.bmax[b]);
  if (a.plain) {
    a.relres[b] = rm / fmax(bm, 1e-300);
    return;
  }
  const FactorInfo fi = a.info[b];
  // a non-finite right-hand side (||b|| is NaN or Inf) or a non-finite pivot
  const bool nonfinite_in = fi.nonfinite || !(bm <= 1.7976931348623157e308);
  if (!a.final_pass) {
    if (fi.singular || nonfinite_in) {
      a.conv[b] = 1;
      a.lastrel[b] = __builtin_nan("");
    } else {
      const double rel = rm / fmax(bm, 1e-300);
      a.conv[b] = (rel <= a.tol) ? 1 : 0;
      a.lastrel[b] = rel;
    }
    a.resmax[b] = 0ull;
    return;
  }
  const double rel = a.lastrel[b];
  if (a.relres) a.relres[b] = rel;
  if (a.status) {
    int st = RLQR_INST_OK;
    // a residual that is NaN or Inf with finite data and nonzero pivots:
    // a non-finite value arose in the recursion itself
    if (nonfinite_in || (!fi.singular && !(fabs(rel) <= 1.7976931348623157e308))) st = RLQR_INST_NONFINITE;
    else if (fi.singular) st = RLQR_INST_SINGULAR;
    else if (!(rel <= a.tol)) st = RLQR_INST_NOT_CONVERGED;
    else if (!fi.verdict) st = RLQR_INST_NOT_PD;
    a.status[b] = st;
  }
}

// Flag bookkeeping between launches (see MaskArgs::kind).
__global__ void k_masks(MaskArgs a) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.batch) return;
  if (a.kind == 0) {
    const int c = a.conv[b], f = a.flag64[b];
    a.run32[b] = (!f && !c) ? 1 : 0;
    a.run64[b] = (f && !c) ? 1 : 0;
    a.runres[b] = (!c) ? 1 : 0;
  } else if (a.kind == 1) {
    if (a.skip && a.skip[b]) return;  // left out of this factorization: keeps its path
    const FactorInfo fi = a.info[b];
    const bool fp64_only = a.pref32 && !a.pref32[b];
    const bool guard = fi.singular || !(fi.minrel >= a.guard) || (a.bad && a.bad[b]);
    a.flag64[b] = (fp64_only || guard) ? 1 : 0;
    if (a.path) a.path[b] = fp64_only ? RLQR_PATH_FP64 : (guard ? RLQR_PATH_FP64_GUARD : RLQR_PATH_FP32);
  } else if (a.kind == 2) {
    const int f = (!a.flag64[b] && a.status[b] == RLQR_INST_NOT_CONVERGED && !(a.skip && a.skip[b])) ? 1 : 0;
    a.fb[b] = f;
    if (f) {
      a.flag64[b] = 1;
      a.conv[b] = 0;
      if (a.path) a.path[b] = RLQR_PATH_FP64_REDO;
    }
  } else if (a.kind == 3) {
    a.run64[b] = (a.fb[b] && !a.conv[b]) ? 1 : 0;
  } else if (a.kind == 5) {
    a.out[b] = (!a.skip[b] && (a.in == nullptr || a.in[b])) ? 1 : 0;
  } else if (a.kind == 6) {
    a.conv[b] = a.skip[b] ? 1 : 0;
  } else {
    a.run1[b] = (a.run32[b] && !a.multi[b]) ? 1 : 0;
  }
}

// Per-instance certificate from its segments (global segment order). The
// first failing pivot in elimination order has the largest code.
__global__ void k_merge_stats(MergeArgs a) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.batch) return;
  if (a.run && !a.run[b]) return;
  int first_bad = -1, nzero = 0, nonfinite = 0;
  long long npos = 0, nneg = 0;
  double minrel = 1.0e300;
  for (int s = a.seg_off[b]; s < a.seg_off[b + 1]; ++s) {
    const SegStats st = a.stats[s];
    first_bad = max(first_bad, st.first_bad);
    nonfinite |= st.nonfinite;
    nzero += st.nzero;
    npos += st.npos;
    nneg += st.nneg;
    minrel = fmin(minrel, st.minrel);
  }
  const InstMeta mt = a.meta[b];
  FactorInfo fi;
  fi.verdict = first_bad < 0 ? 1 : 0;
  fi.first_bad = first_bad;
  fi.singular = nzero > 0 ? 1 : 0;
  fi.nonfinite = nonfinite ? 1 : 0;
  fi.npos = npos;
  fi.nneg = nneg + (long long)(mt.N + 1) * mt.n;
  fi.nzero = nzero;
  fi.minrel = minrel;
  a.info[b] = fi;
}

hipError_t launch_merge(const MergeArgs& a, hipStream_t st) {
  if (a.batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_merge_stats, dim3((a.batch + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

__global__ void k_inertia(InertiaArgs a) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.batch) return;
  const FactorInfo fi = a.info[b];
  if (a.verdict) a.verdict[b] = fi.verdict;
  if (a.first_bad) a.first_bad[b] = fi.first_bad;
  if (a.inertia) {
    a.inertia[3 * b + 0] = fi.npos;
    a.inertia[3 * b + 1] = fi.nneg;
    a.inertia[3 * b + 2] = fi.nzero;
  }
}

__global__ void k_fill_u64(unsigned long long* p, int count, unsigned long long v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}
__global__ void k_fill_i32(int32_t* p, int count, int32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

// ------------------------------------------------------------------ launchers

template <typename TG, int SN, int SM, bool DG = false>
static hipError_t launch_factor_t(const FactorArgs& a, int nblocks, hipStream_t st) {
  hipLaunchKernelGGL((k_factor16<TG, SN, SM, DG>), dim3(nblocks), dim3(64), 0, st, a);
  return hipGetLastError();
}
template <typename TG>
static hipError_t launch_factor_s(const FactorArgs& a, int nblocks, int shape, hipStream_t st) {
  if (a.dd) {  // per-stage diagonal Delta_i
    switch (shape) {
      case SHAPE_4_1: return launch_factor_t<TG, 4, 1, true>(a, nblocks, st);
      case SHAPE_8_2: return launch_factor_t<TG, 8, 2, true>(a, nblocks, st);
      case SHAPE_12_4: return launch_factor_t<TG, 12, 4, true>(a, nblocks, st);
      default: return launch_factor_t<TG, 0, 0, true>(a, nblocks, st);
    }
  }
  switch (shape) {
    case SHAPE_4_1: return launch_factor_t<TG, 4, 1>(a, nblocks, st);
    case SHAPE_8_2: return launch_factor_t<TG, 8, 2>(a, nblocks, st);
    case SHAPE_12_4: return launch_factor_t<TG, 12, 4>(a, nblocks, st);
    default: return launch_factor_t<TG, 0, 0>(a, nblocks, st);
  }
}
hipError_t launch_factor(const FactorArgs& a, int nblocks, bool fp32_products, int shape, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  return fp32_products ? launch_factor_s<float>(a, nblocks, shape, st) : launch_factor_s<double>(a, nblocks, shape, st);
}

// fewer instances than SIMDs: the register-rich build of the generic shape
constexpr int SOLVE16_FEW = 1024;
template <typename TG, int SN, int SM, bool DG = false>
static hipError_t launch_solve_t(const SolveArgs& a, int nblocks, hipStream_t st) {
  if (SN == 0 && nblocks < SOLVE16_FEW) {
    if (a.corr)
      hipLaunchKernelGGL((k_solve16<TG, SN, SM, true, DG, 1>), dim3(nblocks), dim3(64), 0, st, a);
    else
      hipLaunchKernelGGL((k_solve16<TG, SN, SM, false, DG, 1>), dim3(nblocks), dim3(64), 0, st, a);
    return hipGetLastError();
  }
  if (a.corr)
    hipLaunchKernelGGL((k_solve16<TG, SN, SM, true, DG>), dim3(nblocks), dim3(64), 0, st, a);
  else
    hipLaunchKernelGGL((k_solve16<TG, SN, SM, false, DG>), dim3(nblocks), dim3(64), 0, st, a);
  return hipGetLastError();
}
template <typename TG>
static hipError_t launch_solve_s(const SolveArgs& a, int nblocks, int shape, hipStream_t st) {
  if (a.dd) {  // per-stage diagonal Delta_i
    switch (shape) {
      case SHAPE_4_1: return launch_solve_t<TG, 4, 1, true>(a, nblocks, st);
      case SHAPE_8_2: return launch_solve_t<TG, 8, 2, true>(a, nblocks, st);
      case SHAPE_12_4: return launch_solve_t<TG, 12, 4, true>(a, nblocks, st);
      default: return launch_solve_t<TG, 0, 0, true>(a, nblocks, st);
    }
  }
  switch (shape) {
    case SHAPE_4_1: return launch_solve_t<TG, 4, 1>(a, nblocks, st);
    case SHAPE_8_2: return launch_solve_t<TG, 8, 2>(a, nblocks, st);
    case SHAPE_12_4: return launch_solve_t<TG, 12, 4>(a, nblocks, st);
    default: return launch_solve_t<TG, 0, 0>(a, nblocks, st);
  }
}
hipError_t launch_solve(const SolveArgs& a, int nblocks, bool fp32_tiles, int shape, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  return fp32_tiles ? launch_solve_s<float>(a, nblocks, shape, st) : launch_solve_s<double>(a, nblocks, shape, st);
}

hipError_t launch_residual(const ResidualArgs& a, int shape, hipStream_t st) {
  if (a.nchunks <= 0) return hipSuccess;
  const dim3 grid((unsigned)(a.nchunks < (1 << 20) ? a.nchunks : (1 << 20)));
  if (a.dd) {
    if (shape != SHAPE_LARGE) hipLaunchKernelGGL((k_residual<0, 0, true, 1>), grid, dim3(64), 0, st, a);
    hipLaunchKernelGGL((k_residual<0, 0, true, 2>), grid, dim3(64), 0, st, a);
    return hipGetLastError();
  }
  switch (shape) {
    case SHAPE_LARGE: hipLaunchKernelGGL((k_residual<0, 0, false, 2>), grid, dim3(64), 0, st, a); break;
    case SHAPE_4_1: hipLaunchKernelGGL((k_residual<4, 1, false, 1>), grid, dim3(64), 0, st, a); break;
    case SHAPE_8_2: hipLaunchKernelGGL((k_residual<8, 2, false, 1>), grid, dim3(64), 0, st, a); break;
    case SHAPE_12_4: hipLaunchKernelGGL((k_residual<12, 4, false, 1>), grid, dim3(64), 0, st, a); break;
    default:
      hipLaunchKernelGGL((k_residual<0, 0, false, 1>), grid, dim3(64), 0, st, a);
      hipLaunchKernelGGL((k_residual<0, 0, false, 2>), grid, dim3(64), 0, st, a);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_check(const CheckArgs& a, hipStream_t st) {
  if (a.batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_check, dim3((a.batch + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_inertia(const InertiaArgs& a, hipStream_t st) {
  if (a.batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_inertia, dim3((a.batch + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_masks(const MaskArgs& a, hipStream_t st) {
  if (a.batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_masks, dim3((a.batch + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int count, int32_t v, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3((count + 255) / 256), dim3(256), 0, st, p, count, v);
  return hipGetLastError();
}

}  // namespace rlqr
