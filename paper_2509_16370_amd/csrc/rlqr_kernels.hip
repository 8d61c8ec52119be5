// rlqr_kernels.hip -- gfx950 kernels of the dual-regularized Riccati solver.
//
// Factor: the backward recursion of Section "Sequential Algorithm"
// (arXiv 2509.16370), one wavefront per instance, 16 x 16 tiles. Per stage k:
//   X   = I + delta P_{k+1}                 sweep all n pivots -> X = -S_hat^{-1}
//   W   = -P_{k+1} X = P S_hat^{-1}         MFMA, then symmetrized
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
  const int c = lane & 15, grp = lane >> 4;
  double s = 0.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = trow<TL>(grp, v);
    if (r == c && r >= lo && r < hi) s = fmax(s, fabs(X[v]));
  }
  return wave_max(s);
}

// ------------------------------------------------------------------ factor

template <typename TG>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_factor16(FactorArgs a) {
  const int b = a.list ? a.list[blockIdx.x] : (int)blockIdx.x;
  if (a.run && !a.run[b]) return;
  const InstMeta mt = a.meta[b];
  const int N = mt.N, n = mt.n, m = mt.m;
  const double delta = a.delta[b];
  const double* __restrict__ Qg = a.Q + mt.oQ;
  const double* __restrict__ Mg = a.M + mt.oM;
  const double* __restrict__ Rg = a.R + mt.oR;
  const double* __restrict__ Ag = a.A + mt.oA;
  const double* __restrict__ Bg = a.B + mt.oB;
  TG* __restrict__ ws = reinterpret_cast<TG*>(a.ws) + mt.ows;  // tiles: Z_i at 2i, X_i at 2i+1

  const int lane = threadIdx.x, col = lane & 15, grp = lane >> 4;
  __shared__ TG sP[NT * LD], sX[NT * LD], sAB[NT * LD];
  __shared__ double sD[NT * LD];
  __shared__ double colbuf[32];

  PivStats ps;
  ps.init();
  const double eps = 2.220446049250313e-16;

  // P_N = Q_N
  double P[4];
  {
    const double* QN = Qg + (int64_t)N * n * n;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = trow<TG>(grp, v);
      const bool in = r < n && col < n;
      const double x = QN[in ? r * n + col : 0];
      P[v] = in ? x : 0.0;
    }
  }
  tile_store(ws + (int64_t)(2 * N) * 256, P, lane);

  double H[4], abn[4], Hn[4];
  if (N > 0) {
    const int k = N - 1;
    double ab[4];
    load_ab_rowmajor(ab, Ag + (int64_t)k * n * n, Bg + (int64_t)k * n * m, n, m, lane);
#pragma unroll
    for (int t = 0; t < 4; ++t) sAB[((lane + 64 * t) >> 4) * LD + ((lane + 64 * t) & 15)] = (TG)ab[t];
    load_hess<TG>(H, Qg + (int64_t)k * n * n, Mg + (int64_t)k * n * m, Rg + (int64_t)k * m * m, n, m, lane);
  }
  __syncthreads();

  for (int k = N - 1; k >= 0; --k) {
    // prefetch the stage blocks of step k-1
    if (k >= 1) {
      load_ab_rowmajor(abn, Ag + (int64_t)(k - 1) * n * n, Bg + (int64_t)(k - 1) * n * m, n, m, lane);
      load_hess<TG>(Hn, Qg + (int64_t)(k - 1) * n * n, Mg + (int64_t)(k - 1) * n * m,
                Rg + (int64_t)(k - 1) * m * m, n, m, lane);
    }
    // X = I + delta P_{k+1}; sweep -> -S_hat_{k+1}^{-1}
    double X[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) X[v] = (trow<TG>(grp, v) == col ? 1.0 : 0.0) + delta * P[v];
    {
      const double sc = diag_scale<TG>(X, 0, n, lane);
      sweep16<TG>(X, 0, n, lane, colbuf, ps, 2 * (k + 1), 1.0e3 * n * eps * sc, sc);
    }
    tile_store(ws + (int64_t)(2 * (k + 1) + 1) * 256, X, lane);
    tile_to_lds<TG>(sP, P, lane);
    tile_to_lds<TG>(sX, X, lane);
    __syncthreads();
    // W = -P X, symmetrized
    double W[4];
    {
      auto acc = gemm16<TG, false>(sP, sX, lane);
      acc_to_regs<TG>(W, acc, -1.0);
    }
    tile_to_lds<TG>(sD, W, lane);
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) W[v] = 0.5 * (W[v] + sD[col * LD + trow<TG>(grp, v)]);
    tile_to_lds<TG>(sP, W, lane);
    __syncthreads();
    // T = W [A B]
    double T[4];
    {
      auto acc = gemm16<TG, false>(sP, sAB, lane);
      acc_to_regs<TG>(T, acc, 1.0);
    }
    tile_to_lds<TG>(sX, T, lane);
    __syncthreads();
    // Z = [A B]^T T + Hess, symmetrized
    double Z[4];
    {
      auto acc = gemm16<TG, true>(sAB, sX, lane);
#pragma unroll
      for (int v = 0; v < 4; ++v) Z[v] = (double)acc[v] + H[v];
    }
    tile_to_lds<TG>(sD, Z, lane);
    __syncthreads();
#pragma unroll
    for (int v = 0; v < 4; ++v) Z[v] = 0.5 * (Z[v] + sD[col * LD + trow<TG>(grp, v)]);
    // sweep the control block: G_k pivots
    {
      const double sc = diag_scale<TG>(Z, n, n + m, lane);
      sweep16<TG>(Z, n, n + m, lane, colbuf, ps, 2 * k + 1, 1.0e3 * m * eps * sc, sc);
    }
    tile_store(ws + (int64_t)(2 * k) * 256, Z, lane);
#pragma unroll
    for (int v = 0; v < 4; ++v) P[v] = (trow<TG>(grp, v) < n && col < n) ? Z[v] : 0.0;
    __syncthreads();
    if (k >= 1) {
#pragma unroll
      for (int t = 0; t < 4; ++t) sAB[((lane + 64 * t) >> 4) * LD + ((lane + 64 * t) & 15)] = (TG)abn[t];
#pragma unroll
      for (int v = 0; v < 4; ++v) H[v] = Hn[v];
      __syncthreads();
    }
  }
  // S_hat_0
  {
    double X[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) X[v] = (trow<TG>(grp, v) == col ? 1.0 : 0.0) + delta * P[v];
    const double sc = diag_scale<TG>(X, 0, n, lane);
    sweep16<TG>(X, 0, n, lane, colbuf, ps, 0, 1.0e3 * n * eps * sc, sc);
    tile_store(ws + (int64_t)1 * 256, X, lane);
  }
  if (lane == 0) {
    FactorInfo fi;
    fi.verdict = (ps.first_bad < 0) ? 1 : 0;
    fi.first_bad = ps.first_bad;
    fi.singular = ps.nzero > 0 ? 1 : 0;
    fi.pad = 0;
    fi.npos = ps.npos;
    fi.nneg = ps.nneg + (int64_t)(N + 1) * n;
    fi.nzero = ps.nzero;
    fi.minrel = ps.minrel;
    a.info[b] = fi;
  }
}

// ------------------------------------------------------------------ solve

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

// LDS ordering inside a one-wavefront workgroup: the LDS unit executes one
// wavefront's instructions in order, so a compiler-level barrier suffices.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// masked vector element load: v[i] if ok else 0. A masked-off lane reads the
// zero below instead (an empty block may sit at the end of an array).
__device__ double g_zero = 0.0;
__device__ __forceinline__ double ld_or0(const double* __restrict__ v, int64_t i, bool ok) {
  const double* p = ok ? v + i : &g_zero;
  const double x = *p;
  return ok ? x : 0.0;
}

// Solve pass. Backward vector pass and forward rollout (see the file header),
// with the float64 residual of Section "Residual Computation" evaluated on the
// fly: at step k the rows of stage k-1 are completed (they need y_k and x_k).
// corr == NULL: solve K z = -b and write z.  corr != NULL: solve for the
// correction with right-hand side corr (the previous residual), add it to z.
// Either way the residual of the resulting z against the original b is
// written to res_out (if set) and its infinity norm and ||b||_inf to
// resmax/bmax.
template <typename TG>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4, 8))) void k_solve16(SolveArgs a) {
  const int b = a.list ? a.list[blockIdx.x] : (int)blockIdx.x;
  const int lane = threadIdx.x, col = lane & 15, grp = lane >> 4;
  if (a.run && !a.run[b]) return;
  const InstMeta mt = a.meta[b];
  const int N = mt.N, n = mt.n, m = mt.m;
  const double delta = a.delta[b];
  const double* __restrict__ Qg = a.Q + mt.oQ;
  const double* __restrict__ Mg = a.M + mt.oM;
  const double* __restrict__ Rg = a.R + mt.oR;
  const double* __restrict__ Ag = a.A + mt.oA;
  const double* __restrict__ Bg = a.B + mt.oB;
  const TG* __restrict__ ws = reinterpret_cast<const TG*>(a.ws) + mt.ows;
  double* __restrict__ pg = a.pk + mt.opk;                        // p_i at i*n
  double* __restrict__ kg = a.pk + mt.opk + (int64_t)(N + 1) * n;  // k_i at i*m
  const double* __restrict__ q0 = a.q + mt.oq;
  const double* __restrict__ r0 = a.r + mt.or_;
  const double* __restrict__ c0 = a.c + mt.oc;
  const double *qb, *rb, *cb;
  int64_t qs, rs;
  if (a.corr) {
    const double* res = a.corr + mt.ores;
    qb = res; qs = n + m;
    rb = res + n; rs = n + m;
    cb = res + (int64_t)N * (n + m) + n;
  } else {
    qb = q0; qs = n;
    rb = r0; rs = m;
    cb = c0;
  }
  double* __restrict__ xg = a.x + mt.ox;
  double* __restrict__ ug = a.u + mt.ou;
  double* __restrict__ yg = a.y + mt.oy;
  double* __restrict__ rg = a.res_out ? a.res_out + mt.ores : nullptr;
  const bool acc = a.corr != nullptr;

  if (a.info[b].singular) {
    if (!acc) {
      const double nanv = __builtin_nan("");
      for (int i = lane; i < (N + 1) * n; i += 64) { xg[i] = nanv; yg[i] = nanv; }
      for (int i = lane; i < N * m; i += 64) ug[i] = nanv;
    }
    return;
  }

  __shared__ double sv[6][16];
  const bool xr = col < n, ur = (col >= n) && (col < n + m);
  const bool own = grp == 0;  // lanes 0..15 write outputs

  // ---- backward vector pass
  double p = ld_or0(qb, (int64_t)N * qs + col, xr);
  if (own && xr) pg[(int64_t)N * n + col] = p;
  double Zp[4];
  tile_load(Zp, ws + (int64_t)(2 * N) * 256, lane);
  for (int k = N - 1; k >= 0; --k) {
    double Zk[4], Xn[4], ab[4];
    tile_load(Zk, ws + (int64_t)(2 * k) * 256, lane);
    tile_load(Xn, ws + (int64_t)(2 * (k + 1) + 1) * 256, lane);
    {
      const double* A = Ag + (int64_t)k * n * n;
      const double* B = Bg + (int64_t)k * n * m;
#pragma unroll
      for (int v = 0; v < 4; ++v) ab[v] = ab_elem(A, B, n, m, trow<TG>(grp, v), col);
    }
    const double ck = ld_or0(cb, (int64_t)(k + 1) * n + col, xr);
    const double qk = ld_or0(qb, (int64_t)k * qs + col, xr);
    const double rk = ld_or0(rb, (int64_t)k * rs + (col - n), ur);
    wave_sync();
    if (own) sv[0][col] = ck;
    wave_sync();
    const double vv = xr ? p + tmatvec<TG>(Zp, sv[0], lane) : 0.0;  // p + P_{k+1} c_{k+1}
    if (own) sv[1][col] = vv;
    wave_sync();
    const double g = -tmatvec<TG>(Xn, sv[1], lane);                  // S_hat^{-1} v
    if (own) sv[2][col] = xr ? g : 0.0;
    wave_sync();
    const double abg = tmatvec<TG>(ab, sv[2], lane);                 // [A^T g; B^T g]
    const double h = ur ? rk + abg : 0.0;
    if (own) sv[3][col] = h;
    wave_sync();
    const double zh = tmatvec<TG>(Zk, sv[3], lane);                  // [-K^T h; -G^{-1} h]
    p = xr ? qk + abg - zh : 0.0;
    if (own) {
      if (xr) pg[(int64_t)k * n + col] = p;
      if (ur) kg[(int64_t)k * m + (col - n)] = zh;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) Zp[v] = Zk[v];
  }
  __syncthreads();  // p/k written by lanes 0..15 are read by all lanes below

  // ---- forward rollout with the fused residual
  double rmax = 0.0, bmax = 0.0;
  double x;  // correction state x_k
  {
    double X0[4];
    tile_load(X0, ws + (int64_t)1 * 256, lane);
    const double p0 = ld_or0(pg, col, xr);
    const double c00 = ld_or0(cb, col, xr);
    wave_sync();
    if (own) sv[0][col] = xr ? c00 - delta * p0 : 0.0;
    wave_sync();
    x = xr ? -tmatvec<TG>(X0, sv[0], lane) : 0.0;
  }
  // totals of the previous stage, kept for its residual rows
  double xtp = 0.0, utp = 0.0, ytp = 0.0, wtp = 0.0, q0p = 0.0, r0p = 0.0;
  double Hp[4] = {0, 0, 0, 0}, abp[4] = {0, 0, 0, 0};
  for (int k = 0; k <= N; ++k) {
    const bool last = (k == N);
    double Zk[4], Xn[4], abt[4], ab[4], Hk[4];
    tile_load(Zk, ws + (int64_t)(2 * k) * 256, lane);
    const int kn = last ? k : k + 1;
    tile_load(Xn, ws + (int64_t)(2 * kn + 1) * 256, lane);
    const int ks = last ? (k > 0 ? k - 1 : 0) : k;  // stage blocks (unused on the last step)
    {
      const double* A = Ag + (int64_t)ks * n * n;
      const double* B = Bg + (int64_t)ks * n * m;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int j = trow<TG>(grp, v);
        abt[v] = (!last && N > 0) ? ab_elem(A, B, n, m, col, j) : 0.0;   // [A B][col][j]
        ab[v] = (!last && N > 0) ? ab_elem(A, B, n, m, j, col) : 0.0;    // [A B][j][col]
      }
      if (!last && N > 0) {
        load_hess<TG>(Hk, Qg + (int64_t)k * n * n, Mg + (int64_t)k * n * m, Rg + (int64_t)k * m * m, n, m, lane);
      } else {
        // terminal block Q_N for the last row group
        const double* QN = Qg + (int64_t)N * n * n;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = trow<TG>(grp, v);
          Hk[v] = ld_or0(QN, r * n + col, r < n && xr);
        }
      }
    }
    const double pk = ld_or0(pg, (int64_t)k * n + col, xr);
    const double kk = ld_or0(kg, (int64_t)k * m + (col - n), ur && !last);
    const double pn = ld_or0(pg, (int64_t)kn * n + col, xr && !last);
    const double cn = ld_or0(cb, (int64_t)kn * n + col, xr && !last);
    const double q0k = ld_or0(q0, (int64_t)k * n + col, xr);
    const double r0k = ld_or0(r0, (int64_t)k * m + (col - n), ur && !last);
    const double c0k = ld_or0(c0, (int64_t)k * n + col, xr);
    const double xold = acc ? ld_or0(xg, (int64_t)k * n + col, xr) : 0.0;
    const double yold = acc ? ld_or0(yg, (int64_t)k * n + col, xr) : 0.0;
    const double uold = acc ? ld_or0(ug, (int64_t)k * m + (col - n), ur && !last) : 0.0;

    // phase A: [P_k x; -K_k x] for the chain, Hess_{k-1} z_{k-1} for the residual
    wave_sync();
    if (own) {
      sv[0][col] = xr ? x : 0.0;
      sv[1][col] = xr ? xtp : (ur ? utp : 0.0);
    }
    wave_sync();
    const double zx = tmatvec<TG>(Zk, sv[0], lane);
    const double h1 = tmatvec<TG>(Hp, sv[1], lane);
    const double yk = xr ? zx + pk : 0.0;
    const double uk = (ur && !last) ? kk - zx : 0.0;
    const double xt = x + xold, yt = yk + yold, ut = uk + uold;
    if (own) {
      if (xr) {
        yg[(int64_t)k * n + col] = yt;
        xg[(int64_t)k * n + col] = xt;
      }
      if (ur && !last) ug[(int64_t)k * m + (col - n)] = ut;
    }
    // phase B: [A B] z for the chain (correction) and for the totals,
    // [A_{k-1} B_{k-1}]^T y_k for the residual of stage k-1
    wave_sync();
    if (own) {
      sv[2][col] = xr ? x : (ur ? uk : 0.0);
      sv[3][col] = xr ? yt : 0.0;
      sv[4][col] = xr ? xt : (ur ? ut : 0.0);
    }
    wave_sync();
    const double w = tmatvec<TG>(abt, sv[2], lane);
    const double h2 = tmatvec<TG>(abp, sv[3], lane);
    const double wt = acc ? tmatvec<TG>(abt, sv[4], lane) : w;
    // residual rows of stage k-1 (x-row, u-row, dynamics row)
    if (k > 0) {
      const double rx = h1 + h2 + q0p - ytp;        // x rows
      const double ru = h1 + h2 + r0p;              // u rows
      const double rd = wtp + c0k - delta * yt - xt;  // dynamics row of step k-1
      if (own) {
        const int64_t base = (int64_t)(k - 1) * (n + m);
        if (xr) {
          if (rg) rg[base + col] = rx;
          if (rg) rg[(int64_t)N * (n + m) + n + (int64_t)k * n + col] = rd;
          rmax = fmax(rmax, fmax(fabs(rx), fabs(rd)));
        }
        if (ur) {
          if (rg) rg[base + col] = ru;
          rmax = fmax(rmax, fabs(ru));
        }
      }
    } else if (own && xr) {  // initial-state row c_0 - delta y_0 - x_0
      const double ri = c0k - delta * yt - xt;
      if (rg) rg[(int64_t)N * (n + m) + n + col] = ri;
      rmax = fmax(rmax, fabs(ri));
    }
    if (own) bmax = fmax(bmax, fmax(fabs(q0k), fmax(fabs(r0k), fabs(c0k))));
    if (last) {
      // terminal row Q_N x_N + q_N - y_N
      wave_sync();
      if (own) sv[5][col] = xr ? xt : 0.0;
      wave_sync();
      const double rt = tmatvec<TG>(Hk, sv[5], lane) + q0k - yt;
      if (own && xr) {
        if (rg) rg[(int64_t)N * (n + m) + col] = rt;
        rmax = fmax(rmax, fabs(rt));
      }
      break;
    }
    // phase C: x_{k+1} = S_hat_{k+1}^{-1}(A x + B u + c_{k+1} - delta p_{k+1})
    wave_sync();
    if (own) sv[0][col] = xr ? w + cn - delta * pn : 0.0;
    wave_sync();
    x = xr ? -tmatvec<TG>(Xn, sv[0], lane) : 0.0;
    // keep this stage for its residual rows
    xtp = xt; utp = ut; ytp = yt; wtp = wt; q0p = q0k; r0p = r0k;
#pragma unroll
    for (int v = 0; v < 4; ++v) { Hp[v] = Hk[v]; abp[v] = ab[v]; }
  }
  rmax = wave_max(rmax);
  bmax = wave_max(bmax);
  if (lane == 0) {
    a.resmax[b] = (unsigned long long)__double_as_longlong(rmax);
    a.bmax[b] = (unsigned long long)__double_as_longlong(bmax);
  }
}

// ------------------------------------------------------------------ residual

__device__ __forceinline__ void atomic_max_nonneg(unsigned long long* p, double v) {
  // non-negative doubles order like their bit patterns
  atomicMax(p, (unsigned long long)__double_as_longlong(v));
}

// One block of 64 lanes per (instance, stage i = 0..N); stage N also covers
// the terminal row and the c_0 row. Rows are spread over the lanes.
__global__ __launch_bounds__(64) void k_residual(ResidualArgs a) {
  const int64_t gblk = blockIdx.x;
  const int b = a.blk_inst[gblk];
  if (a.run && !a.run[b]) return;
  if (a.skip && a.skip[b]) return;
  if (a.info && a.info[b].singular) return;
  const int i = (int)(gblk - a.stage_off[b]);
  const InstMeta mt = a.meta[b];
  const int N = mt.N, n = mt.n, m = mt.m;
  const double delta = a.delta[b];
  const double* Q = a.Q + mt.oQ; const double* M = a.M + mt.oM; const double* R = a.R + mt.oR;
  const double* A = a.A + mt.oA; const double* B = a.B + mt.oB;
  const double* q = a.q + mt.oq; const double* r = a.r + mt.or_; const double* c = a.c + mt.oc;
  const double* x = a.x + mt.ox; const double* u = a.u + mt.ou; const double* y = a.y + mt.oy;
  double* res = a.res ? a.res + mt.ores : nullptr;
  const int nn = n * n, nm = n * m, mm = m * m;
  double rmax = 0.0, bmax = 0.0;
  if (i < N) {
    const double* Qi = Q + (int64_t)i * nn; const double* Mi = M + (int64_t)i * nm;
    const double* Ri = R + (int64_t)i * mm; const double* Ai = A + (int64_t)i * nn;
    const double* Bi = B + (int64_t)i * nm;
    const double* xi = x + (int64_t)i * n; const double* ui = u + (int64_t)i * m;
    const double* yi = y + (int64_t)i * n; const double* yn = y + (int64_t)(i + 1) * n;
    const double* xn = x + (int64_t)(i + 1) * n;
    for (int row = threadIdx.x; row < 2 * n + m; row += 64) {
      double s, bv;
      int64_t out;
      if (row < n) {           // x-row
        const int a0 = row;
        bv = q[(int64_t)i * n + a0];
        s = bv - yi[a0];
        for (int j = 0; j < n; ++j) s += Qi[a0 * n + j] * xi[j];
        for (int j = 0; j < m; ++j) s += Mi[a0 * m + j] * ui[j];
        for (int j = 0; j < n; ++j) s += Ai[j * n + a0] * yn[j];
        out = (int64_t)i * (n + m) + a0;
      } else if (row < n + m) { // u-row
        const int a0 = row - n;
        bv = r[(int64_t)i * m + a0];
        s = bv;
        for (int j = 0; j < n; ++j) s += Mi[j * m + a0] * xi[j];
        for (int j = 0; j < m; ++j) s += Ri[a0 * m + j] * ui[j];
        for (int j = 0; j < n; ++j) s += Bi[j * m + a0] * yn[j];
        out = (int64_t)i * (n + m) + n + a0;
      } else {                  // dynamics row of step i
        const int a0 = row - n - m;
        bv = c[(int64_t)(i + 1) * n + a0];
        s = bv - delta * yn[a0] - xn[a0];
        for (int j = 0; j < n; ++j) s += Ai[a0 * n + j] * xi[j];
        for (int j = 0; j < m; ++j) s += Bi[a0 * m + j] * ui[j];
        out = (int64_t)N * (n + m) + 2 * n + (int64_t)i * n + a0;
      }
      if (res) res[out] = s;
      rmax = fmax(rmax, fabs(s));
      bmax = fmax(bmax, fabs(bv));
    }
  } else {
    const double* QN = Q + (int64_t)N * nn;
    const double* xN = x + (int64_t)N * n; const double* yN = y + (int64_t)N * n;
    for (int row = threadIdx.x; row < 2 * n; row += 64) {
      double s, bv;
      int64_t out;
      if (row < n) {
        bv = q[(int64_t)N * n + row];
        s = bv - yN[row];
        for (int j = 0; j < n; ++j) s += QN[row * n + j] * xN[j];
        out = (int64_t)N * (n + m) + row;
      } else {
        const int a0 = row - n;
        bv = c[a0];
        s = bv - delta * y[a0] - x[a0];
        out = (int64_t)N * (n + m) + n + a0;
      }
      if (res) res[out] = s;
      rmax = fmax(rmax, fabs(s));
      bmax = fmax(bmax, fabs(bv));
    }
  }
  rmax = wave_max(rmax);
  bmax = wave_max(bmax);
  if (threadIdx.x == 0) {
    atomic_max_nonneg(a.resmax + b, rmax);
    atomic_max_nonneg(a.bmax + b, bmax);
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
  if (!a.final_pass) {
    if (fi.singular) {
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
    if (fi.singular) st = RLQR_INST_SINGULAR;
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
    const FactorInfo fi = a.info[b];
    a.flag64[b] = (fi.singular || !(fi.minrel >= a.guard)) ? 1 : 0;
  } else if (a.kind == 2) {
    const int f = (!a.flag64[b] && a.status[b] == RLQR_INST_NOT_CONVERGED) ? 1 : 0;
    a.fb[b] = f;
    if (f) {
      a.flag64[b] = 1;
      a.conv[b] = 0;
    }
  } else {
    a.run64[b] = (a.fb[b] && !a.conv[b]) ? 1 : 0;
  }
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

hipError_t launch_factor(const FactorArgs& a, int nblocks, bool fp32_products, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  if (fp32_products)
    hipLaunchKernelGGL(k_factor16<float>, dim3(nblocks), dim3(64), 0, st, a);
  else
    hipLaunchKernelGGL(k_factor16<double>, dim3(nblocks), dim3(64), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_solve(const SolveArgs& a, int nblocks, bool fp32_tiles, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  if (fp32_tiles)
    hipLaunchKernelGGL(k_solve16<float>, dim3(nblocks), dim3(64), 0, st, a);
  else
    hipLaunchKernelGGL(k_solve16<double>, dim3(nblocks), dim3(64), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_residual(const ResidualArgs& a, int64_t nblocks, hipStream_t st) {
  if (nblocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_residual, dim3((unsigned)nblocks), dim3(64), 0, st, a);
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
