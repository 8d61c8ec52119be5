// rlqr_spd.hip -- general SPD per-stage regularization Delta_i (include/rlqr_spd.h).
//
// Delta_i = L_i D_i L_i^T (unit lower L_i, positive diagonal D_i); the
// congruence x = L x~, y = L^{-T} y~ turns the problem into one with the
// diagonal regularization D_i, which the handle's per-stage diagonal path
// solves in any mode. Kernels (all float64, one workgroup per (instance,
// stage) slot; elementwise over the stage's small matrices, HBM-bound):
//   k_spd_ldl       LDL^T of Delta_i in LDS (one thread per row, two barriers
//                   per column), L_i^{-1} by forward substitution (one thread
//                   per column); writes L_i, L_i^{-1} (n x n) and D_i.
//   k_spd_lhs       Q~ = L^T Q L (upper triangle computed, mirrored: exactly
//                   symmetric), M~ = L^T M, A~ = L_{i+1}^{-1} A L_i,
//                   B~ = L_{i+1}^{-1} B.
//   k_spd_vec       right-hand side (q~ = L^T q, c~ = L^{-1} c, r copied), a
//                   residual mapped the same way (zero for converged
//                   instances), or the back map x = L x~, y = L^{-T} y~.
//   k_spd_residual  the original system's residual with Delta_i y_i, and the
//                   per-instance maxima of |res| and |[s; c]|.
//   k_spd_check     relative residual, convergence flags, final status.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/rlqr_spd.h"
#include "rlqr_internal.h"

namespace rlqr {
namespace {

struct SpdMeta {
  int32_t N, n, m, pad;
  int64_t oQ, oM, oR, oA, oB, oq, or_, oc, ox, ou, oy, ores;
};

struct SpdSlot {
  int32_t b, i;
};

struct SpdArgs {
  const SpdMeta* meta;
  const SpdSlot* slots;
  int64_t nslots;
  // original data
  const double *Q, *M, *R, *A, *B, *Delta;
  const double *q, *r, *c;
  // factors
  double *L, *Li, *D;
  // transformed left-hand side
  double *tQ, *tM, *tA, *tB;
  // vector kernels: input (q, r, c) or residual; output (q, r, c) / (x, u, y)
  const double *vq, *vr, *vc, *vres;
  double *oq, *or_, *oc;
  const double *zx, *zu, *zy;  // back map: transformed solution
  double *x, *u, *y;           // back map / residual: original solution
  int kind, accumulate;
  const int32_t* conv;  // kind 1: converged instances get a zero right-hand side
  // residual
  double* res;
  unsigned long long *rmax, *bmax;
};

__device__ __forceinline__ void atomic_max_abs(unsigned long long* p, double v) {
  // |v| as a non-negative double orders like its bit pattern; NaN (0x7ff8...)
  // sorts above +Inf, so a NaN is kept
  atomicMax(p, (unsigned long long)__double_as_longlong(fabs(v)));
}

template <int NM>
__global__ __launch_bounds__(64) void k_spd_ldl(SpdArgs a) {
  const SpdSlot sl = a.slots[blockIdx.x];
  const SpdMeta mt = a.meta[sl.b];
  const int n = mt.n, t = threadIdx.x;
  __shared__ double S[NM][NM + 1];
  __shared__ double X[NM][NM + 1];
  const int64_t o = mt.oQ + (int64_t)sl.i * n * n;
  const double* __restrict__ Dl = a.Delta + o;
  for (int e = t; e < n * n; e += 64) {
    const int r = e / n, c = e % n;
    S[r][c] = r >= c ? Dl[r * n + c] : Dl[c * n + r];  // the lower triangle, mirrored
  }
  __syncthreads();
  for (int j = 0; j < n; ++j) {
    const double d = S[j][j];
    if (t > j && t < n) S[t][j] = S[t][j] / d;  // l_tj
    __syncthreads();
    if (t > j && t < n) {
      const double ltd = S[t][j] * d;
      for (int c = j + 1; c <= t; ++c) S[t][c] -= ltd * S[c][j];
    }
    __syncthreads();
  }
  // L^{-1} (unit lower): thread t forms column t by forward substitution
  if (t < n) {
    for (int r = 0; r < t; ++r) X[r][t] = 0.0;
    X[t][t] = 1.0;
    for (int r = t + 1; r < n; ++r) {
      double s = 0.0;
      for (int k = t; k < r; ++k) s += S[r][k] * X[k][t];
      X[r][t] = -s;
    }
  }
  __syncthreads();
  double* __restrict__ L = a.L + o;
  double* __restrict__ Li = a.Li + o;
  for (int e = t; e < n * n; e += 64) {
    const int r = e / n, c = e % n;
    L[e] = r > c ? S[r][c] : (r == c ? 1.0 : 0.0);
    Li[e] = X[r][c];
  }
  if (t < n) a.D[mt.ox + (int64_t)sl.i * n + t] = S[t][t];
}

template <int NM>
__global__ __launch_bounds__(256) void k_spd_lhs(SpdArgs a) {
  const SpdSlot sl = a.slots[blockIdx.x];
  const SpdMeta mt = a.meta[sl.b];
  const int n = mt.n, m = mt.m, i = sl.i, N = mt.N, t = threadIdx.x;
  __shared__ double sL[NM][NM + 1], sLi[NM][NM + 1], sT[NM][NM + 1];
  const int64_t o = mt.oQ + (int64_t)i * n * n;
  for (int e = t; e < n * n; e += 256) sL[e / n][e % n] = a.L[o + e];
  if (i < N)
    for (int e = t; e < n * n; e += 256) sLi[e / n][e % n] = a.Li[o + (int64_t)n * n + e];
  __syncthreads();
  // T = Q L (L lower: k >= c)
  const double* __restrict__ Q = a.Q + o;
  for (int e = t; e < n * n; e += 256) {
    const int r = e / n, c = e % n;
    double s = 0.0;
    for (int k = c; k < n; ++k) s += Q[r * n + k] * sL[k][c];
    sT[r][c] = s;
  }
  __syncthreads();
  // Q~ = L^T T, upper triangle, written to both halves
  double* __restrict__ tQ = a.tQ + o;
  for (int e = t; e < n * n; e += 256) {
    const int r = e / n, c = e % n;
    if (r > c) continue;
    double s = 0.0;
    for (int k = r; k < n; ++k) s += sL[k][r] * sT[k][c];
    tQ[r * n + c] = s;
    tQ[c * n + r] = s;
  }
  if (i == N) return;
  // M~ = L^T M
  const int64_t om = mt.oM + (int64_t)i * n * m;
  for (int e = t; e < n * m; e += 256) {
    const int r = e / m, c = e % m;
    double s = 0.0;
    for (int k = r; k < n; ++k) s += sL[k][r] * a.M[om + k * m + c];
    a.tM[om + e] = s;
  }
  // B~ = L_{i+1}^{-1} B (L^{-1} lower: k <= r)
  for (int e = t; e < n * m; e += 256) {
    const int r = e / m, c = e % m;
    double s = 0.0;
    for (int k = 0; k <= r; ++k) s += sLi[r][k] * a.B[om + k * m + c];
    a.tB[om + e] = s;
  }
  __syncthreads();  // sT is rewritten
  const int64_t oa = mt.oA + (int64_t)i * n * n;
  for (int e = t; e < n * n; e += 256) {
    const int r = e / n, c = e % n;
    double s = 0.0;
    for (int k = c; k < n; ++k) s += a.A[oa + r * n + k] * sL[k][c];
    sT[r][c] = s;
  }
  __syncthreads();
  for (int e = t; e < n * n; e += 256) {
    const int r = e / n, c = e % n;
    double s = 0.0;
    for (int k = 0; k <= r; ++k) s += sLi[r][k] * sT[k][c];
    a.tA[oa + e] = s;
  }
}

// kind 0: (q, r, c) -> (L^T q, r, L^{-1} c); kind 1: the same map applied to
// the residual rows (zero for converged instances); kind 2: (x~, u~, y~) ->
// (L x~, u~, L^{-T} y~), added to (x, u, y) when accumulate is set.
__global__ __launch_bounds__(64) void k_spd_vec(SpdArgs a) {
  const SpdSlot sl = a.slots[blockIdx.x];
  const SpdMeta mt = a.meta[sl.b];
  const int n = mt.n, m = mt.m, i = sl.i, N = mt.N, t = threadIdx.x;
  const int64_t o = mt.oQ + (int64_t)i * n * n;
  const double* __restrict__ L = a.L + o;
  const double* __restrict__ Li = a.Li + o;
  const int64_t ox = mt.ox + (int64_t)i * n, ou = mt.ou + (int64_t)i * m;
  if (a.kind == 2) {
    if (t < n) {
      double sx = 0.0, sy = 0.0;
      for (int k = 0; k <= t; ++k) sx += L[t * n + k] * a.zx[ox + k];        // (L x~)_t
      for (int k = t; k < n; ++k) sy += Li[k * n + t] * a.zy[mt.oy + (int64_t)i * n + k];  // (L^{-T} y~)_t
      if (a.accumulate) {
        a.x[ox + t] += sx;
        a.y[mt.oy + (int64_t)i * n + t] += sy;
      } else {
        a.x[ox + t] = sx;
        a.y[mt.oy + (int64_t)i * n + t] = sy;
      }
    }
    if (i < N)
      for (int j = t; j < m; j += 64) {  // m may exceed 64 (n + m <= 96)
        if (a.accumulate) a.u[ou + j] += a.zu[ou + j];
        else a.u[ou + j] = a.zu[ou + j];
      }
    return;
  }
  const bool zero = a.kind == 1 && a.conv[sl.b];
  const double *vq, *vr = nullptr, *vc;
  if (a.kind == 0) {
    vq = a.vq + mt.oq + (int64_t)i * n;
    if (i < N) vr = a.vr + mt.or_ + (int64_t)i * m;
    vc = a.vc + mt.oc + (int64_t)i * n;
  } else {  // residual rows: primal [x_i; u_i] (i < N) or x_N, then dual row i
    const double* res = a.vres + mt.ores;
    vq = res + (int64_t)i * (n + m);
    if (i < N) vr = vq + n;
    vc = res + (int64_t)N * (n + m) + n + (int64_t)i * n;
  }
  if (t < n) {
    double sq = 0.0, sc = 0.0;
    if (!zero) {
      for (int k = t; k < n; ++k) sq += L[k * n + t] * vq[k];  // (L^T q)_t
      for (int k = 0; k <= t; ++k) sc += Li[t * n + k] * vc[k];  // (L^{-1} c)_t
    }
    a.oq[mt.oq + (int64_t)i * n + t] = sq;
    a.oc[mt.oc + (int64_t)i * n + t] = sc;
  }
  if (i < N)
    for (int j = t; j < m; j += 64) a.or_[mt.or_ + (int64_t)i * m + j] = zero ? 0.0 : vr[j];
}

// Residual of the original system (row order of rlqr_residual), stage slot i:
// the primal rows of stage i and the dual row i.
__global__ __launch_bounds__(128) void k_spd_residual(SpdArgs a) {
  const SpdSlot sl = a.slots[blockIdx.x];
  const SpdMeta mt = a.meta[sl.b];
  const int n = mt.n, m = mt.m, i = sl.i, N = mt.N, t = threadIdx.x;
  const int np = i < N ? n + m : n;
  double rmax = 0.0, bmax = 0.0;
  const double* x = a.x + mt.ox;
  const double* u = a.u + mt.ou;
  const double* y = a.y + mt.oy;
  for (int row = t; row < np + n; row += 128) {
    double s;
    if (row < np) {
      if (i < N) {
        const double* Q = a.Q + mt.oQ + (int64_t)i * n * n;
        const double* M = a.M + mt.oM + (int64_t)i * n * m;
        const double* R = a.R + mt.oR + (int64_t)i * m * m;
        const double* A = a.A + mt.oA + (int64_t)i * n * n;
        const double* B = a.B + mt.oB + (int64_t)i * n * m;
        const double* xi = x + (int64_t)i * n;
        const double* ui = u + (int64_t)i * m;
        const double* y1 = y + (int64_t)(i + 1) * n;
        if (row < n) {
          double b = a.q[mt.oq + (int64_t)i * n + row];
          s = b - y[(int64_t)i * n + row];
          for (int k = 0; k < n; ++k) s += Q[row * n + k] * xi[k] + A[k * n + row] * y1[k];
          for (int k = 0; k < m; ++k) s += M[row * m + k] * ui[k];
          bmax = fmax(bmax, fabs(b));
        } else {
          const int j = row - n;
          double b = a.r[mt.or_ + (int64_t)i * m + j];
          s = b;
          for (int k = 0; k < n; ++k) s += M[k * m + j] * xi[k] + B[k * m + j] * y1[k];
          for (int k = 0; k < m; ++k) s += R[j * m + k] * ui[k];
          bmax = fmax(bmax, fabs(b));
        }
        if (a.res) a.res[mt.ores + (int64_t)i * (n + m) + row] = s;
      } else {
        const double* Q = a.Q + mt.oQ + (int64_t)N * n * n;
        const double* xN = x + (int64_t)N * n;
        double b = a.q[mt.oq + (int64_t)N * n + row];
        s = b - y[(int64_t)N * n + row];
        for (int k = 0; k < n; ++k) s += Q[row * n + k] * xN[k];
        bmax = fmax(bmax, fabs(b));
        if (a.res) a.res[mt.ores + (int64_t)N * (n + m) + row] = s;
      }
    } else {
      const int j = row - np;
      const double* Dl = a.Delta + mt.oQ + (int64_t)i * n * n;
      const double* yi = y + (int64_t)i * n;
      double b = a.c[mt.oc + (int64_t)i * n + j];
      s = b - x[(int64_t)i * n + j];
      for (int k = 0; k < n; ++k) s -= (j >= k ? Dl[j * n + k] : Dl[k * n + j]) * yi[k];  // lower triangle
      if (i > 0) {
        const double* A = a.A + mt.oA + (int64_t)(i - 1) * n * n;
        const double* B = a.B + mt.oB + (int64_t)(i - 1) * n * m;
        const double* xp = x + (int64_t)(i - 1) * n;
        const double* up = u + (int64_t)(i - 1) * m;
        for (int k = 0; k < n; ++k) s += A[j * n + k] * xp[k];
        for (int k = 0; k < m; ++k) s += B[j * m + k] * up[k];
      }
      bmax = fmax(bmax, fabs(b));
      if (a.res) a.res[mt.ores + (int64_t)N * (n + m) + n + (int64_t)i * n + j] = s;
    }
    rmax = (s != s || rmax != rmax) ? __builtin_nan("") : fmax(rmax, fabs(s));
  }
  // per-thread maxima straight to the instance's maxima (small blocks: no reduction tree)
  if (t < np + n) {
    atomic_max_abs(a.rmax + sl.b, rmax);
    atomic_max_abs(a.bmax + sl.b, bmax);
  }
}

struct SpdCheckArgs {
  int batch, final_pass;
  double tol;
  unsigned long long *rmax, *bmax;
  int32_t* conv;
  int32_t* count;           // instances above tol (non-final passes)
  const int32_t* istat;     // status of the transformed problem's solve
  const int32_t* verdict;   // certificate of the transformed factorization
  int32_t* status;
  double* relres;
};

__global__ void k_spd_check(SpdCheckArgs a) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.batch) return;
  const double rm = __longlong_as_double((long long)a.rmax[b]);
  const double bm = __longlong_as_double((long long)a.bmax[b]);
  const double rel = rm / fmax(bm, 1e-300);
  const int is = a.istat[b];
  const bool dead = is == RLQR_INST_SINGULAR || is == RLQR_INST_NONFINITE;
  const bool ok = dead || rel <= a.tol;
  a.conv[b] = ok ? 1 : 0;
  a.rmax[b] = 0ull;
  a.bmax[b] = 0ull;
  if (!a.final_pass) {
    if (!ok) atomicAdd(a.count, 1);
    return;
  }
  if (a.relres) a.relres[b] = rel;
  if (a.status) {
    int st;
    if (dead) st = is;
    else if (!(fabs(rel) <= 1.7976931348623157e308) || !(bm <= 1.7976931348623157e308)) st = RLQR_INST_NONFINITE;
    else if (!(rel <= a.tol)) st = RLQR_INST_NOT_CONVERGED;
    else st = a.verdict[b] ? RLQR_INST_OK : RLQR_INST_NOT_PD;
    a.status[b] = st;
  }
}

template <int NM>
hipError_t launch_ldl_lhs(const SpdArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_spd_ldl<NM>, dim3((unsigned)a.nslots), dim3(64), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_spd_lhs<NM>, dim3((unsigned)a.nslots), dim3(256), 0, st, a);
  return hipGetLastError();
}

}  // namespace
}  // namespace rlqr

using namespace rlqr;

struct rlqr_spd {
  rlqr_handle* h = nullptr;
  int B = 0, nmax = 0;
  int64_t nslots = 0;
  SpdMeta* meta = nullptr;
  SpdSlot* slots = nullptr;
  double *L = nullptr, *Li = nullptr, *D = nullptr;
  double *tQ = nullptr, *tM = nullptr, *tA = nullptr, *tB = nullptr;
  double *tq = nullptr, *tr = nullptr, *tc = nullptr, *tx = nullptr, *tu = nullptr, *ty = nullptr;
  double *res = nullptr, *relres = nullptr;
  unsigned long long *rmax = nullptr, *bmax = nullptr;
  int32_t *conv = nullptr, *istat = nullptr, *verdict = nullptr, *count = nullptr;
  rlqr_lhs lhs{};
  const double* Delta = nullptr;
  bool factored = false;
  size_t bytes = 0;
  std::vector<void*> allocs;
};

namespace {

void spd_release(rlqr_spd* c) {
  if (!c) return;
  (void)hipDeviceSynchronize();
  for (void* p : c->allocs) (void)hipFree(p);
  c->allocs.clear();
}

SpdArgs base_args(const rlqr_spd* c) {
  SpdArgs a{};
  a.meta = c->meta; a.slots = c->slots; a.nslots = c->nslots;
  a.Q = c->lhs.Q; a.M = c->lhs.M; a.R = c->lhs.R; a.A = c->lhs.A; a.B = c->lhs.B; a.Delta = c->Delta;
  a.L = c->L; a.Li = c->Li; a.D = c->D;
  a.tQ = c->tQ; a.tM = c->tM; a.tA = c->tA; a.tB = c->tB;
  a.rmax = c->rmax; a.bmax = c->bmax;
  return a;
}

#define SPD_TRY(x)                \
  do {                            \
    if ((x) != hipSuccess) {      \
      (void)hipGetLastError();    \
      return RLQR_E_HIP;          \
    }                             \
  } while (0)

#define SPD_TRYS(x)                        \
  do {                                     \
    const rlqr_status s_ = (x);            \
    if (s_ != RLQR_OK) return s_;          \
  } while (0)

rlqr_status launch_vec(const rlqr_spd* c, SpdArgs a, hipStream_t st) {
  hipLaunchKernelGGL(k_spd_vec, dim3((unsigned)c->nslots), dim3(64), 0, st, a);
  SPD_TRY(hipGetLastError());
  return RLQR_OK;
}

// original residual at z into c->res (and res_out if given), maxima accumulated
rlqr_status residual_pass(rlqr_spd* c, const rlqr_rhs* rhs, const rlqr_sol* z, double* res_out, hipStream_t st) {
  SpdArgs a = base_args(c);
  a.q = rhs->q; a.r = rhs->r; a.c = rhs->c;
  a.x = z->x; a.u = z->u; a.y = z->y;
  a.res = res_out;
  hipLaunchKernelGGL(k_spd_residual, dim3((unsigned)c->nslots), dim3(128), 0, st, a);
  SPD_TRY(hipGetLastError());
  return RLQR_OK;
}

rlqr_status check_pass(rlqr_spd* c, int final_pass, double tol, int32_t* status, double* relres, hipStream_t st) {
  SpdCheckArgs k{};
  k.batch = c->B; k.final_pass = final_pass; k.tol = tol;
  k.rmax = c->rmax; k.bmax = c->bmax; k.conv = c->conv; k.count = c->count;
  k.istat = c->istat; k.verdict = c->verdict; k.status = status; k.relres = relres ? relres : c->relres;
  hipLaunchKernelGGL(k_spd_check, dim3((c->B + 255) / 256), dim3(256), 0, st, k);
  SPD_TRY(hipGetLastError());
  return RLQR_OK;
}

}  // namespace

extern "C" {

rlqr_status rlqr_spd_create(rlqr_spd** ctx, rlqr_handle* h, size_t* workspace_bytes) {
  if (!ctx) return RLQR_E_INVALID;
  *ctx = nullptr;
  if (!h) return RLQR_E_INVALID;
  int B = 0;
  const int32_t *N = nullptr, *n = nullptr, *m = nullptr;
  handle_shapes(h, &B, &N, &n, &m);
  std::vector<int64_t> off[RLQR_ARR_COUNT];
  for (int k = 0; k < RLQR_ARR_COUNT; ++k) {
    off[k].assign((size_t)B + 1, 0);
    if (rlqr_layout_offsets(h, k, off[k].data()) != RLQR_OK) return RLQR_E_INVALID;
  }
  rlqr_spd* c = new (std::nothrow) rlqr_spd();
  if (!c) return RLQR_E_NOMEM;
  c->h = h;
  c->B = B;
  std::vector<SpdMeta> meta((size_t)B);
  std::vector<SpdSlot> slots;
  for (int b = 0; b < B; ++b) {
    SpdMeta& e = meta[b];
    e.N = N[b]; e.n = n[b]; e.m = m[b]; e.pad = 0;
    e.oQ = off[RLQR_ARR_Q][b]; e.oM = off[RLQR_ARR_M][b]; e.oR = off[RLQR_ARR_R][b];
    e.oA = off[RLQR_ARR_A][b]; e.oB = off[RLQR_ARR_B][b];
    e.oq = off[RLQR_ARR_q][b]; e.or_ = off[RLQR_ARR_r][b]; e.oc = off[RLQR_ARR_c][b];
    e.ox = off[RLQR_ARR_x][b]; e.ou = off[RLQR_ARR_u][b]; e.oy = off[RLQR_ARR_y][b];
    e.ores = off[RLQR_ARR_RES][b];
    c->nmax = std::max(c->nmax, (int)n[b]);
    for (int i = 0; i <= N[b]; ++i) slots.push_back(SpdSlot{b, i});
  }
  c->nslots = (int64_t)slots.size();
  if (c->nslots > (int64_t)INT32_MAX) {
    delete c;
    return RLQR_E_INVALID;
  }
  rlqr_status st = RLQR_OK;
  auto A = [&](void** p, size_t count, size_t elem) {
    if (st != RLQR_OK) return;
    const size_t bytes = std::max<size_t>(count, 1) * elem;
    if (hipMalloc(p, bytes) != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      st = RLQR_E_NOMEM;
      return;
    }
    c->allocs.push_back(*p);
    c->bytes += bytes;
  };
  const size_t nQ = (size_t)off[RLQR_ARR_Q][B], nM = (size_t)off[RLQR_ARR_M][B], nA = (size_t)off[RLQR_ARR_A][B],
               nq = (size_t)off[RLQR_ARR_q][B], nr = (size_t)off[RLQR_ARR_r][B], nc = (size_t)off[RLQR_ARR_c][B],
               nx = (size_t)off[RLQR_ARR_x][B], nu = (size_t)off[RLQR_ARR_u][B], ny = (size_t)off[RLQR_ARR_y][B],
               nres = (size_t)off[RLQR_ARR_RES][B];
  A((void**)&c->meta, (size_t)B, sizeof(SpdMeta));
  A((void**)&c->slots, slots.size(), sizeof(SpdSlot));
  A((void**)&c->L, nQ, 8); A((void**)&c->Li, nQ, 8); A((void**)&c->D, nx, 8);
  A((void**)&c->tQ, nQ, 8); A((void**)&c->tM, nM, 8); A((void**)&c->tA, nA, 8); A((void**)&c->tB, nM, 8);
  A((void**)&c->tq, nq, 8); A((void**)&c->tr, nr, 8); A((void**)&c->tc, nc, 8);
  A((void**)&c->tx, nx, 8); A((void**)&c->tu, nu, 8); A((void**)&c->ty, ny, 8);
  A((void**)&c->res, nres, 8);
  A((void**)&c->relres, (size_t)B, 8);
  A((void**)&c->rmax, (size_t)B, 8); A((void**)&c->bmax, (size_t)B, 8);
  A((void**)&c->conv, (size_t)B, 4); A((void**)&c->istat, (size_t)B, 4); A((void**)&c->verdict, (size_t)B, 4);
  A((void**)&c->count, 1, 4);
  if (st == RLQR_OK && B > 0) {
    if (hipMemcpy(c->meta, meta.data(), sizeof(SpdMeta) * meta.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(c->slots, slots.data(), sizeof(SpdSlot) * slots.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(c->rmax, 0, 8 * (size_t)B) != hipSuccess || hipMemset(c->bmax, 0, 8 * (size_t)B) != hipSuccess) {
      (void)hipGetLastError();
      st = RLQR_E_HIP;
    }
  }
  if (st != RLQR_OK) {
    spd_release(c);
    delete c;
    return st;
  }
  if (workspace_bytes) *workspace_bytes = c->bytes;
  *ctx = c;
  return RLQR_OK;
}

rlqr_status rlqr_spd_factor(rlqr_spd* c, const rlqr_lhs* lhs, const double* Delta, rlqr_stream stv) {
  if (!c || !lhs) return RLQR_E_INVALID;
  if (c->B == 0) {
    c->factored = true;
    return RLQR_OK;
  }
  if (!lhs->Q || !lhs->M || !lhs->R || !lhs->A || !lhs->B || !Delta) return RLQR_E_INVALID;
  hipStream_t st = (hipStream_t)stv;
  c->lhs = *lhs;
  c->Delta = Delta;
  c->factored = false;
  SpdArgs a = base_args(c);
  hipError_t e;
  if (c->nmax <= 16) e = launch_ldl_lhs<16>(a, st);
  else if (c->nmax <= 32) e = launch_ldl_lhs<32>(a, st);
  else e = launch_ldl_lhs<64>(a, st);
  SPD_TRY(e);
  rlqr_lhs t{};
  t.Q = c->tQ; t.M = c->tM; t.R = lhs->R; t.A = c->tA; t.B = c->tB;
  t.delta = nullptr;
  t.delta_diag = c->D;
  SPD_TRYS(rlqr_factor(c->h, &t, stv));
  c->factored = true;
  return RLQR_OK;
}

rlqr_status rlqr_spd_residual(rlqr_spd* c, const rlqr_rhs* rhs, const rlqr_sol* z, double* res, double* inst_relres,
                              rlqr_stream stv) {
  if (!c || !rhs || !z) return RLQR_E_INVALID;
  if (!c->factored) return RLQR_E_STATE;
  if (c->B == 0) return RLQR_OK;
  if (!rhs->q || !rhs->r || !rhs->c || !z->x || !z->u || !z->y) return RLQR_E_INVALID;
  hipStream_t st = (hipStream_t)stv;
  SPD_TRYS(residual_pass(c, rhs, z, res, st));
  // relative residual only: the check's status path is not taken (status NULL);
  // istat may hold anything, but dead instances only change conv, not relres
  SpdCheckArgs k{};
  k.batch = c->B; k.final_pass = 1; k.tol = 0.0;
  k.rmax = c->rmax; k.bmax = c->bmax; k.conv = c->conv; k.count = c->count;
  k.istat = c->istat; k.verdict = c->verdict; k.status = nullptr; k.relres = inst_relres ? inst_relres : c->relres;
  hipLaunchKernelGGL(k_spd_check, dim3((c->B + 255) / 256), dim3(256), 0, st, k);
  SPD_TRY(hipGetLastError());
  return RLQR_OK;
}

rlqr_status rlqr_spd_solve(rlqr_spd* c, const rlqr_rhs* rhs, rlqr_sol* out, double rel_tol, int32_t max_refine,
                           int32_t* inst_status, double* inst_relres, rlqr_stream stv) {
  if (!c || !rhs || !out) return RLQR_E_INVALID;
  if (!c->factored) return RLQR_E_STATE;
  if (!(rel_tol >= 0.0) || max_refine < 0) return RLQR_E_INVALID;
  if (c->B == 0) return RLQR_OK;
  if (!rhs->q || !rhs->r || !rhs->c || !out->x || !out->u || !out->y) return RLQR_E_INVALID;
  hipStream_t st = (hipStream_t)stv;
  rlqr_rhs trhs{c->tq, c->tr, c->tc};
  rlqr_sol tsol{c->tx, c->tu, c->ty};
  // transformed right-hand side, solve, back map
  SpdArgs a = base_args(c);
  a.kind = 0;
  a.vq = rhs->q; a.vr = rhs->r; a.vc = rhs->c;
  a.oq = c->tq; a.or_ = c->tr; a.oc = c->tc;
  SPD_TRYS(launch_vec(c, a, st));
  SPD_TRYS(rlqr_solve(c->h, &trhs, &tsol, rel_tol, max_refine, c->istat, nullptr, stv));
  SPD_TRYS(rlqr_pivot_inertia(c->h, c->verdict, nullptr, nullptr, stv));
  a = base_args(c);
  a.kind = 2; a.accumulate = 0;
  a.zx = c->tx; a.zu = c->tu; a.zy = c->ty;
  a.x = out->x; a.u = out->u; a.y = out->y;
  SPD_TRYS(launch_vec(c, a, st));
  for (int pass = 0;; ++pass) {
    SPD_TRYS(residual_pass(c, rhs, out, c->res, st));
    if (pass == max_refine) break;
    SPD_TRY(launch_fill_i32(c->count, 1, 0, st));
    SPD_TRYS(check_pass(c, 0, rel_tol, nullptr, nullptr, st));
    int32_t above = 0;
    SPD_TRY(hipMemcpyAsync(&above, c->count, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    SPD_TRY(hipStreamSynchronize(st));
    if (above == 0) {  // every instance converged: the final check needs the maxima again
      SPD_TRYS(residual_pass(c, rhs, out, c->res, st));
      break;
    }
    // correction: z += T solve(T^T res), converged instances get a zero right-hand side
    a = base_args(c);
    a.kind = 1; a.vres = c->res; a.conv = c->conv;
    a.oq = c->tq; a.or_ = c->tr; a.oc = c->tc;
    SPD_TRYS(launch_vec(c, a, st));
    // a loose inner tolerance: the correction only has to shrink the error,
    // and a float32 handle must not be sent to its float64 redo by it
    SPD_TRYS(rlqr_solve(c->h, &trhs, &tsol, 1e-3, 1, nullptr, nullptr, stv));
    a = base_args(c);
    a.kind = 2; a.accumulate = 1;
    a.zx = c->tx; a.zu = c->tu; a.zy = c->ty;
    a.x = out->x; a.u = out->u; a.y = out->y;
    SPD_TRYS(launch_vec(c, a, st));
  }
  SPD_TRYS(check_pass(c, 1, rel_tol, inst_status, inst_relres, st));
  return RLQR_OK;
}

void rlqr_spd_destroy(rlqr_spd* c) {
  if (!c) return;
  spd_release(c);
  delete c;
}

}  // extern "C"
