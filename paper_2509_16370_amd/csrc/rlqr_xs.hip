// rlqr_xs.hip -- cross-stage variables: the arrowhead Newton step of Section
// "Cross-Stage Variables" (eqs. cross-stage-kkt, cross-stage-schur).
//
// Built on the public LQR calls (rlqr_factor, rlqr_solve_multi, rlqr_solve,
// rlqr_residual, rlqr_pivot_inertia): one factorization of K serves the p
// column solves K^{-1} J and every later solve. What is added here is
// HBM-bound vector work over each instance's rows plus p x p algebra:
//   k_xs_dots   J^T Y over work units of up to XS_CHUNK rows (partial sums
//               per unit, summed in unit order by k_xs_small: deterministic);
//   k_xs_small  one wavefront per instance: S = H - J^T K^{-1} J and its
//               LDL^T, the p x p solve for dtheta, the theta rows of the
//               residual and the convergence test;
//   k_xs_elem   dw = s + V dtheta, r_w + J theta, the scatter of the LQR
//               residual into right-hand-side layout, inf-norms.
// Sign convention: rlqr_solve(v) returns z with K z = -v, so with
// Vs_j = rlqr_solve(J_j) = -K^{-1} J_j the Schur complement is S = H + J^T Vs,
// and for a right-hand side b = (b_w, b_theta) (system A d = -b) with
// s = rlqr_solve(b_w): t = b_theta + J^T s, dtheta = -S^{-1} t,
// dw = s + Vs dtheta. Checked: K dw + J dtheta = -b_w and
// J^T dw + H dtheta = J^T s + S dtheta = -b_theta.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "../../include/rlqr_xs.h"
#include "rlqr_internal.h"

namespace {

#define XS_HIP(expr)                         \
  do {                                       \
    if ((expr) != hipSuccess) return RLQR_E_HIP; \
  } while (0)
#define XS_CALL(expr)                        \
  do {                                       \
    rlqr_status s_ = (expr);                 \
    if (s_ != RLQR_OK) return s_;            \
  } while (0)

constexpr int XS_THREADS = 256;
constexpr int XS_CHUNK = 8192;  // rows per work unit

// One work unit: rows [start, start + len) of array arr of instance b
// (arr 0: q / x rows, 1: r / u rows, 2: c / y rows, 3: LQR residual rows).
struct XChunk {
  int32_t b, arr, start, len;
};
struct XInst {
  int32_t N, n, m, pad;
  int64_t o[4];  // first element of the instance in q, r, c and residual arrays
};
struct Vec3 {
  const double* a[3];
};
struct MVec3 {
  double* a[3];
};

struct DotArgs {
  const XChunk* ch;
  const XInst* inst;
  Vec3 J, Y;        // J: p stacked columns; Y: NY stacked columns
  int64_t L[3];     // column stride of each array (batch length)
  double* part;     // [unit][P][NY]
};

// Element k of a 3- or 4-entry argument array by selects (a dynamic index
// would copy the array to private memory).
template <class T>
__device__ inline T pick3(const T* v, int k) { return k == 0 ? v[0] : (k == 1 ? v[1] : v[2]); }

// NaN-propagating maximum of non-negative values (a NaN residual must not
// read as converged).
__device__ inline double nmax(double a, double b) { return (b > a || b != b) ? b : a; }

__device__ inline double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ inline double wave_nmax(double v) {
  for (int off = 32; off > 0; off >>= 1) v = nmax(v, __shfl_xor(v, off, 64));
  return v;
}

// J_i . Y_j over one work unit, i < P, j < NY.
template <int P, int NY>
__global__ __launch_bounds__(XS_THREADS) void k_xs_dots(DotArgs a) {
  const XChunk c = a.ch[blockIdx.x];
  const XInst in = a.inst[c.b];
  const int64_t base = pick3(in.o, c.arr) + c.start;
  const int64_t L = pick3(a.L, c.arr);
  const double* ja = pick3(a.J.a, c.arr) + base;
  const double* ya = pick3(a.Y.a, c.arr) + base;
  double acc[P][NY];
#pragma unroll
  for (int i = 0; i < P; ++i)
#pragma unroll
    for (int j = 0; j < NY; ++j) acc[i][j] = 0.0;
  for (int e = threadIdx.x; e < c.len; e += XS_THREADS) {
    double jv[P], yv[NY];
#pragma unroll
    for (int i = 0; i < P; ++i) jv[i] = ja[i * L + e];
#pragma unroll
    for (int j = 0; j < NY; ++j) yv[j] = ya[j * L + e];
#pragma unroll
    for (int i = 0; i < P; ++i)
#pragma unroll
      for (int j = 0; j < NY; ++j) acc[i][j] = fma(jv[i], yv[j], acc[i][j]);
  }
  __shared__ double red[XS_THREADS / 64][P * NY];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < P; ++i)
#pragma unroll
    for (int j = 0; j < NY; ++j) {
      const double v = wave_sum(acc[i][j]);
      if (lane == 0) red[w][i * NY + j] = v;
    }
  __syncthreads();
  if (threadIdx.x < P * NY) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < XS_THREADS / 64; ++k) s += red[k][threadIdx.x];
    a.part[(int64_t)blockIdx.x * (P * NY) + threadIdx.x] = s;
  }
}

enum { EL_MAXABS = 0, EL_UPDATE = 1, EL_RHS = 2, EL_SCATTER = 3 };

struct ElemArgs {
  int mode, p, first;
  const XChunk* ch;
  const XInst* inst;
  int64_t L[3];
  Vec3 src;                  // MAXABS: r_w; UPDATE: s; RHS: r_w
  Vec3 cols;                 // UPDATE: Vs; RHS: J
  const double* coef;        // [B][p] UPDATE: this pass's dtheta; RHS: theta
  MVec3 dst;                 // UPDATE: dw; RHS: r_w + J theta; SCATTER: residual in rhs layout
  const double* res;         // SCATTER: LQR residual
  const int32_t* skip;       // [B] UPDATE (not first): converged, left unchanged
  unsigned long long* amax;  // [B] MAXABS, SCATTER: inf-norm (bits of a non-negative double)
};

__global__ __launch_bounds__(XS_THREADS) void k_xs_elem(ElemArgs a) {
  const XChunk c = a.ch[blockIdx.x];
  const XInst in = a.inst[c.b];
  double mx = 0.0;
  if (a.mode == EL_SCATTER) {
    // residual order: [x_i-row (n); u_i-row (m)] for i < N, x_N-row, then the
    // N + 1 dual rows, which are the c layout
    const int n = in.n, m = in.m, nm = in.n + in.m;
    const int sN = in.N * nm;
    for (int e = threadIdx.x; e < c.len; e += XS_THREADS) {
      const int t = c.start + e;
      const double v = a.res[in.o[3] + t];
      mx = nmax(mx, fabs(v));
      if (t < sN) {
        const int i = t / nm, k = t - i * nm;
        if (k < n)
          a.dst.a[0][in.o[0] + (int64_t)i * n + k] = v;
        else
          a.dst.a[1][in.o[1] + (int64_t)i * m + (k - n)] = v;
      } else if (t < sN + n) {
        a.dst.a[0][in.o[0] + (int64_t)in.N * n + (t - sN)] = v;
      } else {
        a.dst.a[2][in.o[2] + (t - sN - n)] = v;
      }
    }
  } else {
    if (a.mode == EL_UPDATE && !a.first && a.skip[c.b]) return;  // uniform over the block
    const int64_t base = pick3(in.o, c.arr) + c.start;
    const int64_t L = pick3(a.L, c.arr);
    const double* s = pick3(a.src.a, c.arr) + base;
    if (a.mode == EL_MAXABS) {
      for (int e = threadIdx.x; e < c.len; e += XS_THREADS) mx = nmax(mx, fabs(s[e]));
    } else {
      double co[RLQR_XS_MAX_P];
#pragma unroll
      for (int j = 0; j < RLQR_XS_MAX_P; ++j) co[j] = j < a.p ? a.coef[(int64_t)c.b * a.p + j] : 0.0;
      const double* cl = pick3(a.cols.a, c.arr) + base;
      double* d = pick3(a.dst.a, c.arr) + base;
      const bool acc = a.mode == EL_UPDATE && !a.first;
      for (int e = threadIdx.x; e < c.len; e += XS_THREADS) {
        double v = s[e];
#pragma unroll
        for (int j = 0; j < RLQR_XS_MAX_P; ++j)
          if (j < a.p) v = fma(co[j], cl[j * L + e], v);
        d[e] = acc ? d[e] + v : v;
      }
      return;
    }
  }
  // inf-norm of the unit, merged per instance
  __shared__ double red[XS_THREADS / 64];
  mx = wave_nmax(mx);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int k = 1; k < XS_THREADS / 64; ++k) r = nmax(r, red[k]);
    atomicMax(&a.amax[c.b], (unsigned long long)__double_as_longlong(r));
  }
}

enum { SM_FACTOR = 0, SM_SCHUR = 1, SM_RESID = 2 };

struct SmallArgs {
  int mode, p, ny, first, batch;
  double tol;
  const int32_t* coff;       // [B + 1] dot work units of each instance
  const double* part;        // [unit][p][ny]
  const double* H;           // [B][p][p]
  double* S;                 // [B][p][p]: d on the diagonal, L below
  int32_t* sinfo;            // [B][4]: positive, negative, zero pivots of S; singular
  const int32_t* kst;        // [p][B] statuses of the column solves (FACTOR)
  int32_t* ksing;            // [B] K singular
  const int32_t* kverdict;   // [B] K's certificate
  const double* rth;         // [B][p]
  double* rho;               // [B][p] theta rows of the residual
  double* theta;             // [B][p]
  double* dlt;               // [B][p] this pass's dtheta
  int32_t* conv;             // [B]
  const unsigned long long* wmax;  // [B] |res_w|_inf
  const unsigned long long* bmax;  // [B] |r_w|_inf
  double* relres;            // [B]
  int32_t* status;           // [B]
  int32_t* count;            // unconverged, non-singular instances
};

// One 64-lane workgroup per instance; p <= 8, so p * p <= 64 lanes.
__global__ __launch_bounds__(64) void k_xs_small(SmallArgs a) {
  const int b = blockIdx.x;
  const int p = a.p, ny = a.ny, t = threadIdx.x;
  __shared__ double sm[RLQR_XS_MAX_P * RLQR_XS_MAX_P];
  __shared__ double vec[RLQR_XS_MAX_P];
  // sum of the instance's partial dot products, entry t of [p][ny]
  double dsum = 0.0;
  if (t < p * ny)
    for (int u = a.coff[b]; u < a.coff[b + 1]; ++u) dsum += a.part[(int64_t)u * p * ny + t];
  const double* Hb = a.H + (int64_t)b * p * p;

  if (a.mode == SM_FACTOR) {
    const int i = t / p, j = t - (t / p) * p;
    if (t < p * p) sm[t] = Hb[t] + dsum;
    __syncthreads();
    double v = 0.0;
    if (t < p * p) v = 0.5 * (sm[i * p + j] + sm[j * p + i]);
    __syncthreads();
    if (t < p * p) sm[t] = v;
    __syncthreads();
    double dmax = 0.0;
    for (int k = 0; k < p; ++k) dmax = fmax(dmax, fabs(sm[k * p + k]));
    __syncthreads();
    // right-looking LDL^T without pivoting: after step k, row k holds d_k and
    // the untouched column entries below it
    for (int k = 0; k < p; ++k) {
      const double piv = sm[k * p + k];
      double nv = 0.0;
      const bool upd = t < p * p && i > k && j > k && piv != 0.0;
      if (upd) nv = sm[i * p + j] - sm[i * p + k] * sm[k * p + j] / piv;
      __syncthreads();
      if (upd) sm[i * p + j] = nv;
      __syncthreads();
    }
    if (t < p * p)
      a.S[(int64_t)b * p * p + t] = i > j ? sm[i * p + j] / sm[j * p + j] : (i == j ? sm[t] : 0.0);
    if (t == 0) {
      const double zt = 1.0e3 * p * 2.220446049250313e-16 * dmax;
      int pos = 0, neg = 0, zero = 0, bad = 0;
      for (int k = 0; k < p; ++k) {
        const double d = sm[k * p + k];
        if (!(d == d) || isinf(d)) bad = 1;
        if (fabs(d) <= zt || !(d == d)) ++zero;
        else if (d > 0.0) ++pos;
        else ++neg;
      }
      int32_t* si = a.sinfo + 4 * b;
      si[0] = pos; si[1] = neg; si[2] = zero; si[3] = (zero > 0 || bad) ? 1 : 0;
      int ks = 0;
      for (int c = 0; c < p; ++c) ks |= a.kst[(int64_t)c * a.batch + b] == RLQR_INST_SINGULAR;
      a.ksing[b] = ks;
    }
    return;
  }

  const double* th = a.theta + (int64_t)b * p;
  if (a.mode == SM_SCHUR) {
    // t_i = b_theta_i + (J^T s)_i; dtheta = -S^{-1} t by the stored LDL^T
    if (t < p) vec[t] = (a.first ? a.rth[(int64_t)b * p + t] : a.rho[(int64_t)b * p + t]) + dsum;
    __syncthreads();
    if (t == 0) {
      const double* F = a.S + (int64_t)b * p * p;
      double z[RLQR_XS_MAX_P];
      const bool hold = !a.first && a.conv[b];
      for (int k = 0; k < p; ++k) z[k] = -vec[k];
      for (int k = 0; k < p; ++k)
        for (int r = k + 1; r < p; ++r) z[r] -= F[r * p + k] * z[k];
      for (int k = 0; k < p; ++k) z[k] /= F[k * p + k];
      for (int k = p - 1; k >= 0; --k)
        for (int r = k + 1; r < p; ++r) z[k] -= F[r * p + k] * z[r];
      for (int k = 0; k < p; ++k) {
        const double d = hold ? 0.0 : z[k];
        a.dlt[(int64_t)b * p + k] = d;
        a.theta[(int64_t)b * p + k] = a.first ? d : th[k] + d;
      }
    }
    return;
  }

  // SM_RESID: theta rows J^T dw + H theta + r_theta, relative residual, status
  double rmax = 0.0, tmax = 0.0;
  if (t < p) {
    double r = dsum + a.rth[(int64_t)b * p + t];
    for (int j = 0; j < p; ++j) r += 0.5 * (Hb[t * p + j] + Hb[j * p + t]) * th[j];
    a.rho[(int64_t)b * p + t] = r;
    rmax = fabs(r);
    tmax = fabs(a.rth[(int64_t)b * p + t]);
  }
  rmax = wave_nmax(rmax);
  tmax = wave_nmax(tmax);
  if (t == 0) {
    rmax = nmax(rmax, __longlong_as_double((long long)a.wmax[b]));
    const double bn = nmax(tmax, __longlong_as_double((long long)a.bmax[b]));
    const double rel = bn > 0.0 ? rmax / bn : (rmax > 0.0 ? INFINITY : 0.0);
    const bool ok = rel <= a.tol;
    const int32_t* si = a.sinfo + 4 * b;
    const bool sing = si[3] || a.ksing[b];
    a.conv[b] = ok ? 1 : 0;
    a.relres[b] = rel;
    a.status[b] = sing ? RLQR_INST_SINGULAR
                       : (!ok ? RLQR_INST_NOT_CONVERGED
                              : ((a.kverdict[b] && si[0] == p) ? RLQR_INST_OK : RLQR_INST_NOT_PD));
    if (!ok && !sing) atomicAdd(a.count, 1);
  }
}

struct InertiaXArgs {
  int batch;
  const int32_t* kverdict;
  const int64_t* kin;
  const int32_t* sinfo;
  int p;
  int32_t* verdict;
  int64_t* inertia;
};

__global__ void k_xs_inertia(InertiaXArgs a) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.batch) return;
  const int32_t* si = a.sinfo + 4 * b;
  if (a.verdict) a.verdict[b] = (a.kverdict[b] && si[0] == a.p) ? 1 : 0;
  if (a.inertia)
    for (int k = 0; k < 3; ++k) a.inertia[3 * b + k] = a.kin[3 * b + k] + si[k];
}

__global__ void k_xs_fill(int32_t* p, int64_t count, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

template <int P>
hipError_t launch_dots_p(const DotArgs& a, int units, int ny, hipStream_t st) {
  if (ny == 1)
    hipLaunchKernelGGL((k_xs_dots<P, 1>), dim3(units), dim3(XS_THREADS), 0, st, a);
  else
    hipLaunchKernelGGL((k_xs_dots<P, P>), dim3(units), dim3(XS_THREADS), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_dots(const DotArgs& a, int units, int p, int ny, hipStream_t st) {
  if (units == 0) return hipSuccess;
  switch (p) {
    case 1: return launch_dots_p<1>(a, units, ny, st);
    case 2: return launch_dots_p<2>(a, units, ny, st);
    case 3: return launch_dots_p<3>(a, units, ny, st);
    case 4: return launch_dots_p<4>(a, units, ny, st);
    case 5: return launch_dots_p<5>(a, units, ny, st);
    case 6: return launch_dots_p<6>(a, units, ny, st);
    case 7: return launch_dots_p<7>(a, units, ny, st);
    case 8: return launch_dots_p<8>(a, units, ny, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t fill(int32_t* p, int64_t count, int32_t v, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_xs_fill, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, st, p, count, v);
  return hipGetLastError();
}

}  // namespace

struct rlqr_xs {
  rlqr_handle* h = nullptr;
  int B = 0, p = 0;
  int64_t L[3] = {0, 0, 0}, Lres = 0;
  XInst* inst = nullptr;
  XChunk* dch = nullptr;  // units over the q, r, c rows, instance by instance
  int ndch = 0;
  XChunk* rch = nullptr;  // units over the LQR residual rows
  int nrch = 0;
  int32_t* coff = nullptr;
  double *V[3] = {}, *SA[3] = {}, *W[3] = {}, *C[3] = {};
  double *res = nullptr, *part = nullptr, *S = nullptr, *rho = nullptr, *dlt = nullptr, *relres = nullptr;
  int32_t *sinfo = nullptr, *kst = nullptr, *ksing = nullptr, *kverd = nullptr, *conv = nullptr,
          *count = nullptr, *status = nullptr;
  int64_t* kin = nullptr;
  unsigned long long *wmax = nullptr, *bmax = nullptr;
  int32_t* host_count = nullptr;  // pinned
  size_t bytes = 0;
  bool factored = false;
  rlqr_xs_lhs xl{};
  std::vector<void*> allocs;
};

namespace {

template <class T>
bool xs_alloc(rlqr_xs* x, T** p, size_t count) {
  const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  void* q = nullptr;
  if (hipMalloc(&q, bytes) != hipSuccess) return false;
  x->allocs.push_back(q);
  x->bytes += bytes;
  *p = static_cast<T*>(q);
  return true;
}

void xs_release(rlqr_xs* x) {
  (void)hipDeviceSynchronize();
  for (void* p : x->allocs) (void)hipFree(p);
  if (x->host_count) (void)hipHostFree(x->host_count);
  delete x;
}

DotArgs dot_args(rlqr_xs* x, const rlqr_xs_lhs* xl, const double* const* Y) {
  DotArgs a{};
  a.ch = x->dch; a.inst = x->inst;
  a.J.a[0] = xl->Jq; a.J.a[1] = xl->Jr; a.J.a[2] = xl->Jc;
  for (int k = 0; k < 3; ++k) { a.Y.a[k] = Y[k]; a.L[k] = x->L[k]; }
  a.part = x->part;
  return a;
}

ElemArgs elem_args(rlqr_xs* x, int mode) {
  ElemArgs a{};
  a.mode = mode; a.p = x->p; a.ch = mode == EL_SCATTER ? x->rch : x->dch; a.inst = x->inst;
  for (int k = 0; k < 3; ++k) a.L[k] = x->L[k];
  return a;
}

SmallArgs small_args(rlqr_xs* x, int mode, int ny) {
  SmallArgs a{};
  a.mode = mode; a.p = x->p; a.ny = ny; a.batch = x->B;
  a.coff = x->coff; a.part = x->part; a.H = x->xl.H; a.S = x->S; a.sinfo = x->sinfo;
  a.kst = x->kst; a.ksing = x->ksing; a.kverdict = x->kverd;
  a.rho = x->rho; a.dlt = x->dlt; a.conv = x->conv;
  a.wmax = x->wmax; a.bmax = x->bmax; a.relres = x->relres; a.status = x->status; a.count = x->count;
  return a;
}

hipError_t launch_elem(const ElemArgs& a, int units, hipStream_t st) {
  if (units == 0) return hipSuccess;
  hipLaunchKernelGGL(k_xs_elem, dim3(units), dim3(XS_THREADS), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_small(const SmallArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(k_xs_small, dim3(a.batch), dim3(64), 0, st, a);
  return hipGetLastError();
}

// One Schur-route solve for b = (b_w, b_theta): s = rlqr_solve(b_w) into SA,
// dtheta = -S^{-1}(b_theta + J^T s), dw (+)= s + Vs dtheta.
rlqr_status schur_pass(rlqr_xs* x, const rlqr_rhs* bw, const double* rtheta, rlqr_sol* dw, double* dtheta,
                       bool first, double rel_tol, int32_t max_refine, hipStream_t st) {
  rlqr_sol s{x->SA[0], x->SA[1], x->SA[2]};
  XS_CALL(rlqr_solve(x->h, bw, &s, rel_tol, max_refine, nullptr, nullptr, st));
  const double* Y[3] = {x->SA[0], x->SA[1], x->SA[2]};
  XS_HIP(launch_dots(dot_args(x, &x->xl, Y), x->ndch, x->p, 1, st));
  SmallArgs sa = small_args(x, SM_SCHUR, 1);
  sa.first = first ? 1 : 0; sa.rth = rtheta; sa.theta = dtheta;
  XS_HIP(launch_small(sa, st));
  ElemArgs ea = elem_args(x, EL_UPDATE);
  ea.first = first ? 1 : 0;
  for (int k = 0; k < 3; ++k) { ea.src.a[k] = x->SA[k]; ea.cols.a[k] = x->V[k]; }
  ea.coef = x->dlt;
  ea.dst.a[0] = dw->x; ea.dst.a[1] = dw->u; ea.dst.a[2] = dw->y;
  ea.skip = x->conv;
  XS_HIP(launch_elem(ea, x->ndch, st));
  return RLQR_OK;
}

}  // namespace

extern "C" rlqr_status rlqr_xs_create(rlqr_xs** xp, rlqr_handle* h, int32_t p, size_t* workspace_bytes) {
  if (!xp) return RLQR_E_INVALID;
  *xp = nullptr;
  if (!h || p < 1 || p > RLQR_XS_MAX_P) return RLQR_E_INVALID;
  rlqr_xs* x = new (std::nothrow) rlqr_xs();
  if (!x) return RLQR_E_NOMEM;
  x->h = h; x->p = p;
  const int32_t *N, *n, *m;
  int B = 0;
  rlqr::handle_shapes(h, &B, &N, &n, &m);
  x->B = B;
  std::vector<int64_t> off[4];
  const int arrs[4] = {RLQR_ARR_q, RLQR_ARR_r, RLQR_ARR_c, RLQR_ARR_RES};
  for (int k = 0; k < 4; ++k) {
    off[k].resize(B + 1);
    if (rlqr_layout_offsets(h, arrs[k], off[k].data()) != RLQR_OK) { xs_release(x); return RLQR_E_INVALID; }
  }
  for (int k = 0; k < 3; ++k) x->L[k] = off[k][B];
  x->Lres = off[3][B];
  std::vector<XInst> inst(B);
  std::vector<XChunk> dch, rch;
  std::vector<int32_t> coff(B + 1, 0);
  for (int b = 0; b < B; ++b) {
    inst[b].N = N[b]; inst[b].n = n[b]; inst[b].m = m[b]; inst[b].pad = 0;
    for (int k = 0; k < 4; ++k) inst[b].o[k] = off[k][b];
    for (int k = 0; k < 3; ++k)
      for (int64_t s = 0; s < off[k][b + 1] - off[k][b]; s += XS_CHUNK)
        dch.push_back({b, k, (int32_t)s, (int32_t)std::min<int64_t>(XS_CHUNK, off[k][b + 1] - off[k][b] - s)});
    coff[b + 1] = (int32_t)dch.size();
    for (int64_t s = 0; s < off[3][b + 1] - off[3][b]; s += XS_CHUNK)
      rch.push_back({b, 3, (int32_t)s, (int32_t)std::min<int64_t>(XS_CHUNK, off[3][b + 1] - off[3][b] - s)});
  }
  x->ndch = (int)dch.size();
  x->nrch = (int)rch.size();
  bool ok = xs_alloc(x, &x->inst, B) && xs_alloc(x, &x->dch, dch.size()) && xs_alloc(x, &x->rch, rch.size()) &&
            xs_alloc(x, &x->coff, B + 1) && xs_alloc(x, &x->res, x->Lres) &&
            xs_alloc(x, &x->part, (size_t)x->ndch * p * p) && xs_alloc(x, &x->S, (size_t)B * p * p) &&
            xs_alloc(x, &x->rho, (size_t)B * p) && xs_alloc(x, &x->dlt, (size_t)B * p) &&
            xs_alloc(x, &x->relres, B) && xs_alloc(x, &x->sinfo, (size_t)4 * B) &&
            xs_alloc(x, &x->kst, (size_t)p * B) && xs_alloc(x, &x->ksing, B) && xs_alloc(x, &x->kverd, B) &&
            xs_alloc(x, &x->conv, B) && xs_alloc(x, &x->count, 1) && xs_alloc(x, &x->status, B) &&
            xs_alloc(x, &x->kin, (size_t)3 * B) && xs_alloc(x, &x->wmax, B) && xs_alloc(x, &x->bmax, B);
  for (int k = 0; k < 3 && ok; ++k)
    ok = xs_alloc(x, &x->V[k], (size_t)p * x->L[k]) && xs_alloc(x, &x->SA[k], x->L[k]) &&
         xs_alloc(x, &x->W[k], x->L[k]) && xs_alloc(x, &x->C[k], x->L[k]);
  if (!ok) { xs_release(x); return RLQR_E_NOMEM; }
  if (hipHostMalloc((void**)&x->host_count, sizeof(int32_t), hipHostMallocDefault) != hipSuccess) {
    x->host_count = nullptr;
    xs_release(x);
    return RLQR_E_NOMEM;
  }
  auto up_copy = [](void* dst, const void* src, size_t bytes) {
    return bytes == 0 || hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess;
  };
  bool up = up_copy(x->inst, inst.data(), sizeof(XInst) * B) &&
            up_copy(x->dch, dch.data(), sizeof(XChunk) * dch.size()) &&
            up_copy(x->rch, rch.data(), sizeof(XChunk) * rch.size()) &&
            up_copy(x->coff, coff.data(), sizeof(int32_t) * (B + 1));
  if (!up) { xs_release(x); return RLQR_E_HIP; }
  if (workspace_bytes) *workspace_bytes = x->bytes;
  *xp = x;
  return RLQR_OK;
}

extern "C" rlqr_status rlqr_xs_factor(rlqr_xs* x, const rlqr_lhs* lhs, const rlqr_xs_lhs* xl, double rel_tol,
                                      int32_t max_refine, rlqr_stream stv) {
  if (!x || !lhs || !xl) return RLQR_E_INVALID;
  if (!(rel_tol >= 0.0) || max_refine < 0) return RLQR_E_INVALID;
  hipStream_t st = (hipStream_t)stv;
  x->factored = false;
  XS_CALL(rlqr_factor(x->h, lhs, stv));
  if (x->B == 0) { x->factored = true; x->xl = *xl; return RLQR_OK; }
  if (!xl->Jq || !xl->Jr || !xl->Jc || !xl->H) return RLQR_E_INVALID;
  x->xl = *xl;
  // Vs_j = rlqr_solve(J_j) = -K^{-1} J_j
  rlqr_rhs J{xl->Jq, xl->Jr, xl->Jc};
  rlqr_sol V{x->V[0], x->V[1], x->V[2]};
  XS_CALL(rlqr_solve_multi(x->h, x->p, &J, &V, rel_tol, max_refine, x->kst, nullptr, stv));
  XS_CALL(rlqr_pivot_inertia(x->h, x->kverd, nullptr, x->kin, stv));
  const double* Y[3] = {x->V[0], x->V[1], x->V[2]};
  XS_HIP(launch_dots(dot_args(x, xl, Y), x->ndch, x->p, x->p, st));
  XS_HIP(launch_small(small_args(x, SM_FACTOR, x->p), st));
  x->factored = true;
  return RLQR_OK;
}

extern "C" rlqr_status rlqr_xs_solve(rlqr_xs* x, const rlqr_rhs* rw, const double* rtheta, rlqr_sol* dw,
                                     double* dtheta, double rel_tol, int32_t max_refine, int32_t* inst_status,
                                     double* inst_relres, rlqr_stream stv) {
  if (!x || !rw || !dw) return RLQR_E_INVALID;
  if (!x->factored) return RLQR_E_STATE;
  if (!(rel_tol >= 0.0) || max_refine < 0) return RLQR_E_INVALID;
  if (x->B == 0) return RLQR_OK;
  if (!rw->q || !rw->r || !rw->c || !rtheta || !dw->x || !dw->u || !dw->y || !dtheta) return RLQR_E_INVALID;
  hipStream_t st = (hipStream_t)stv;
  const int B = x->B;

  XS_HIP(fill(x->conv, B, 0, st));
  XS_HIP(fill(reinterpret_cast<int32_t*>(x->bmax), 2 * (int64_t)B, 0, st));
  ElemArgs mx = elem_args(x, EL_MAXABS);
  mx.src.a[0] = rw->q; mx.src.a[1] = rw->r; mx.src.a[2] = rw->c;
  mx.amax = x->bmax;
  XS_HIP(launch_elem(mx, x->ndch, st));

  XS_CALL(schur_pass(x, rw, rtheta, dw, dtheta, true, rel_tol, max_refine, st));
  for (int pass = 0;; ++pass) {
    // residual of the arrowhead system: res_w = K dw + (r_w + J theta) by the
    // LQR residual, res_theta = J^T dw + H theta + r_theta
    ElemArgs rh = elem_args(x, EL_RHS);
    rh.src.a[0] = rw->q; rh.src.a[1] = rw->r; rh.src.a[2] = rw->c;
    rh.cols.a[0] = x->xl.Jq; rh.cols.a[1] = x->xl.Jr; rh.cols.a[2] = x->xl.Jc;
    rh.coef = dtheta;
    for (int k = 0; k < 3; ++k) rh.dst.a[k] = x->W[k];
    XS_HIP(launch_elem(rh, x->ndch, st));
    rlqr_rhs wr{x->W[0], x->W[1], x->W[2]};
    XS_CALL(rlqr_residual(x->h, &wr, dw, x->res, nullptr, stv));
    XS_HIP(fill(reinterpret_cast<int32_t*>(x->wmax), 2 * (int64_t)B, 0, st));
    XS_HIP(fill(x->count, 1, 0, st));
    ElemArgs sc = elem_args(x, EL_SCATTER);
    sc.res = x->res;
    for (int k = 0; k < 3; ++k) sc.dst.a[k] = x->C[k];
    sc.amax = x->wmax;
    XS_HIP(launch_elem(sc, x->nrch, st));
    const double* Y[3] = {dw->x, dw->u, dw->y};
    XS_HIP(launch_dots(dot_args(x, &x->xl, Y), x->ndch, x->p, 1, st));
    SmallArgs rs = small_args(x, SM_RESID, 1);
    rs.tol = rel_tol; rs.rth = rtheta; rs.theta = dtheta;
    XS_HIP(launch_small(rs, st));
    if (pass >= max_refine) break;
    XS_HIP(hipMemcpyAsync(x->host_count, x->count, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    XS_HIP(hipStreamSynchronize(st));
    if (*x->host_count == 0) break;
    // correction for b = residual (A d = -res): instances already converged keep their values
    rlqr_rhs cr{x->C[0], x->C[1], x->C[2]};
    XS_CALL(schur_pass(x, &cr, x->rho, dw, dtheta, false, rel_tol, max_refine, st));
  }
  if (inst_status) XS_HIP(hipMemcpyAsync(inst_status, x->status, sizeof(int32_t) * B, hipMemcpyDeviceToDevice, st));
  if (inst_relres) XS_HIP(hipMemcpyAsync(inst_relres, x->relres, sizeof(double) * B, hipMemcpyDeviceToDevice, st));
  return RLQR_OK;
}

extern "C" rlqr_status rlqr_xs_inertia(rlqr_xs* x, int32_t* pd_verdict, int64_t* inertia, rlqr_stream stv) {
  if (!x) return RLQR_E_INVALID;
  if (!x->factored) return RLQR_E_STATE;
  if (x->B == 0) return RLQR_OK;
  InertiaXArgs a{};
  a.batch = x->B; a.kverdict = x->kverd; a.kin = x->kin; a.sinfo = x->sinfo; a.p = x->p;
  a.verdict = pd_verdict; a.inertia = inertia;
  hipLaunchKernelGGL(k_xs_inertia, dim3((x->B + 255) / 256), dim3(256), 0, (hipStream_t)stv, a);
  XS_HIP(hipGetLastError());
  return RLQR_OK;
}

extern "C" void rlqr_xs_destroy(rlqr_xs* x) {
  if (x) xs_release(x);
}
