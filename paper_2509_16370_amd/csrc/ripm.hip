// ripm.hip -- batched regularized interior-point driver (include/ripm.h).
//
// Every per-stage computation of the interior-point iteration runs here on
// the GPU: model evaluation (dynamics, tanh Jacobians and second
// derivatives, inequalities), assembly of the reduced Newton-KKT system as
// dual-regularized LQR stage blocks, recovery of dz and ds, the fraction to
// the boundary, the merit along the step ladder, the update and the error
// measures. The Newton step itself is rlqr_factor / rlqr_solve.
//
// Layout (instance-major, float64): x [B][N+1][n], u [B][N][m], y [B][N+1][n],
// s, z, ds, dz [B][N+1][ng]; the Newton LQR arrays in the packed layout of
// rlqr.h for a uniform batch. Reductions over stages are done by one
// workgroup per problem in a fixed order, so every decision (step length,
// mu update, convergence) is deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "../../include/ripm.h"

namespace {

constexpr int LADDER = 12;    // step ladder alpha_max 2^-k, k = 0..LADDER-1
constexpr double C1 = 1.0e-4;  // Armijo constant
constexpr int MAXD = 32;      // n + m bound of the driver
constexpr int MAXE = 8;       // stagewise equality rows bound

struct Dims {
  int B, N, n, m, ng;
  int ne;                     // stagewise equality rows E_u u_i = b_i per stage (0: none)
  double dt, wx, wu, wN, xmax, umax, eta;
};

// Problem and iterate pointers handed to every kernel.
struct IpmArgs {
  Dims d;
  const double* model;  // A (n x n), B (n x m), a (2 x n), E_u (ne x m)
  const double *x0, *goal;
  const double* eb;     // [B][N][ne] right-hand sides b_i of the equality rows
  double* ye;           // [B][N][ne] their multipliers
  double *x, *u, *y, *s, *z, *ds, *dz;
  double *mu, *rho, *merit, *slope, *alpha, *err;
  unsigned long long *amax_s, *amax_z;  // fraction-to-boundary steps (bit patterns of positive doubles)
  int32_t *conv, *iters, *fail;
  // Newton LQR arrays (rlqr.h packed layout, uniform shapes) and its solution
  double *Q, *M, *R, *Al, *Bl, *q, *r, *c;
  const double *dx, *du, *dy;
  const int32_t* verdict;
  // LQR instances left out of the factor and solve (rlqr_set_skip):
  // converged problems, and in later inertia-correction rounds also those
  // whose certificate already holds; k_ipm_build skips them too when set
  int32_t* skip;
  const int32_t* build_skip;
};

__device__ __forceinline__ const double* mA(const IpmArgs& a) { return a.model; }
__device__ __forceinline__ const double* mB(const IpmArgs& a) { return a.model + a.d.n * a.d.n; }
__device__ __forceinline__ const double* ma(const IpmArgs& a) { return a.model + a.d.n * a.d.n + a.d.n * a.d.m; }
__device__ __forceinline__ const double* mE(const IpmArgs& a) { return ma(a) + 2 * a.d.n; }

// equality row k of stage i at u: e_k = E_u[k] u - b_k  (Section "Applying
// the regularized IPM to optimal control": stagewise rows other than the
// dynamics, eliminated through their -1/eta block like the dynamics duals)
__device__ __forceinline__ double e_row(const IpmArgs& a, int b, int i, int k, const double* u) {
  const double* E = mE(a) + k * a.d.m;
  double v = 0.0;
  for (int j = 0; j < a.d.m; ++j) v = fma(E[j], u[j], v);
  return v - a.eb[((int64_t)b * a.d.N + i) * a.d.ne + k];
}
// (E_u v)_k
__device__ __forceinline__ double e_lin(const IpmArgs& a, int k, const double* v) {
  const double* E = mE(a) + k * a.d.m;
  double s = 0.0;
  for (int j = 0; j < a.d.m; ++j) s = fma(E[j], v[j], s);
  return s;
}

// inequality row l of stage i at (x, u): rows 0, 1: a_l^T x - xmax; 2..2+m: u - umax; 2+m..: -u - umax
__device__ __forceinline__ double g_row(const IpmArgs& a, int l, const double* x, const double* u) {
  const int n = a.d.n, m = a.d.m;
  if (l < 2) {
    const double* al = ma(a) + l * n;
    double v = 0.0;
    for (int j = 0; j < n; ++j) v = fma(al[j], x[j], v);
    return v - a.d.xmax;
  }
  if (l < 2 + m) return u[l - 2] - a.d.umax;
  return -u[l - 2 - m] - a.d.umax;
}
__device__ __forceinline__ int rows_of(const Dims& d, int i) { return i < d.N ? d.ng : 2; }

// block-wide fixed-order reductions (blockDim.x == 256)
__device__ double block_sum(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}
__device__ double block_max(double v, double* red) {
  const int t = threadIdx.x;
  red[t] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) red[t] = fmax(red[t], red[t + o]);
    __syncthreads();
  }
  const double r = red[0];
  __syncthreads();
  return r;
}

__device__ __forceinline__ void atomic_min_pos(unsigned long long* p, double v) {
  atomicMin(p, (unsigned long long)__double_as_longlong(v));  // positive doubles order like their bits
}

// ---------------------------------------------------------------- start

// Cold or warm starting point (stage i = blockIdx.x, problem b = blockIdx.y).
__global__ void k_ipm_init(IpmArgs a, const double* warm) {
  const Dims d = a.d;
  const int i = blockIdx.x, b = blockIdx.y, t = threadIdx.x;
  const int n = d.n, m = d.m, ng = d.ng;
  double* x = a.x + ((int64_t)b * (d.N + 1) + i) * n;
  double* y = a.y + ((int64_t)b * (d.N + 1) + i) * n;
  double* u = a.u + ((int64_t)b * d.N + i) * m;
  double* s = a.s + ((int64_t)b * (d.N + 1) + i) * ng;
  double* z = a.z + ((int64_t)b * (d.N + 1) + i) * ng;
  const int64_t wstride = (int64_t)(d.N + 1) * n * 2 + (int64_t)d.N * m + (int64_t)(d.N + 1) * ng;
  const double* w = warm ? warm + b * wstride : nullptr;
  for (int k = t; k < n; k += blockDim.x) {
    x[k] = w ? w[(int64_t)i * n + k] : a.x0[(int64_t)b * n + k];
    y[k] = w ? w[(int64_t)(d.N + 1) * n + (int64_t)d.N * m + (int64_t)i * n + k] : 0.0;
  }
  if (i < d.N) {
    for (int k = t; k < m; k += blockDim.x) u[k] = w ? w[(int64_t)(d.N + 1) * n + (int64_t)i * m + k] : 0.0;
    for (int k = t; k < d.ne; k += blockDim.x) a.ye[((int64_t)b * d.N + i) * d.ne + k] = 0.0;
  }
  __syncthreads();
  const double mu0 = 0.1;
  for (int l = t; l < ng; l += blockDim.x) {
    if (l < rows_of(d, i)) {
      const double sl = fmax(-g_row(a, l, x, u), 1.0e-2);
      s[l] = sl;
      z[l] = w ? exp(w[2 * (int64_t)(d.N + 1) * n + (int64_t)d.N * m + (int64_t)i * ng + l]) : mu0 / sl;
    } else {
      s[l] = 1.0;
      z[l] = 0.0;
    }
  }
  if (i == 0 && t == 0) {
    a.rho[b] = 0.0;
    a.iters[b] = 0;
    a.conv[b] = 0;
    a.mu[b] = mu0;  // warm starts overwrite it in k_ipm_errors(mode 0)
  }
}

// ---------------------------------------------------------------- Newton LQR assembly

// Stage blocks of the reduced Newton-KKT system (the dual-regularized LQR):
// Q, M, R = Hessian of L (with the tanh second derivatives weighted by y)
// + G^T Sigma G + rho I, q, r = grad L + G^T Sigma r_z, A_i, B_i = dynamics
// Jacobians, c = constraint values. Sigma = (S Z^{-1} + 1/eta)^{-1},
// r_z = g + mu / z.
__global__ __launch_bounds__(256) void k_ipm_build(IpmArgs a) {
  const Dims d = a.d;
  const int i = blockIdx.x, b = blockIdx.y, t = threadIdx.x;
  if (a.conv[b] || (a.build_skip && a.build_skip[b])) return;
  const int n = d.n, m = d.m, ng = d.ng, N = d.N, nz = n + m;
  const double mu = a.mu[b], rho = a.rho[b];
  __shared__ double xs[MAXD], us[MAXD], yi[MAXD], yn[MAXD], th[MAXD], se[MAXD], wdd[MAXD];
  __shared__ double sig[2 + 2 * MAXD], rz[2 + 2 * MAXD];
  __shared__ double ev[MAXE], yev[MAXE];  // equality residuals and multipliers of the stage
  const double* xg = a.x + ((int64_t)b * (N + 1) + i) * n;
  const double* yg = a.y + (int64_t)b * (N + 1) * n;
  const double* sg = a.s + ((int64_t)b * (N + 1) + i) * ng;
  const double* zg = a.z + ((int64_t)b * (N + 1) + i) * ng;
  for (int k = t; k < n; k += 256) {
    xs[k] = xg[k];
    yi[k] = yg[(int64_t)i * n + k];
    yn[k] = i < N ? yg[(int64_t)(i + 1) * n + k] : 0.0;
  }
  for (int k = t; k < m; k += 256) us[k] = i < N ? a.u[((int64_t)b * N + i) * m + k] : 0.0;
  __syncthreads();
  const double* A = mA(a);
  const double* Bm = mB(a);
  const double* av = ma(a);
  if (t < n && i < N) {
    double v = 0.0;
    for (int j = 0; j < n; ++j) v = fma(A[t * n + j], xs[j], v);
    for (int j = 0; j < m; ++j) v = fma(Bm[t * m + j], us[j], v);
    const double tv = tanh(v), sv = 1.0 - tv * tv;
    th[t] = tv;
    se[t] = sv;
    wdd[t] = d.dt * yn[t] * (-2.0 * tv * sv);
  }
  if (t >= 192 && t < 192 + d.ne && i < N) {
    const int k = t - 192;
    ev[k] = e_row(a, b, i, k, us);
    yev[k] = a.ye[((int64_t)b * N + i) * d.ne + k];
  }
  const int rows = rows_of(d, i);
  for (int l = t; l < 2 + 2 * m; l += 256) {
    if (l < rows) {
      const double sl = sg[l], zl = zg[l];
      sig[l] = 1.0 / (sl / zl + 1.0 / d.eta);
      rz[l] = g_row(a, l, xs, us) + mu / zl;
    } else {
      sig[l] = 0.0;
      rz[l] = 0.0;
    }
  }
  __syncthreads();
  if (i < N) {
    double* Q = a.Q + ((int64_t)b * (N + 1) + i) * n * n;
    double* M = a.M + ((int64_t)b * N + i) * n * m;
    double* R = a.R + ((int64_t)b * N + i) * m * m;
    for (int e = t; e < nz * nz; e += 256) {
      const int rr = e / nz, cc = e % nz;
      if (rr >= n && cc < n) continue;  // M^T part
      double h = 0.0;
      for (int j = 0; j < n; ++j) {
        const double pr = rr < n ? A[j * n + rr] : Bm[j * m + rr - n];
        const double pc = cc < n ? A[j * n + cc] : Bm[j * m + cc - n];
        h = fma(wdd[j] * pr, pc, h);
      }
      if (rr < n && cc < n) {
        double gq = sig[0] * av[rr] * av[cc] + sig[1] * av[n + rr] * av[n + cc];
        Q[rr * n + cc] = (rr == cc ? d.wx + rho : 0.0) + h + gq;
      } else if (rr < n) {
        M[rr * m + (cc - n)] = h;
      } else {
        const int k = rr - n;
        // eliminated equality rows: + eta E_u^T E_u
        double ee = 0.0;
        for (int l = 0; l < d.ne; ++l) ee = fma(mE(a)[l * m + k], mE(a)[l * m + (cc - n)], ee);
        R[k * m + (cc - n)] = (rr == cc ? d.wu + rho + sig[2 + k] + sig[2 + m + k] : 0.0) + h + d.eta * ee;
      }
    }
    double* Al = a.Al + ((int64_t)b * N + i) * n * n;
    double* Bl = a.Bl + ((int64_t)b * N + i) * n * m;
    for (int e = t; e < n * n; e += 256) {
      const int rr = e / n, cc = e % n;
      Al[e] = (rr == cc ? 1.0 : 0.0) + d.dt * se[rr] * A[rr * n + cc];
    }
    for (int e = t; e < n * m; e += 256) {
      const int rr = e / m, cc = e % m;
      Bl[e] = d.dt * se[rr] * Bm[rr * m + cc];
    }
    if (t < n) {
      // grad_x L = wx (x - goal) + (I + dt diag(se) A)^T y_{i+1} - y_i + G_x^T z
      double gx = d.wx * (xs[t] - a.goal[(int64_t)b * n + t]) + yn[t] - yi[t];
      for (int j = 0; j < n; ++j) gx = fma(d.dt * se[j] * yn[j], A[j * n + t], gx);
      gx += av[t] * zg[0] + av[n + t] * zg[1];
      a.q[((int64_t)b * (N + 1) + i) * n + t] = gx + av[t] * sig[0] * rz[0] + av[n + t] * sig[1] * rz[1];
      // c_{i+1} = d(x_i, u_i) - x_{i+1}
      const double xn = a.x[((int64_t)b * (N + 1) + i + 1) * n + t];
      a.c[((int64_t)b * (N + 1) + i + 1) * n + t] = xs[t] + d.dt * th[t] - xn;
      if (i == 0) a.c[(int64_t)b * (N + 1) * n + t] = a.x0[(int64_t)b * n + t] - xs[t];
    } else if (t < n + m) {
      const int k = t - n;
      double gu = d.wu * us[k] + zg[2 + k] - zg[2 + m + k];
      for (int j = 0; j < n; ++j) gu = fma(d.dt * se[j] * yn[j], Bm[j * m + k], gu);
      // E_u^T y_e (gradient of the Lagrangian) + eta E_u^T e (the eliminated rows' right-hand side)
      for (int l = 0; l < d.ne; ++l) gu = fma(mE(a)[l * m + k], yev[l] + d.eta * ev[l], gu);
      a.r[((int64_t)b * N + i) * m + k] = gu + sig[2 + k] * rz[2 + k] - sig[2 + m + k] * rz[2 + m + k];
    }
  } else {
    double* Q = a.Q + ((int64_t)b * (N + 1) + N) * n * n;
    for (int e = t; e < n * n; e += 256) {
      const int rr = e / n, cc = e % n;
      Q[e] = (rr == cc ? d.wN + rho : 0.0) + sig[0] * av[rr] * av[cc] + sig[1] * av[n + rr] * av[n + cc];
    }
    if (t < n) {
      double gx = d.wN * (xs[t] - a.goal[(int64_t)b * n + t]) - yi[t] + av[t] * zg[0] + av[n + t] * zg[1];
      a.q[((int64_t)b * (N + 1) + N) * n + t] = gx + av[t] * sig[0] * rz[0] + av[n + t] * sig[1] * rz[1];
    }
  }
}

// Inertia correction: problems whose certificate failed get rho <- max(1e-8, 10 rho).
__global__ void k_ipm_rho(IpmArgs a) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.d.B || a.conv[b]) return;
  if (!a.verdict[b]) {
    a.rho[b] = fmax(1.0e-8, 10.0 * a.rho[b]);
    atomicAdd(a.fail, 1);
  }
}

// ---------------------------------------------------------------- step recovery

// dz = Sigma (G dx + r_z), ds = -W (dz - mu S^{-1} e + z) = -(s / z)(dz + z) + mu / z,
// and the largest steps keeping s and z inside tau times their distance to 0.
__global__ __launch_bounds__(64) void k_ipm_recover(IpmArgs a) {
  const Dims d = a.d;
  const int i = blockIdx.x, b = blockIdx.y, t = threadIdx.x;
  if (a.conv[b]) return;
  const int n = d.n, m = d.m, ng = d.ng, N = d.N;
  const double mu = a.mu[b], tau = fmax(0.99, 1.0 - mu);
  const double* x = a.x + ((int64_t)b * (N + 1) + i) * n;
  const double* u = a.u + ((int64_t)b * N + i) * m;
  const double* dx = a.dx + ((int64_t)b * (N + 1) + i) * n;
  const double* du = a.du + ((int64_t)b * N + i) * m;
  const int64_t o = ((int64_t)b * (N + 1) + i) * ng;
  double as = 1.0, az = 1.0;
  const int rows = rows_of(d, i);
  for (int l = t; l < ng; l += 64) {
    if (l >= rows) {
      a.ds[o + l] = 0.0;
      a.dz[o + l] = 0.0;
      continue;
    }
    const double sl = a.s[o + l], zl = a.z[o + l];
    const double sg = 1.0 / (sl / zl + 1.0 / d.eta);
    const double rzl = g_row(a, l, x, u) + mu / zl;
    double gdx;
    if (l < 2) {
      const double* al = ma(a) + l * n;
      gdx = 0.0;
      for (int j = 0; j < n; ++j) gdx = fma(al[j], dx[j], gdx);
    } else {
      gdx = l < 2 + m ? du[l - 2] : -du[l - 2 - m];
    }
    const double dzl = sg * (gdx + rzl);
    const double dsl = -(sl / zl) * (dzl + zl) + mu / zl;
    a.ds[o + l] = dsl;
    a.dz[o + l] = dzl;
    if (dsl < 0.0) as = fmin(as, -tau * sl / dsl);
    if (dzl < 0.0) az = fmin(az, -tau * zl / dzl);
  }
  for (int k = 32; k > 0; k >>= 1) {
    as = fmin(as, __shfl_xor(as, k));
    az = fmin(az, __shfl_xor(az, k));
  }
  if (t == 0) {
    atomic_min_pos(a.amax_s + b, as);
    atomic_min_pos(a.amax_z + b, az);
  }
}

// ---------------------------------------------------------------- merit along the ladder

// blockIdx.x = 0: merit and its slope along (dx, du, ds) at the current point;
// blockIdx.x = k + 1: merit at alpha_k = alpha_max 2^-k. One workgroup per
// (problem, trial), stages strided over the threads, fixed-order sums.
__global__ __launch_bounds__(256) void k_ipm_merit(IpmArgs a) {
  const Dims d = a.d;
  const int k = (int)blockIdx.x - 1, b = blockIdx.y, t = threadIdx.x;
  if (a.conv[b]) return;
  const int n = d.n, m = d.m, ng = d.ng, N = d.N;
  __shared__ double red[256];
  const double mu = a.mu[b];
  const double amax = __longlong_as_double((long long)a.amax_s[b]);
  const double al = k < 0 ? 0.0 : ldexp(amax, -k);
  const double* A = mA(a);
  const double* Bm = mB(a);
  const double* goal = a.goal + (int64_t)b * n;
  double mer = 0.0, slope = 0.0;
  double xt[MAXD], ut[MAXD], xn[MAXD];
  for (int i = t; i <= N; i += 256) {
    const double* x = a.x + ((int64_t)b * (N + 1) + i) * n;
    const double* dx = a.dx + ((int64_t)b * (N + 1) + i) * n;
    const double* y = a.y + ((int64_t)b * (N + 1)) * n;
    const int64_t o = ((int64_t)b * (N + 1) + i) * ng;
    for (int j = 0; j < n; ++j) xt[j] = x[j] + al * dx[j];
    if (i < N) {
      const double* u = a.u + ((int64_t)b * N + i) * m;
      const double* du = a.du + ((int64_t)b * N + i) * m;
      for (int j = 0; j < m; ++j) ut[j] = u[j] + al * du[j];
    } else {
      for (int j = 0; j < m; ++j) ut[j] = 0.0;
    }
    // cost
    const double w = i < N ? d.wx : d.wN;
    for (int j = 0; j < n; ++j) {
      const double e = xt[j] - goal[j];
      mer += 0.5 * w * e * e;
      if (k < 0) slope += w * e * dx[j];
    }
    if (i < N)
      for (int j = 0; j < m; ++j) {
        mer += 0.5 * d.wu * ut[j] * ut[j];
        if (k < 0) slope += d.wu * ut[j] * a.du[((int64_t)b * N + i) * m + j];
      }
    // stagewise equality rows: y_e^T e + eta/2 |e|^2
    if (i < N)
      for (int l = 0; l < d.ne; ++l) {
        const double ev = e_row(a, b, i, l, ut);
        const double yv = a.ye[((int64_t)b * N + i) * d.ne + l];
        mer += yv * ev + 0.5 * d.eta * ev * ev;
        if (k < 0) slope += (yv + d.eta * ev) * e_lin(a, l, a.du + ((int64_t)b * N + i) * m);
      }
    // inequalities with slacks
    const int rows = rows_of(d, i);
    for (int l = 0; l < rows; ++l) {
      const double sl = a.s[o + l] + al * a.ds[o + l];
      const double gs = g_row(a, l, xt, ut) + sl;
      const double zl = a.z[o + l];
      mer += -mu * log(sl) + zl * gs + 0.5 * d.eta * gs * gs;
      if (k < 0) {
        double gd;
        if (l < 2) {
          const double* av = ma(a) + l * n;
          gd = 0.0;
          for (int j = 0; j < n; ++j) gd = fma(av[j], dx[j], gd);
        } else {
          const double* du = a.du + ((int64_t)b * N + i) * m;
          gd = l < 2 + m ? du[l - 2] : -du[l - 2 - m];
        }
        const double dsl = a.ds[o + l];
        slope += (zl + d.eta * gs) * (gd + dsl) - mu / sl * dsl;
      }
    }
    // equality constraints: c_0 = x0 - x_0 (stage 0), c_{i+1} = d(x_i, u_i) - x_{i+1}
    if (i == 0) {
      for (int j = 0; j < n; ++j) {
        const double cv = a.x0[(int64_t)b * n + j] - xt[j];
        mer += y[j] * cv + 0.5 * d.eta * cv * cv;
        if (k < 0) slope += (y[j] + d.eta * cv) * (-dx[j]);
      }
    }
    if (i < N) {
      const double* x1 = a.x + ((int64_t)b * (N + 1) + i + 1) * n;
      const double* dx1 = a.dx + ((int64_t)b * (N + 1) + i + 1) * n;
      const double* du = a.du + ((int64_t)b * N + i) * m;
      for (int j = 0; j < n; ++j) xn[j] = x1[j] + al * dx1[j];
      for (int r = 0; r < n; ++r) {
        double v = 0.0;
        for (int j = 0; j < n; ++j) v = fma(A[r * n + j], xt[j], v);
        for (int j = 0; j < m; ++j) v = fma(Bm[r * m + j], ut[j], v);
        const double tv = tanh(v);
        const double cv = xt[r] + d.dt * tv - xn[r];
        const double yv = y[(int64_t)(i + 1) * n + r];
        mer += yv * cv + 0.5 * d.eta * cv * cv;
        if (k < 0) {
          double jd = 0.0;  // row r of (A dx + B du)
          for (int j = 0; j < n; ++j) jd = fma(A[r * n + j], dx[j], jd);
          for (int j = 0; j < m; ++j) jd = fma(Bm[r * m + j], du[j], jd);
          const double lin = dx[r] + d.dt * (1.0 - tv * tv) * jd - dx1[r];
          slope += (yv + d.eta * cv) * lin;
        }
      }
    }
  }
  mer = block_sum(mer, red);
  if (k < 0) slope = block_sum(slope, red);
  if (t == 0) {
    a.merit[(int64_t)b * (LADDER + 1) + k + 1] = mer;
    if (k < 0) a.slope[b] = slope;
  }
}

// First ladder step passing Armijo, else the last.
__global__ void k_ipm_select(IpmArgs a) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.d.B || a.conv[b]) return;
  const double amax = __longlong_as_double((long long)a.amax_s[b]);
  const double* mr = a.merit + (int64_t)b * (LADDER + 1);
  const double m0 = mr[0], sl = a.slope[b];
  double al = ldexp(amax, -(LADDER - 1));
  for (int k = 0; k < LADDER; ++k) {
    const double ak = ldexp(amax, -k);
    if (mr[k + 1] <= m0 + C1 * ak * sl) {
      al = ak;
      break;
    }
  }
  a.alpha[b] = al;
}

__global__ __launch_bounds__(64) void k_ipm_update(IpmArgs a) {
  const Dims d = a.d;
  const int i = blockIdx.x, b = blockIdx.y, t = threadIdx.x;
  if (a.conv[b]) return;
  const int n = d.n, m = d.m, ng = d.ng, N = d.N;
  const double al = a.alpha[b];
  const double az = __longlong_as_double((long long)a.amax_z[b]);
  const int64_t ox = ((int64_t)b * (N + 1) + i) * n;
  for (int j = t; j < n; j += 64) {
    a.x[ox + j] += al * a.dx[ox + j];
    a.y[ox + j] += a.dy[ox + j];
  }
  if (i < N) {
    const int64_t ou = ((int64_t)b * N + i) * m;
    // equality multipliers, full step: dy_e = eta (E_u du + e(u)) at the u before the update
    if (t < d.ne) {
      const double dye = d.eta * (e_lin(a, t, a.du + ou) + e_row(a, b, i, t, a.u + ou));
      a.ye[((int64_t)b * N + i) * d.ne + t] += dye;
    }
    __syncthreads();
    for (int j = t; j < m; j += 64) a.u[ou + j] += al * a.du[ou + j];
  }
  const int64_t o = ((int64_t)b * (N + 1) + i) * ng;
  const int rows = rows_of(d, i);
  for (int l = t; l < rows; l += 64) {
    a.s[o + l] += al * a.ds[o + l];
    a.z[o + l] += az * a.dz[o + l];
  }
}

// ---------------------------------------------------------------- errors, mu, convergence

// mode 0: after (re)start (warm starts set mu0 = mean(s z) clipped to [1e-9, 0.1]);
// mode 1: after an update (mu decrease, rho / 3, iteration count).
// Both set conv[b] = (max(|grad L|, |c|, |g + s|, |s z|) <= tol).
__global__ __launch_bounds__(256) void k_ipm_errors(IpmArgs a, int mode, int warm, double tol) {
  const Dims d = a.d;
  const int b = blockIdx.x, t = threadIdx.x;
  if (a.conv[b]) return;
  const int n = d.n, m = d.m, ng = d.ng, N = d.N;
  __shared__ double red[256];
  const double mu = a.mu[b];
  const double* A = mA(a);
  const double* Bm = mB(a);
  const double* av = ma(a);
  const double* goal = a.goal + (int64_t)b * n;
  const double* y = a.y + (int64_t)b * (N + 1) * n;
  double eg = 0.0, ec = 0.0, egs = 0.0, esz_mu = 0.0, esz = 0.0, sz = 0.0;
  double thv[MAXD], sev[MAXD];
  for (int i = t; i <= N; i += 256) {
    const double* x = a.x + ((int64_t)b * (N + 1) + i) * n;
    const double* u = a.u + ((int64_t)b * N + i) * m;
    const double* s = a.s + ((int64_t)b * (N + 1) + i) * ng;
    const double* z = a.z + ((int64_t)b * (N + 1) + i) * ng;
    const int rows = rows_of(d, i);
    if (i < N) {
      for (int r = 0; r < n; ++r) {
        double v = 0.0;
        for (int j = 0; j < n; ++j) v = fma(A[r * n + j], x[j], v);
        for (int j = 0; j < m; ++j) v = fma(Bm[r * m + j], u[j], v);
        thv[r] = tanh(v);
        sev[r] = 1.0 - thv[r] * thv[r];
        const double cv = x[r] + d.dt * thv[r] - x[n + r];  // x_{i+1} follows x_i in memory
        ec = fmax(ec, fabs(cv));
      }
    }
    if (i == 0)
      for (int j = 0; j < n; ++j) ec = fmax(ec, fabs(a.x0[(int64_t)b * n + j] - x[j]));
    for (int r = 0; r < n; ++r) {
      double gx = (i < N ? d.wx : d.wN) * (x[r] - goal[r]) - y[(int64_t)i * n + r] + av[r] * z[0] + av[n + r] * z[1];
      if (i < N) {
        gx += y[(int64_t)(i + 1) * n + r];
        for (int j = 0; j < n; ++j) gx = fma(d.dt * sev[j] * y[(int64_t)(i + 1) * n + j], A[j * n + r], gx);
      }
      eg = fmax(eg, fabs(gx));
    }
    if (i < N) {
      const double* ye = a.ye + ((int64_t)b * N + i) * d.ne;
      for (int k = 0; k < m; ++k) {
        double gu = d.wu * u[k] + z[2 + k] - z[2 + m + k];
        for (int j = 0; j < n; ++j) gu = fma(d.dt * sev[j] * y[(int64_t)(i + 1) * n + j], Bm[j * m + k], gu);
        for (int l = 0; l < d.ne; ++l) gu = fma(ye[l], mE(a)[l * m + k], gu);
        eg = fmax(eg, fabs(gu));
      }
      for (int l = 0; l < d.ne; ++l) ec = fmax(ec, fabs(e_row(a, b, i, l, u)));
    }
    for (int l = 0; l < rows; ++l) {
      egs = fmax(egs, fabs(g_row(a, l, x, u) + s[l]));
      esz_mu = fmax(esz_mu, fabs(s[l] * z[l] - mu));
      esz = fmax(esz, fabs(s[l] * z[l]));
      sz += s[l] * z[l];
    }
  }
  eg = block_max(eg, red);
  ec = block_max(ec, red);
  egs = block_max(egs, red);
  esz_mu = block_max(esz_mu, red);
  esz = block_max(esz, red);
  if (mode == 0 && warm) sz = block_sum(sz, red);
  if (t == 0) {
    double* e = a.err + (int64_t)b * 4;
    e[0] = eg; e[1] = ec; e[2] = egs; e[3] = esz;
    if (mode == 1) {
      if (fmax(fmax(eg, ec), fmax(egs, esz_mu)) <= 10.0 * mu) a.mu[b] = fmax(mu / 10.0, 1.0e-9);
      a.rho[b] = a.rho[b] / 3.0;
      a.iters[b] += 1;
    } else if (warm) {
      const int cnt = N * ng + 2;
      a.mu[b] = fmin(fmax(sz / cnt, 1.0e-9), 0.1);
    }
    a.conv[b] = fmax(fmax(eg, ec), fmax(egs, esz)) <= tol ? 1 : 0;
  }
}

__global__ void k_ipm_reset_steps(IpmArgs a) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.d.B) return;
  const unsigned long long one = (unsigned long long)__double_as_longlong(1.0);
  a.amax_s[b] = one;
  a.amax_z[b] = one;
}

__global__ void k_ipm_zero(int32_t* p) { *p = 0; }

// skip = conv (mode 0), or conv || verdict (mode 1: later inertia-correction
// rounds refactor only the problems whose certificate failed)
__global__ void k_ipm_skip(IpmArgs a, int mode) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.d.B) return;
  a.skip[b] = (a.conv[b] || (mode == 1 && a.verdict[b])) ? 1 : 0;
}

__global__ void k_ipm_count_active(const int32_t* conv, int B, int32_t* out) {
  __shared__ int red[256];
  int c = 0;
  for (int b = threadIdx.x; b < B; b += 256) c += conv[b] ? 0 : 1;
  red[threadIdx.x] = c;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

}  // namespace

// ---------------------------------------------------------------- host

struct ripm_handle {
  Dims d{};
  double tol = 1e-6;
  int lqr_mode = RLQR_SEQ_MIXED;
  rlqr_handle* lqr = nullptr;
  bool warm = false;
  std::vector<void*> allocs;
  size_t bytes = 0;
  IpmArgs a{};
  double *delta = nullptr, *dxv = nullptr, *duv = nullptr, *dyv = nullptr;
  int32_t* verdict = nullptr;
  int32_t* counter = nullptr;  // [0] certificate failures, [1] active problems
};

static rlqr_status ipm_alloc(ripm_handle* h, void** p, size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return RLQR_E_NOMEM;
  }
  h->allocs.push_back(*p);
  h->bytes += bytes;
  return RLQR_OK;
}

static void ipm_release(ripm_handle* h) {
  (void)hipDeviceSynchronize();
  if (h->lqr) rlqr_destroy(h->lqr);
  h->lqr = nullptr;
  for (void* p : h->allocs) (void)hipFree(p);
  h->allocs.clear();
}

#define IPM_TRY(x)                            \
  do {                                        \
    if ((x) != hipSuccess) return RLQR_E_HIP; \
  } while (0)

extern "C" {

rlqr_status ripm_create(ripm_handle** hp, const ripm_problem* p, size_t* workspace_bytes) {
  if (!hp) return RLQR_E_INVALID;
  *hp = nullptr;
  if (!p || p->batch < 1 || p->N < 1 || p->n < 1 || p->m < 1 || p->n + p->m > MAXD || !p->A || !p->B || !p->a)
    return RLQR_E_INVALID;
  if (!(p->eta > 0) || !(p->dt > 0) || !(p->tol > 0) || !(p->umax > 0)) return RLQR_E_INVALID;
  if (p->lqr_mode != RLQR_SEQ_FP64 && p->lqr_mode != RLQR_SEQ_MIXED) return RLQR_E_INVALID;
  if (p->ne < 0 || p->ne > MAXE || p->ne > p->m || (p->ne > 0 && !p->Eu)) return RLQR_E_INVALID;
  ripm_handle* h = new (std::nothrow) ripm_handle();
  if (!h) return RLQR_E_NOMEM;
  Dims& d = h->d;
  d.B = p->batch; d.N = p->N; d.n = p->n; d.m = p->m; d.ng = 2 + 2 * p->m; d.ne = p->ne;
  d.dt = p->dt; d.wx = p->wx; d.wu = p->wu; d.wN = p->wN; d.xmax = p->xmax; d.umax = p->umax; d.eta = p->eta;
  h->tol = p->tol;
  h->lqr_mode = p->lqr_mode;
  const int64_t B = d.B, N = d.N, n = d.n, m = d.m, ng = d.ng;
  std::vector<int32_t> Nv(B, (int32_t)N), nv(B, (int32_t)n), mv(B, (int32_t)m);
  rlqr_shape sh{(int32_t)B, Nv.data(), nv.data(), mv.data()};
  size_t lqr_bytes = 0;
  rlqr_status st = rlqr_create(&h->lqr, &sh, (rlqr_mode)p->lqr_mode, &lqr_bytes);
  auto A = [&](void* pp, size_t bytes) {
    if (st == RLQR_OK) st = ipm_alloc(h, reinterpret_cast<void**>(pp), bytes);
  };
  IpmArgs& a = h->a;
  a.d = d;
  const size_t D = sizeof(double);
  const int64_t ne = d.ne;
  A(&a.model, D * (size_t)(n * n + n * m + 2 * n + ne * m));
  A(&a.x0, D * B * n);
  A(&a.eb, D * B * N * ne);
  A(&a.ye, D * B * N * ne);
  A(&a.goal, D * B * n);
  A(&a.x, D * B * (N + 1) * n);
  A(&a.u, D * B * N * m);
  A(&a.y, D * B * (N + 1) * n);
  A(&a.s, D * B * (N + 1) * ng);
  A(&a.z, D * B * (N + 1) * ng);
  A(&a.ds, D * B * (N + 1) * ng);
  A(&a.dz, D * B * (N + 1) * ng);
  A(&a.mu, D * B);
  A(&a.rho, D * B);
  A(&a.merit, D * B * (LADDER + 1));
  A(&a.slope, D * B);
  A(&a.alpha, D * B);
  A(&a.err, D * B * 4);
  A(&a.amax_s, 8 * B);
  A(&a.amax_z, 8 * B);
  A(&a.conv, 4 * B);
  A(&a.iters, 4 * B);
  A(&h->counter, 8);
  A(&a.Q, D * B * (N + 1) * n * n);
  A(&a.M, D * B * N * n * m);
  A(&a.R, D * B * N * m * m);
  A(&a.Al, D * B * N * n * n);
  A(&a.Bl, D * B * N * n * m);
  A(&a.q, D * B * (N + 1) * n);
  A(&a.r, D * B * N * m);
  A(&a.c, D * B * (N + 1) * n);
  A(&h->delta, D * B);
  A(&h->dxv, D * B * (N + 1) * n);
  A(&h->duv, D * B * N * m);
  A(&h->dyv, D * B * (N + 1) * n);
  A(&h->verdict, 4 * B);
  A(&a.skip, 4 * B);
  if (st == RLQR_OK) {
    a.dx = h->dxv; a.du = h->duv; a.dy = h->dyv; a.verdict = h->verdict; a.fail = h->counter;
    a.build_skip = nullptr;
    if (rlqr_set_skip(h->lqr, a.skip) != RLQR_OK) st = RLQR_E_HIP;
    std::vector<double> model;
    model.insert(model.end(), p->A, p->A + n * n);
    model.insert(model.end(), p->B, p->B + n * m);
    model.insert(model.end(), p->a, p->a + 2 * n);
    if (ne > 0) model.insert(model.end(), p->Eu, p->Eu + ne * m);
    std::vector<double> dl(B, 1.0 / d.eta);
    if (hipMemcpy((void*)a.model, model.data(), D * model.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->delta, dl.data(), D * B, hipMemcpyHostToDevice) != hipSuccess)
      st = RLQR_E_HIP;
  }
  if (st != RLQR_OK) {
    ipm_release(h);
    delete h;
    return st;
  }
  if (workspace_bytes) *workspace_bytes = h->bytes + lqr_bytes;
  *hp = h;
  return RLQR_OK;
}

rlqr_status ripm_start(ripm_handle* h, const double* x0, const double* goal, const double* warm, const double* eb,
                       rlqr_stream stv) {
  if (!h || !x0 || !goal) return RLQR_E_INVALID;
  if (h->d.ne > 0 && !eb) return RLQR_E_INVALID;
  hipStream_t st = (hipStream_t)stv;
  const Dims& d = h->d;
  if (d.ne > 0)
    IPM_TRY(hipMemcpyAsync((void*)h->a.eb, eb, sizeof(double) * d.B * d.N * d.ne, hipMemcpyDeviceToDevice, st));
  IPM_TRY(hipMemcpyAsync((void*)h->a.x0, x0, sizeof(double) * d.B * d.n, hipMemcpyDeviceToDevice, st));
  IPM_TRY(hipMemcpyAsync((void*)h->a.goal, goal, sizeof(double) * d.B * d.n, hipMemcpyDeviceToDevice, st));
  h->warm = warm != nullptr;
  hipLaunchKernelGGL(k_ipm_init, dim3(d.N + 1, d.B), dim3(64), 0, st, h->a, warm);
  IPM_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_ipm_errors, dim3(d.B), dim3(256), 0, st, h->a, 0, warm ? 1 : 0, h->tol);
  IPM_TRY(hipGetLastError());
  return RLQR_OK;
}

rlqr_status ripm_iterate(ripm_handle* h, int32_t* active, rlqr_stream stv) {
  if (!h) return RLQR_E_INVALID;
  hipStream_t st = (hipStream_t)stv;
  const Dims& d = h->d;
  IpmArgs& a = h->a;
  const int64_t B = d.B, N = d.N, n = d.n, m = d.m;
  const dim3 stages(d.N + 1, d.B), small((d.B + 255) / 256);
  rlqr_lhs lhs{a.Q, a.M, a.R, a.Al, a.Bl, h->delta};
  rlqr_rhs rhs{a.q, a.r, a.c};
  rlqr_sol sol{h->dxv, h->duv, h->dyv};
  rlqr_status s;
  // Newton direction with the inertia correction; converged problems are left
  // out of the LQR calls, and after the first round only the problems whose
  // certificate failed are rebuilt (with their larger rho) and refactored
  for (int round = 0; round < 60; ++round) {
    hipLaunchKernelGGL(k_ipm_skip, small, dim3(256), 0, st, a, round > 0 ? 1 : 0);
    IpmArgs ab = a;
    ab.build_skip = round > 0 ? a.skip : nullptr;
    hipLaunchKernelGGL(k_ipm_build, stages, dim3(256), 0, st, ab);
    IPM_TRY(hipGetLastError());
    if ((s = rlqr_factor_rhs(h->lqr, &lhs, &rhs, stv)) != RLQR_OK) return s;
    if ((s = rlqr_pivot_inertia(h->lqr, h->verdict, nullptr, nullptr, stv)) != RLQR_OK) return s;
    hipLaunchKernelGGL(k_ipm_zero, dim3(1), dim3(1), 0, st, h->counter);
    hipLaunchKernelGGL(k_ipm_rho, small, dim3(256), 0, st, a);
    IPM_TRY(hipGetLastError());
    int32_t fails = 0;
    IPM_TRY(hipMemcpyAsync(&fails, h->counter, 4, hipMemcpyDeviceToHost, st));
    IPM_TRY(hipStreamSynchronize(st));
    if (fails == 0) break;
  }
  hipLaunchKernelGGL(k_ipm_skip, small, dim3(256), 0, st, a, 0);
  IPM_TRY(hipGetLastError());
  if ((s = rlqr_solve(h->lqr, &rhs, &sol, 1e-10, 4, nullptr, nullptr, stv)) != RLQR_OK) return s;
  hipLaunchKernelGGL(k_ipm_reset_steps, small, dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_ipm_recover, stages, dim3(64), 0, st, a);
  hipLaunchKernelGGL(k_ipm_merit, dim3(LADDER + 1, d.B), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_ipm_select, small, dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_ipm_update, stages, dim3(64), 0, st, a);
  hipLaunchKernelGGL(k_ipm_errors, dim3(d.B), dim3(256), 0, st, a, 1, 0, h->tol);
  hipLaunchKernelGGL(k_ipm_count_active, dim3(1), dim3(256), 0, st, (const int32_t*)a.conv, d.B, h->counter + 1);
  IPM_TRY(hipGetLastError());
  int32_t act = 0;
  IPM_TRY(hipMemcpyAsync(&act, h->counter + 1, 4, hipMemcpyDeviceToHost, st));
  IPM_TRY(hipStreamSynchronize(st));
  if (active) *active = act;
  (void)B; (void)N; (void)n; (void)m;
  return RLQR_OK;
}

rlqr_status ripm_solve(ripm_handle* h, int32_t max_iter, int32_t* iters, int32_t* converged, rlqr_stream stv) {
  if (!h || max_iter < 0) return RLQR_E_INVALID;
  hipStream_t st = (hipStream_t)stv;
  const Dims& d = h->d;
  hipLaunchKernelGGL(k_ipm_count_active, dim3(1), dim3(256), 0, st, (const int32_t*)h->a.conv, d.B, h->counter + 1);
  int32_t act = 0;
  IPM_TRY(hipMemcpyAsync(&act, h->counter + 1, 4, hipMemcpyDeviceToHost, st));
  IPM_TRY(hipStreamSynchronize(st));
  for (int it = 0; it < max_iter && act > 0; ++it) {
    rlqr_status s = ripm_iterate(h, &act, stv);
    if (s != RLQR_OK) return s;
  }
  if (iters) IPM_TRY(hipMemcpyAsync(iters, h->a.iters, 4 * d.B, hipMemcpyDeviceToHost, st));
  if (converged) IPM_TRY(hipMemcpyAsync(converged, h->a.conv, 4 * d.B, hipMemcpyDeviceToHost, st));
  IPM_TRY(hipStreamSynchronize(st));
  return RLQR_OK;
}

rlqr_status ripm_solution(ripm_handle* h, double* x, double* u, double* y, double* z, double* ye,
                          rlqr_stream stv) {
  if (!h) return RLQR_E_INVALID;
  hipStream_t st = (hipStream_t)stv;
  const Dims& d = h->d;
  const size_t D = sizeof(double);
  const size_t B = d.B, N = d.N, n = d.n, m = d.m, ng = d.ng;
  if (x) IPM_TRY(hipMemcpyAsync(x, h->a.x, D * B * (N + 1) * n, hipMemcpyDeviceToDevice, st));
  if (u) IPM_TRY(hipMemcpyAsync(u, h->a.u, D * B * N * m, hipMemcpyDeviceToDevice, st));
  if (y) IPM_TRY(hipMemcpyAsync(y, h->a.y, D * B * (N + 1) * n, hipMemcpyDeviceToDevice, st));
  if (z) IPM_TRY(hipMemcpyAsync(z, h->a.z, D * B * (N + 1) * ng, hipMemcpyDeviceToDevice, st));
  if (ye && d.ne > 0) IPM_TRY(hipMemcpyAsync(ye, h->a.ye, D * B * N * d.ne, hipMemcpyDeviceToDevice, st));
  return RLQR_OK;
}

void ripm_destroy(ripm_handle* h) {
  if (!h) return;
  ipm_release(h);
  delete h;
}

}  // extern "C"
