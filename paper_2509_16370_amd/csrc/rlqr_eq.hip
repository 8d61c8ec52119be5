// rlqr_eq.hip -- stagewise equality rows eliminated into the dual-regularized
// LQR (Section "Applying the regularized IPM to optimal control" of arXiv
// 2509.16370): the rows E z - D^{-1} w = -r_e leave w = D (E z + r_e), and
// the stage Hessian and gradient gain E^T D E and E^T D r_e. Both kernels are
// elementwise over the caller's packed arrays (HBM-bound): one wavefront per
// (stage, instance) for the reduction, one thread per (stage, row) for w.
#include <new>
#include <vector>

#include "../../include/rlqr_eq.h"
#include "rlqr_internal.h"

namespace rlqr {
namespace {

struct EqMeta {
  int32_t N, n, m, ne;
  int64_t oQ, oM, oR, oq, or_, ox, ou, oE, ov;
};

struct EqReduceArgs {
  const EqMeta* meta;
  const double *Q, *M, *R, *q, *r;
  const double *E, *re, *eta;
  double *Qo, *Mo, *Ro, *qo, *ro;
  int lds_e;  // doubles of E staged per wavefront (max ne (n + m) of the batch)
};

struct EqRecoverArgs {
  const EqMeta* meta;
  const double *E, *re, *eta, *x, *u;
  double* w;
  int lds_e;  // as in EqReduceArgs
};

// Four stages per workgroup, one wavefront each: stage i = 4 blockIdx.x + w
// of instance blockIdx.y. The outputs may alias the inputs: every element is
// read, then written, by one lane. E_i is staged in the wavefront's LDS
// slice; each output element adds sum_k eta_k E[k][a] E[k][b] (the pair
// product first, so the reduced Q and R stay exactly symmetric) or
// sum_k E[k][a] eta_k r_k.
constexpr int EQ_SPB = 4;  // stages (wavefronts) per workgroup
__global__ __launch_bounds__(64 * EQ_SPB) void k_eq_reduce(EqReduceArgs a) {
  const EqMeta mt = a.meta[blockIdx.y];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * EQ_SPB + w;
  const int N = mt.N, n = mt.n, m = mt.m, ne = mt.ne;
  if (i > N) return;  // no workgroup barrier below: each wavefront works alone
  const int s = i < N ? n + m : n;  // columns of E_i
  extern __shared__ double sEall[];  // EQ_SPB slices of lds_e doubles
  __shared__ double sEtaAll[EQ_SPB][RLQR_EQ_MAX_NE], sDrAll[EQ_SPB][RLQR_EQ_MAX_NE];
  double* sE = sEall + (size_t)w * a.lds_e;
  double* sEta = sEtaAll[w];
  double* sDr = sDrAll[w];
  const double* __restrict__ E = a.E + mt.oE + (int64_t)i * ne * (n + m);
  const double* __restrict__ re = a.re + mt.ov + (int64_t)i * ne;
  const double* __restrict__ eta = a.eta + mt.ov + (int64_t)i * ne;
  for (int x = lane; x < ne * s; x += 64) sE[x] = E[x];
  if (lane < ne) {
    sEta[lane] = eta[lane];
    sDr[lane] = eta[lane] * re[lane];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  {
    const double* Q = a.Q + mt.oQ + (int64_t)i * n * n;
    double* Qo = a.Qo + mt.oQ + (int64_t)i * n * n;
    for (int x = lane; x < n * n; x += 64) {
      const int r0 = x / n, c0 = x % n;
      double v = Q[x];
      for (int k = 0; k < ne; ++k) v = fma(sEta[k], sE[k * s + r0] * sE[k * s + c0], v);
      Qo[x] = v;
    }
    const double* q = a.q + mt.oq + (int64_t)i * n;
    double* qo = a.qo + mt.oq + (int64_t)i * n;
    for (int x = lane; x < n; x += 64) {
      double v = q[x];
      for (int k = 0; k < ne; ++k) v = fma(sE[k * s + x], sDr[k], v);
      qo[x] = v;
    }
  }
  if (i < N) {
    const double* M = a.M + mt.oM + (int64_t)i * n * m;
    double* Mo = a.Mo + mt.oM + (int64_t)i * n * m;
    for (int x = lane; x < n * m; x += 64) {
      const int r0 = x / m, c0 = x % m;
      double v = M[x];
      for (int k = 0; k < ne; ++k) v = fma(sEta[k], sE[k * s + r0] * sE[k * s + n + c0], v);
      Mo[x] = v;
    }
    const double* R = a.R + mt.oR + (int64_t)i * m * m;
    double* Ro = a.Ro + mt.oR + (int64_t)i * m * m;
    for (int x = lane; x < m * m; x += 64) {
      const int r0 = x / m, c0 = x % m;
      double v = R[x];
      for (int k = 0; k < ne; ++k) v = fma(sEta[k], sE[k * s + n + r0] * sE[k * s + n + c0], v);
      Ro[x] = v;
    }
    const double* r = a.r + mt.or_ + (int64_t)i * m;
    double* ro = a.ro + mt.or_ + (int64_t)i * m;
    for (int x = lane; x < m; x += 64) {
      double v = r[x];
      for (int k = 0; k < ne; ++k) v = fma(sE[k * s + n + x], sDr[k], v);
      ro[x] = v;
    }
  }
}

// Sixteen lanes per stage, four stages per workgroup (one wavefront): stage
// i = 4 blockIdx.x + g (g = lane / 16) of instance blockIdx.y. The sixteen
// lanes copy E_i and z_i = (x_i, u_i) into their LDS slice with contiguous
// loads, then lane 16 g + k, k < ne, forms row k's multiplier. LDS: four
// slices of at most 16 * 96 + 96 doubles (52 KB).
constexpr int EQ_RSPB = 4;  // stages per workgroup
__global__ __launch_bounds__(64) void k_eq_recover(EqRecoverArgs a) {
  const EqMeta mt = a.meta[blockIdx.y];
  const int lane = threadIdx.x, g = lane >> 4, l = lane & 15;
  const int i = blockIdx.x * EQ_RSPB + g;
  const int N = mt.N, n = mt.n, m = mt.m, ne = mt.ne;
  extern __shared__ double sRec[];  // per stage: lds_e doubles of E, then RLQR_MAX_NXU of z
  double* sE = sRec + (size_t)g * (a.lds_e + RLQR_MAX_NXU);
  double* sz = sE + a.lds_e;
  const bool live = i <= N && ne > 0;
  const int s = i < N ? n + m : n;
  if (live) {
    const double* __restrict__ E = a.E + mt.oE + (int64_t)i * ne * (n + m);
    for (int x = l; x < ne * s; x += 16) sE[x] = E[x];
    const double* __restrict__ xi = a.x + mt.ox + (int64_t)i * n;
    for (int x = l; x < n; x += 16) sz[x] = xi[x];
    if (i < N) {
      const double* __restrict__ ui = a.u + mt.ou + (int64_t)i * m;
      for (int x = l; x < m; x += 16) sz[n + x] = ui[x];
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (!live || l >= ne) return;
  const int64_t v = mt.ov + (int64_t)i * ne + l;
  double acc = a.re[v];
  for (int j = 0; j < s; ++j) acc = fma(sE[l * s + j], sz[j], acc);
  a.w[v] = a.eta[v] * acc;
}

}  // namespace
}  // namespace rlqr

using namespace rlqr;

struct rlqr_eq {
  const rlqr_handle* h = nullptr;
  int B = 0, maxN = 0, lds_e = 1;
  int64_t max_rows = 0;  // max over the batch of (N + 1) ne
  std::vector<int64_t> offE, offV;
  EqMeta* meta = nullptr;
  size_t bytes = 0;
};

extern "C" {

rlqr_status rlqr_eq_create(rlqr_eq** ctx, const rlqr_handle* h, const int32_t* ne, size_t* workspace_bytes) {
  if (!ctx) return RLQR_E_INVALID;
  *ctx = nullptr;
  if (!h) return RLQR_E_INVALID;
  int B = 0;
  const int32_t *N = nullptr, *n = nullptr, *m = nullptr;
  handle_shapes(h, &B, &N, &n, &m);
  if (B > 65535 || (B > 0 && !ne)) return RLQR_E_INVALID;
  for (int b = 0; b < B; ++b)
    if (ne[b] < 0 || ne[b] > RLQR_EQ_MAX_NE) return RLQR_E_INVALID;
  rlqr_eq* c = new (std::nothrow) rlqr_eq();
  if (!c) return RLQR_E_NOMEM;
  c->h = h;
  c->B = B;
  c->offE.assign(B + 1, 0);
  c->offV.assign(B + 1, 0);
  std::vector<int64_t> off[RLQR_ARR_COUNT];
  for (int k = 0; k < RLQR_ARR_COUNT; ++k) {
    off[k].assign(B + 1, 0);
    if (rlqr_layout_offsets(h, k, off[k].data()) != RLQR_OK) {
      delete c;
      return RLQR_E_INVALID;
    }
  }
  std::vector<EqMeta> meta((size_t)B);
  for (int b = 0; b < B; ++b) {
    EqMeta& e = meta[b];
    e.N = N[b]; e.n = n[b]; e.m = m[b]; e.ne = ne[b];
    e.oQ = off[RLQR_ARR_Q][b]; e.oM = off[RLQR_ARR_M][b]; e.oR = off[RLQR_ARR_R][b];
    e.oq = off[RLQR_ARR_q][b]; e.or_ = off[RLQR_ARR_r][b];
    e.ox = off[RLQR_ARR_x][b]; e.ou = off[RLQR_ARR_u][b];
    e.oE = c->offE[b];
    e.ov = c->offV[b];
    c->offE[b + 1] = c->offE[b] + (int64_t)ne[b] * ((int64_t)N[b] * (n[b] + m[b]) + n[b]);
    c->offV[b + 1] = c->offV[b] + (int64_t)ne[b] * (N[b] + 1);
    c->maxN = N[b] > c->maxN ? N[b] : c->maxN;
    const int64_t rows = (int64_t)(N[b] + 1) * ne[b];
    c->max_rows = rows > c->max_rows ? rows : c->max_rows;
    const int le = ne[b] * (n[b] + m[b]);
    c->lds_e = le > c->lds_e ? le : c->lds_e;
  }
  if (B > 0) {
    c->bytes = sizeof(EqMeta) * (size_t)B;
    if (hipMalloc((void**)&c->meta, c->bytes) != hipSuccess) {
      (void)hipGetLastError();
      delete c;
      return RLQR_E_NOMEM;
    }
    if (hipMemcpy(c->meta, meta.data(), c->bytes, hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(c->meta);
      delete c;
      return RLQR_E_HIP;
    }
  }
  if (workspace_bytes) *workspace_bytes = c->bytes;
  *ctx = c;
  return RLQR_OK;
}

rlqr_status rlqr_eq_offsets(const rlqr_eq* ctx, int32_t array, int64_t* off) {
  if (!ctx || !off || (array != RLQR_EQ_ARR_E && array != RLQR_EQ_ARR_V)) return RLQR_E_INVALID;
  const std::vector<int64_t>& v = array == RLQR_EQ_ARR_E ? ctx->offE : ctx->offV;
  for (int b = 0; b <= ctx->B; ++b) off[b] = v[b];
  return RLQR_OK;
}

rlqr_status rlqr_eq_reduce(rlqr_eq* ctx, const rlqr_lhs* lhs, const rlqr_rhs* rhs, const rlqr_eq_data* eq,
                           double* Qo, double* Mo, double* Ro, double* qo, double* ro, rlqr_stream stv) {
  if (!ctx || !lhs || !rhs || !eq) return RLQR_E_INVALID;
  if (ctx->B == 0) return RLQR_OK;
  if (!lhs->Q || !lhs->M || !lhs->R || !rhs->q || !rhs->r || !eq->E || !eq->r || !eq->eta || !Qo || !Mo ||
      !Ro || !qo || !ro)
    return RLQR_E_INVALID;
  EqReduceArgs a{};
  a.meta = ctx->meta;
  a.Q = lhs->Q; a.M = lhs->M; a.R = lhs->R; a.q = rhs->q; a.r = rhs->r;
  a.E = eq->E; a.re = eq->r; a.eta = eq->eta;
  a.Qo = Qo; a.Mo = Mo; a.Ro = Ro; a.qo = qo; a.ro = ro;
  a.lds_e = ctx->lds_e;
  const unsigned gx = (unsigned)((ctx->maxN + 1 + EQ_SPB - 1) / EQ_SPB);
  const size_t lds = sizeof(double) * (size_t)EQ_SPB * (size_t)ctx->lds_e;  // <= 48 KB
  hipLaunchKernelGGL(k_eq_reduce, dim3(gx, ctx->B), dim3(64 * EQ_SPB), lds, (hipStream_t)stv, a);
  return hipGetLastError() == hipSuccess ? RLQR_OK : RLQR_E_HIP;
}

rlqr_status rlqr_eq_recover(rlqr_eq* ctx, const rlqr_eq_data* eq, const rlqr_sol* z, double* w, rlqr_stream stv) {
  if (!ctx || !eq || !z) return RLQR_E_INVALID;
  if (ctx->B == 0) return RLQR_OK;
  if (!eq->E || !eq->r || !eq->eta || !z->x || !z->u || !w) return RLQR_E_INVALID;
  EqRecoverArgs a{};
  a.meta = ctx->meta;
  a.E = eq->E; a.re = eq->r; a.eta = eq->eta; a.x = z->x; a.u = z->u; a.w = w;
  if (ctx->max_rows == 0) return RLQR_OK;
  a.lds_e = ctx->lds_e;
  const unsigned gx = (unsigned)((ctx->maxN + 1 + EQ_RSPB - 1) / EQ_RSPB);
  const size_t lds = sizeof(double) * (size_t)EQ_RSPB * (size_t)(ctx->lds_e + RLQR_MAX_NXU);  // <= 52 KB
  hipLaunchKernelGGL(k_eq_recover, dim3(gx, ctx->B), dim3(64), lds, (hipStream_t)stv, a);
  return hipGetLastError() == hipSuccess ? RLQR_OK : RLQR_E_HIP;
}

void rlqr_eq_destroy(rlqr_eq* ctx) {
  if (!ctx) return;
  if (ctx->meta) (void)hipFree(ctx->meta);
  delete ctx;
}

}  // extern "C"
