// rlqr_api.hip -- host side of the C ABI declared in include/rlqr.h.
//
// Owns the handle: shape metadata, packed-layout offsets, the factorization
// workspace (two 16 x 16 tiles per stage and instance) and the per-instance
// flags that steer the mixed-precision path:
//   flag64[b]  instance uses the float64 factorization (always in RLQR_SEQ_FP64;
//              in RLQR_SEQ_MIXED when a pivot falls inside the guard band or
//              refinement in float32 did not converge)
//   conv[b]    refinement converged
// All launches are asynchronous on the caller's stream; no call after
// rlqr_create allocates memory, synchronizes or copies to the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "rlqr_internal.h"

using namespace rlqr;

namespace {

// |pivot| / max|diag| below this (in a float32-product factorization) sends the
// instance to the float64 factorization, so the certificate is decided in float64.
constexpr double kGuard = 1.0e-4;

}  // namespace

struct rlqr_handle {
  int B = 0;
  rlqr_mode mode = RLQR_SEQ_FP64;
  std::vector<int32_t> N, n, m;
  std::vector<int64_t> off[RLQR_ARR_COUNT];
  int64_t total_stage_blocks = 0;  // sum of N_b + 1
  size_t bytes = 0;

  InstMeta* meta = nullptr;
  int64_t* stage_off = nullptr;
  int32_t* blk_inst = nullptr;  // residual block -> instance
  void* ws64 = nullptr;   // float64 tiles
  void* ws32 = nullptr;   // float32 tiles (mixed mode)
  double* pk = nullptr;   // p_i / k_i scratch
  double* res[2] = {nullptr, nullptr};  // residual vectors (ping-pong between passes)
  FactorInfo* info = nullptr;
  int32_t* fused = nullptr;  // instance's solve kernel computes its residual itself
  // instances grouped by tile class: device id lists and counts
  int32_t* list[TILE_CLASSES] = {};
  int count[TILE_CLASSES] = {};
  unsigned long long *resmax = nullptr, *bmax = nullptr;
  int32_t *flag64 = nullptr, *conv = nullptr, *run32 = nullptr, *run64 = nullptr,
          *runres = nullptr, *fb = nullptr, *status = nullptr;
  double *lastrel = nullptr, *relres = nullptr;

  rlqr_lhs lhs{};
  bool factored = false;
  std::vector<void*> allocs;
};

static rlqr_status dev_alloc(rlqr_handle* h, void** p, size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return RLQR_E_NOMEM;
  }
  h->allocs.push_back(*p);
  h->bytes += bytes;
  return RLQR_OK;
}

static void release(rlqr_handle* h) {
  if (!h) return;
  (void)hipDeviceSynchronize();
  for (void* p : h->allocs) (void)hipFree(p);
  h->allocs.clear();
}

extern "C" {

const char* rlqr_status_string(rlqr_status s) {
  switch (s) {
    case RLQR_OK: return "ok";
    case RLQR_E_INVALID: return "invalid argument";
    case RLQR_E_NOMEM: return "out of device memory";
    case RLQR_E_HIP: return "HIP runtime error";
    case RLQR_E_STATE: return "no factorization (call rlqr_factor first)";
    case RLQR_E_UNSUPPORTED: return "unsupported mode for these shapes";
  }
  return "unknown status";
}

rlqr_status rlqr_create(rlqr_handle** hp, const rlqr_shape* s, rlqr_mode mode, size_t* workspace_bytes) {
  if (!hp) return RLQR_E_INVALID;
  *hp = nullptr;
  if (!s || s->batch < 0) return RLQR_E_INVALID;
  if (mode != RLQR_SEQ_FP64 && mode != RLQR_SEQ_MIXED) return RLQR_E_INVALID;
  const int B = s->batch;
  if (B > 0 && (!s->N || !s->nx || !s->nu)) return RLQR_E_INVALID;
  for (int b = 0; b < B; ++b) {
    const int N = s->N[b], n = s->nx[b], m = s->nu[b];
    if (N < 0 || n < 1 || m < 1 || n > RLQR_MAX_NX || n + m > RLQR_MAX_NXU) return RLQR_E_INVALID;
    if (tile_class(n, m) < 0) return RLQR_E_INVALID;
  }
  rlqr_handle* h = new (std::nothrow) rlqr_handle();
  if (!h) return RLQR_E_NOMEM;
  h->B = B;
  h->mode = mode;
  h->N.assign(s->N, s->N + B);
  h->n.assign(s->nx, s->nx + B);
  h->m.assign(s->nu, s->nu + B);
  for (auto& o : h->off) o.assign(B + 1, 0);
  std::vector<InstMeta> meta(B);
  std::vector<int64_t> stage_off(B + 1, 0);
  std::vector<int32_t> cls(B), fused(B);
  std::vector<std::vector<int32_t>> lists(TILE_CLASSES);
  int64_t ws_elems = 0, pk_elems = 0;
  for (int b = 0; b < B; ++b) {
    const int64_t N = h->N[b], n = h->n[b], m = h->m[b];
    const int64_t cnt[RLQR_ARR_COUNT] = {(N + 1) * n * n, N * n * m, N * m * m, N * n * n, N * n * m,
                                         (N + 1) * n,     N * m,     (N + 1) * n, (N + 1) * n, N * m,
                                         (N + 1) * n,     N * (n + m) + n + (N + 1) * n};
    for (int k = 0; k < RLQR_ARR_COUNT; ++k) h->off[k][b + 1] = h->off[k][b] + cnt[k];
    InstMeta& mt = meta[b];
    mt.N = (int32_t)N; mt.n = (int32_t)n; mt.m = (int32_t)m; mt.pad = 0;
    mt.oQ = h->off[RLQR_ARR_Q][b]; mt.oM = h->off[RLQR_ARR_M][b]; mt.oR = h->off[RLQR_ARR_R][b];
    mt.oA = h->off[RLQR_ARR_A][b]; mt.oB = h->off[RLQR_ARR_B][b];
    mt.oq = h->off[RLQR_ARR_q][b]; mt.or_ = h->off[RLQR_ARR_r][b]; mt.oc = h->off[RLQR_ARR_c][b];
    mt.ox = h->off[RLQR_ARR_x][b]; mt.ou = h->off[RLQR_ARR_u][b]; mt.oy = h->off[RLQR_ARR_y][b];
    mt.ores = h->off[RLQR_ARR_RES][b];
    mt.ows = ws_elems;
    mt.opk = pk_elems;
    cls[b] = tile_class((int)n, (int)m);
    fused[b] = cls[b] == TILE_16 ? 1 : 0;
    lists[cls[b]].push_back(b);
    ws_elems += (N + 1) * tile_blocks_per_stage(cls[b]) * 256;
    pk_elems += (N + 1) * n + N * m;
    stage_off[b + 1] = stage_off[b] + N + 1;
  }
  h->total_stage_blocks = stage_off[B];
  std::vector<int32_t> blk_inst(h->total_stage_blocks > 0 ? h->total_stage_blocks : 1, 0);
  for (int b = 0; b < B; ++b)
    for (int64_t i = stage_off[b]; i < stage_off[b + 1]; ++i) blk_inst[i] = b;

  rlqr_status st = RLQR_OK;
  auto A = [&](void** p, size_t bytes) {
    if (st == RLQR_OK) st = dev_alloc(h, p, bytes);
  };
  A((void**)&h->meta, sizeof(InstMeta) * (size_t)B);
  A((void**)&h->stage_off, sizeof(int64_t) * (size_t)(B + 1));
  A((void**)&h->blk_inst, sizeof(int32_t) * blk_inst.size());
  A(&h->ws64, sizeof(double) * (size_t)ws_elems);
  if (mode == RLQR_SEQ_MIXED) A(&h->ws32, sizeof(float) * (size_t)ws_elems);
  A((void**)&h->pk, sizeof(double) * (size_t)pk_elems);
  A((void**)&h->res[0], sizeof(double) * (size_t)h->off[RLQR_ARR_RES][B]);
  A((void**)&h->res[1], sizeof(double) * (size_t)h->off[RLQR_ARR_RES][B]);
  A((void**)&h->info, sizeof(FactorInfo) * (size_t)B);
  A((void**)&h->fused, sizeof(int32_t) * (size_t)B);
  for (int c = 0; c < TILE_CLASSES; ++c) {
    h->count[c] = (int)lists[c].size();
    if (h->count[c] > 0) A((void**)&h->list[c], sizeof(int32_t) * lists[c].size());
  }
  A((void**)&h->resmax, sizeof(unsigned long long) * (size_t)B);
  A((void**)&h->bmax, sizeof(unsigned long long) * (size_t)B);
  int32_t** i32s[] = {&h->flag64, &h->conv, &h->run32, &h->run64, &h->runres, &h->fb, &h->status};
  for (auto pp : i32s) A((void**)pp, sizeof(int32_t) * (size_t)B);
  A((void**)&h->lastrel, sizeof(double) * (size_t)B);
  A((void**)&h->relres, sizeof(double) * (size_t)B);
  if (st == RLQR_OK && B > 0) {
    if (hipMemcpy(h->meta, meta.data(), sizeof(InstMeta) * B, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->stage_off, stage_off.data(), sizeof(int64_t) * (B + 1), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->blk_inst, blk_inst.data(), sizeof(int32_t) * blk_inst.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(h->fused, fused.data(), sizeof(int32_t) * B, hipMemcpyHostToDevice) != hipSuccess)
      st = RLQR_E_HIP;
    for (int c = 0; c < TILE_CLASSES && st == RLQR_OK; ++c)
      if (h->count[c] > 0 &&
          hipMemcpy(h->list[c], lists[c].data(), sizeof(int32_t) * lists[c].size(), hipMemcpyHostToDevice) != hipSuccess)
        st = RLQR_E_HIP;
    std::vector<int32_t> f(B, mode == RLQR_SEQ_FP64 ? 1 : 0);
    if (st == RLQR_OK && hipMemcpy(h->flag64, f.data(), sizeof(int32_t) * B, hipMemcpyHostToDevice) != hipSuccess)
      st = RLQR_E_HIP;
  }
  if (st != RLQR_OK) {
    release(h);
    delete h;
    return st;
  }
  if (workspace_bytes) *workspace_bytes = h->bytes;
  *hp = h;
  return RLQR_OK;
}

rlqr_status rlqr_layout_offsets(const rlqr_handle* h, int32_t array, int64_t* off) {
  if (!h || !off || array < 0 || array >= RLQR_ARR_COUNT) return RLQR_E_INVALID;
  std::memcpy(off, h->off[array].data(), sizeof(int64_t) * (h->B + 1));
  return RLQR_OK;
}

static FactorArgs factor_args(rlqr_handle* h, void* ws, const int32_t* run) {
  FactorArgs a{};
  a.meta = h->meta; a.list = nullptr; a.run = run;
  a.Q = h->lhs.Q; a.M = h->lhs.M; a.R = h->lhs.R; a.A = h->lhs.A; a.B = h->lhs.B; a.delta = h->lhs.delta;
  a.ws = ws; a.info = h->info;
  return a;
}

// one factor launch per tile class
static hipError_t factor_all(rlqr_handle* h, void* ws, const int32_t* run, bool fp32, hipStream_t st) {
  for (int c = 0; c < TILE_CLASSES; ++c) {
    if (h->count[c] == 0) continue;
    FactorArgs a = factor_args(h, ws, run);
    a.list = h->list[c];
    hipError_t e = (c == TILE_16) ? launch_factor(a, h->count[c], fp32, st)
                                  : launch_factor_mw(c, a, h->count[c], fp32, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

rlqr_status rlqr_factor(rlqr_handle* h, const rlqr_lhs* lhs, rlqr_stream stv) {
  if (!h || !lhs) return RLQR_E_INVALID;
  if (h->B > 0 && (!lhs->Q || !lhs->M || !lhs->R || !lhs->A || !lhs->B || !lhs->delta)) return RLQR_E_INVALID;
  h->lhs = *lhs;
  h->factored = true;
  if (h->B == 0) return RLQR_OK;
  hipStream_t st = (hipStream_t)stv;
  if (h->mode == RLQR_SEQ_FP64) {
    if (factor_all(h, h->ws64, nullptr, false, st) != hipSuccess) return RLQR_E_HIP;
    return RLQR_OK;
  }
  // mixed: float32 products everywhere, then float64 for instances whose pivots
  // fall inside the guard band
  if (factor_all(h, h->ws32, nullptr, true, st) != hipSuccess) return RLQR_E_HIP;
  MaskArgs m{};
  m.batch = h->B; m.kind = 1; m.guard = kGuard; m.info = h->info; m.flag64 = h->flag64;
  if (launch_masks(m, st) != hipSuccess) return RLQR_E_HIP;
  if (factor_all(h, h->ws64, h->flag64, false, st) != hipSuccess) return RLQR_E_HIP;
  return RLQR_OK;
}

static SolveArgs solve_args(rlqr_handle* h, const rlqr_rhs* rhs, rlqr_sol* out, bool fp32, const int32_t* run,
                            const double* corr, double* res_out) {
  SolveArgs a{};
  a.meta = h->meta; a.list = nullptr; a.run = run;
  a.Q = h->lhs.Q; a.M = h->lhs.M; a.R = h->lhs.R; a.A = h->lhs.A; a.B = h->lhs.B; a.delta = h->lhs.delta;
  a.ws = fp32 ? h->ws32 : h->ws64;
  a.info = h->info;
  a.q = rhs->q; a.r = rhs->r; a.c = rhs->c;
  a.corr = corr;
  a.x = out->x; a.u = out->u; a.y = out->y;
  a.pk = h->pk;
  a.res_out = res_out;
  a.resmax = h->resmax; a.bmax = h->bmax;
  return a;
}

static ResidualArgs residual_args(rlqr_handle* h, const rlqr_rhs* rhs, const rlqr_sol* z, double* res,
                                  const int32_t* run) {
  ResidualArgs a{};
  a.batch = h->B; a.meta = h->meta; a.blk_inst = h->blk_inst; a.stage_off = h->stage_off;
  a.run = run; a.skip = nullptr; a.info = h->info;
  a.Q = h->lhs.Q; a.M = h->lhs.M; a.R = h->lhs.R; a.A = h->lhs.A; a.B = h->lhs.B; a.delta = h->lhs.delta;
  a.q = rhs->q; a.r = rhs->r; a.c = rhs->c;
  a.x = z->x; a.u = z->u; a.y = z->y;
  a.res = res; a.resmax = h->resmax; a.bmax = h->bmax;
  return a;
}

static CheckArgs check_args(rlqr_handle* h, int final_pass, double tol, const int32_t* run) {
  CheckArgs a{};
  a.batch = h->B; a.final_pass = final_pass; a.plain = 0; a.tol = tol; a.info = h->info; a.run = run;
  a.resmax = h->resmax; a.bmax = h->bmax; a.conv = h->conv; a.lastrel = h->lastrel;
  a.status = h->status; a.relres = h->relres;
  return a;
}

#define RLQR_TRY(x)                        \
  do {                                     \
    if ((x) != hipSuccess) return RLQR_E_HIP; \
  } while (0)

// one solve launch per tile class and precision; run masks select instances
static rlqr_status solve_launch(rlqr_handle* h, const rlqr_rhs* rhs, rlqr_sol* out, bool fp32, const int32_t* run,
                                const double* corr, double* res_out, hipStream_t st) {
  for (int c = 0; c < TILE_CLASSES; ++c) {
    if (h->count[c] == 0) continue;
    SolveArgs a = solve_args(h, rhs, out, fp32, run, corr, res_out);
    a.list = h->list[c];
    hipError_t e = (c == TILE_16) ? launch_solve(a, h->count[c], fp32, st)
                                  : launch_solve_mw(c, a, h->count[c], fp32, st);
    if (e != hipSuccess) return RLQR_E_HIP;
  }
  return RLQR_OK;
}

// Pass p of the refinement: solve (p == 0) or correct (p > 0) every
// instance not yet converged, then its residual (fused for one-wavefront
// instances, a separate kernel for the others) and the convergence check.
static rlqr_status solve_pass(rlqr_handle* h, const rlqr_rhs* rhs, rlqr_sol* out, int pass, double tol,
                              const int32_t* run64_override, hipStream_t st) {
  const double* corr = pass == 0 ? nullptr : h->res[(pass - 1) & 1];
  double* res_out = h->res[pass & 1];
  const int32_t *r32 = nullptr, *r64 = nullptr, *rres = nullptr;
  if (run64_override) {
    r64 = run64_override;
    rres = run64_override;
  } else {
    MaskArgs m{};
    m.batch = h->B; m.kind = 0; m.flag64 = h->flag64; m.conv = h->conv;
    m.run32 = h->run32; m.run64 = h->run64; m.runres = h->runres;
    RLQR_TRY(launch_masks(m, st));
    r32 = h->run32; r64 = h->run64; rres = h->runres;
  }
  rlqr_status s;
  if (h->mode == RLQR_SEQ_MIXED && !run64_override)
    if ((s = solve_launch(h, rhs, out, true, r32, corr, res_out, st)) != RLQR_OK) return s;
  if ((s = solve_launch(h, rhs, out, false, r64, corr, res_out, st)) != RLQR_OK) return s;
  bool any_unfused = false;
  for (int c = 1; c < TILE_CLASSES; ++c) any_unfused |= h->count[c] > 0;
  if (any_unfused) {
    ResidualArgs ra = residual_args(h, rhs, out, res_out, rres);
    ra.skip = h->fused;
    RLQR_TRY(launch_residual(ra, h->total_stage_blocks, st));
  }
  RLQR_TRY(launch_check(check_args(h, 0, tol, rres), st));
  return RLQR_OK;
}

rlqr_status rlqr_solve(rlqr_handle* h, const rlqr_rhs* rhs, rlqr_sol* out, double rel_tol, int32_t max_refine,
                       int32_t* inst_status, double* inst_relres, rlqr_stream stv) {
  if (!h || !rhs || !out) return RLQR_E_INVALID;
  if (!h->factored) return RLQR_E_STATE;
  if (h->B == 0) return RLQR_OK;
  if (!rhs->q || !rhs->r || !rhs->c || !out->x || !out->u || !out->y) return RLQR_E_INVALID;
  if (!(rel_tol >= 0.0) || max_refine < 0) return RLQR_E_INVALID;
  hipStream_t st = (hipStream_t)stv;
  rlqr_status s;

  RLQR_TRY(launch_fill_i32(h->conv, h->B, 0, st));
  for (int pass = 0; pass <= max_refine; ++pass)
    if ((s = solve_pass(h, rhs, out, pass, rel_tol, nullptr, st)) != RLQR_OK) return s;
  RLQR_TRY(launch_check(check_args(h, 1, rel_tol, nullptr), st));

  if (h->mode == RLQR_SEQ_MIXED) {
    // instances that did not converge from float32 tiles: redo them in float64
    MaskArgs m{};
    m.batch = h->B; m.kind = 2; m.flag64 = h->flag64; m.conv = h->conv; m.status = h->status; m.fb = h->fb;
    RLQR_TRY(launch_masks(m, st));
    RLQR_TRY(factor_all(h, h->ws64, h->fb, false, st));
    const int extra = std::min<int32_t>(max_refine, 2);
    for (int pass = 0; pass <= extra; ++pass) {
      if (pass > 0) {
        MaskArgs mm{};
        mm.batch = h->B; mm.kind = 3; mm.fb = h->fb; mm.conv = h->conv; mm.run64 = h->run64;
        RLQR_TRY(launch_masks(mm, st));
      }
      if ((s = solve_pass(h, rhs, out, pass, rel_tol, pass == 0 ? h->fb : h->run64, st)) != RLQR_OK) return s;
    }
    RLQR_TRY(launch_check(check_args(h, 1, rel_tol, h->fb), st));
  }
  if (inst_status)
    RLQR_TRY(hipMemcpyAsync(inst_status, h->status, sizeof(int32_t) * h->B, hipMemcpyDeviceToDevice, st));
  if (inst_relres)
    RLQR_TRY(hipMemcpyAsync(inst_relres, h->relres, sizeof(double) * h->B, hipMemcpyDeviceToDevice, st));
  return RLQR_OK;
}

rlqr_status rlqr_pivot_inertia(rlqr_handle* h, int32_t* pd_verdict, int32_t* first_bad, int64_t* inertia,
                               rlqr_stream stv) {
  if (!h) return RLQR_E_INVALID;
  if (!h->factored) return RLQR_E_STATE;
  InertiaArgs a{};
  a.batch = h->B; a.info = h->info; a.verdict = pd_verdict; a.first_bad = first_bad; a.inertia = inertia;
  RLQR_TRY(launch_inertia(a, (hipStream_t)stv));
  return RLQR_OK;
}

rlqr_status rlqr_residual(rlqr_handle* h, const rlqr_rhs* rhs, const rlqr_sol* z, double* res,
                          double* inst_relres, rlqr_stream stv) {
  if (!h || !rhs || !z) return RLQR_E_INVALID;
  if (!h->factored) return RLQR_E_STATE;
  if (h->B == 0) return RLQR_OK;
  if (!rhs->q || !rhs->r || !rhs->c || !z->x || !z->u || !z->y) return RLQR_E_INVALID;
  hipStream_t st = (hipStream_t)stv;
  // clear the per-instance maxima (a fill kernel over their 32-bit halves)
  RLQR_TRY(launch_fill_i32(reinterpret_cast<int32_t*>(h->resmax), 2 * h->B, 0, st));
  RLQR_TRY(launch_fill_i32(reinterpret_cast<int32_t*>(h->bmax), 2 * h->B, 0, st));
  ResidualArgs a = residual_args(h, rhs, z, res, nullptr);
  a.info = nullptr;  // evaluate every instance at the given z, singular ones included
  RLQR_TRY(launch_residual(a, h->total_stage_blocks, st));
  if (inst_relres) {
    CheckArgs c = check_args(h, 1, 0.0, nullptr);
    c.plain = 1;
    c.relres = inst_relres;
    RLQR_TRY(launch_check(c, st));
  }
  return RLQR_OK;
}

void rlqr_destroy(rlqr_handle* h) {
  if (!h) return;
  release(h);
  delete h;
}

}  // extern "C"
