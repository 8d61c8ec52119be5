// rlqr_api.hip -- host side of the C ABI declared in include/rlqr.h.
//
// Owns the handle: shape metadata, packed-layout offsets, the factorization
// workspace and the per-instance flags that steer the precision of each
// instance:
//   flag64[b]  instance uses the float64 factorization (always in RLQR_SEQ_FP64;
//              otherwise when a pivot falls inside the guard band, the scan
//              failed, or refinement from float32 tiles did not converge)
//   conv[b]    refinement converged
// Work is cut into segments (SegDesc): in the sequential modes one segment
// per instance; in the scan modes the horizon of an instance is cut into
// segments of L stages whose boundary cost-to-go comes from the scan.
// All launches are asynchronous on the caller's stream; no call after
// rlqr_create allocates memory or synchronizes with the host.
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

// element tile size of the scan for state size n (16, 32 or 64 rows)
inline int scan_tx(int n) { return n <= 16 ? 1 : (n <= 32 ? 2 : 4); }
inline int scan_group(int n) { return n <= 16 ? 0 : (n <= 32 ? 1 : 2); }

struct SegList {
  SegDesc* d = nullptr;
  int count = 0;
};

// Instances of one element tile size that take part in the scan.
struct ScanGroup {
  int tx = 0, tm = 0, ninst = 0, maxN = 0, maxchunks = 0;
  int32_t* insts = nullptr;
  int64_t *eoff = nullptr, *aoff = nullptr;
  float* elems = nullptr;
  float* aggr[2] = {nullptr, nullptr};
  float* pce = nullptr;                  // carried p, c (scan_carry_pc)
  float* pca[2] = {nullptr, nullptr};
};

}  // namespace

struct rlqr_handle {
  int B = 0;
  rlqr_mode mode = RLQR_SEQ_FP64;
  int chunk = 0;  // scan mode: stages per segment
  int shape16 = SHAPE_ANY;  // fixed stage shape shared by every one-wavefront instance
  int shape_all = SHAPE_ANY;  // fixed stage shape shared by every instance of the batch
  std::vector<int32_t> N, n, m;
  std::vector<int64_t> off[RLQR_ARR_COUNT];
  size_t bytes = 0;

  InstMeta* meta = nullptr;
  ResChunk* chunks = nullptr;     // residual work units
  int64_t nchunks = 0;
  void* ws64 = nullptr;   // float64 tiles
  void* ws32 = nullptr;   // float32 tiles (mixed and scan modes)
  double* pk = nullptr;   // p_i / k_i scratch
  double* res[2] = {nullptr, nullptr};  // residual vectors (ping-pong between passes)
  FactorInfo* info = nullptr;

  // one segment per instance, by tile class (factor); instance lists (solve)
  SegList whole[TILE_CLASSES];
  int32_t* list[TILE_CLASSES] = {};
  int count[TILE_CLASSES] = {};
  int32_t* whole_off = nullptr;   // [B + 1]: b
  SegStats* whole_stats = nullptr;

  // scan mode
  SegList fseg[TILE_CLASSES];     // every segment (factor)
  SegList sseg[TILE_CLASSES];     // segments of multi-segment instances (solve, transfer)
  int32_t* seg_off = nullptr;     // [B + 1]
  SegStats* seg_stats = nullptr;
  ScanGroup grp[3];
  int32_t* multi_list = nullptr;  // instances with two or more segments
  int nmulti = 0;
  int32_t* multi = nullptr;       // [B] 1 if the instance has two or more segments
  int32_t* bad = nullptr;         // [B] scan failed
  int32_t* run1 = nullptr;        // [B] float32 run mask of single-segment instances
  double *psi = nullptr, *plo = nullptr, *xhi = nullptr;

  unsigned long long *resmax = nullptr, *bmax = nullptr;
  int32_t *flag64 = nullptr, *conv = nullptr, *run32 = nullptr, *run64 = nullptr,
          *runres = nullptr, *fb = nullptr, *status = nullptr;
  double *lastrel = nullptr, *relres = nullptr;

  int32_t* path = nullptr;       // [B] precision path of the last factor / solve (RLQR_PATH_*)
  int32_t* pref32 = nullptr;     // [B] float32 attempt allowed (mixed and scan modes)
  const int32_t* skip = nullptr;  // [B] caller's mask of instances left out (rlqr_set_skip)
  int32_t *runf = nullptr, *runf2 = nullptr;  // [B] factor run masks under the skip mask
  bool any_pref64 = false;

  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;

  // Batches with instances in two or more tile classes run the classes'
  // factor and solve launches side by side: class c > first on side[c],
  // forked from and joined back to the caller's stream with events (the same
  // in graph capture). Each class launch is bound by its longest instance's
  // sequential stage loop, so one after another they would add up.
  hipStream_t side[TILE_CLASSES] = {};
  hipEvent_t ev_fork = nullptr, ev_join[TILE_CLASSES] = {};
  bool owns_streams = false;

  rlqr_lhs lhs{};
  bool factored = false;
  bool pk_fused = false;  // pk holds the backward vector pass for pk_rhs (rlqr_factor_rhs)
  int32_t* resfuse = nullptr;        // [B] residual computed by the one-wavefront solve (n + m <= 16, one segment)
  ResChunk* chunks_nf = nullptr;     // residual chunks of the other instances
  int64_t nchunks_nf = 0;
  // the same chunks by tile class: in float64 mode each class's residual runs
  // on its own stream right after its solve, beside the other classes' solves
  ResChunk* cls_chunks[TILE_CLASSES] = {};
  int64_t cls_nchunks[TILE_CLASSES] = {};
  bool cls_res = false;
  rlqr_rhs pk_rhs{};
  // scan_carry_pc: the last rlqr_factor_rhs carried p through the scan and
  // wrote the segments' boundary p for this right-hand side into plo
  bool carry_pc = false, pc_valid = false;
  rlqr_rhs pc_rhs{};
  std::vector<void*> allocs;

  // Stacked right-hand sides (rlqr_solve_multi, sequential modes): mv is a
  // handle over a virtual batch of max_rhs * B instances, instance j*B + b
  // being right-hand side j of instance b. It shares this handle's tiles and
  // left-hand side; its vectors sit at j times the batch lengths. A call
  // with r right-hand sides uses the first r*B virtual instances.
  int max_rhs = 1;
  int mw_waves = 4;  // wavefronts per workgroup of the multi-wavefront classes up to 32 x 48 (1, 2, 4 or 8)
  rlqr_handle* mv = nullptr;
  int Bbase = 0;                                   // (mv) instances per right-hand side
  int base_count[TILE_CLASSES] = {};               // (mv) per right-hand side
  int64_t base_nchunks = 0, base_nchunks_nf = 0;   // (mv) per right-hand side
  std::vector<int32_t*> mlist[TILE_CLASSES];       // (mv) [r - 1]: launch order for r right-hand sides
  double* vdelta = nullptr;                        // (mv) delta per virtual instance
};

static bool is_scan(rlqr_mode m) { return m == RLQR_SCAN_FP32 || m == RLQR_SCAN_BF16; }

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

static void drop_graph(rlqr_handle* h) {
  if (h->graph_exec) (void)hipGraphExecDestroy(h->graph_exec);
  if (h->graph) (void)hipGraphDestroy(h->graph);
  h->graph_exec = nullptr;
  h->graph = nullptr;
}

static void release(rlqr_handle* h) {
  if (!h) return;
  (void)hipDeviceSynchronize();
  drop_graph(h);
  if (h->owns_streams) {
    for (int c = 0; c < TILE_CLASSES; ++c) {
      if (h->side[c]) (void)hipStreamDestroy(h->side[c]);
      if (h->ev_join[c]) (void)hipEventDestroy(h->ev_join[c]);
    }
    if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  }
  for (int c = 0; c < TILE_CLASSES; ++c) { h->side[c] = nullptr; h->ev_join[c] = nullptr; }
  h->ev_fork = nullptr;
  h->owns_streams = false;
  if (h->mv) {
    release(h->mv);
    delete h->mv;
    h->mv = nullptr;
  }
  for (void* p : h->allocs) (void)hipFree(p);
  h->allocs.clear();
}

template <typename T>
static bool upload(T* dst, const std::vector<T>& src) {
  if (src.empty()) return true;
  return hipMemcpy(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice) == hipSuccess;
}

#define RLQR_TRY(x)                           \
  do {                                        \
    if ((x) != hipSuccess) return RLQR_E_HIP; \
  } while (0)

// Virtual instance j*B + b (right-hand side j of instance b) takes b's
// certificate bookkeeping, float64 flag and delta at the start of each
// stacked solve (the factorization of b may have changed them).
struct ReplicateArgs {
  int B, total;
  const FactorInfo* info;
  const int32_t* flag64;
  const double* delta;
  FactorInfo* vinfo;
  int32_t* vflag64;
  double* vdelta;
};

__global__ void k_replicate(ReplicateArgs a) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= a.total) return;
  const int b = v % a.B;
  a.vinfo[v] = a.info[b];
  a.vflag64[v] = a.flag64[b];
  a.vdelta[v] = a.delta ? a.delta[b] : 0.0;  // NULL with a per-stage diagonal
}

// The virtual handle of rlqr_handle::mv for R right-hand sides (sequential
// modes). Launch order of class c for r right-hand sides: the class's
// instances in groups of 8 consecutive list positions t = 8s + x; right-hand
// side j of position t goes to launch index (s*r + j)*8 + x, so the r
// workgroups of one instance are 8 apart, which places them on the same XCD
// (workgroups are dealt round-robin to the 8 XCDs) at about the same time;
// the last C mod 8 positions follow in order.
static rlqr_status build_multi(rlqr_handle* h, int R, const std::vector<InstMeta>& meta,
                               const std::vector<ResChunk>& chunks, const std::vector<ResChunk>& chunks_nf,
                               const std::vector<int32_t>& resfuse, const std::vector<std::vector<int32_t>>& lists,
                               const std::vector<int32_t>& pref64, int64_t pk_elems) {
  const int B = h->B;
  if ((int64_t)R * B > (int64_t)INT32_MAX / 2) return RLQR_E_INVALID;
  const int VB = R * B;
  rlqr_handle* v = new (std::nothrow) rlqr_handle();
  if (!v) return RLQR_E_NOMEM;
  v->B = VB; v->mode = h->mode; v->chunk = h->chunk; v->shape16 = h->shape16; v->shape_all = h->shape_all;
  v->mw_waves = h->mw_waves;
  v->ws64 = h->ws64; v->ws32 = h->ws32;  // shared, owned by h
  for (int c = 0; c < TILE_CLASSES; ++c) { v->side[c] = h->side[c]; v->ev_join[c] = h->ev_join[c]; }
  v->ev_fork = h->ev_fork;  // shared, owned by h (v->owns_streams stays false)
  v->any_pref64 = h->any_pref64;
  v->Bbase = B;
  const int64_t Lq = h->off[RLQR_ARR_q][B], Lr = h->off[RLQR_ARR_r][B], Lc = h->off[RLQR_ARR_c][B],
                Lres = h->off[RLQR_ARR_RES][B];
  std::vector<InstMeta> vm((size_t)VB);
  std::vector<int32_t> vres((size_t)VB), vwoff((size_t)VB + 1), vflag((size_t)VB), vpref((size_t)VB);
  for (int j = 0; j < R; ++j)
    for (int b = 0; b < B; ++b) {
      InstMeta mt = meta[b];
      mt.oq += j * Lq; mt.or_ += j * Lr; mt.oc += j * Lc;
      mt.ox += j * Lq; mt.ou += j * Lr; mt.oy += j * Lc;
      mt.ores += j * Lres; mt.opk += j * pk_elems;
      const int vi = j * B + b;
      vm[vi] = mt;
      vres[vi] = resfuse[b];
      vflag[vi] = (h->mode == RLQR_SEQ_FP64 || pref64[b]) ? 1 : 0;
      vpref[vi] = pref64[b] ? 0 : 1;
    }
  for (int i = 0; i <= VB; ++i) vwoff[i] = i;
  std::vector<ResChunk> vch, vchnf;
  for (int j = 0; j < R; ++j) {
    for (ResChunk c : chunks) { c.inst += j * B; vch.push_back(c); }
    for (ResChunk c : chunks_nf) { c.inst += j * B; vchnf.push_back(c); }
  }
  v->base_nchunks = (int64_t)chunks.size();
  v->base_nchunks_nf = (int64_t)chunks_nf.size();
  v->nchunks = (int64_t)vch.size();
  v->nchunks_nf = (int64_t)vchnf.size();

  rlqr_status st = RLQR_OK;
  auto A = [&](void** p, size_t bytes) {
    if (st == RLQR_OK) st = dev_alloc(v, p, bytes);
  };
  A((void**)&v->meta, sizeof(InstMeta) * (size_t)VB);
  A((void**)&v->chunks, sizeof(ResChunk) * std::max<size_t>(vch.size(), 1));
  A((void**)&v->chunks_nf, sizeof(ResChunk) * std::max<size_t>(vchnf.size(), 1));
  A((void**)&v->resfuse, sizeof(int32_t) * (size_t)VB);
  A((void**)&v->pk, sizeof(double) * (size_t)(R * pk_elems));
  A((void**)&v->res[0], sizeof(double) * (size_t)(R * Lres));
  A((void**)&v->res[1], sizeof(double) * (size_t)(R * Lres));
  A((void**)&v->info, sizeof(FactorInfo) * (size_t)VB);
  A((void**)&v->whole_off, sizeof(int32_t) * (size_t)(VB + 1));
  A((void**)&v->whole_stats, sizeof(SegStats) * (size_t)VB);
  A((void**)&v->resmax, sizeof(unsigned long long) * (size_t)VB);
  A((void**)&v->bmax, sizeof(unsigned long long) * (size_t)VB);
  int32_t** i32s[] = {&v->flag64, &v->conv, &v->run32, &v->run64, &v->runres, &v->fb, &v->status};
  for (auto pp : i32s) A((void**)pp, sizeof(int32_t) * (size_t)VB);
  A((void**)&v->lastrel, sizeof(double) * (size_t)VB);
  A((void**)&v->relres, sizeof(double) * (size_t)VB);
  A((void**)&v->vdelta, sizeof(double) * (size_t)VB);
  if (h->mode != RLQR_SEQ_FP64) A((void**)&v->pref32, sizeof(int32_t) * (size_t)VB);
  std::vector<std::vector<int32_t>> mlist_h[TILE_CLASSES];
  std::vector<std::vector<SegDesc>> whole_d(TILE_CLASSES);
  for (int c = 0; c < TILE_CLASSES; ++c) {
    const int C = (int)lists[c].size();
    v->base_count[c] = C;
    v->count[c] = R * C;
    v->whole[c].count = R * C;
    if (C == 0) continue;
    for (int j = 0; j < R; ++j)
      for (int b : lists[c]) {
        SegDesc d{};
        d.inst = j * B + b; d.lo = 0; d.hi = h->N[b]; d.p0_ld = 0; d.gidx = j * B + b; d.s = 0; d.P0 = nullptr;
        whole_d[c].push_back(d);
      }
    A((void**)&v->whole[c].d, sizeof(SegDesc) * whole_d[c].size());
    const int S8 = C / 8, T = C % 8;
    for (int r = 1; r <= R; ++r) {
      std::vector<int32_t> L((size_t)r * C, -1);
      for (int t = 0; t < C; ++t) {
        const int b = lists[c][t];
        for (int j = 0; j < r; ++j) {
          const int64_t i = t < 8 * S8 ? ((int64_t)(t / 8) * r + j) * 8 + (t % 8)
                                       : (int64_t)8 * S8 * r + (int64_t)j * T + (t - 8 * S8);
          L[(size_t)i] = j * B + b;
        }
      }
      mlist_h[c].push_back(L);
      int32_t* d = nullptr;
      A((void**)&d, sizeof(int32_t) * L.size());
      v->mlist[c].push_back(d);
    }
    v->list[c] = v->mlist[c][R - 1];
  }
  if (st == RLQR_OK) {
    bool ok = upload(v->meta, vm) && upload(v->chunks, vch) && upload(v->chunks_nf, vchnf) &&
              upload(v->resfuse, vres) && upload(v->whole_off, vwoff) && upload(v->flag64, vflag);
    if (ok && h->mode != RLQR_SEQ_FP64) ok = upload(v->pref32, vpref);
    for (int c = 0; c < TILE_CLASSES && ok; ++c) {
      if (lists[c].empty()) continue;
      ok = upload(v->whole[c].d, whole_d[c]);
      for (int r = 0; r < R && ok; ++r) ok = upload(v->mlist[c][r], mlist_h[c][r]);
    }
    if (!ok) st = RLQR_E_HIP;
  }
  if (st != RLQR_OK) {
    release(v);
    delete v;
    return st;
  }
  h->bytes += v->bytes;
  h->mv = v;
  h->max_rhs = R;
  return RLQR_OK;
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

rlqr_status rlqr_create_tuned(rlqr_handle** hp, const rlqr_shape* s, rlqr_mode mode, const rlqr_tuning* tune,
                              size_t* workspace_bytes) {
  if (!hp) return RLQR_E_INVALID;
  *hp = nullptr;
  if (!s || s->batch < 0) return RLQR_E_INVALID;
  if (mode != RLQR_SEQ_FP64 && mode != RLQR_SEQ_MIXED && mode != RLQR_SCAN_FP32 && mode != RLQR_SCAN_BF16)
    return RLQR_E_INVALID;
  if (tune && (tune->scan_chunk < 0 || tune->max_rhs < 0)) return RLQR_E_INVALID;
  if (tune && tune->mw_waves != 0 && tune->mw_waves != 1 && tune->mw_waves != 2 && tune->mw_waves != 4 &&
      tune->mw_waves != 8)
    return RLQR_E_INVALID;
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
  const bool scan = is_scan(mode);
  h->carry_pc = scan && tune && tune->scan_carry_pc != 0;
  h->mw_waves = (tune && tune->mw_waves != 0) ? tune->mw_waves : 4;

  // segment length: about one segment per compute unit (256) over the whole
  // batch, so the chunk folds and the segment recursions run in one round and
  // the boundary chains stay short
  int64_t total_elems = 0;
  for (int b = 0; b < B; ++b) total_elems += h->N[b] + 1;
  const int L = tune && tune->scan_chunk > 0 ? tune->scan_chunk : (int)std::min<int64_t>(
                                                                      std::max<int64_t>((total_elems + 255) / 256, 8), 1 << 20);
  h->chunk = L;
  std::vector<int32_t> Lb(B, L), pref64(B, 0);
  if (tune && tune->inst_chunk)
    for (int b = 0; b < B; ++b) {
      if (tune->inst_chunk[b] < 0) { delete h; return RLQR_E_INVALID; }
      Lb[b] = tune->inst_chunk[b] > 0 ? tune->inst_chunk[b] : std::max(h->N[b], 1);
    }
  if (tune && tune->inst_fp64 && mode != RLQR_SEQ_FP64)
    for (int b = 0; b < B; ++b) pref64[b] = tune->inst_fp64[b] ? 1 : 0;
  for (int b = 0; b < B; ++b) h->any_pref64 = h->any_pref64 || pref64[b];

  for (auto& o : h->off) o.assign(B + 1, 0);
  std::vector<InstMeta> meta(B);
  std::vector<int32_t> cls(B), nseg(B, 1), seg_off(B + 1, 0), whole_off(B + 1, 0), multi(B, 0), multi_list;
  std::vector<std::vector<int32_t>> lists(TILE_CLASSES);
  int64_t ws_elems = 0, pk_elems = 0, vec_elems = 0, psi_elems = 0;
  for (int b = 0; b < B; ++b) {
    const int64_t N = h->N[b], n = h->n[b], m = h->m[b];
    const int64_t cnt[RLQR_ARR_COUNT] = {(N + 1) * n * n, N * n * m, N * m * m, N * n * n, N * n * m,
                                         (N + 1) * n,     N * m,     (N + 1) * n, (N + 1) * n, N * m,
                                         (N + 1) * n,     N * (n + m) + n + (N + 1) * n};
    for (int k = 0; k < RLQR_ARR_COUNT; ++k) h->off[k][b + 1] = h->off[k][b] + cnt[k];
    cls[b] = tile_class((int)n, (int)m);
    lists[cls[b]].push_back(b);
    if (scan && !pref64[b] && N > Lb[b]) nseg[b] = (int)((N + Lb[b] - 1) / Lb[b]);
    if (nseg[b] > 1) {
      multi[b] = 1;
      multi_list.push_back(b);
    }
    InstMeta& mt = meta[b];
    mt.N = (int32_t)N; mt.n = (int32_t)n; mt.m = (int32_t)m; mt.nseg = nseg[b];
    mt.chunk = Lb[b]; mt.pad = 0;
    mt.oQ = h->off[RLQR_ARR_Q][b]; mt.oM = h->off[RLQR_ARR_M][b]; mt.oR = h->off[RLQR_ARR_R][b];
    mt.oA = h->off[RLQR_ARR_A][b]; mt.oB = h->off[RLQR_ARR_B][b];
    mt.oq = h->off[RLQR_ARR_q][b]; mt.or_ = h->off[RLQR_ARR_r][b]; mt.oc = h->off[RLQR_ARR_c][b];
    mt.ox = h->off[RLQR_ARR_x][b]; mt.ou = h->off[RLQR_ARR_u][b]; mt.oy = h->off[RLQR_ARR_y][b];
    mt.od = mt.ox;
    mt.ores = h->off[RLQR_ARR_RES][b];
    mt.ows = ws_elems;
    mt.opk = pk_elems;
    mt.ovec = vec_elems;
    mt.opsi = psi_elems;
    ws_elems += (N + 1) * tile_blocks_per_stage(cls[b]) * 256;
    pk_elems += (N + 1) * n + N * m;
    if (nseg[b] > 1) {
      vec_elems += nseg[b] * n;
      psi_elems += (int64_t)nseg[b] * 2 * n * n;
    }
    seg_off[b + 1] = seg_off[b] + nseg[b];
    whole_off[b + 1] = b + 1;
  }
  // Longest first: a class launch whose workgroups do not all fit on the GPU
  // at once dispatches them in list order, and a workgroup's time is its
  // instance's sequential stage loop, so the longest loops start first.
  for (auto& l : lists)
    std::stable_sort(l.begin(), l.end(), [&](int32_t x, int32_t y) { return h->N[x] > h->N[y]; });
  // one fixed-shape kernel serves the one-wavefront class if all its instances share the shape
  {
    int sn = -1, sm = -1;
    bool same = true;
    for (int b : lists[TILE_16]) {
      if (sn < 0) { sn = h->n[b]; sm = h->m[b]; }
      same = same && h->n[b] == sn && h->m[b] == sm;
    }
    h->shape16 = (sn > 0 && same) ? fixed_shape(sn, sm) : SHAPE_ANY;
    h->shape_all = (B > 0 && (int)lists[TILE_16].size() == B) ? h->shape16 : SHAPE_ANY;
  }
  std::vector<ResChunk> chunks, chunks_nf;
  std::vector<int32_t> resfuse(B, 0);
  for (int b = 0; b < B; ++b) {
    resfuse[b] = (cls[b] == TILE_16 && nseg[b] == 1) ? 1 : 0;
    // stages with n + m > 16 take one lane per (stage, row) of each kind of
    // row: 64 / n stages per chunk fill a wavefront
    const int len = cls[b] == TILE_16 ? RES_CHUNK : std::max(1, 64 / h->n[b]);
    for (int i0 = 0; i0 <= h->N[b]; i0 += len) {
      const ResChunk ch{b, i0, std::min(i0 + len, h->N[b] + 1), 0};
      chunks.push_back(ch);
      if (!resfuse[b]) chunks_nf.push_back(ch);
    }
  }
  h->nchunks = (int64_t)chunks.size();
  h->nchunks_nf = (int64_t)chunks_nf.size();
  std::vector<std::vector<ResChunk>> cls_chunks(TILE_CLASSES);
  for (const ResChunk& ch : chunks_nf) cls_chunks[cls[ch.inst]].push_back(ch);

  // scan groups: instances with two or more segments, by element tile size
  std::vector<int32_t> g_insts[3];
  std::vector<int64_t> g_eoff[3], g_aoff[3], inst_aoff(B, 0);
  int64_t g_elem[3] = {0, 0, 0}, g_aggr[3] = {0, 0, 0};
  for (int b = 0; b < B; ++b) {
    if (nseg[b] < 2) continue;
    const int g = scan_group(h->n[b]);
    ScanGroup& G = h->grp[g];
    const int N = h->N[b], n = h->n[b], m = h->m[b];
    const int nch = (N + 1 + Lb[b] - 1) / Lb[b];
    G.tx = scan_tx(n);
    G.tm = std::max(G.tm, (m + 15) / 16);
    G.maxN = std::max(G.maxN, N);
    G.maxchunks = std::max(G.maxchunks, nch);
    g_insts[g].push_back(b);
    g_eoff[g].push_back(g_elem[g]);
    g_aoff[g].push_back(g_aggr[g]);
    inst_aoff[b] = g_aggr[g];
    g_elem[g] += N + 1;
    g_aggr[g] += nch;
  }

  rlqr_status st = RLQR_OK;
  auto A = [&](void** p, size_t bytes) {
    if (st == RLQR_OK) st = dev_alloc(h, p, bytes);
  };
  A((void**)&h->meta, sizeof(InstMeta) * (size_t)B);
  A((void**)&h->chunks, sizeof(ResChunk) * std::max<size_t>(chunks.size(), 1));
  A((void**)&h->chunks_nf, sizeof(ResChunk) * std::max<size_t>(chunks_nf.size(), 1));
  for (int c = 0; c < TILE_CLASSES; ++c) {
    h->cls_nchunks[c] = (int64_t)cls_chunks[c].size();
    if (h->cls_nchunks[c] > 0) A((void**)&h->cls_chunks[c], sizeof(ResChunk) * cls_chunks[c].size());
  }
  A((void**)&h->resfuse, sizeof(int32_t) * std::max<size_t>((size_t)B, 1));
  A(&h->ws64, sizeof(double) * (size_t)ws_elems);
  if (mode != RLQR_SEQ_FP64) A(&h->ws32, sizeof(float) * (size_t)ws_elems);
  A((void**)&h->pk, sizeof(double) * (size_t)pk_elems);
  A((void**)&h->res[0], sizeof(double) * (size_t)h->off[RLQR_ARR_RES][B]);
  A((void**)&h->res[1], sizeof(double) * (size_t)h->off[RLQR_ARR_RES][B]);
  A((void**)&h->info, sizeof(FactorInfo) * (size_t)B);
  A((void**)&h->whole_off, sizeof(int32_t) * (size_t)(B + 1));
  A((void**)&h->whole_stats, sizeof(SegStats) * (size_t)B);
  for (int c = 0; c < TILE_CLASSES; ++c) {
    h->count[c] = (int)lists[c].size();
    h->whole[c].count = h->count[c];
    if (h->count[c] > 0) {
      A((void**)&h->list[c], sizeof(int32_t) * lists[c].size());
      A((void**)&h->whole[c].d, sizeof(SegDesc) * lists[c].size());
    }
  }
  A((void**)&h->resmax, sizeof(unsigned long long) * (size_t)B);
  A((void**)&h->bmax, sizeof(unsigned long long) * (size_t)B);
  int32_t** i32s[] = {&h->flag64, &h->conv, &h->run32, &h->run64, &h->runres, &h->fb, &h->status};
  for (auto pp : i32s) A((void**)pp, sizeof(int32_t) * (size_t)B);
  A((void**)&h->lastrel, sizeof(double) * (size_t)B);
  A((void**)&h->relres, sizeof(double) * (size_t)B);
  if (mode != RLQR_SEQ_FP64) A((void**)&h->pref32, sizeof(int32_t) * (size_t)B);
  A((void**)&h->path, sizeof(int32_t) * (size_t)B);
  if (!scan) {
    A((void**)&h->runf, sizeof(int32_t) * (size_t)B);
    A((void**)&h->runf2, sizeof(int32_t) * (size_t)B);
  }
  if (scan) {
    A((void**)&h->seg_off, sizeof(int32_t) * (size_t)(B + 1));
    A((void**)&h->seg_stats, sizeof(SegStats) * (size_t)std::max(seg_off[B], 1));
    A((void**)&h->multi, sizeof(int32_t) * (size_t)B);
    A((void**)&h->bad, sizeof(int32_t) * (size_t)B);
    A((void**)&h->run1, sizeof(int32_t) * (size_t)B);
    h->nmulti = (int)multi_list.size();
    if (h->nmulti > 0) {
      A((void**)&h->multi_list, sizeof(int32_t) * multi_list.size());
      A((void**)&h->psi, sizeof(double) * (size_t)psi_elems);
      A((void**)&h->plo, sizeof(double) * (size_t)vec_elems);
      A((void**)&h->xhi, sizeof(double) * (size_t)vec_elems);
    }
    for (int g = 0; g < 3; ++g) {
      ScanGroup& G = h->grp[g];
      G.ninst = (int)g_insts[g].size();
      if (G.ninst == 0) continue;
      const size_t elem = 3ull * (16 * G.tx) * (16 * G.tx);
      A((void**)&G.insts, sizeof(int32_t) * (size_t)G.ninst);
      A((void**)&G.eoff, sizeof(int64_t) * (size_t)G.ninst);
      A((void**)&G.aoff, sizeof(int64_t) * (size_t)G.ninst);
      A((void**)&G.elems, sizeof(float) * elem * (size_t)g_elem[g]);
      A((void**)&G.aggr[0], sizeof(float) * elem * (size_t)g_aggr[g]);
      A((void**)&G.aggr[1], sizeof(float) * elem * (size_t)g_aggr[g]);
      if (h->carry_pc) {
        const size_t vec = 2ull * (16 * G.tx);
        A((void**)&G.pce, sizeof(float) * vec * (size_t)g_elem[g]);
        A((void**)&G.pca[0], sizeof(float) * vec * (size_t)g_aggr[g]);
        A((void**)&G.pca[1], sizeof(float) * vec * (size_t)g_aggr[g]);
      }
    }
  }
  // segment descriptors (device pointers into the scan buffers are known now)
  std::vector<std::vector<SegDesc>> whole_d(TILE_CLASSES), fseg_d(TILE_CLASSES), sseg_d(TILE_CLASSES);
  if (st == RLQR_OK) {
    for (int c = 0; c < TILE_CLASSES; ++c)
      for (int b : lists[c]) {
        SegDesc d{};
        d.inst = b; d.lo = 0; d.hi = h->N[b]; d.p0_ld = 0; d.gidx = b; d.s = 0; d.P0 = nullptr;
        whole_d[c].push_back(d);
      }
    for (int b = 0; b < B; ++b) {
      if (!scan) break;
      const int N = h->N[b];
      const ScanGroup* G = nseg[b] > 1 ? &h->grp[scan_group(h->n[b])] : nullptr;
      for (int s2 = 0; s2 < nseg[b]; ++s2) {
        SegDesc e{};
        e.inst = b;
        e.lo = s2 * Lb[b];
        e.hi = nseg[b] > 1 ? std::min(e.lo + Lb[b], N) : N;
        e.gidx = seg_off[b] + s2;
        e.s = s2;
        e.P0 = nullptr;
        e.p0_ld = 0;
        if (G && e.hi < N) {
          const int NX = 16 * G->tx;
          const int rb = scan_result_buffer(G->maxchunks);
          e.P0 = G->aggr[rb] + (size_t)(inst_aoff[b] + s2 + 1) * 3 * NX * NX;
          e.p0_ld = NX;
        }
        fseg_d[cls[b]].push_back(e);
        if (nseg[b] > 1) sseg_d[cls[b]].push_back(e);
      }
    }
    for (int c = 0; c < TILE_CLASSES; ++c) {
      if (!scan) break;
      h->fseg[c].count = (int)fseg_d[c].size();
      h->sseg[c].count = (int)sseg_d[c].size();
      if (h->fseg[c].count > 0) A((void**)&h->fseg[c].d, sizeof(SegDesc) * fseg_d[c].size());
      if (h->sseg[c].count > 0) A((void**)&h->sseg[c].d, sizeof(SegDesc) * sseg_d[c].size());
    }
  }
  if (st == RLQR_OK && B > 0) {
    bool ok = upload(h->meta, meta) && upload(h->chunks, chunks) && upload(h->whole_off, whole_off) &&
              upload(h->chunks_nf, chunks_nf) && upload(h->resfuse, resfuse);
    for (int c = 0; c < TILE_CLASSES && ok; ++c)
      if (h->cls_nchunks[c] > 0) ok = upload(h->cls_chunks[c], cls_chunks[c]);
    h->cls_res = ok;
    for (int c = 0; c < TILE_CLASSES && ok; ++c) {
      if (h->count[c] > 0) ok = upload(h->list[c], lists[c]) && upload(h->whole[c].d, whole_d[c]);
      if (ok && scan && h->fseg[c].count > 0) ok = upload(h->fseg[c].d, fseg_d[c]);
      if (ok && scan && h->sseg[c].count > 0) ok = upload(h->sseg[c].d, sseg_d[c]);
    }
    if (ok && scan) {
      ok = upload(h->seg_off, seg_off) && upload(h->multi, multi);
      if (ok && h->nmulti > 0) ok = upload(h->multi_list, multi_list);
      for (int g = 0; g < 3 && ok; ++g)
        if (h->grp[g].ninst > 0)
          ok = upload(h->grp[g].insts, g_insts[g]) && upload(h->grp[g].eoff, g_eoff[g]) &&
               upload(h->grp[g].aoff, g_aoff[g]);
    }
    std::vector<int32_t> f(B, mode == RLQR_SEQ_FP64 ? 1 : 0);
    for (int b = 0; b < B; ++b) f[b] = f[b] || pref64[b];
    if (ok) ok = upload(h->flag64, f);
    if (ok) {  // before the first factorization: the float64-only instances are known
      std::vector<int32_t> pth(B);
      for (int b = 0; b < B; ++b) pth[b] = f[b] ? RLQR_PATH_FP64 : RLQR_PATH_FP32;
      ok = upload(h->path, pth);
    }
    if (ok && mode != RLQR_SEQ_FP64) {
      std::vector<int32_t> p32(B);
      for (int b = 0; b < B; ++b) p32[b] = pref64[b] ? 0 : 1;
      ok = upload(h->pref32, p32);
    }
    if (ok && scan && scan_prepare() != hipSuccess) ok = false;
    if (!ok) st = RLQR_E_HIP;
  }
  if (st == RLQR_OK) {
    int nclass = 0;
    for (int c = 0; c < TILE_CLASSES; ++c) nclass += lists[c].empty() ? 0 : 1;
    if (nclass > 1) {
      h->owns_streams = true;
      bool ok = hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming) == hipSuccess;
      for (int c = 0; c < TILE_CLASSES && ok; ++c) {
        if (lists[c].empty()) continue;
        ok = hipStreamCreateWithFlags(&h->side[c], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&h->ev_join[c], hipEventDisableTiming) == hipSuccess;
      }
      if (!ok) st = RLQR_E_HIP;
    }
  }
  if (st == RLQR_OK && tune && tune->max_rhs > 1 && !scan && B > 0)
    st = build_multi(h, tune->max_rhs, meta, chunks, chunks_nf, resfuse, lists, pref64, pk_elems);
  if (st != RLQR_OK) {
    release(h);
    delete h;
    return st;
  }
  if (workspace_bytes) *workspace_bytes = h->bytes;
  *hp = h;
  return RLQR_OK;
}

rlqr_status rlqr_create(rlqr_handle** hp, const rlqr_shape* s, rlqr_mode mode, size_t* workspace_bytes) {
  return rlqr_create_tuned(hp, s, mode, nullptr, workspace_bytes);
}

rlqr_status rlqr_get_tuning(const rlqr_handle* h, rlqr_tuning* t) {
  if (!h || !t) return RLQR_E_INVALID;
  t->scan_chunk = h->chunk;
  t->inst_chunk = nullptr;
  t->inst_fp64 = nullptr;
  t->max_rhs = h->max_rhs;
  t->scan_carry_pc = h->carry_pc ? 1 : 0;
  t->mw_waves = h->mw_waves;
  return RLQR_OK;
}

rlqr_status rlqr_layout_offsets(const rlqr_handle* h, int32_t array, int64_t* off) {
  if (!h || !off || array < 0 || array >= RLQR_ARR_COUNT) return RLQR_E_INVALID;
  std::memcpy(off, h->off[array].data(), sizeof(int64_t) * (h->B + 1));
  return RLQR_OK;
}

}  // extern "C"

// One factor launch per tile class over the given segment lists, then the
// per-instance merge of the segments' pivot statistics.
// Run launch(c, stream) for every class c with count[c] > 0: the first on st,
// the others on their side streams between a fork and a join event.
template <class F>
static hipError_t per_class(rlqr_handle* h, const int* count, hipStream_t st, F&& launch) {
  int first = -1, nclass = 0;
  for (int c = 0; c < TILE_CLASSES; ++c)
    if (count[c] > 0) {
      if (first < 0) first = c;
      ++nclass;
    }
  if (nclass <= 1 || !h->ev_fork) {
    for (int c = 0; c < TILE_CLASSES; ++c) {
      if (count[c] <= 0) continue;
      hipError_t e = launch(c, st);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  hipError_t e = hipEventRecord(h->ev_fork, st);
  if (e != hipSuccess) return e;
  for (int c = 0; c < TILE_CLASSES; ++c) {
    if (count[c] <= 0) continue;
    if (c == first) {
      e = launch(c, st);
    } else {
      e = hipStreamWaitEvent(h->side[c], h->ev_fork, 0);
      if (e == hipSuccess) e = launch(c, h->side[c]);
      if (e == hipSuccess) e = hipEventRecord(h->ev_join[c], h->side[c]);
    }
    if (e != hipSuccess) return e;
  }
  for (int c = 0; c < TILE_CLASSES; ++c) {
    if (count[c] <= 0 || c == first) continue;
    e = hipStreamWaitEvent(st, h->ev_join[c], 0);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static hipError_t factor_segments(rlqr_handle* h, const SegList* lists, const int32_t* off, SegStats* stats,
                                  void* ws, const int32_t* run, bool fp32, hipStream_t st,
                                  const rlqr_rhs* rhs = nullptr) {
  int count[TILE_CLASSES];
  for (int c = 0; c < TILE_CLASSES; ++c) count[c] = lists[c].count;
  hipError_t e = per_class(h, count, st, [&](int c, hipStream_t s2) {
    FactorArgs a{};
    a.meta = h->meta; a.segs = lists[c].d; a.run = run;
    a.Q = h->lhs.Q; a.M = h->lhs.M; a.R = h->lhs.R; a.A = h->lhs.A; a.B = h->lhs.B; a.delta = h->lhs.delta;
    a.dd = h->lhs.delta_diag;
    a.ws = ws; a.stats = stats;
    if (rhs && c == TILE_16) {
      a.q = rhs->q; a.r = rhs->r; a.c = rhs->c; a.pk = h->pk;
    }
    return (c == TILE_16) ? launch_factor(a, lists[c].count, fp32, h->shape16, s2)
                          : launch_factor_mw(c, a, lists[c].count, fp32, s2, h->mw_waves);
  });
  if (e != hipSuccess) return e;
  MergeArgs m{};
  m.batch = h->B; m.meta = h->meta; m.seg_off = off; m.run = run; m.stats = stats; m.info = h->info;
  return launch_merge(m, st);
}

static hipError_t factor_whole(rlqr_handle* h, void* ws, const int32_t* run, bool fp32, hipStream_t st,
                               const rlqr_rhs* rhs = nullptr) {
  return factor_segments(h, h->whole, h->whole_off, h->whole_stats, ws, run, fp32, st, rhs);
}

// Scan mode: elements, chunk reduce and suffix scan per group, then every
// segment factored from its boundary cost-to-go, then the transfer matrices.
// With rhs (scan_carry_pc) the scan also carries p and c, and the segments'
// boundary p for that right-hand side goes to plo.
static hipError_t factor_scan(rlqr_handle* h, hipStream_t st, const rlqr_rhs* rhs = nullptr) {
  hipError_t e = launch_fill_i32(h->bad, h->B, 0, st);
  if (e != hipSuccess) return e;
  const bool pc = h->carry_pc && rhs != nullptr;
  h->pc_valid = false;
  for (int g = 0; g < 3; ++g) {
    ScanGroup& G = h->grp[g];
    if (G.ninst == 0) continue;
    ScanArgs a{};
    a.meta = h->meta; a.insts = G.insts; a.eoff = G.eoff; a.aoff = G.aoff;
    a.Q = h->lhs.Q; a.M = h->lhs.M; a.R = h->lhs.R; a.A = h->lhs.A; a.B = h->lhs.B; a.delta = h->lhs.delta;
    a.dd = h->lhs.delta_diag;
    a.elems = G.elems; a.aggr[0] = G.aggr[0]; a.aggr[1] = G.aggr[1];
    a.maxN = G.maxN; a.maxchunks = G.maxchunks; a.bad = h->bad;
    if (pc) {
      a.pc = 1; a.q = rhs->q; a.r = rhs->r; a.c = rhs->c;
      a.pce = G.pce; a.pca[0] = G.pca[0]; a.pca[1] = G.pca[1];
    }
    if ((e = launch_scan_elements(a, G.ninst, G.tx, G.tm, st)) != hipSuccess) return e;
    if ((e = launch_scan_tree(a, G.ninst, G.tx, h->mode == RLQR_SCAN_BF16, st)) != hipSuccess) return e;
    if (pc) {
      a.pca_in = G.pca[scan_result_buffer(G.maxchunks)];
      if ((e = launch_scan_pc_boundary(a, G.ninst, G.tx, h->plo, st)) != hipSuccess) return e;
    }
  }
  if (pc) {
    h->pc_valid = true;
    h->pc_rhs = *rhs;
  }
  const int32_t* run32 = h->any_pref64 ? h->pref32 : nullptr;
  if ((e = factor_segments(h, h->fseg, h->seg_off, h->seg_stats, h->ws32, run32, true, st)) != hipSuccess)
    return e;
  for (int c = 0; c < TILE_CLASSES; ++c) {
    if (h->sseg[c].count == 0) continue;
    TransferArgs t{};
    t.meta = h->meta; t.segs = h->sseg[c].d; t.A = h->lhs.A; t.B = h->lhs.B; t.ws = h->ws32; t.psi = h->psi;
    t.dd = h->lhs.delta_diag;
    if ((e = launch_transfer(c, t, h->sseg[c].count, st)) != hipSuccess) return e;
  }
  return hipSuccess;
}

static rlqr_status factor_impl(rlqr_handle* h, const rlqr_lhs* lhs, const rlqr_rhs* rhs, hipStream_t st) {
  if (!h || !lhs) return RLQR_E_INVALID;
  if (h->B > 0 && (!lhs->Q || !lhs->M || !lhs->R || !lhs->A || !lhs->B || (!lhs->delta && !lhs->delta_diag)))
    return RLQR_E_INVALID;
  if (rhs && h->B > 0 && (!rhs->q || !rhs->r || !rhs->c)) return RLQR_E_INVALID;
  h->lhs = *lhs;
  h->factored = true;
  h->pk_fused = false;
  if (h->B == 0) return RLQR_OK;
  const rlqr_rhs* scan_rhs = rhs;       // scan_carry_pc: the scan carries p and c for it
  if (is_scan(h->mode)) rhs = nullptr;  // the segment recursions do not carry the vector pass
  // run mask of a factor launch under the skip mask: !skip && in
  auto masked = [&](const int32_t* in, int32_t* out, const int32_t** run) -> hipError_t {
    *run = in;
    if (!h->skip) return hipSuccess;
    MaskArgs k{};
    k.batch = h->B; k.kind = 5; k.skip = h->skip; k.in = in; k.out = out;
    *run = out;
    return launch_masks(k, st);
  };
  const int32_t* run = nullptr;
  if (h->mode == RLQR_SEQ_FP64) {
    RLQR_TRY(masked(nullptr, h->runf, &run));
    RLQR_TRY(factor_whole(h, h->ws64, run, false, st, rhs));
  } else {
    // float32 products everywhere, then float64 for instances whose pivots fall
    // inside the guard band (or whose scan failed)
    if (h->mode == RLQR_SEQ_MIXED) {
      RLQR_TRY(masked(h->any_pref64 ? h->pref32 : nullptr, h->runf, &run));
      RLQR_TRY(factor_whole(h, h->ws32, run, true, st, rhs));
    } else {
      RLQR_TRY(factor_scan(h, st, scan_rhs));
    }
    MaskArgs m{};
    m.batch = h->B; m.kind = 1; m.guard = kGuard; m.info = h->info; m.flag64 = h->flag64;
    m.path = h->path; m.skip = h->skip;
    m.bad = is_scan(h->mode) ? h->bad : nullptr;
    m.pref32 = h->any_pref64 ? h->pref32 : nullptr;
    RLQR_TRY(launch_masks(m, st));
    RLQR_TRY(masked(h->flag64, h->runf2, &run));
    RLQR_TRY(factor_whole(h, h->ws64, run, false, st, rhs));
  }
  if (rhs) {
    h->pk_fused = true;
    h->pk_rhs = *rhs;
  }
  return RLQR_OK;
}

extern "C" rlqr_status rlqr_factor(rlqr_handle* h, const rlqr_lhs* lhs, rlqr_stream stv) {
  return factor_impl(h, lhs, nullptr, (hipStream_t)stv);
}

extern "C" rlqr_status rlqr_factor_rhs(rlqr_handle* h, const rlqr_lhs* lhs, const rlqr_rhs* rhs, rlqr_stream stv) {
  if (!rhs) return RLQR_E_INVALID;
  return factor_impl(h, lhs, rhs, (hipStream_t)stv);
}

static SolveArgs solve_args(rlqr_handle* h, const rlqr_rhs* rhs, rlqr_sol* out, bool fp32, const int32_t* run,
                            const double* corr) {
  SolveArgs a{};
  a.meta = h->meta; a.run = run;
  a.Q = h->lhs.Q; a.M = h->lhs.M; a.R = h->lhs.R; a.A = h->lhs.A; a.B = h->lhs.B; a.delta = h->lhs.delta;
  a.dd = h->lhs.delta_diag;
  a.ws = fp32 ? h->ws32 : h->ws64;
  a.info = h->info;
  a.q = rhs->q; a.r = rhs->r; a.c = rhs->c;
  a.corr = corr;
  a.x = out->x; a.u = out->u; a.y = out->y;
  a.pk = h->pk;
  a.plo = h->plo; a.xhi = h->xhi;
  return a;
}

static ResidualArgs residual_args(rlqr_handle* h, const rlqr_rhs* rhs, const rlqr_sol* z, double* res,
                                  const int32_t* run) {
  ResidualArgs a{};
  a.batch = h->B; a.meta = h->meta; a.chunks = h->chunks; a.nchunks = h->nchunks;
  a.run = run; a.skip = nullptr; a.info = h->info;
  a.Q = h->lhs.Q; a.M = h->lhs.M; a.R = h->lhs.R; a.A = h->lhs.A; a.B = h->lhs.B; a.delta = h->lhs.delta;
  a.dd = h->lhs.delta_diag;
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

// Whole-instance solves, one launch per tile class; run masks select instances.
// skip (scan mode) leaves the multi-segment instances to the segment solve.
static ResidualArgs residual_args(rlqr_handle* h, const rlqr_rhs* rhs, const rlqr_sol* z, double* res,
                                  const int32_t* run);

// res_run: if set, each class's residual (its instances outside the fused
// one-wavefront residual, run mask res_run) follows its solve on the class's
// stream, beside the other classes' solves, instead of one launch after all.
static rlqr_status solve_whole(rlqr_handle* h, const rlqr_rhs* rhs, rlqr_sol* out, bool fp32, const int32_t* run,
                               const double* corr, hipStream_t st, bool fwd_only = false, double* res_out = nullptr,
                               const int32_t* res_run = nullptr) {
  hipError_t e = per_class(h, h->count, st, [&](int c, hipStream_t s2) {
    SolveArgs a = solve_args(h, rhs, out, fp32, run, corr);
    a.list = h->list[c];
    a.fwd_only = (fwd_only && c == TILE_16) ? 1 : 0;
    if (res_out && c == TILE_16) {
      a.res = res_out; a.resmax = h->resmax; a.bmax = h->bmax; a.resfuse = h->resfuse;
    }
    hipError_t e2 = (c == TILE_16) ? launch_solve(a, h->count[c], fp32, h->shape16, s2)
                                   : launch_solve_mw(c, a, h->count[c], fp32, s2, h->mw_waves);
    if (e2 == hipSuccess && res_run && h->cls_nchunks[c] > 0) {
      ResidualArgs ra = residual_args(h, rhs, out, res_out, res_run);
      ra.chunks = h->cls_chunks[c];
      ra.nchunks = h->cls_nchunks[c];
      e2 = launch_residual(ra, c == TILE_16 ? h->shape16 : SHAPE_LARGE, s2);
    }
    return e2;
  });
  return e == hipSuccess ? RLQR_OK : RLQR_E_HIP;
}

// Scan mode: the segments of multi-segment instances in three phases joined
// by the boundary chains (see k_solve_mw and k_chain).
static rlqr_status solve_segments(rlqr_handle* h, const rlqr_rhs* rhs, rlqr_sol* out, const int32_t* run,
                                  const double* corr, hipStream_t st) {
  if (h->nmulti == 0) return RLQR_OK;
  // the boundary p carried by the scan serves the first solve of its
  // right-hand side; phase 1 and the backward chain overwrite it
  const bool use_pc = h->pc_valid && corr == nullptr && rhs->q == h->pc_rhs.q && rhs->r == h->pc_rhs.r &&
                      rhs->c == h->pc_rhs.c;
  h->pc_valid = false;
  for (int phase = use_pc ? 2 : 1; phase <= 3; ++phase) {
    for (int c = 0; c < TILE_CLASSES; ++c) {
      if (h->sseg[c].count == 0) continue;
      SolveArgs a = solve_args(h, rhs, out, true, run, corr);
      a.segs = h->sseg[c].d;
      a.phase = phase;
      RLQR_TRY(launch_seg_solve(c, a, h->sseg[c].count, st));
    }
    if (phase < 3) {
      ChainArgs ch{};
      ch.meta = h->meta; ch.insts = h->multi_list; ch.run = run; ch.psi = h->psi;
      ch.vec = phase == 1 ? h->plo : h->xhi;
      ch.forward = phase == 2 ? 1 : 0;
      RLQR_TRY(launch_chain(ch, h->nmulti, st));
    }
  }
  return RLQR_OK;
}

// Pass p of the refinement: solve (p == 0) or correct (p > 0) every
// instance not yet converged, then its residual and the convergence check.
static rlqr_status solve_pass(rlqr_handle* h, const rlqr_rhs* rhs, rlqr_sol* out, int pass, double tol,
                              const int32_t* run64_override, hipStream_t st, bool fwd_only = false) {
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
  if (h->mode != RLQR_SEQ_FP64 && !run64_override) {
    if (is_scan(h->mode)) {
      // single-segment instances take the whole-instance kernels
      MaskArgs m{};
      m.batch = h->B; m.kind = 4; m.run32 = h->run32; m.multi = h->multi; m.run1 = h->run1;
      RLQR_TRY(launch_masks(m, st));
      if ((s = solve_whole(h, rhs, out, true, h->run1, corr, st, false, res_out)) != RLQR_OK) return s;
      if ((s = solve_segments(h, rhs, out, r32, corr, st)) != RLQR_OK) return s;
    } else if ((s = solve_whole(h, rhs, out, true, r32, corr, st, fwd_only, res_out)) != RLQR_OK) {
      return s;
    }
  }
  // float64 mode: every instance is solved by this one call, so each class's
  // residual can follow its own solve (the one-wavefront solves write theirs)
  const bool cls_res = h->cls_res && h->mode == RLQR_SEQ_FP64 && !run64_override;
  if ((s = solve_whole(h, rhs, out, false, r64, corr, st, fwd_only, res_out, cls_res ? rres : nullptr)) != RLQR_OK)
    return s;
  if (!cls_res) {
    // the one-wavefront solves wrote their instances' residuals; the others here
    ResidualArgs ra = residual_args(h, rhs, out, res_out, rres);
    ra.chunks = h->chunks_nf;
    ra.nchunks = h->nchunks_nf;
    RLQR_TRY(launch_residual(ra, h->shape_all, st));
  }
  RLQR_TRY(launch_check(check_args(h, 0, tol, rres), st));
  return RLQR_OK;
}

static rlqr_status solve_impl(rlqr_handle* h, const rlqr_rhs* rhs, rlqr_sol* out, double rel_tol, int32_t max_refine,
                              int32_t* inst_status, double* inst_relres, hipStream_t st) {
  rlqr_status s;

  if (h->skip) {  // left-out instances start converged: no pass touches them
    MaskArgs k{};
    k.batch = h->B; k.kind = 6; k.skip = h->skip; k.conv = h->conv;
    RLQR_TRY(launch_masks(k, st));
  } else {
    RLQR_TRY(launch_fill_i32(h->conv, h->B, 0, st));
  }
  // per-instance residual maxima start at zero (the check kernel clears resmax after each pass)
  RLQR_TRY(launch_fill_i32(reinterpret_cast<int32_t*>(h->resmax), 2 * h->B, 0, st));
  RLQR_TRY(launch_fill_i32(reinterpret_cast<int32_t*>(h->bmax), 2 * h->B, 0, st));
  // the first pass may start at the forward rollout (rlqr_factor_rhs with these rhs arrays)
  const bool fused = h->pk_fused && h->pk_rhs.q == rhs->q && h->pk_rhs.r == rhs->r && h->pk_rhs.c == rhs->c;
  h->pk_fused = false;  // the passes below overwrite pk
  for (int pass = 0; pass <= max_refine; ++pass)
    if ((s = solve_pass(h, rhs, out, pass, rel_tol, nullptr, st, fused && pass == 0)) != RLQR_OK) return s;
  RLQR_TRY(launch_check(check_args(h, 1, rel_tol, nullptr), st));

  if (h->mode != RLQR_SEQ_FP64) {
    // instances that did not converge from float32 tiles: redo them in float64
    MaskArgs m{};
    m.batch = h->B; m.kind = 2; m.flag64 = h->flag64; m.conv = h->conv; m.status = h->status; m.fb = h->fb;
    m.skip = h->skip; m.path = h->path;
    RLQR_TRY(launch_masks(m, st));
    RLQR_TRY(factor_whole(h, h->ws64, h->fb, false, st));
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

extern "C" rlqr_status rlqr_solve(rlqr_handle* h, const rlqr_rhs* rhs, rlqr_sol* out, double rel_tol,
                                  int32_t max_refine, int32_t* inst_status, double* inst_relres, rlqr_stream stv) {
  if (!h || !rhs || !out) return RLQR_E_INVALID;
  if (!h->factored) return RLQR_E_STATE;
  if (h->B == 0) return RLQR_OK;
  if (!rhs->q || !rhs->r || !rhs->c || !out->x || !out->u || !out->y) return RLQR_E_INVALID;
  if (!(rel_tol >= 0.0) || max_refine < 0) return RLQR_E_INVALID;
  return solve_impl(h, rhs, out, rel_tol, max_refine, inst_status, inst_relres, (hipStream_t)stv);
}

namespace rlqr {
void handle_shapes(const rlqr_handle* h, int* batch, const int32_t** N, const int32_t** n, const int32_t** m) {
  *batch = h->B;
  *N = h->N.data(); *n = h->n.data(); *m = h->m.data();
}
}  // namespace rlqr

extern "C" rlqr_status rlqr_solve_multi(rlqr_handle* h, int32_t nrhs, const rlqr_rhs* rhs, rlqr_sol* out,
                                        double rel_tol, int32_t max_refine, int32_t* inst_status,
                                        double* inst_relres, rlqr_stream stv) {
  if (!h || !rhs || !out || nrhs < 0) return RLQR_E_INVALID;
  if (!h->factored) return RLQR_E_STATE;
  if (h->B == 0 || nrhs == 0) return RLQR_OK;
  if (nrhs >= 2 && h->mv && nrhs <= h->max_rhs) {
    if (!rhs->q || !rhs->r || !rhs->c || !out->x || !out->u || !out->y) return RLQR_E_INVALID;
    if (!(rel_tol >= 0.0) || max_refine < 0) return RLQR_E_INVALID;
    hipStream_t st = (hipStream_t)stv;
    rlqr_handle* v = h->mv;
    const int B = h->B;
    v->B = nrhs * B;
    for (int c = 0; c < TILE_CLASSES; ++c) {
      v->count[c] = nrhs * v->base_count[c];
      v->whole[c].count = v->count[c];
      if (v->base_count[c] > 0) v->list[c] = v->mlist[c][nrhs - 1];
    }
    v->nchunks = nrhs * v->base_nchunks;
    v->nchunks_nf = nrhs * v->base_nchunks_nf;
    ReplicateArgs ra{};
    ra.B = B; ra.total = v->B; ra.info = h->info; ra.flag64 = h->flag64; ra.delta = h->lhs.delta;
    ra.vinfo = v->info; ra.vflag64 = v->flag64; ra.vdelta = v->vdelta;
    hipLaunchKernelGGL(k_replicate, dim3((v->B + 255) / 256), dim3(256), 0, st, ra);
    RLQR_TRY(hipGetLastError());
    v->lhs = h->lhs;
    v->lhs.delta = v->vdelta;
    v->factored = true;
    v->pk_fused = false;
    return solve_impl(v, rhs, out, rel_tol, max_refine, inst_status, inst_relres, st);
  }
  const int64_t Lq = h->off[RLQR_ARR_q][h->B], Lr = h->off[RLQR_ARR_r][h->B], Lc = h->off[RLQR_ARR_c][h->B];
  for (int32_t j = 0; j < nrhs; ++j) {
    rlqr_rhs b{rhs->q + j * Lq, rhs->r + j * Lr, rhs->c + j * Lc};
    rlqr_sol z{out->x + j * Lq, out->u + j * Lr, out->y + j * Lc};
    rlqr_status s = rlqr_solve(h, &b, &z, rel_tol, max_refine, inst_status ? inst_status + (int64_t)j * h->B : nullptr,
                               inst_relres ? inst_relres + (int64_t)j * h->B : nullptr, stv);
    if (s != RLQR_OK) return s;
  }
  return RLQR_OK;
}

extern "C" rlqr_status rlqr_set_skip(rlqr_handle* h, const int32_t* skip) {
  if (!h) return RLQR_E_INVALID;
  if (skip && is_scan(h->mode)) return RLQR_E_UNSUPPORTED;
  h->skip = skip;
  return RLQR_OK;
}

extern "C" rlqr_status rlqr_pivot_inertia(rlqr_handle* h, int32_t* pd_verdict, int32_t* first_bad, int64_t* inertia,
                                          rlqr_stream stv) {
  if (!h) return RLQR_E_INVALID;
  if (!h->factored) return RLQR_E_STATE;
  InertiaArgs a{};
  a.batch = h->B; a.info = h->info; a.verdict = pd_verdict; a.first_bad = first_bad; a.inertia = inertia;
  RLQR_TRY(launch_inertia(a, (hipStream_t)stv));
  return RLQR_OK;
}

extern "C" rlqr_status rlqr_precision_path(rlqr_handle* h, int32_t* path, rlqr_stream stv) {
  if (!h) return RLQR_E_INVALID;
  if (!h->factored) return RLQR_E_STATE;
  if (h->B == 0) return RLQR_OK;
  if (!path) return RLQR_E_INVALID;
  RLQR_TRY(hipMemcpyAsync(path, h->path, sizeof(int32_t) * h->B, hipMemcpyDeviceToDevice, (hipStream_t)stv));
  return RLQR_OK;
}

extern "C" rlqr_status rlqr_residual(rlqr_handle* h, const rlqr_rhs* rhs, const rlqr_sol* z, double* res,
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
  RLQR_TRY(launch_residual(a, h->shape_all, st));
  if (inst_relres) {
    CheckArgs c = check_args(h, 1, 0.0, nullptr);
    c.plain = 1;
    c.relres = inst_relres;
    RLQR_TRY(launch_check(c, st));
  }
  return RLQR_OK;
}

extern "C" rlqr_status rlqr_graph_capture(rlqr_handle* h, const rlqr_lhs* lhs, const rlqr_rhs* rhs, rlqr_sol* out,
                                          double rel_tol, int32_t max_refine, int32_t* inst_status,
                                          double* inst_relres, rlqr_stream stv) {
  if (!h || !lhs || !rhs || !out || !stv) return RLQR_E_INVALID;
  if (h->B > 0 && (!lhs->Q || !lhs->M || !lhs->R || !lhs->A || !lhs->B || (!lhs->delta && !lhs->delta_diag) ||
                   !rhs->q || !rhs->r || !rhs->c || !out->x || !out->u || !out->y))
    return RLQR_E_INVALID;
  if (!(rel_tol >= 0.0) || max_refine < 0) return RLQR_E_INVALID;
  hipStream_t st = (hipStream_t)stv;
  drop_graph(h);
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    return RLQR_E_HIP;
  }
  rlqr_status s = rlqr_factor_rhs(h, lhs, rhs, stv);
  if (s == RLQR_OK) s = rlqr_solve(h, rhs, out, rel_tol, max_refine, inst_status, inst_relres, stv);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(st, &g);
  if (s != RLQR_OK || e != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return s != RLQR_OK ? s : RLQR_E_HIP;
  }
  hipGraphExec_t x = nullptr;
  if (hipGraphInstantiate(&x, g, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return RLQR_E_HIP;
  }
  h->graph = g;
  h->graph_exec = x;
  return RLQR_OK;
}

extern "C" rlqr_status rlqr_graph_launch(rlqr_handle* h, rlqr_stream stv) {
  if (!h) return RLQR_E_INVALID;
  if (!h->graph_exec) return RLQR_E_STATE;
  RLQR_TRY(hipGraphLaunch(h->graph_exec, (hipStream_t)stv));
  return RLQR_OK;
}

extern "C" void rlqr_destroy(rlqr_handle* h) {
  if (!h) return;
  release(h);
  delete h;
}
