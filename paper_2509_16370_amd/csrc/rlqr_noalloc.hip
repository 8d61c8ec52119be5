// rlqr_noalloc.hip -- rlqr_residual_noalloc: the float64 residual of Section
// "Residual Computation" for a batch, without a handle and without any device
// allocation.
//
// The residual kernels need per-instance metadata (shape and offsets into the
// packed arrays), a list of stage chunks and two per-instance maxima. A handle
// keeps them in workspace it allocated at create; here they live in one
// file-scope device array, `scratch`, of RLQR_NOALLOC_SCRATCH_BYTES, which
// every GPU that runs this code holds until the process ends. Host code never
// passes the array's name to a kernel (on the host it is only a stand-in for
// the symbol): the device address is looked up once per device with
// hipGetSymbolAddress and kept in `g_scratch`.
//
// Per call the metadata are built on the host and uploaded with a copy from
// pageable host memory (HIP performs such a copy synchronously with respect
// to the host, in stream order), the maxima are cleared by a fill kernel, then
// the residual and the per-instance relative residual run on the caller's
// stream. Calls on one stream are ordered; calls that overlap on one GPU (two
// streams, two host threads) share the array and race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "rlqr_internal.h"

using namespace rlqr;

static __device__ __align__(256) unsigned char scratch[RLQR_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
rlqr_status scratch_address(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return RLQR_E_HIP;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return RLQR_E_HIP;
    }
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return RLQR_OK;
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

#define NA_TRY(x)                             \
  do {                                        \
    if ((x) != hipSuccess) {                  \
      (void)hipGetLastError();                \
      return RLQR_E_HIP;                      \
    }                                         \
  } while (0)

}  // namespace

extern "C" rlqr_status rlqr_residual_noalloc(const rlqr_shape* s, const rlqr_lhs* lhs, const rlqr_rhs* rhs,
                                             const rlqr_sol* z, double* res, double* inst_relres,
                                             rlqr_stream stv) {
  if (!s || !lhs || !rhs || !z || s->batch < 0) return RLQR_E_INVALID;
  const int B = s->batch;
  if (B == 0) return RLQR_OK;
  if (!s->N || !s->nx || !s->nu) return RLQR_E_INVALID;
  if (!lhs->Q || !lhs->M || !lhs->R || !lhs->A || !lhs->B || (!lhs->delta && !lhs->delta_diag) || !rhs->q ||
      !rhs->r || !rhs->c || !z->x || !z->u || !z->y)
    return RLQR_E_INVALID;

  // metadata and residual chunks, exactly as a handle lays them out
  std::vector<InstMeta> meta((size_t)B);
  std::vector<ResChunk> chunks;
  int64_t off[RLQR_ARR_COUNT] = {};
  int sn = -1, sm = -1;
  bool same16 = true;
  for (int b = 0; b < B; ++b) {
    const int64_t N = s->N[b], n = s->nx[b], m = s->nu[b];
    if (N < 0 || n < 1 || m < 1 || n > RLQR_MAX_NX || n + m > RLQR_MAX_NXU) return RLQR_E_INVALID;
    const int cls = tile_class((int)n, (int)m);
    if (cls < 0) return RLQR_E_INVALID;
    InstMeta& mt = meta[b];
    mt = InstMeta{};
    mt.N = (int32_t)N; mt.n = (int32_t)n; mt.m = (int32_t)m; mt.nseg = 1; mt.chunk = (int32_t)std::max<int64_t>(N, 1);
    mt.oQ = off[RLQR_ARR_Q]; mt.oM = off[RLQR_ARR_M]; mt.oR = off[RLQR_ARR_R];
    mt.oA = off[RLQR_ARR_A]; mt.oB = off[RLQR_ARR_B];
    mt.oq = off[RLQR_ARR_q]; mt.or_ = off[RLQR_ARR_r]; mt.oc = off[RLQR_ARR_c];
    mt.ox = off[RLQR_ARR_x]; mt.ou = off[RLQR_ARR_u]; mt.oy = off[RLQR_ARR_y];
    mt.od = mt.ox;
    mt.ores = off[RLQR_ARR_RES];
    const int64_t cnt[RLQR_ARR_COUNT] = {(N + 1) * n * n, N * n * m, N * m * m, N * n * n, N * n * m,
                                         (N + 1) * n,     N * m,     (N + 1) * n, (N + 1) * n, N * m,
                                         (N + 1) * n,     N * (n + m) + n + (N + 1) * n};
    for (int k = 0; k < RLQR_ARR_COUNT; ++k) off[k] += cnt[k];
    if (cls == TILE_16) {
      if (sn < 0) { sn = (int)n; sm = (int)m; }
      same16 = same16 && n == sn && m == sm;
    } else {
      same16 = false;
    }
    // stages with n + m > 16: 64 / n stages per chunk (one lane per stage and row)
    const int64_t len = cls == TILE_16 ? RES_CHUNK : std::max<int64_t>(1, 64 / n);
    for (int64_t i0 = 0; i0 <= N; i0 += len)
      chunks.push_back(ResChunk{b, (int32_t)i0, (int32_t)std::min<int64_t>(i0 + len, N + 1), 0});
  }
  const int shape = (same16 && sn > 0) ? fixed_shape(sn, sm) : SHAPE_ANY;

  // carve the scratch array: meta | resmax | bmax | chunks
  const size_t o_meta = 0;
  const size_t o_rmax = align256(o_meta + sizeof(InstMeta) * (size_t)B);
  const size_t o_bmax = align256(o_rmax + sizeof(unsigned long long) * (size_t)B);
  const size_t o_chunks = align256(o_bmax + sizeof(unsigned long long) * (size_t)B);
  const size_t total = o_chunks + sizeof(ResChunk) * chunks.size();
  if (total > (size_t)RLQR_NOALLOC_SCRATCH_BYTES) return RLQR_E_INVALID;

  void* base = nullptr;
  const rlqr_status as = scratch_address(&base);
  if (as != RLQR_OK) return as;
  unsigned char* p = static_cast<unsigned char*>(base);
  InstMeta* d_meta = reinterpret_cast<InstMeta*>(p + o_meta);
  unsigned long long* d_rmax = reinterpret_cast<unsigned long long*>(p + o_rmax);
  unsigned long long* d_bmax = reinterpret_cast<unsigned long long*>(p + o_bmax);
  ResChunk* d_chunks = reinterpret_cast<ResChunk*>(p + o_chunks);
  hipStream_t st = (hipStream_t)stv;

  NA_TRY(hipMemcpyAsync(d_meta, meta.data(), sizeof(InstMeta) * meta.size(), hipMemcpyHostToDevice, st));
  NA_TRY(hipMemcpyAsync(d_chunks, chunks.data(), sizeof(ResChunk) * chunks.size(), hipMemcpyHostToDevice, st));
  // the maxima accumulate by atomic max from zero: clear them (fill kernel over their 32-bit halves)
  NA_TRY(launch_fill_i32(reinterpret_cast<int32_t*>(d_rmax), 2 * B, 0, st));
  NA_TRY(launch_fill_i32(reinterpret_cast<int32_t*>(d_bmax), 2 * B, 0, st));

  ResidualArgs a{};
  a.batch = B; a.meta = d_meta; a.chunks = d_chunks; a.nchunks = (int64_t)chunks.size();
  a.run = nullptr; a.skip = nullptr; a.info = nullptr;  // every instance, at the given z
  a.Q = lhs->Q; a.M = lhs->M; a.R = lhs->R; a.A = lhs->A; a.B = lhs->B; a.delta = lhs->delta;
  a.dd = lhs->delta_diag;
  a.q = rhs->q; a.r = rhs->r; a.c = rhs->c;
  a.x = z->x; a.u = z->u; a.y = z->y;
  a.res = res; a.resmax = d_rmax; a.bmax = d_bmax;
  NA_TRY(launch_residual(a, shape, st));
  if (inst_relres) {
    CheckArgs c{};
    c.batch = B; c.final_pass = 1; c.plain = 1; c.tol = 0.0;
    c.resmax = d_rmax; c.bmax = d_bmax; c.relres = inst_relres;
    NA_TRY(launch_check(c, st));
  }
  return RLQR_OK;
}
