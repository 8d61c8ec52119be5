// rlqr_internal.h -- argument blocks shared by the host API and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rlqr.h"

namespace rlqr {

// Per-instance metadata: shape and element offsets into every packed array
// (ows in workspace elements, opk in float64 elements of the p/k scratch).
// Scan mode only: nseg stage segments, ovec the first boundary vector (n
// float64 per segment), opsi the first transfer matrix pair (2 n^2 float64
// per segment). od: offset of the instance's per-stage diagonals Delta_i
// (laid out like x; a stacked right-hand side keeps its base instance's).
struct InstMeta {
  int32_t N, n, m, nseg;
  int32_t chunk, pad;  // scan mode: stages per segment and per scan chunk
  int64_t oQ, oM, oR, oA, oB, oq, or_, oc, ox, ou, oy, ores, ows, opk, ovec, opsi, od;
};

// Certificate bookkeeping written by the factor kernels.
struct FactorInfo {
  int32_t verdict, first_bad, singular;
  int32_t nonfinite;  // a pivot was NaN or +-Inf (non-finite data reached the factorization)
  int64_t npos, nneg, nzero;
  double minrel;  // min |pivot| / max|diag| over all pivots
};

// A stage range [lo, hi) of one instance run by one factor workgroup. The
// recursion starts from P_hi: Q_N when hi == N, else the float32 tile P0
// (row-major, stride 16 * TX) produced by the parallel scan.
struct SegDesc {
  int32_t inst, lo, hi, p0_ld;  // p0_ld: row stride of P0
  int32_t gidx, s;              // index of this segment's SegStats; segment number in its instance
  const float* P0;
};

// Pivot bookkeeping of one segment, merged per instance by k_merge_stats.
struct SegStats {
  int32_t first_bad, nzero;
  int32_t npos, nneg;
  double minrel;
  int32_t nonfinite, pad;
};

struct FactorArgs {
  const InstMeta* meta;
  const SegDesc* segs;    // block -> segment
  const int32_t* run;     // if set, only instances with run[b] != 0 are touched
  const double *Q, *M, *R, *A, *B, *delta;
  const double* dd;       // if set: per-stage diagonal Delta_i (at InstMeta::od), delta unused
  void* ws;
  SegStats* stats;        // one per segment (indexed like segs)
  // optional right-hand side (one-wavefront kernels, whole instances): the
  // backward vector pass is run inside the stage loop and p_i / k_i written to pk
  const double *q, *r, *c;
  double* pk;
};

struct MergeArgs {
  int batch;
  const InstMeta* meta;
  const int32_t* seg_off;    // exclusive prefix of segments per instance (global segment order)
  const int32_t* run;
  const SegStats* stats;
  FactorInfo* info;
};

// Parallel-in-time scan over a list of instances (blockIdx.y indexes the list).
struct ScanArgs {
  const InstMeta* meta;
  const int32_t* insts;    // instances handled by this launch
  const int64_t* eoff;     // per instance: element offset (in elements) into elems
  const int64_t* aoff;     // per instance: chunk-aggregate offset (in elements) into aggr
  const double *Q, *M, *R, *A, *B, *delta;
  const double* dd;        // if set: per-stage diagonal Delta_i (at InstMeta::od), delta unused
  float* elems;            // N + 1 interval elements per instance
  float* aggr[2];          // chunk aggregates, ping-pong
  const float* aggr_in;
  float* aggr_out;
  int dist, maxN, maxchunks;
  int32_t* bad;            // per instance: set when the scan cannot be used
  // pc != 0: the elements also carry p and c (eq. lqr-gpu-combo), built from
  // the right-hand side q, r, c; 2 NX floats per element / aggregate (p at 0,
  // c at NX), indexed like elems / aggr
  int pc;
  const double *q, *r, *c;
  float* pce;
  float* pca[2];
  const float* pca_in;
  float* pca_out;
};
hipError_t launch_scan_elements(const ScanArgs& a, int ninst, int tx, int tm, hipStream_t st);
hipError_t launch_scan_tree(const ScanArgs& a, int ninst, int tx, bool bf16, hipStream_t st);
// Carried p: write p_{lo(s)} of every segment s >= 1 of the launch's
// multi-segment instances into the boundary vectors (InstMeta::ovec) from the
// finished suffix scan (the pca buffer given as pca_in).
hipError_t launch_scan_pc_boundary(const ScanArgs& a, int ninst, int tx, double* plo, hipStream_t st);
int scan_result_buffer(int maxchunks);
hipError_t scan_prepare();  // once per device before the first scan launch
hipError_t launch_merge(const MergeArgs& a, hipStream_t st);

// Transfer matrix of a segment [lo, hi): Psi = F_{hi-1} ... F_lo with
// F_k = S_hat_{k+1}^{-1} (A_k + B_k K_k), from the float32 factor tiles.
struct TransferArgs {
  const InstMeta* meta;
  const SegDesc* segs;
  const double *A, *B;
  const void* ws;          // float32 factor tiles
  double* psi;             // per segment: Psi (row-major n x n), then Psi^T
  const double* dd;        // if set: per-stage diagonal Delta_i; the X tiles then hold D X D
};
hipError_t launch_transfer(int cls, const TransferArgs& a, int nblocks, hipStream_t st);

// Sequential pass over the segment boundaries of each instance (one
// wavefront per instance): backward p_lo(s) += Psi_s^T p_lo(s+1), or forward
// xhi(s) += Psi_s xhi(s-1).
struct ChainArgs {
  const InstMeta* meta;
  const int32_t* insts;
  const int32_t* run;
  const double* psi;
  double* vec;
  int forward;
};
hipError_t launch_chain(const ChainArgs& a, int ninst, hipStream_t st);

struct SolveArgs {
  const InstMeta* meta;
  const int32_t* list;    // whole-instance solves: block -> instance
  const SegDesc* segs;    // segment solves: block -> segment
  int phase;              // segment solves: 1, 2 or 3 (see k_solve_mw)
  double *plo, *xhi;      // segment boundary vectors (n per segment, at InstMeta::ovec)
  const int32_t* run;     // if set, only instances with run[b] != 0 are touched
  const double *Q, *M, *R, *A, *B, *delta;
  const double* dd;       // if set: per-stage diagonal Delta_i (at InstMeta::od), delta unused
  const void* ws;
  const FactorInfo* info;
  const double *q, *r, *c;  // the original right-hand side
  const double* corr;       // if set: correction pass, right-hand side = this residual, z += dz
  double *x, *u, *y;
  double* pk;               // p_i / k_i scratch
  int fwd_only;             // whole-instance one-wavefront solves: p_i / k_i already in pk (fused factor)
  // whole-instance one-wavefront solves: the forward rollout also writes the
  // float64 residual of the updated solution (layout of k_residual) for the
  // instances with resfuse[b] != 0, and their maxima to resmax / bmax
  double* res;
  unsigned long long *resmax, *bmax;
  const int32_t* resfuse;
};
hipError_t launch_seg_solve(int cls, const SolveArgs& a, int nblocks, hipStream_t st);

// RES_CHUNK consecutive stage slots [i0, i1) of one instance (slots 0..N)
constexpr int RES_CHUNK = 16;
struct ResChunk {
  int32_t inst, i0, i1, pad;
};

struct ResidualArgs {
  int batch;
  const InstMeta* meta;
  const ResChunk* chunks;
  int64_t nchunks;
  const int32_t* run;
  const int32_t* skip;       // if set, instances with skip[b] != 0 are left alone
  const FactorInfo* info;
  const double *Q, *M, *R, *A, *B, *delta;
  const double* dd;          // if set: per-stage diagonal Delta_i (at InstMeta::od), delta unused
  const double *q, *r, *c;
  const double *x, *u, *y;
  double* res;
  unsigned long long *resmax, *bmax;
};

struct CheckArgs {
  int batch;
  int final_pass;
  int plain;              // only relres = resmax / bmax (no certificate, no flags)
  double tol;
  const FactorInfo* info;
  const int32_t* run;
  unsigned long long *resmax, *bmax;
  int32_t* conv;
  double* lastrel;
  int32_t* status;
  double* relres;
};

struct InertiaArgs {
  int batch;
  const FactorInfo* info;
  int32_t *verdict, *first_bad;
  int64_t* inertia;
};

// Tile classes: TILE_16 is the one-wavefront kernel (n + m <= 16); the others
// are (TX, TZ) = (ceil16 bound of n, of n + m) for the multi-wavefront kernels.
enum {
  TILE_16 = 0, TILE_X1_Z2, TILE_X2_Z2, TILE_X2_Z3, TILE_X3_Z3, TILE_X4_Z4, TILE_X4_Z6, TILE_CLASSES
};
// smallest class holding (n, m), or -1
inline int tile_class(int n, int m) {
  if (n + m <= 16) return TILE_16;
  static const int tx[] = {1, 1, 2, 2, 3, 4, 4}, tz[] = {1, 2, 2, 3, 3, 4, 6};
  for (int c = 1; c < TILE_CLASSES; ++c)
    if (n <= 16 * tx[c] && n + m <= 16 * tz[c]) return c;
  return -1;
}
int tile_blocks_per_stage(int cls);  // 16x16 blocks of workspace per stage

// Stage shapes of the one-wavefront kernels compiled with n and m fixed (the
// paper's cart-pole / acrobot and quad-pendulum sizes and a quadrotor); a
// launch over instances that all share one of them takes the fixed-shape
// kernel, any other launch the general one (SHAPE_ANY).
enum { SHAPE_ANY = 0, SHAPE_4_1, SHAPE_8_2, SHAPE_12_4 };
// launch_residual only: every chunk of the launch has n + m > 16
constexpr int SHAPE_LARGE = -1;
inline int fixed_shape(int n, int m) {
  if (n == 4 && m == 1) return SHAPE_4_1;
  if (n == 8 && m == 2) return SHAPE_8_2;
  if (n == 12 && m == 4) return SHAPE_12_4;
  return SHAPE_ANY;
}
hipError_t launch_factor(const FactorArgs& a, int nblocks, bool fp32_products, int shape, hipStream_t st);
// waves: wavefronts per workgroup of the multi-wavefront kernels for the tile
// classes up to 32 x 48 (TILE_X1_Z2, TILE_X2_Z2, TILE_X2_Z3): 1, 2, 4 or 8
// (the 32-wide classes take at least 2); the larger classes have their own
// fixed counts (9, 16)
hipError_t launch_factor_mw(int cls, const FactorArgs& a, int nblocks, bool fp32, hipStream_t st, int waves = 4);
hipError_t launch_solve_mw(int cls, const SolveArgs& a, int nblocks, bool fp32, hipStream_t st, int waves = 4);
hipError_t launch_solve(const SolveArgs& a, int nblocks, bool fp32_tiles, int shape, hipStream_t st);
hipError_t launch_residual(const ResidualArgs& a, int shape, hipStream_t st);
hipError_t launch_check(const CheckArgs& a, hipStream_t st);
hipError_t launch_inertia(const InertiaArgs& a, hipStream_t st);
hipError_t launch_fill_i32(int32_t* p, int count, int32_t v, hipStream_t st);

struct MaskArgs {
  int batch;
  int kind;               // 0: run masks, 1: guard band, 2: pick fallback instances, 3: fallback run mask,
                          // 4: single-segment float32 run mask, 5: out = !skip && in (in NULL: 1),
                          // 6: conv = skip
  double guard;
  const FactorInfo* info;
  const int32_t* status;
  const int32_t* bad;     // kind 1: instances whose scan failed also go to float64
  const int32_t* pref32;  // kind 1: if set, instances with pref32[b] == 0 always use float64
  const int32_t* multi;   // kind 4: instances with two or more segments
  const int32_t* skip;    // kinds 2, 5, 6: instances left out (rlqr_set_skip)
  const int32_t* in;      // kind 5
  int32_t* out;           // kind 5
  int32_t *flag64, *conv, *run32, *run64, *runres, *fb, *run1;
  int32_t* path;          // kinds 1, 2: if set, the precision path (RLQR_PATH_*) of each instance
};
hipError_t launch_masks(const MaskArgs& a, hipStream_t st);

// Shapes of a handle's batch (host arrays owned by the handle), for the
// cross-stage layer built on the public calls.
void handle_shapes(const rlqr_handle* h, int* batch, const int32_t** N, const int32_t** n, const int32_t** m);

}  // namespace rlqr
