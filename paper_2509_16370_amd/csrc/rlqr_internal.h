// rlqr_internal.h -- argument blocks shared by the host API and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rlqr.h"

namespace rlqr {

// Per-instance metadata: shape and element offsets into every packed array
// (ows in workspace elements, opk in float64 elements of the p/k scratch).
struct InstMeta {
  int32_t N, n, m, pad;
  int64_t oQ, oM, oR, oA, oB, oq, or_, oc, ox, ou, oy, ores, ows, opk;
};

// Certificate bookkeeping written by the factor kernels.
struct FactorInfo {
  int32_t verdict, first_bad, singular, pad;
  int64_t npos, nneg, nzero;
  double minrel;  // min |pivot| / max|diag| over all pivots
};

struct FactorArgs {
  const InstMeta* meta;
  const int32_t* list;    // block -> instance (NULL: identity)
  const int32_t* run;     // if set, only instances with run[b] != 0 are touched
  const double *Q, *M, *R, *A, *B, *delta;
  void* ws;
  FactorInfo* info;
};

struct SolveArgs {
  const InstMeta* meta;
  const int32_t* list;
  const int32_t* run;     // if set, only instances with run[b] != 0 are touched
  const double *Q, *M, *R, *A, *B, *delta;
  const void* ws;
  const FactorInfo* info;
  const double *q, *r, *c;  // the original right-hand side
  const double* corr;       // if set: correction pass, right-hand side = this residual, z += dz
  double *x, *u, *y;
  double* pk;               // p_i / k_i scratch
  double* res_out;          // residual of the resulting z (fused kernels), may be NULL
  unsigned long long *resmax, *bmax;  // written by fused kernels
};

struct ResidualArgs {
  int batch;
  const InstMeta* meta;
  const int32_t* blk_inst;   // block -> instance (one block per stage i = 0..N of each instance)
  const int64_t* stage_off;  // exclusive prefix of N_b + 1
  const int32_t* run;
  const int32_t* skip;       // if set, instances with skip[b] != 0 are left alone
  const FactorInfo* info;
  const double *Q, *M, *R, *A, *B, *delta;
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

hipError_t launch_factor(const FactorArgs& a, int nblocks, bool fp32_products, hipStream_t st);
hipError_t launch_factor_mw(int cls, const FactorArgs& a, int nblocks, bool fp32, hipStream_t st);
hipError_t launch_solve_mw(int cls, const SolveArgs& a, int nblocks, bool fp32, hipStream_t st);
hipError_t launch_solve(const SolveArgs& a, int nblocks, bool fp32_tiles, hipStream_t st);
hipError_t launch_residual(const ResidualArgs& a, int64_t nblocks, hipStream_t st);
hipError_t launch_check(const CheckArgs& a, hipStream_t st);
hipError_t launch_inertia(const InertiaArgs& a, hipStream_t st);
hipError_t launch_fill_i32(int32_t* p, int count, int32_t v, hipStream_t st);

struct MaskArgs {
  int batch;
  int kind;               // 0: run masks, 1: guard band, 2: pick fallback instances, 3: fallback run mask
  double guard;
  const FactorInfo* info;
  const int32_t* status;
  int32_t *flag64, *conv, *run32, *run64, *runres, *fb;
};
hipError_t launch_masks(const MaskArgs& a, hipStream_t st);

}  // namespace rlqr
