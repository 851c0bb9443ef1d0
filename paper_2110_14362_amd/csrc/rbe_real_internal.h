// Internal declarations of the real-space pair kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "../../include/rbe.h"

namespace rbe {

constexpr int kCellMax = 2048;     // members of one cell the sort kernel can order
constexpr int kCellAxisMax = 64;   // cells per axis

struct RealArgs {
  const double* x; const double* y; const double* z;
  double* fx; double* fy; double* fz;
  double* virial6; double* energy;
  const double* q; const int32_t* type;   // type may be NULL
  const double* lj;                        // [ntypes*ntypes][2] = (c12, c6)
  int32_t ntypes, accumulate;
  int64_t n;
  double alpha, rc, coulomb;
  double box[3];                           // used when box_ptr is NULL
  const double* box_ptr;                   // device cell (3 doubles) or NULL
  int32_t nc_cap[3];
  // scratch (context-owned)
  int32_t* cellof; int32_t* count; int32_t* start; int32_t* cursor; int32_t* list;
  double* xs; double* ys; double* zs; double* qs; int32_t* ts; int32_t* cs;
  int32_t* grid;                           // cells per axis of the last binning
  double* part;                            // [blocks][8]
  uint32_t* cnt;
  int32_t* err;                            // bit 1: rc > l/3 or cell cap; bit 2: cell overflow
};

hipError_t launch_real(const RealArgs& a, int ncell_cap, hipStream_t s);

}  // namespace rbe
