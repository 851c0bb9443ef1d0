// Internal declarations of the real-space pair kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "../../include/rbe.h"

namespace rbe {

constexpr int kCellMax = 2048;     // members of one cell the sort kernel can order
constexpr int kCellAxisMax = 96;   // cells per axis
constexpr int kPairWaves = 4;      // pair kernel: waves per block
constexpr int kPairPerWave = 1;    // particles i a wave takes in turn
constexpr int kPairPerBlock = kPairWaves * kPairPerWave;
constexpr int kPairQueue = 512;    // accepted-pair queue of a wave
constexpr int kSegments = 50;      // neighbour segments: 25 rows of 5 cells, split at x wraps

constexpr int kBinPer = 2048;      // particles a binning block takes (256 threads)
constexpr int kBinLds = 8192;      // cells counted in LDS by the binning kernels

__host__ __device__ inline int64_t bin_blocks(int64_t n) { return (n + kBinPer - 1) / kBinPer; }

__host__ __device__ inline int64_t pair_blocks(int64_t n) {
  return (n + kPairPerBlock - 1) / kPairPerBlock;
}

struct RealArgs {
  const double* x; const double* y; const double* z;
  double* fx; double* fy; double* fz;
  double* virial6; double* energy;
  const double* q; const int32_t* type;   // type may be NULL
  const double* lj;                        // [ntypes*ntypes][2] = (c12, c6)
  int32_t ntypes, accumulate;
  int32_t prec32, pad;                     // 1: single-precision pair arithmetic
  int64_t n;
  double alpha, rc, coulomb;
  double box[3];                           // used when box_ptr is NULL
  const double* box_ptr;                   // device cell (3 doubles) or NULL
  int32_t nc_cap[3];
  // scratch (context-owned)
  int32_t* cellof; int32_t* count; int32_t* start; int32_t* cursor; int32_t* list;
  double4* xq;                             // cell order: wrapped x, y, z and q
  float4* xf;                              // the same positions in FP32 (candidate tests)
  int32_t* ts; int32_t* cs;
  int32_t* grid;                           // cells per axis of the last binning
  double* part;                            // [pair_blocks(n)][8]
  uint32_t* cnt;
  int32_t* err;                            // bit 1: rc > 2l/5 or cell cap; bit 2: cell overflow
};

hipError_t launch_real(const RealArgs& a, int ncell_cap, hipStream_t s);
hipError_t launch_real_multi(const RealArgs* d_tab, const int* d_bstart_p, int total_p,
                             const int* d_bstart_c, int total_c, const int* d_bstart_q, int total_q,
                             int nsys, int prec32, hipStream_t s);

// host side of rbe_real_forces without the launches
rbe_status real_step_args(rbe_real_ctx c, const double* d_x, const double* d_y, const double* d_z,
                          double* d_fx, double* d_fy, double* d_fz, int accumulate,
                          double* d_virial6, double* d_energy, RealArgs* out, int* ncell_cap);
// device bytes rbe_real_init allocates (each buffer rounded up to 256 bytes)
int64_t real_footprint(const rbe_real_config* cfg, const double* box);

}  // namespace rbe
