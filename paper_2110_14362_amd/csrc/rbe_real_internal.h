// Internal declarations of the real-space pair kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "../../include/rbe.h"

namespace rbe {

constexpr int kCellMax = 2048;     // members of one cell the sort kernel can order
constexpr int kCellAxisMax = 96;   // cells per axis
constexpr int kPairWaves = 4;      // pair kernel: waves per block
// particles a wave of the pair kernels takes in turn: two on the FP32 path
// (the block's fixed costs and the arrival atomic are spread over more work),
// one on the FP64 path (its registers allow three waves per SIMD only)
constexpr int kPairPerWave64 = 1, kPairPerWave32 = 2;
__host__ __device__ constexpr int pair_per_wave(bool p32) { return p32 ? kPairPerWave32 : kPairPerWave64; }
constexpr int kPairQueue = 512;    // accepted-pair queue of a wave
// neighbour-list entries: the cell-order index in the low 25 bits, the
// Lennard-Jones type above them; lists hold at least 128 entries
constexpr int kListTypeShift = 25;
constexpr int kListIdxMask = (1 << kListTypeShift) - 1;
constexpr int kListMin = 128;
constexpr int kLjLds = 16;         // list pair kernel: LJ table in LDS up to this many types
constexpr int kSegments = 50;      // neighbour segments: 25 rows of 5 cells, split at x wraps
// list mode: cells at least (rc + skin)/kListReach wide, the list build's
// neighbourhood kListReach cells each way
constexpr int kListReach = 2;

constexpr int kBinPer = 2048;      // particles a binning block takes (256 threads)
constexpr int kBinLds = 8192;      // cells counted in LDS by the binning kernels

__host__ __device__ inline int64_t bin_blocks(int64_t n) { return (n + kBinPer - 1) / kBinPer; }

__host__ __device__ inline int64_t pair_blocks(int64_t n, bool p32) {
  const int per = kPairWaves * pair_per_wave(p32);
  return (n + per - 1) / per;
}
// the list pair kernel: a wave takes several particles in turn, requesting
// the next one's list while it works on the current one
constexpr int kListPerWave64 = 4, kListPerWave32 = 4;
__host__ __device__ constexpr int list_per_wave(bool p32) { return p32 ? kListPerWave32 : kListPerWave64; }
__host__ __device__ inline int64_t list_blocks(int64_t n, bool p32) {
  const int per = kPairWaves * list_per_wave(p32);
  return (n + per - 1) / per;
}
// the list build: one particle per wave
__host__ __device__ inline int64_t build_blocks(int64_t n) { return (n + kPairWaves - 1) / kPairWaves; }
// the most pair blocks of either path (sizes the block partials)
__host__ __device__ inline int64_t pair_blocks_max(int64_t n) { return build_blocks(n); }

// energy / virial reduction of the pair kernels: block partials summed by
// the last block of each group of kRedGroup blocks, group partials by the
// last group
constexpr int kRedGroup = 256;
__host__ __device__ inline int64_t red_groups(int64_t blocks) {
  return (blocks + kRedGroup - 1) / kRedGroup;
}
// list pair kernel: list entries staged in LDS per wave, this many at a time
constexpr int kListChunk = 1024;

struct RealArgs {
  const double* x; const double* y; const double* z;
  double* fx; double* fy; double* fz;
  double* virial6; double* energy;
  const double* q; const int32_t* type;   // type may be NULL
  const double* lj;                        // [ntypes*ntypes][2] = (c12, c6)
  int32_t ntypes, accumulate;
  int32_t prec32;                          // 1: single-precision pair arithmetic
  int32_t erfcx_short;                     // 1: the bounded-range erfcx series (short_series)
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
  double* part;                            // [pair_blocks_max(n)][8] block partials, then
                                           // [red_groups][8] group partials
  uint32_t* cnt;                           // [red_groups + 1] arrival counters
  int32_t* err;                            // bit 1: rc > 2l/5 or cell cap; bit 2: cell overflow;
                                           // bit 3: a neighbour list over capacity
  // neighbour lists (skin > 0): pairs closer than rc + skin at the last
  // build, rebuilt when 2 max|displacement| + sqrt(3) max|cell change| >= skin
  double skin;
  int32_t kcap, pad2;                      // list slots per particle
  int32_t* nbr;                            // [n][kcap] cell-ordered j of particle t (cell order)
  int32_t* ncount;                         // [n] list lengths
  double* ref;                             // [3][n] positions at the last build (input order)
  double* ref_box;                         // [3] cell at the last build
  double4* xc;                             // [n] current positions (unwrapped) and q, cell order
  unsigned long long* dmax;                // max squared displacement (FP64 bits)
  int32_t* state;                          // [0] 1: this evaluation rebuilds; [1] 1: built once
  uint32_t* vcnt;                          // arrival counter of the check kernel
};

// search radius of the cell grid: the cutoff, plus the skin with lists
__host__ __device__ inline double search_radius(const RealArgs& a) { return a.rc + a.skin; }

hipError_t launch_real(const RealArgs& a, int ncell_cap, hipStream_t s);
// The pair kernels take the bounded-range erfcx series (fewer terms) when
// every evaluated pair has x = sqrt(alpha) r < sqrt(alpha) rc within its
// range [0, 4]: decided once on the host at set-up (RealArgs::erfcx_short),
// per system, and read by the launches and the kernels alike.
constexpr double kErfcxRange = 4.0;
__host__ __device__ inline bool short_series(const RealArgs& a) { return a.erfcx_short != 0; }
// list-mode evaluation (a.skin > 0): check (and gather), conditional rebuild, pairs
hipError_t launch_real_list(const RealArgs& a, int ncell_cap, hipStream_t s);
hipError_t launch_real_multi(const RealArgs* d_tab, const int* d_bstart_p, int total_p,
                             const int* d_bstart_c, int total_c, const int* d_bstart_q, int total_q,
                             const int* d_bstart_b, int total_b,
                             const int* d_bstart_v, int total_v, int any_list, int any_cells,
                             int max_types, int nsys, int prec32, int series, hipStream_t s);

// host side of rbe_real_forces without the launches
rbe_status real_step_args(rbe_real_ctx c, const double* d_x, const double* d_y, const double* d_z,
                          double* d_fx, double* d_fy, double* d_fz, int accumulate,
                          double* d_virial6, double* d_energy, RealArgs* out, int* ncell_cap);
// device bytes rbe_real_init allocates (each buffer rounded up to 256 bytes),
// plus the neighbour lists of rbe_real_set_skin when skin > 0
int64_t real_footprint(const rbe_real_config* cfg, const double* box, double skin = 0.0);
// list slots per particle for a skin (rbe_real_set_skin)
int32_t list_capacity(int64_t n, const double* box, double rc, double skin);

}  // namespace rbe
