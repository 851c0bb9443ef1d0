// Internal declarations of the Langevin NPT integrator kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "../../include/rbe.h"

namespace rbe {

// Cell and barostat state (internal units: forces x ftm).
struct MDCell {
  int32_t mode;      // 0 isotropic (V, pV), 1 semi-isotropic (A, pA, L, pL),
                     // 2 anisotropic rectangular (l, pl)
  int32_t err;       // bit 0: non-positive or non-finite cell
  double V, pV, M;
  double A, pA, MA, L, pL, ML;
  double l[3];       // side lengths (the state itself in mode 2)
  double pl[3], Ml[3];  // mode 2: momenta and masses of the side lengths
  double asp[3];     // isotropic mode: l = asp * V^(1/3), asp fixed (product 1)
  double P_ins[6];   // pressure tensor xx yy zz xy xz yz (internal units)
  double K[6];       // kinetic tensor sum p p^T / m (rigid molecules: P P^T / M)
  double C[6];       // rigid molecules: sum sym((r - R_mol) F), force x length units
  uint64_t step;
};

struct MDArgs {
  double* x; double* y; double* z;
  double* px; double* py; double* pz;
  const double* fx; const double* fy; const double* fz;
  const double* virial_k; const double* virial_r;
  const double* mass;
  int64_t n;
  double dt, kT, P, gp, gc, ftm;
  uint64_t seed, sysid, step;
  const MDCell* cell_in;
  MDCell* cell_out;
  double* part;      // [blocks][16] block partials, then [md_groups][16] group partials
  uint32_t* cnt;     // [md_groups + 1] arrival counters
  // rigid 3-site molecules: atoms rig_first + 3k (O), +1, +2 (H) for
  // k < rig_count; one thread per molecule, one per remaining atom
  int64_t rig_first, rig_count;
  double ra, rb, rc;   // the molecule in its centre-of-mass frame: O at (0, ra),
                       // H at (-rc, -rb) and (rc, -rb)
  int32_t* flags;      // bit 0: a position constraint had no solution
};

// threads (units) of the integrator kernels: molecules plus free atoms
__host__ __device__ inline int64_t md_units(const MDArgs& a) { return a.n - 2 * a.rig_count; }

// integrator blocks hold one wave of units: a rigid molecule's update is
// long FP64 work, so small blocks spread a system's molecules over more CUs
// (k_md_first adds three waves for the noise and the cell replay)
constexpr int kMdThreads = 64;
// threads of a k_md_first block (its kMdThreads units, four waves)
constexpr int kMdFirstThreads = 4 * 64;
static_assert(kMdThreads == 64, "k_md_first: a unit per lane of one wave");
__host__ __device__ inline int64_t md_blocks(int64_t units) { return (units + kMdThreads - 1) / kMdThreads; }
// pressure reduction: block partials summed by the last block of each group
// of kMdGroup blocks, group partials by the last group
constexpr int kMdGroup = kMdThreads;
__host__ __device__ inline int64_t md_groups(int64_t blocks) { return (blocks + kMdGroup - 1) / kMdGroup; }

hipError_t launch_md_first(const MDArgs& a, hipStream_t s);
hipError_t launch_md_second(const MDArgs& a, int prime, hipStream_t s);
hipError_t launch_md_first_multi(const MDArgs* d_tab, const int* d_bstart, int nsys, int total,
                                 hipStream_t s);
hipError_t launch_md_second_multi(const MDArgs* d_tab, const int* d_bstart, int nsys, int total,
                                  int prime, hipStream_t s);

// host side of rbe_md_first_half / rbe_md_second_half without the launches
rbe_status md_first_args(rbe_md_ctx c, uint64_t step, double* d_x, double* d_y, double* d_z,
                         double* d_px, double* d_py, double* d_pz, const double* d_fx,
                         const double* d_fy, const double* d_fz, MDArgs* out);
rbe_status md_second_args(rbe_md_ctx c, const double* d_x, const double* d_y, const double* d_z,
                          double* d_px, double* d_py, double* d_pz,
                          const double* d_fx, const double* d_fy, const double* d_fz,
                          const double* d_virial_k, const double* d_virial_r, MDArgs* out);
// device bytes rbe_md_init allocates (each buffer rounded up to 256 bytes)
int64_t md_footprint(int64_t n);

}  // namespace rbe
