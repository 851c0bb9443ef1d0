// Internal declarations of the Langevin NPT integrator kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "../../include/rbe.h"

namespace rbe {

// Cell and barostat state (internal units: forces x ftm).
struct MDCell {
  int32_t mode;      // 0 isotropic (V, pV), 1 semi-isotropic (A, pA, L, pL)
  int32_t err;       // bit 0: non-positive or non-finite cell
  double V, pV, M;
  double A, pA, MA, L, pL, ML;
  double l[3];       // side lengths
  double P_ins[6];   // pressure tensor xx yy zz xy xz yz (internal units)
  double K[6];       // kinetic tensor sum p p^T / m
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
  double* part;      // [blocks][8]
  uint32_t* cnt;
};

hipError_t launch_md_first(const MDArgs& a, hipStream_t s);
hipError_t launch_md_second(const MDArgs& a, int prime, hipStream_t s);

}  // namespace rbe
