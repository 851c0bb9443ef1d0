// Real-space part of the Ewald split on gfx950 (section 4.1 eq. (U2) and
// eq. (force); section 4.2: nearest image, pairs closer than the cutoff),
// with an optional Lennard-Jones 12-6 term per type pair.  FP64 throughout.
//
// One evaluation is five launches:
//   k_bin     cell of each particle (cells at least rc wide, >= 3 per axis)
//   k_scan    exclusive scan of the cell counts (one block), counts cleared
//   k_fill    scatter particle indices into their cells
//   k_csort   per cell: sort the member indices (bitonic, LDS) so every sum
//             below has a fixed order, and gather positions/charges/types
//             into cell order
//   k_pairs   one lane per particle (in cell order): the 27 neighbour cells,
//             forces, and per-block energy/virial partials summed in a
//             fixed order by the last-arriving block
#include "rbe_real_internal.h"
#include <math.h>

namespace rbe {

__device__ __forceinline__ int cell_coord(double x, double inv_l, int nc) {
  double s = x * inv_l;
  s -= floor(s);
  int c = (int)(s * nc);
  return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__device__ __forceinline__ void real_box(const RealArgs& a, double l[3]) {
  if (a.box_ptr) { l[0] = a.box_ptr[0]; l[1] = a.box_ptr[1]; l[2] = a.box_ptr[2]; }
  else { l[0] = a.box[0]; l[1] = a.box[1]; l[2] = a.box[2]; }
}

// cells per axis: floor(l / rc), clamped to [3, cap]; err bit 1 if clamped
__device__ __forceinline__ void cell_grid(const RealArgs& a, const double l[3], int nc[3], int& err) {
  for (int d = 0; d < 3; ++d) {
    const double f = floor(l[d] / a.rc);
    int v = (f >= 3.0 && f <= (double)a.nc_cap[d]) ? (int)f : -1;
    if (v < 0) { err |= (f < 3.0 || !(f == f)) ? 2 : 0; v = (f >= 3.0) ? a.nc_cap[d] : 3; }
    nc[d] = v;
  }
}

__device__ __forceinline__ void bin_body(const RealArgs& a, int bx) {
  const int64_t i = (int64_t)bx * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  double l[3];
  real_box(a, l);
  int nc[3], err = 0;
  cell_grid(a, l, nc, err);
  const int cx = cell_coord(a.x[i], 1.0 / l[0], nc[0]);
  const int cy = cell_coord(a.y[i], 1.0 / l[1], nc[1]);
  const int cz = cell_coord(a.z[i], 1.0 / l[2], nc[2]);
  const int c = (cz * nc[1] + cy) * nc[0] + cx;
  a.cellof[i] = c;
  atomicAdd(&a.count[c], 1);
  if (i == 0 && err) atomicOr(a.err, err);
}

__device__ __forceinline__ void scan_body(const RealArgs& a) {
  __shared__ int sh[1024];
  double l[3];
  real_box(a, l);
  int nc[3], err = 0;
  cell_grid(a, l, nc, err);
  const int ncell = nc[0] * nc[1] * nc[2];
  const int t = threadIdx.x;
  const int seg = (ncell + 1023) / 1024;
  const int b0 = min(ncell, t * seg), b1 = min(ncell, b0 + seg);
  int loc = 0, mx = 0;
  for (int c = b0; c < b1; ++c) { const int v = a.count[c]; loc += v; mx = max(mx, v); }
  sh[t] = loc;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {      // inclusive Hillis-Steele scan
    const int v = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += v;
    __syncthreads();
  }
  int run = sh[t] - loc;
  for (int c = b0; c < b1; ++c) {
    const int v = a.count[c];
    a.start[c] = run;
    a.cursor[c] = run;
    run += v;
    a.count[c] = 0;                               // ready for the next evaluation
  }
  if (t == 1023) a.start[ncell] = sh[1023];
  if (mx > kCellMax) atomicOr(a.err, 4);
  __syncthreads();
  if (t == 0) a.grid[0] = nc[0], a.grid[1] = nc[1], a.grid[2] = nc[2];
}

__device__ __forceinline__ void fill_body(const RealArgs& a, int bx) {
  const int64_t i = (int64_t)bx * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const int pos = atomicAdd(&a.cursor[a.cellof[i]], 1);
  a.list[pos] = (int)i;
}

// one block per cell: sort member indices, then gather in that order
__device__ __forceinline__ void csort_body(const RealArgs& a, int c) {
  __shared__ int key[kCellMax];
  const int ncell = a.grid[0] * a.grid[1] * a.grid[2];
  if (c >= ncell) return;
  const int s0 = a.start[c], cnt = min(a.start[c + 1] - s0, kCellMax);
  int np2 = 1;
  while (np2 < cnt) np2 <<= 1;
  for (int k = threadIdx.x; k < np2; k += blockDim.x) key[k] = k < cnt ? a.list[s0 + k] : INT32_MAX;
  __syncthreads();
  for (int size = 2; size <= np2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int k = threadIdx.x; k < np2; k += blockDim.x) {
        const int o = k ^ stride;
        if (o > k) {
          const bool up = (k & size) == 0;
          const int u = key[k], v = key[o];
          if ((u > v) == up) { key[k] = v; key[o] = u; }
        }
      }
      __syncthreads();
    }
  }
  for (int k = threadIdx.x; k < cnt; k += blockDim.x) {
    const int i = key[k];
    const int d = s0 + k;
    a.list[d] = i;
    a.xs[d] = a.x[i]; a.ys[d] = a.y[i]; a.zs[d] = a.z[i];
    a.qs[d] = a.q[i];
    a.ts[d] = a.type ? a.type[i] : 0;
    a.cs[d] = c;
  }
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ void pairs_body(const RealArgs& a, int bx, int nbx) {
  __shared__ double sh[4][8];
  __shared__ int sh_last;
  const int64_t t = (int64_t)bx * blockDim.x + threadIdx.x;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  double l[3];
  real_box(a, l);
  const int nx = a.grid[0], ny = a.grid[1], nz = a.grid[2];
  const double rc2 = a.rc * a.rc, sa = sqrt(a.alpha);
  const double two_sa_pi = 2.0 * sa / sqrt(M_PI);
  double fx = 0, fy = 0, fz = 0, u = 0, w[6] = {0, 0, 0, 0, 0, 0};
  if (t < a.n) {
    const double xi = a.xs[t], yi = a.ys[t], zi = a.zs[t], qi = a.qs[t];
    const int ti = a.ts[t];
    const int c = a.cs[t];
    const int cx = c % nx, cy = (c / nx) % ny, cz = c / (nx * ny);
    for (int dz = -1; dz <= 1; ++dz) {
      const int zz = (cz + dz + nz) % nz;
      for (int dy = -1; dy <= 1; ++dy) {
        const int yy = (cy + dy + ny) % ny;
        for (int dx = -1; dx <= 1; ++dx) {
          const int xx = (cx + dx + nx) % nx;
          const int cc = (zz * ny + yy) * nx + xx;
          const int j0 = a.start[cc], j1 = a.start[cc + 1];
          for (int j = j0; j < j1; ++j) {
            if (j == t) continue;
            double ex = a.xs[j] - xi, ey = a.ys[j] - yi, ez = a.zs[j] - zi;
            ex -= l[0] * rint(ex / l[0]);
            ey -= l[1] * rint(ey / l[1]);
            ez -= l[2] * rint(ez / l[2]);
            const double r2 = ex * ex + ey * ey + ez * ez;
            if (r2 >= rc2) continue;
            const double r = sqrt(r2), ir = 1.0 / r;
            // Coulomb: phi = C qi qj erfc(sa r)/r,  -phi' = C qi qj G(r)
            const double qq = a.coulomb * qi * a.qs[j];
            const double er = erfc(sa * r);
            double dU = -qq * (er * ir * ir + two_sa_pi * exp(-a.alpha * r2) * ir);   // U'(r)
            u += qq * er * ir;
            if (a.ntypes > 0) {
              const int k = ti * a.ntypes + a.ts[j];
              const double c12 = a.lj[2 * k], c6 = a.lj[2 * k + 1];
              const double i2 = ir * ir, i6 = i2 * i2 * i2;
              u += c12 * i6 * i6 - c6 * i6;
              dU += (-12.0 * c12 * i6 * i6 + 6.0 * c6 * i6) * ir;
            }
            // force on i: U'(r) x/r;  virial: (1/2) (-U'(r)) x x^T / r per ordered pair
            const double g = dU * ir;
            fx += g * ex; fy += g * ey; fz += g * ez;
            w[0] -= g * ex * ex; w[1] -= g * ey * ey; w[2] -= g * ez * ez;
            w[3] -= g * ex * ey; w[4] -= g * ex * ez; w[5] -= g * ey * ez;
          }
        }
      }
    }
    const int i = a.list[t];
    if (a.accumulate) { a.fx[i] += fx; a.fy[i] += fy; a.fz[i] += fz; }
    else { a.fx[i] = fx; a.fy[i] = fy; a.fz[i] = fz; }
  }
  // block partial of (U, W), fixed order: wave sums, then waves in order
  double v[7] = {u, w[0], w[1], w[2], w[3], w[4], w[5]};
  for (int k = 0; k < 7; ++k) {
    const double s = wsum(v[k]);
    if (lane == 0) sh[wave][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < 7) {
    const double s = sh[0][threadIdx.x] + sh[1][threadIdx.x] + sh[2][threadIdx.x] + sh[3][threadIdx.x];
    __hip_atomic_store(&a.part[bx * 8 + threadIdx.x], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0)
    sh_last = __hip_atomic_fetch_add(a.cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (unsigned)nbx - 1u;
  __syncthreads();
  if (!sh_last) return;
  // the last block: sum the block partials in block order (thread k: component k)
  if (threadIdx.x < 7) {
    double s = 0.0;
    for (int b = 0; b < nbx; ++b)
      s += __hip_atomic_load(&a.part[b * 8 + threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (threadIdx.x == 0) { if (a.energy) a.energy[0] = 0.5 * s; }
    else if (a.virial6) a.virial6[threadIdx.x - 1] = 0.5 * s;
  }
  if (threadIdx.x == 0) *a.cnt = 0u;
}

__global__ void __launch_bounds__(256) k_bin(RealArgs a) { bin_body(a, blockIdx.x); }
__global__ void __launch_bounds__(1024) k_scan(RealArgs a) { scan_body(a); }
__global__ void __launch_bounds__(256) k_fill(RealArgs a) { fill_body(a, blockIdx.x); }
__global__ void __launch_bounds__(256) k_csort(RealArgs a) { csort_body(a, blockIdx.x); }
__global__ void __launch_bounds__(256) k_pairs(RealArgs a) { pairs_body(a, blockIdx.x, gridDim.x); }

hipError_t launch_real(const RealArgs& a, int ncell_cap, hipStream_t s) {
  const unsigned pb = (unsigned)((a.n + 255) / 256);
  hipLaunchKernelGGL(k_bin, dim3(pb), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, a);
  hipLaunchKernelGGL(k_fill, dim3(pb), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_csort, dim3(ncell_cap), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_pairs, dim3(pb), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// many systems per launch: block b of a launch belongs to system s with
// bstart[s] <= b < bstart[s+1] (one table per kernel shape); the system's
// arguments are copied to LDS.

__device__ __forceinline__ int find_sys_r(const int* bstart, int nsys, int b) {
  int lo = 0, hi = nsys - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bstart[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

#define REAL_MULTI_PROLOGUE                                \
  __shared__ RealArgs sa;                                  \
  const int b = blockIdx.x;                                \
  const int sys = find_sys_r(bstart, nsys, b);             \
  if (threadIdx.x == 0) sa = tab[sys];                     \
  __syncthreads();                                         \
  const int lb = b - bstart[sys], nb = bstart[sys + 1] - bstart[sys];

__global__ void __launch_bounds__(256) k_bin_m(const RealArgs* tab, const int* bstart, int nsys) {
  REAL_MULTI_PROLOGUE
  (void)nb;
  bin_body(sa, lb);
}
__global__ void __launch_bounds__(1024) k_scan_m(const RealArgs* tab, int nsys) {
  __shared__ RealArgs sa;
  if (threadIdx.x == 0) sa = tab[blockIdx.x];
  __syncthreads();
  (void)nsys;
  scan_body(sa);
}
__global__ void __launch_bounds__(256) k_fill_m(const RealArgs* tab, const int* bstart, int nsys) {
  REAL_MULTI_PROLOGUE
  (void)nb;
  fill_body(sa, lb);
}
__global__ void __launch_bounds__(256) k_csort_m(const RealArgs* tab, const int* bstart, int nsys) {
  REAL_MULTI_PROLOGUE
  (void)nb;
  csort_body(sa, lb);
}
__global__ void __launch_bounds__(256) k_pairs_m(const RealArgs* tab, const int* bstart, int nsys) {
  REAL_MULTI_PROLOGUE
  pairs_body(sa, lb, nb);
}

// bstart_p: per-particle blocks (256 particles each); bstart_c: cell blocks
hipError_t launch_real_multi(const RealArgs* d_tab, const int* d_bstart_p, int total_p,
                             const int* d_bstart_c, int total_c, int nsys, hipStream_t s) {
  hipLaunchKernelGGL(k_bin_m, dim3(total_p), dim3(256), 0, s, d_tab, d_bstart_p, nsys);
  hipLaunchKernelGGL(k_scan_m, dim3(nsys), dim3(1024), 0, s, d_tab, nsys);
  hipLaunchKernelGGL(k_fill_m, dim3(total_p), dim3(256), 0, s, d_tab, d_bstart_p, nsys);
  hipLaunchKernelGGL(k_csort_m, dim3(total_c), dim3(256), 0, s, d_tab, d_bstart_c, nsys);
  hipLaunchKernelGGL(k_pairs_m, dim3(total_p), dim3(256), 0, s, d_tab, d_bstart_p, nsys);
  return hipGetLastError();
}

}  // namespace rbe
