// Langevin NPT integrator on gfx950 (section 3.2 eq. (24); appendix A eq.
// (99999); section 3.3 splitting B_V B_R A_V A_R O^p O A_R A_V | forces |
// B_R B_V), FP64.  Two kernels per step around the force evaluation:
//   k_md_first   every block replays the cell sub-steps (B_V, A_V, O^p, A_V:
//                scalar work, identical in every block) and applies B_R, A_R,
//                O, A_R to its particles; block 0 stores the mid-step cell
//   k_md_second  B_R on every particle, the kinetic tensor summed in a fixed
//                order by the last-arriving block, which forms the pressure
//                tensor and applies the closing B_V
// The start-of-step and mid-step cells live in two buffers, so no block reads
// a cell another block of the same launch writes.
#include "rbe_md_internal.h"
#include <math.h>

namespace rbe {

__device__ __forceinline__ void philox_md(uint64_t c[4], uint64_t k0, uint64_t k1) {
  // Philox4x64-10 (Salmon et al., SC'11)
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) { k0 += W0; k1 += W1; }
    const uint64_t lo0 = M0 * c[0], hi0 = __umul64hi(M0, c[0]);
    const uint64_t lo1 = M1 * c[2], hi1 = __umul64hi(M1, c[2]);
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
  }
}

constexpr uint64_t kTagNoise = 0x6E6F6973ull;   // 'nois'
constexpr uint64_t kTagCell = 0x63656C6Cull;    // 'cell'

// three standard normals (Box-Muller on the four uniforms of one counter)
__device__ __forceinline__ void normals3(uint64_t seed, uint64_t sysid, uint64_t step,
                                         uint64_t index, uint64_t tag, double z[3]) {
  uint64_t c[4] = {step, index, tag, 0ull};
  philox_md(c, seed, sysid);
  double u[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) u[j] = (double)(c[j] >> 11) * 0x1.0p-53;
  const double a = sqrt(-2.0 * log(1.0 - u[0]));
  const double b = sqrt(-2.0 * log(1.0 - u[2]));
  double s1, c1, s3, c3;
  sincospi(2.0 * u[1], &s1, &c1);
  sincospi(2.0 * u[3], &s3, &c3);
  z[0] = a * c1; z[1] = a * s1; z[2] = b * c3;
}

// (e^{a h} - 1)/a, h at a = 0
__device__ __forceinline__ double expm1_over(double a, double h) {
  return a == 0.0 ? h : expm1(a * h) / a;
}

__device__ __forceinline__ double cell_volume(const MDCell& c) {
  return c.mode == 0 ? c.V : c.A * c.L;
}

__device__ __forceinline__ void cell_rates(const MDCell& c, double a[3]) {
  if (c.mode == 0) {
    const double r = c.pV / (3.0 * c.M * c.V);
    a[0] = a[1] = a[2] = r;
  } else {
    a[0] = a[1] = c.pA / (2.0 * c.MA * c.A);
    a[2] = c.pL / (c.ML * c.L);
  }
}

__device__ __forceinline__ void cell_lengths(MDCell& c) {
  if (c.mode == 0) {
    const double L = cbrt(c.V);
    c.l[0] = c.asp[0] * L; c.l[1] = c.asp[1] * L; c.l[2] = c.asp[2] * L;
  } else {
    const double s = sqrt(c.A);
    c.l[0] = c.l[1] = s;
    c.l[2] = c.L;
  }
  if (!(c.l[0] > 0.0 && c.l[2] > 0.0)) c.err |= 1;    // collapsed or non-finite cell
}

__device__ __forceinline__ void B_V(const MDArgs& a, MDCell& c, double h) {
  const double P = a.ftm * a.P;
  const double* Pt = c.P_ins;
  if (c.mode == 0) c.pV += h * ((Pt[0] + Pt[1] + Pt[2]) / 3.0 - P);
  else {
    c.pA += h * c.L * (0.5 * (Pt[0] + Pt[1]) - P);
    c.pL += h * c.A * (Pt[2] - P);
  }
}

__device__ __forceinline__ void A_V(MDCell& c, double h) {
  if (c.mode == 0) c.V += h * c.pV / c.M;
  else { c.A += h * c.pA / c.MA; c.L += h * c.pL / c.ML; }
}

__device__ __forceinline__ void md_first_body(const MDArgs& a, int bx) {
  __shared__ MDCell sc;
  __shared__ double rate[3][3];
  const double h = 0.5 * a.dt;
  if (threadIdx.x == 0) {
    MDCell c = *a.cell_in;
    B_V(a, c, h);
    cell_rates(c, rate[0]);                 // B_R
    A_V(c, h);
    cell_rates(c, rate[1]);                 // first A_R
    double z[3];
    normals3(a.seed, a.sysid, a.step, 0, kTagCell, z);
    const double c1 = exp(-a.gc * a.dt);
    const double amp = sqrt(a.ftm * a.kT * (1.0 - c1 * c1));
    if (c.mode == 0) c.pV = c1 * c.pV + amp * sqrt(c.M) * z[0];
    else {
      c.pA = c1 * c.pA + amp * sqrt(c.MA) * z[0];
      c.pL = c1 * c.pL + amp * sqrt(c.ML) * z[1];
    }
    cell_rates(c, rate[2]);                 // second A_R
    A_V(c, h);
    cell_lengths(c);
    c.step = a.step;
    sc = c;
  }
  __syncthreads();
  if (bx == 0 && threadIdx.x == 0) *a.cell_out = sc;
  const int64_t i = (int64_t)bx * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const double m = a.mass[i], im = 1.0 / m;
  double r[3] = {a.x[i], a.y[i], a.z[i]};
  double p[3] = {a.px[i], a.py[i], a.pz[i]};
  const double F[3] = {a.fx[i], a.fy[i], a.fz[i]};
  double z[3];
  normals3(a.seed, a.sysid, a.step, (uint64_t)i, kTagNoise, z);
  const double c1 = exp(-a.gp * a.dt);
  const double amp = sqrt(a.ftm * a.kT * m * (1.0 - c1 * c1));
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    p[d] = p[d] * exp(-rate[0][d] * h) + a.ftm * F[d] * expm1_over(-rate[0][d], h);   // B_R
    r[d] = r[d] * exp(rate[1][d] * h) + p[d] * im * expm1_over(rate[1][d], h);        // A_R
    p[d] = c1 * p[d] + amp * z[d];                                                    // O
    r[d] = r[d] * exp(rate[2][d] * h) + p[d] * im * expm1_over(rate[2][d], h);        // A_R
  }
  a.x[i] = r[0]; a.y[i] = r[1]; a.z[i] = r[2];
  a.px[i] = p[0]; a.py[i] = p[1]; a.pz[i] = p[2];
}

__device__ __forceinline__ double wsum_md(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// mode 0: closing half step (B_R, pressure, B_V); mode 1: pressure only
__device__ __forceinline__ void md_second_body(const MDArgs& a, int prime, int bx, int nbx) {
  __shared__ MDCell sc;
  __shared__ double sh[4][6];
  __shared__ int sh_last;
  const double h = 0.5 * a.dt;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (threadIdx.x == 0) sc = *a.cell_in;
  __syncthreads();
  double rate[3];
  cell_rates(sc, rate);
  const int64_t i = (int64_t)bx * blockDim.x + threadIdx.x;
  double k6[6] = {0, 0, 0, 0, 0, 0};
  if (i < a.n) {
    double p[3] = {a.px[i], a.py[i], a.pz[i]};
    if (!prime) {
      const double F[3] = {a.fx[i], a.fy[i], a.fz[i]};
#pragma unroll
      for (int d = 0; d < 3; ++d)
        p[d] = p[d] * exp(-rate[d] * h) + a.ftm * F[d] * expm1_over(-rate[d], h);
      a.px[i] = p[0]; a.py[i] = p[1]; a.pz[i] = p[2];
    }
    const double im = 1.0 / a.mass[i];
    k6[0] = p[0] * p[0] * im; k6[1] = p[1] * p[1] * im; k6[2] = p[2] * p[2] * im;
    k6[3] = p[0] * p[1] * im; k6[4] = p[0] * p[2] * im; k6[5] = p[1] * p[2] * im;
  }
  for (int k = 0; k < 6; ++k) {
    const double s = wsum_md(k6[k]);
    if (lane == 0) sh[wave][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const double s = sh[0][threadIdx.x] + sh[1][threadIdx.x] + sh[2][threadIdx.x] + sh[3][threadIdx.x];
    __hip_atomic_store(&a.part[bx * 8 + threadIdx.x], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0)
    sh_last = __hip_atomic_fetch_add(a.cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (unsigned)nbx - 1u;
  __syncthreads();
  if (!sh_last) return;
  __shared__ double ksum[6];
  if (threadIdx.x < 6) {
    double s = 0.0;
    for (int b = 0; b < nbx; ++b)
      s += __hip_atomic_load(&a.part[b * 8 + threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    ksum[threadIdx.x] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    MDCell c = sc;
    const double V = cell_volume(c);
    for (int k = 0; k < 6; ++k) {
      double w = 0.0;
      if (a.virial_k) w += a.virial_k[k];
      if (a.virial_r) w += a.virial_r[k];
      c.K[k] = ksum[k];
      c.P_ins[k] = (ksum[k] + a.ftm * w) / V;
    }
    if (!prime) B_V(a, c, h);
    *a.cell_out = c;
    *a.cnt = 0u;
  }
}

__global__ void __launch_bounds__(256) k_md_first(MDArgs a) { md_first_body(a, blockIdx.x); }
__global__ void __launch_bounds__(256) k_md_second(MDArgs a, int prime) {
  md_second_body(a, prime, blockIdx.x, gridDim.x);
}

hipError_t launch_md_first(const MDArgs& a, hipStream_t s) {
  const unsigned blocks = (unsigned)((a.n + 255) / 256);
  hipLaunchKernelGGL(k_md_first, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_md_second(const MDArgs& a, int prime, hipStream_t s) {
  const unsigned blocks = (unsigned)((a.n + 255) / 256);
  hipLaunchKernelGGL(k_md_second, dim3(blocks), dim3(256), 0, s, a, prime);
  return hipGetLastError();
}

// many systems per launch (block b -> system s with bstart[s] <= b < bstart[s+1])
__device__ __forceinline__ int find_sys_m(const int* bstart, int nsys, int b) {
  int lo = 0, hi = nsys - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bstart[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ void __launch_bounds__(256) k_md_first_m(const MDArgs* tab, const int* bstart, int nsys) {
  __shared__ MDArgs sa;
  const int sys = find_sys_m(bstart, nsys, blockIdx.x);
  if (threadIdx.x == 0) sa = tab[sys];
  __syncthreads();
  md_first_body(sa, blockIdx.x - bstart[sys]);
}

__global__ void __launch_bounds__(256) k_md_second_m(const MDArgs* tab, const int* bstart, int nsys,
                                                     int prime) {
  __shared__ MDArgs sa;
  const int sys = find_sys_m(bstart, nsys, blockIdx.x);
  if (threadIdx.x == 0) sa = tab[sys];
  __syncthreads();
  md_second_body(sa, prime, blockIdx.x - bstart[sys], bstart[sys + 1] - bstart[sys]);
}

hipError_t launch_md_first_multi(const MDArgs* d_tab, const int* d_bstart, int nsys, int total,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_md_first_m, dim3(total), dim3(256), 0, s, d_tab, d_bstart, nsys);
  return hipGetLastError();
}

hipError_t launch_md_second_multi(const MDArgs* d_tab, const int* d_bstart, int nsys, int total,
                                  int prime, hipStream_t s) {
  hipLaunchKernelGGL(k_md_second_m, dim3(total), dim3(256), 0, s, d_tab, d_bstart, nsys, prime);
  return hipGetLastError();
}

}  // namespace rbe
