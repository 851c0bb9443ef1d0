// Real-space part of the Ewald split on gfx950 (section 4.1 eq. (U2) and
// eq. (force); section 4.2: nearest image, pairs closer than the cutoff),
// with an optional Lennard-Jones 12-6 term per type pair.  Pair arithmetic
// in FP64 (the candidate test in FP32, with FP64 at the cutoff's edge).
//
// One evaluation is five launches:
//   k_bin     cell of each particle (cells at least rc/2 wide, >= 5 per axis)
//   k_scan    exclusive scan of the cell counts (one block), counts cleared
//   k_fill    scatter particle indices into their cells
//   k_csort   per cell: sort the member indices (bitonic, LDS) so every sum
//             below has a fixed order, and gather positions (wrapped into
//             the cell, consistently with the binning)/charges/types into
//             cell order
//   k_pairs   a wave per particle i at a time (in cell order): the 125
//             neighbour cells form up to 50 contiguous segments, laid end
//             to end as one candidate list that the lanes test 64 at a time
//             (each lane applying its segment's periodic shift to i), append
//             the pairs inside the cutoff to a wave-private LDS queue, and
//             evaluate the queue 64 pairs at a time with every lane busy;
//             the force on i is a fixed-order wave sum per batch, energy and
//             virial are per-lane sums reduced in a fixed order by the
//             last-arriving block
#include "rbe_real_internal.h"
#include "erfcx_poly.h"
#include "exp_table.h"
#include <math.h>

namespace rbe {

// fractional coordinate in [0, 1] (1 only by rounding) and its cell
__device__ __forceinline__ double frac_coord(double x, double inv_l) {
  const double s = x * inv_l;
  return s - floor(s);
}
__device__ __forceinline__ int cell_of(double s, int nc) {
  const int c = (int)(s * nc);
  return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}
__device__ __forceinline__ int cell_coord(double x, double inv_l, int nc) {
  return cell_of(frac_coord(x, inv_l), nc);
}

__device__ __forceinline__ void real_box(const RealArgs& a, double l[3]) {
  if (a.box_ptr) { l[0] = a.box_ptr[0]; l[1] = a.box_ptr[1]; l[2] = a.box_ptr[2]; }
  else { l[0] = a.box[0]; l[1] = a.box[1]; l[2] = a.box[2]; }
}

// cells per axis: floor(2 l / rs) (cells at least rs/2 wide, rs the search
// radius), clamped to [5, cap]; err bit 1 if clamped below (l < 2.5 rs)
__device__ __forceinline__ void cell_grid(const RealArgs& a, const double l[3], int nc[3], int& err) {
  for (int d = 0; d < 3; ++d) {
    const double f = floor(2.0 * l[d] / search_radius(a));
    int v = (f >= 5.0 && f <= (double)a.nc_cap[d]) ? (int)f : -1;
    if (v < 0) { err |= (f < 5.0 || !(f == f)) ? 2 : 0; v = (f >= 5.0) ? a.nc_cap[d] : 5; }
    nc[d] = v;
  }
}

// A block bins kBinPer particles; with at most kBinLds cells it counts them
// in LDS first and adds one total per cell to the global counts (far fewer
// contended global atomics).
// list mode: the cell list is rebuilt only with the neighbour lists
__device__ __forceinline__ bool skip_cells(const RealArgs& a) {
  return a.skin > 0.0 && __hip_atomic_load(&a.state[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
}

__device__ __forceinline__ void bin_body(const RealArgs& a, int bx) {
  __shared__ int hist[kBinLds];
  if (skip_cells(a)) return;
  double l[3];
  real_box(a, l);
  int nc[3], err = 0;
  cell_grid(a, l, nc, err);
  const int ncell = nc[0] * nc[1] * nc[2];
  const bool lds = ncell <= kBinLds;
  if (lds) {
    for (int c = threadIdx.x; c < ncell; c += blockDim.x) hist[c] = 0;
    __syncthreads();
  }
  const double il[3] = {1.0 / l[0], 1.0 / l[1], 1.0 / l[2]};
  for (int k = 0; k < kBinPer; k += blockDim.x) {
    const int64_t i = (int64_t)bx * kBinPer + k + threadIdx.x;
    if (i >= a.n) break;
    const int cx = cell_coord(a.x[i], il[0], nc[0]);
    const int cy = cell_coord(a.y[i], il[1], nc[1]);
    const int cz = cell_coord(a.z[i], il[2], nc[2]);
    const int c = (cz * nc[1] + cy) * nc[0] + cx;
    a.cellof[i] = c;
    if (lds) atomicAdd(&hist[c], 1);
    else atomicAdd(&a.count[c], 1);
  }
  if (lds) {
    __syncthreads();
    for (int c = threadIdx.x; c < ncell; c += blockDim.x)
      if (hist[c]) atomicAdd(&a.count[c], hist[c]);
  }
  if (bx == 0 && threadIdx.x == 0 && err) atomicOr(a.err, err);
}

__device__ __forceinline__ void scan_body(const RealArgs& a) {
  __shared__ int sh[1024];
  if (skip_cells(a)) return;
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

// Scatter particle indices into their cells' ranges: with at most kBinLds
// cells, ranks within the block come from LDS atomics and each cell's range
// for the block from one global atomic.
__device__ __forceinline__ void fill_body(const RealArgs& a, int bx) {
  __shared__ int hist[kBinLds];
  if (skip_cells(a)) return;
  const int ncell = a.grid[0] * a.grid[1] * a.grid[2];
  const bool lds = ncell <= kBinLds;
  constexpr int kPer = kBinPer / 256;
  int cell[kPer], rank[kPer];
  if (lds) {
    for (int c = threadIdx.x; c < ncell; c += blockDim.x) hist[c] = 0;
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int64_t i = (int64_t)bx * kBinPer + k * 256 + threadIdx.x;
    cell[k] = -1;
    if (i < a.n) {
      cell[k] = a.cellof[i];
      rank[k] = lds ? atomicAdd(&hist[cell[k]], 1) : atomicAdd(&a.cursor[cell[k]], 1);
    }
  }
  if (lds) {
    __syncthreads();
    for (int c = threadIdx.x; c < ncell; c += blockDim.x)
      if (hist[c]) hist[c] = atomicAdd(&a.cursor[c], hist[c]);
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int64_t i = (int64_t)bx * kBinPer + k * 256 + threadIdx.x;
    if (cell[k] >= 0) a.list[(lds ? hist[cell[k]] : 0) + rank[k]] = (int)i;
  }
}

// one block per cell: sort member indices, then gather in that order
__device__ __forceinline__ void csort_body(const RealArgs& a, int c) {
  __shared__ int key[kCellMax];
  if (skip_cells(a)) return;
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
  double l[3];
  real_box(a, l);
  for (int k = threadIdx.x; k < cnt; k += blockDim.x) {
    const int i = key[k];
    const int d = s0 + k;
    a.list[d] = i;
    // wrapped with the binning's own fractional coordinate, so a particle
    // lies in (or on the boundary of) the cell it was binned into
    double4 v;
    v.x = frac_coord(a.x[i], 1.0 / l[0]) * l[0];
    v.y = frac_coord(a.y[i], 1.0 / l[1]) * l[1];
    v.z = frac_coord(a.z[i], 1.0 / l[2]) * l[2];
    v.w = a.q[i];
    a.xq[d] = v;
    // the type rides in the FP32 copy's fourth word (the list build stores it
    // with each entry and so needs no load of its own)
    a.xf[d] = make_float4((float)v.x, (float)v.y, (float)v.z,
                          __int_as_float(a.type ? a.type[i] : 0));
    a.ts[d] = a.type ? a.type[i] : 0;
    a.cs[d] = c;
  }
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Accepted pairs of one wave: cell-ordered index of j and the periodic shift
// it was seen through (3 trits); the erfcx coefficients (a copy per wave).
struct PairQueue {
  int j[kPairQueue];
  int s[kPairQueue];
  double poly[kErfcxTerms];
  float poly32[kErfcxTerms32];
  double etab[64];              // 2^(j/64) for exp_nonpos
  int seg_off[kSegments + 1];   // candidate offset of each neighbour segment (exclusive scan)
  int seg_j0[kSegments];        // its first cell-ordered index
  int seg_code[kSegments];      // its periodic shift
  float4 seg_io[kSegments];     // i seen from the segment's image, FP32
};

// The list build's segments of a wave (reach R cells): as PairQueue's, for
// 2 (2R+1)^2 segments
template <int R>
struct ListSegs {
  static constexpr int kSeg = 2 * (2 * R + 1) * (2 * R + 1);
  int seg_off[kSeg + 1];
  int seg_j0[kSeg];
  int seg_code[kSeg];
  float4 seg_io[kSeg];
};

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// erfcx(x) = exp(x^2) erfc(x) for x >= 0 as a polynomial in
// t = (x - K)/(x + K) (Horner's rule: one FMA per term); erfc(x) =
// exp(-x^2) erfcx(x) then shares exp(-x^2) with the force term.  The
// coefficients are read from LDS, which keeps them out of the scalar
// registers.
// 1/d for d > 0: the hardware estimate refined by two Newton steps (an ulp or
// two; the correctly rounded division takes twice the instructions)
__device__ __forceinline__ double rcp_nr(double d) {
  double y = __builtin_amdgcn_rcp(d);
  y = fma(fma(-d, y, 1.0), y, y);
  return fma(fma(-d, y, 1.0), y, y);
}

// 1/sqrt(d) for a finite d > 0: the hardware estimate y refined by one
// second-order Newton step, y (1 + e/2 + 3 e^2/8) with e = 1 - d y^2 (the
// library's steps without its handling of zero, infinite and denormal d, which
// a pair separation never is)
__device__ __forceinline__ double rsqrt_pos(double d) {
  const double y = __builtin_amdgcn_rsq(d);
  const double e = fma(-d * y, y, 1.0);
  return fma(y * e, fma(e, 0.375, 0.5), y);
}

// e^x for x <= 0 by Tang's table-driven method (ACM TOMS 15 (1989) 144):
// x = (64 m + j) ln2/64 + r with |r| <= ln2/128 and e^x = 2^m 2^(j/64) e^r,
// e^r - 1 from its Taylor polynomial of degree 6 (truncated below 2e-20 of
// it); 2^(j/64) is read from the table in LDS.  Within about an ulp; 0 below
// e^-745.  Two thirds of the instructions of the library exp, which also
// handles overflow and non-finite arguments that a pair's -alpha r^2 never is.
__device__ __forceinline__ double exp_nonpos(double x, const double* etab) {
  const double n = rint(x * kExpInvL);
  const double r = fma(-n, kExpLlo, fma(-n, kExpLhi, x));
  const int ni = (int)n;
  double p = fma(r, 1.0 / 720.0, 1.0 / 120.0);
  p = fma(p, r, 1.0 / 24.0);
  p = fma(p, r, 1.0 / 6.0);
  p = fma(p, r, 0.5);
  p = fma(p, r, 1.0);
  const double t = etab[ni & 63];
  return ldexp(fma(t, p * r, t), ni >> 6);
}

// S: the series for 0 <= x <= kErfcxShortX only, in u = (A x - K)/(x + K)
// (six fewer terms), which the kernels take when sqrt(alpha) rc is in that range
template <bool S>
__device__ __forceinline__ double erfcx_pos(double x, const double* poly) {
  constexpr int n = S ? kErfcxTermsS : kErfcxTerms;
  const double t = (S ? fma(kErfcxShortA, x, -kErfcxK) : x - kErfcxK) * rcp_nr(x + kErfcxK);
  double y = poly[n - 1];
#pragma unroll
  for (int k = n - 2; k >= 0; --k) y = fma(y, t, poly[k]);
  return y;
}

// A queued pair as loaded for evaluation: j's position and charge, its
// type, and the shift code.
// A queued pair as loaded for evaluation: the separation x_j - x_i (the
// image the candidate test chose), q_j and type_j.
struct PairLoad {
  double ex, ey, ez, qj;
  int tj;
};

// cell path: the queue holds (j, shift code); the same arithmetic as the test
__device__ __forceinline__ PairLoad pair_load(const RealArgs& a, const PairQueue& Q, int e,
                                              const double4& vi, const double l[3]) {
  PairLoad p;
  const int j = Q.j[e], code = Q.s[e];
  const double4 v = a.xq[j];
  p.ex = v.x - (vi.x - l[0] * (double)(code % 3 - 1));
  p.ey = v.y - (vi.y - l[1] * (double)((code / 3) % 3 - 1));
  p.ez = v.z - (vi.z - l[2] * (double)(code / 9 - 1));
  p.qj = v.w;
  p.tj = a.ntypes > 0 ? a.ts[j] : 0;
  return p;
}

// Whether type t has a nonzero Lennard-Jones pair with some type (wave-
// uniform for a uniform t).  In the FP64 pair kernels a particle whose row is
// all zeros, such as a water hydrogen, skips the Lennard-Jones terms (they
// would add exact zeros); the FP32 ones measured slower with the branch.
__device__ __forceinline__ bool lj_row_nonzero(const RealArgs& a, const double* lj, int t) {
  if (a.ntypes <= 0) return false;
  int any = 0;
  for (int v = 0; v < a.ntypes; ++v) {
    const int k = t * a.ntypes + v;
    any |= (lj[2 * k] != 0.0 || lj[2 * k + 1] != 0.0) ? 1 : 0;
  }
  return uniform(any) != 0;
}

// Evaluate one loaded pair per lane (lanes with valid = false add nothing):
// the force on i is added as a wave sum (the same value in every lane, summed
// in a fixed order); energy and virial accumulate per lane.
// one pair's force on i (g), energy and virial terms (FP64)
template <bool S>
__device__ __forceinline__ void pair_core(const RealArgs& a, const PairLoad& p, bool valid,
                                          const double4& vi, int ti, double sa, double two_sa_pi,
                                          const double* poly, const double* etab, const double* lj,
                                          bool lj_on, double& gx, double& gy, double& gz, double& u,
                                          double w[6]) {
  gx = 0.0; gy = 0.0; gz = 0.0;
  if (valid) {
    const double ex = p.ex, ey = p.ey, ez = p.ez;
    const double r2 = ex * ex + ey * ey + ez * ez;
    const double ir = rsqrt_pos(r2), ir2 = ir * ir, r = r2 * ir;
    // Coulomb: U = C qi qj erfc(sa r)/r = qq A,
    // U'(r)/r = -qq (A + (2 sa/sqrt(pi)) exp(-sa^2 r^2))/r^2
    const double qq = a.coulomb * vi.w * p.qj;
    const double g2 = exp_nonpos(-a.alpha * r2, etab);
    const double A = g2 * erfcx_pos<S>(sa * r, poly) * ir;
    double rdU = -qq * fma(two_sa_pi, g2, A);                 // r U'(r)
    u = fma(qq, A, u);
    if (lj_on) {
      // U = c12/r^12 - c6/r^6,  r U'(r) = -12 c12/r^12 + 6 c6/r^6
      const int k = ti * a.ntypes + p.tj;
      const double i6 = ir2 * ir2 * ir2;
      const double t12 = lj[2 * k] * i6 * i6, t6 = lj[2 * k + 1] * i6;
      u += t12 - t6;
      rdU = fma(-12.0, t12, fma(6.0, t6, rdU));
    }
    // force on i: U'(r) x/r;  virial: (1/2) (-U'(r)) x x^T / r per ordered pair
    const double g = rdU * ir2;
    gx = g * ex; gy = g * ey; gz = g * ez;
    w[0] -= g * ex * ex; w[1] -= g * ey * ey; w[2] -= g * ez * ez;
    w[3] -= g * ex * ey; w[4] -= g * ex * ez; w[5] -= g * ey * ez;
  }
}

template <bool S>
__device__ __forceinline__ void pair_eval(const RealArgs& a, const PairLoad& p, bool valid,
                                          const double4& vi, int ti, const double l[3], double sa,
                                          double two_sa_pi, const double* poly, const double* etab,
                                          bool lj_on, double f[3], double& u, double w[6]) {
  double gx, gy, gz;
  pair_core<S>(a, p, valid, vi, ti, sa, two_sa_pi, poly, etab, a.lj, lj_on, gx, gy, gz, u, w);
  f[0] += wsum(gx);
  f[1] += wsum(gy);
  f[2] += wsum(gz);
}

// Single-precision pair arithmetic (the FP32 real-space option): the
// separation is formed in FP64 and rounded once; erfcx from the shorter
// series, exp(-x^2) and 1/sqrt from the hardware approximations (a few ulp);
// energy and virial summed per lane in FP32 over one particle's pairs, then
// folded into FP64; the force's wave sum is formed in FP32 and added in FP64.
// erfcx is always the full-range series here: the bounded-range one measured
// no faster in this kernel, which waits on its loads more than it issues.
__device__ __forceinline__ float erfcx_pos32(float x, const float* poly) {
  const float t = (x - (float)kErfcxK) * __builtin_amdgcn_rcpf(x + (float)kErfcxK);
  float y = poly[kErfcxTerms32 - 1];
#pragma unroll
  for (int k = kErfcxTerms32 - 2; k >= 0; --k) y = fmaf(y, t, poly[k]);
  return y;
}

__device__ __forceinline__ float wsumf(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ void pair_core32(const RealArgs& a, const PairLoad& p, bool valid,
                                            const double4& vi, int ti, float sa, float two_sa_pi,
                                            float alpha, const float* poly, const double* lj,
                                            bool lj_on, float& gx, float& gy, float& gz, float& u,
                                            float w[6]) {
  gx = 0.0f; gy = 0.0f; gz = 0.0f;
  if (valid) {
    const float ex = (float)p.ex, ey = (float)p.ey, ez = (float)p.ez;
    const float r2 = ex * ex + ey * ey + ez * ez;
    const float ir = __builtin_amdgcn_rsqf(r2), ir2 = ir * ir, r = r2 * ir;
    const float qq = (float)(a.coulomb * vi.w * p.qj);
    const float g2 = __expf(-alpha * r2);
    const float A = g2 * erfcx_pos32(sa * r, poly) * ir;
    float rdU = -qq * fmaf(two_sa_pi, g2, A);                 // r U'(r)
    u = fmaf(qq, A, u);
    if (lj_on) {
      const int k = ti * a.ntypes + p.tj;
      const float i6 = ir2 * ir2 * ir2;
      const float t12 = (float)lj[2 * k] * i6 * i6, t6 = (float)lj[2 * k + 1] * i6;
      u += t12 - t6;
      rdU = fmaf(-12.0f, t12, fmaf(6.0f, t6, rdU));
    }
    const float g = rdU * ir2;
    gx = g * ex; gy = g * ey; gz = g * ez;
    w[0] -= g * ex * ex; w[1] -= g * ey * ey; w[2] -= g * ez * ez;
    w[3] -= g * ex * ey; w[4] -= g * ex * ez; w[5] -= g * ey * ez;
  }
}

__device__ __forceinline__ void pair_eval32(const RealArgs& a, const PairLoad& p, bool valid,
                                            const double4& vi, int ti, const double l[3], float sa,
                                            float two_sa_pi, float alpha, const float* poly,
                                            bool lj_on, double f[3], float& u, float w[6]) {
  float gx, gy, gz;
  pair_core32(a, p, valid, vi, ti, sa, two_sa_pi, alpha, poly, a.lj, lj_on, gx, gy, gz, u, w);
  f[0] += (double)wsumf(gx);
  f[1] += (double)wsumf(gy);
  f[2] += (double)wsumf(gz);
}

// The segment table of particle vi in cell c, trimmed: of the (2R+1)^3
// cells around c, only those that can hold a partner closer than rs (the
// cutoff on the cell path, rc + skin for the list build): a row of cells
// along x (fixed dy, dz) is dropped when its y-z distance from the particle
// reaches rs, and a kept row keeps only the cells whose x distance from the
// particle is below what rs leaves (distances from the particle's own
// position to the nearest faces of the cells, with a relative margin of
// 1e-12 on rs^2, so the set only shrinks by cells that cannot hold a pair
// closer than rs).  Segments in the order of the untrimmed table (rows by dz,
// then dy; a row's part before a wrap in x, then after), so the accepted
// candidates keep their order.  Lane s + 64 k describes segment s + 64 k;
// returns the number of candidates.  T: a PairQueue or ListSegs<R>.
template <int R, class T>
__device__ __forceinline__ int trimmed_segment_table(const RealArgs& a, T& S, const double4& vi,
                                                     int c, int nx, int ny, int nz,
                                                     const double l[3], double rs, int lane) {
  constexpr int kRow = 2 * R + 1, kSeg = ListSegs<R>::kSeg;
  const int cx = c % nx, cy = (c / nx) % ny, cz = c / (nx * ny);
  const double wx = l[0] / nx, wy = l[1] / ny, wz = l[2] / nz;
  const double rs2 = rs * rs * (1.0 + 1e-12);
  int carry = 0;
#pragma unroll
  for (int pass = 0; pass < (kSeg + 63) / 64; ++pass) {
    const int sgi = pass * 64 + lane;
    int len = 0;
    if (sgi < kSeg) {
      const int row = sgi >> 1, half = sgi & 1;
      const int dz = row / kRow - R, dy = row % kRow - R;
      // the particle's distance to the row's nearest y and z faces
      const double gy = dy > 0 ? (cy + dy) * wy - vi.y : (dy < 0 ? vi.y - (cy + dy + 1) * wy : 0.0);
      const double gz = dz > 0 ? (cz + dz) * wz - vi.z : (dz < 0 ? vi.z - (cz + dz + 1) * wz : 0.0);
      const double hy = fmax(gy, 0.0), hz = fmax(gz, 0.0);
      const double rem = rs2 - hy * hy - hz * hz;
      bool on = false;
      int c0 = 0, c1 = -1, code = 13;
      if (rem > 0.0) {
        const double h = sqrt(rem);
        const int xa = cx + max(-R, (int)floor((vi.x - h) / wx) - cx);
        const int xb = cx + min(R, (int)floor((vi.x + h) / wx) - cx);
        int zz = cz + dz, yy = cy + dy, kz = 1, ky = 1, kx = 1;
        if (zz < 0) { zz += nz; kz = 0; } else if (zz >= nz) { zz -= nz; kz = 2; }
        if (yy < 0) { yy += ny; ky = 0; } else if (yy >= ny) { yy -= ny; ky = 2; }
        int x0 = 0, x1 = -1;
        if (xa < 0) {                              // cells xa .. -1 wrap to the far end
          if (half == 0) { x0 = nx + xa; x1 = nx - 1; kx = 0; } else { x0 = 0; x1 = xb; }
          on = true;
        } else if (xb > nx - 1) {                  // cells nx .. xb wrap to the start
          if (half == 0) { x0 = xa; x1 = nx - 1; } else { x0 = 0; x1 = xb - nx; kx = 2; }
          on = true;
        } else if (half == 0) {
          x0 = xa; x1 = xb;
          on = true;
        }
        if (on) {
          const int rbase = (zz * ny + yy) * nx;
          c0 = rbase + x0;
          c1 = rbase + x1;
          code = (kz * 3 + ky) * 3 + kx;
        }
      }
      if (on) {
        const int j0 = a.start[c0];
        len = a.start[c1 + 1] - j0;
        S.seg_j0[sgi] = j0;
        S.seg_io[sgi] = make_float4((float)(vi.x - l[0] * (double)(code % 3 - 1)),
                                    (float)(vi.y - l[1] * (double)((code / 3) % 3 - 1)),
                                    (float)(vi.z - l[2] * (double)(code / 9 - 1)), 0.0f);
      } else {
        S.seg_j0[sgi] = 0;
        S.seg_io[sgi] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      }
      S.seg_code[sgi] = code;
    }
    int incl = len;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(incl, off, 64);
      if (lane >= off) incl += v;
    }
    if (sgi < kSeg) S.seg_off[sgi] = carry + incl - len;
    carry += __shfl(incl, 63, 64);
  }
  if (lane == 0) S.seg_off[kSeg] = carry;
  wave_sync();
  return uniform(carry);
}

// FP32 bounds of the squared search radius outside of which the FP32 test
// decides as FP64 would: positions in [0, l] carry an error below 2^-24 l
// each, so a squared separation near rs errs by less than 8 rs 2^-24 lmax
__device__ __forceinline__ void radius_band(double rs, const double l[3], float& lo, float& hi) {
  const double lmax = fmax(l[0], fmax(l[1], l[2]));
  const double band = 16.0 * rs * lmax * 0x1.0p-24 + 8.0 * lmax * lmax * 0x1.0p-48;
  lo = (float)(rs * rs - band);
  hi = (float)(rs * rs + band);
}

// Sum 7 x m values held in LDS (red[k][j], j < m <= 256) in a fixed order:
// threads (k, c) add j = c, c + 32, ... in turn, then thread k adds its 32
// chunk sums in order.  Every thread of the block calls it.
__device__ __forceinline__ void fixed_sum7(double (*red)[kRedGroup + 1], double (*red2)[33], int m,
                                           double out[7]) {
  if (threadIdx.x < 7 * 32) {
    const int k = threadIdx.x / 32, ch = threadIdx.x % 32;
    double s = 0.0;
    for (int j = ch; j < m; j += 32) s += red[k][j];
    red2[k][ch] = s;
  }
  __syncthreads();
  if (threadIdx.x < 7) {
    double s = 0.0;
    for (int ch = 0; ch < 32; ++ch) s += red2[threadIdx.x][ch];
    out[threadIdx.x] = s;
  }
}

// Block partial of (U, W) in a fixed order (wave sums, then waves in order).
// The last-arriving block of each group of kRedGroup blocks sums the group's
// partials (every thread loads its block's seven at once) and the last group
// sums the group partials; both sums have a fixed order, so the result does
// not depend on which block arrives last.  Writes half of each total (every
// pair was counted from both ends).
// scratch: LDS of at least kRedScratch doubles that the caller no longer
// needs (its queue or list staging), written only after a block barrier.
constexpr int kRedScratch = 7 * (kRedGroup + 1) + 7 * 33;
__device__ __forceinline__ void block_energy_virial(const RealArgs& a, double u, const double w[6],
                                                    double (*sh)[8], int& sh_last, int bx, int nbx,
                                                    int wave, int lane, double* scratch) {
  double (*red)[kRedGroup + 1] = reinterpret_cast<double (*)[kRedGroup + 1]>(scratch);
  double (*red2)[33] = reinterpret_cast<double (*)[33]>(scratch + 7 * (kRedGroup + 1));
  __shared__ double tot[7];
  double v[7] = {u, w[0], w[1], w[2], w[3], w[4], w[5]};
  for (int k = 0; k < 7; ++k) {
    const double s = wsum(v[k]);
    if (lane == 0) sh[wave][k] = s;
  }
  __syncthreads();
  if (threadIdx.x < 7) {
    double s = 0.0;
    for (int q = 0; q < kPairWaves; ++q) s += sh[q][threadIdx.x];
    __hip_atomic_store(&a.part[bx * 8 + threadIdx.x], s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  const int g = bx / kRedGroup, ng = (nbx + kRedGroup - 1) / kRedGroup;
  const int gsize = min(kRedGroup, nbx - g * kRedGroup);
  if (threadIdx.x == 0)
    sh_last = __hip_atomic_fetch_add(&a.cnt[g], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (unsigned)gsize - 1u;
  __syncthreads();
  if (!sh_last) return;
  // the group's last block
  for (int j = threadIdx.x; j < kRedGroup; j += blockDim.x) {
    double pv[7];
#pragma unroll
    for (int k = 0; k < 7; ++k)
      pv[k] = j < gsize ? __hip_atomic_load(&a.part[(g * kRedGroup + j) * 8 + k], __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT) : 0.0;
#pragma unroll
    for (int k = 0; k < 7; ++k) red[k][j] = pv[k];
  }
  __syncthreads();
  fixed_sum7(red, red2, gsize, tot);
  double* gp = a.part + (int64_t)nbx * 8;
  if (threadIdx.x < 7)
    __hip_atomic_store(&gp[g * 8 + threadIdx.x], tot[threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (threadIdx.x == 0) __hip_atomic_store(&a.cnt[g], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0)
    sh_last = __hip_atomic_fetch_add(&a.cnt[ng], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (unsigned)ng - 1u;
  __syncthreads();
  if (!sh_last) return;
  // the last group: thread t adds groups t, t + 256, ... in turn, then the
  // thread sums in the fixed order above
  double pv[7] = {0, 0, 0, 0, 0, 0, 0};
  if (threadIdx.x < kRedGroup)
    for (int gi = threadIdx.x; gi < ng; gi += kRedGroup) {
#pragma unroll
      for (int k = 0; k < 7; ++k)
        pv[k] += __hip_atomic_load(&gp[gi * 8 + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  if (threadIdx.x < kRedGroup) {
#pragma unroll
    for (int k = 0; k < 7; ++k) red[k][threadIdx.x] = pv[k];
  }
  __syncthreads();
  fixed_sum7(red, red2, min(ng, kRedGroup), tot);
  if (threadIdx.x < 7) {
    const double s = tot[threadIdx.x];
    if (threadIdx.x == 0) { if (a.energy) a.energy[0] = 0.5 * s; }
    else if (a.virial6) a.virial6[threadIdx.x - 1] = 0.5 * s;
  }
  if (threadIdx.x == 0) __hip_atomic_store(&a.cnt[ng], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool P32, bool S>
__device__ __forceinline__ void pairs_body(const RealArgs& a, int bx, int nbx) {
  __shared__ PairQueue queue[kPairWaves];
  __shared__ double sh[kPairWaves][8];
  __shared__ int sh_last;
  if (a.skin > 0.0) return;                     // list mode: k_pairs_list
  if (short_series(a) != S) return;             // the other series' instance
  const int wave = uniform(threadIdx.x / 64), lane = threadIdx.x % 64;
  PairQueue& Q = queue[wave];
  if (lane < (S ? kErfcxTermsS : kErfcxTerms)) Q.poly[lane] = S ? kErfcxPolyS[lane] : kErfcxPoly[lane];
  Q.etab[lane] = kExpTab[lane];
  if (lane < kErfcxTerms32) Q.poly32[lane] = kErfcxPoly32[lane];
  wave_sync();
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  double l[3];
  real_box(a, l);
  const int nx = a.grid[0], ny = a.grid[1], nz = a.grid[2];
  const double rc2 = a.rc * a.rc, sa = sqrt(a.alpha);
  const double two_sa_pi = 2.0 * sa / sqrt(M_PI);
  float rc2_lo, rc2_hi;
  radius_band(a.rc, l, rc2_lo, rc2_hi);
  double u = 0, w[6] = {0, 0, 0, 0, 0, 0};
  float u32 = 0.0f, w32[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};   // FP32 option: one particle's sums
  constexpr int ppw = pair_per_wave(P32);
  for (int k = 0; k < ppw; ++k) {
    const int t = (int)((int64_t)bx * kPairWaves * ppw + wave * ppw + k);   // the wave's i
    if (t >= a.n) break;
    const double4 vi = a.xq[t];
    const int ti = uniform(a.ts[t]);
    const bool lj_i = P32 ? a.ntypes > 0 : lj_row_nonzero(a, a.lj, ti);
    const int c = uniform(a.cs[t]);
    double f[3] = {0.0, 0.0, 0.0};
    int qn = 0;                                   // queued pairs (wave-uniform)
    // the neighbour segments, lane s describing segment s, and their
    // candidate offsets (an exclusive scan): the candidates of the cells that
    // can hold a partner become one flat list, tested 64 at a time with every
    // lane in use
    static_assert(ListSegs<2>::kSeg == kSegments, "the cell path's segments");
    const int total = trimmed_segment_table<2>(a, Q, vi, c, nx, ny, nz, l, a.rc, lane);
    // Alternate between testing candidates into the queue until it is
    // nearly full (or the candidates are exhausted) and evaluating the
    // queue, so the two phases' registers are never live together.
    // candidate batches: the next batch's position load is issued before the
    // current batch is tested (two register sets, alternating)
    int base = 0, sg = 0;                         // next batch; this lane's segment
    int nj = -1, ncode = 13;                      // the loaded batch's j and shift
    float4 nv = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    auto fetch = [&](int b) {                     // candidate b + lane: j, shift, position
      const int cf = b + lane;
      nj = -1;
      if (cf < total) {
        while (Q.seg_off[sg + 1] <= cf) ++sg;
        nj = Q.seg_j0[sg] + (cf - Q.seg_off[sg]);
        ncode = sg;
        nv = a.xf[nj];
      }
    };
    fetch(0);
    bool done = false;
    while (!done) {
      while (qn <= kPairQueue - 64) {
        if (base >= total) { done = true; break; }
        const int j = nj, sj = ncode;
        const float4 v = nv;
        fetch(base + 64);
        bool acc = false;
        int code = 13;
        if (j >= 0 && j != t) {
          code = Q.seg_code[sj];
          // FP32 test; pairs within the FP32 error band of the cutoff are
          // decided in FP64, so the accepted set is the FP64 one
          const float4 io = Q.seg_io[sj];
          const float ex = v.x - io.x, ey = v.y - io.y, ez = v.z - io.z;
          const float r2 = ex * ex + ey * ey + ez * ez;
          if (r2 < rc2_lo) acc = true;
          else if (r2 <= rc2_hi) {
            const double xo = vi.x - l[0] * (double)(code % 3 - 1);
            const double yo = vi.y - l[1] * (double)((code / 3) % 3 - 1);
            const double zo = vi.z - l[2] * (double)(code / 9 - 1);
            const double4 d = a.xq[j];
            const double dx = d.x - xo, dy = d.y - yo, dz = d.z - zo;
            acc = dx * dx + dy * dy + dz * dz < rc2;
          }
        }
        const uint64_t bal = __ballot(acc);
        if (acc) {
          const int pos = qn + __popcll(bal & below);
          Q.j[pos] = j;
          Q.s[pos] = code;
        }
        qn += __popcll(bal);
        base += 64;
      }
      // evaluate: every full batch, and the last partial one when done
      wave_sync();
      const int m = done ? qn : (qn & ~63);
      for (int from = 0; from < m; from += 64) {
        PairLoad cur;
        if (from + lane < m) cur = pair_load(a, Q, from + lane, vi, l);
        if (P32)
          pair_eval32(a, cur, from + lane < m, vi, ti, l, (float)sa, (float)two_sa_pi,
                      (float)a.alpha, Q.poly32, lj_i, f, u32, w32);
        else
          pair_eval<S>(a, cur, from + lane < m, vi, ti, l, sa, two_sa_pi, Q.poly, Q.etab, lj_i, f, u,
                       w);
      }
      wave_sync();
      if (lane < qn - m) { Q.j[lane] = Q.j[m + lane]; Q.s[lane] = Q.s[m + lane]; }
      wave_sync();
      qn -= m;
    }
    if (lane == 0) {
      const int i = a.list[t];
      if (a.accumulate) { a.fx[i] += f[0]; a.fy[i] += f[1]; a.fz[i] += f[2]; }
      else { a.fx[i] = f[0]; a.fy[i] = f[1]; a.fz[i] = f[2]; }
    }
    if (P32) {
      u += (double)u32;
      u32 = 0.0f;
#pragma unroll
      for (int q = 0; q < 6; ++q) { w[q] += (double)w32[q]; w32[q] = 0.0f; }
    }
  }
  static_assert(sizeof(queue) >= kRedScratch * sizeof(double), "reduction scratch");
  block_energy_virial(a, u, w, sh, sh_last, bx, nbx, wave, lane, reinterpret_cast<double*>(queue));
}

__global__ void __launch_bounds__(256) k_bin(RealArgs a) { bin_body(a, blockIdx.x); }
__global__ void __launch_bounds__(1024) k_scan(RealArgs a) { scan_body(a); }
__global__ void __launch_bounds__(256) k_fill(RealArgs a) { fill_body(a, blockIdx.x); }
__global__ void __launch_bounds__(256) k_csort(RealArgs a) { csort_body(a, blockIdx.x); }
// ---------------------------------------------------------------------------
// neighbour lists (skin > 0)

// Displacement since the last build: the block maximum of |r - r_ref|^2 into
// *dmax (FP64 bits order as the values, all being >= 0); the last-arriving
// block decides whether this evaluation rebuilds the lists and resets *dmax.
__device__ __forceinline__ void vcheck_body(const RealArgs& a, int bx, int nbx) {
  __shared__ double sh[4];
  __shared__ int sh_last;
  if (!(a.skin > 0.0)) return;
  // thread t takes the particle at place t of the last build's cell order and
  // also gathers its current position and charge there for the pair kernel
  // (a rebuilding evaluation rewrites them in the new order)
  const bool built = __hip_atomic_load(&a.state[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) > 0;
  const int64_t t = (int64_t)bx * blockDim.x + threadIdx.x;
  double d2 = built ? 0.0 : 1e300;              // no lists yet: build them
  if (built && t < a.n) {
    const int i = a.list[t];
    const double x = a.x[i], y = a.y[i], z = a.z[i];
    a.xc[t] = make_double4(x, y, z, a.q[i]);
    const double dx = x - a.ref[i], dy = y - a.ref[a.n + i], dz = z - a.ref[2 * a.n + i];
    d2 = dx * dx + dy * dy + dz * dz;
    if (!(d2 == d2)) d2 = 1e300;                // non-finite: rebuild (and fail there)
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) d2 = fmax(d2, __shfl_xor(d2, off, 64));
  if (threadIdx.x % 64 == 0) sh[threadIdx.x / 64] = d2;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double m = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    atomicMax(a.dmax, (unsigned long long)__double_as_longlong(m));
  }
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0)
    sh_last = __hip_atomic_fetch_add(a.vcnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == (unsigned)nbx - 1u;
  __syncthreads();
  if (!sh_last || threadIdx.x != 0) return;
  const double dm = __longlong_as_double((long long)__hip_atomic_load(a.dmax, __ATOMIC_RELAXED,
                                                                      __HIP_MEMORY_SCOPE_AGENT));
  double l[3];
  real_box(a, l);
  double dl = 0.0;
  for (int d = 0; d < 3; ++d) dl = fmax(dl, fabs(l[d] - a.ref_box[d]));
  const int rebuild = (!built || 2.0 * sqrt(dm) + 1.7320508075688772 * dl >= a.skin) ? 1 : 0;
  __hip_atomic_store(&a.state[0], rebuild, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(a.dmax, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(a.vcnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Build the lists (a rebuilding evaluation only): a wave per particle t (cell
// order) tests the flat candidate list of its 125 cells against rc + skin and
// appends the cell-ordered indices in candidate order; it records the
// reference positions and, in block 0, the reference cell.
__device__ __forceinline__ void build_body(const RealArgs& a, int bx) {
  __shared__ ListSegs<kListReach> queue[kPairWaves];
  if (!(a.skin > 0.0) || skip_cells(a)) return;
  const int wave = uniform(threadIdx.x / 64), lane = threadIdx.x % 64;
  ListSegs<kListReach>& Q = queue[wave];
  const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  double l[3];
  real_box(a, l);
  if (bx == 0 && threadIdx.x < 3) a.ref_box[threadIdx.x] = l[threadIdx.x];
  const int nx = a.grid[0], ny = a.grid[1], nz = a.grid[2];
  const double rs = search_radius(a), rs2 = rs * rs;
  float lo, hi;
  radius_band(rs, l, lo, hi);
  {
    const int t = (int)((int64_t)bx * kPairWaves + wave);
    if (t >= a.n) goto done;
    const double4 vi = a.xq[t];
    const int c = uniform(a.cs[t]);
    const int total = trimmed_segment_table<kListReach>(a, Q, vi, c, nx, ny, nz, l, rs, lane);
    int cnt = 0, sg = 0;
    int32_t* out = a.nbr + (int64_t)t * a.kcap;
    // candidate b + lane: its index, segment and FP32 position (with the
    // type), requested one batch ahead of its test
    int nj = -1, nsg = 0;
    float4 nv = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    auto fetch = [&](int b) {
      const int cf = b + lane;
      nj = -1;
      if (cf < total) {
        while (Q.seg_off[sg + 1] <= cf) ++sg;
        nj = Q.seg_j0[sg] + (cf - Q.seg_off[sg]);
        nsg = sg;
        nv = a.xf[nj];
      }
    };
    fetch(0);
    for (int base = 0; base < total; base += 64) {
      const int j = nj, sj = nsg;
      const float4 v = nv;
      fetch(base + 64);
      bool acc = false;
      if (j >= 0 && j != t) {
        const float4 io = Q.seg_io[sj];
        const float ex = v.x - io.x, ey = v.y - io.y, ez = v.z - io.z;
        const float r2 = ex * ex + ey * ey + ez * ez;
        if (r2 < lo) acc = true;
        else if (r2 <= hi) {
          const int code = Q.seg_code[sj];
          const double4 d = a.xq[j];
          const double dx = d.x - (vi.x - l[0] * (double)(code % 3 - 1));
          const double dy = d.y - (vi.y - l[1] * (double)((code / 3) % 3 - 1));
          const double dz = d.z - (vi.z - l[2] * (double)(code / 9 - 1));
          acc = dx * dx + dy * dy + dz * dz < rs2;
        }
      }
      const uint64_t bal = __ballot(acc);
      if (acc) {
        const int pos = cnt + __popcll(bal & below);
        if (pos < a.kcap)
          out[pos] = a.ntypes > 0 ? (j | (__float_as_int(v.w) << kListTypeShift)) : j;
      }
      cnt += __popcll(bal);
    }
    if (lane == 0) {
      a.ncount[t] = min(cnt, a.kcap);
      if (cnt > a.kcap) atomicOr(a.err, 8);
      const int i = a.list[t];
      const double x = a.x[i], y = a.y[i], z = a.z[i];
      a.ref[i] = x; a.ref[a.n + i] = y; a.ref[2 * a.n + i] = z;
      a.xc[t] = make_double4(x, y, z, a.q[i]);
    }
    wave_sync();
  }
done:
  if (bx == 0 && threadIdx.x == 0)          // the build count
    __hip_atomic_store(&a.state[1], a.state[1] + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}


// Entries [c0, c0 + kListChunk) of particle t's list copied to LDS without
// passing through registers (global_load_lds: lane i's 16 bytes land at
// L + 16 i); entries past the row's slots are clamped to its last slots.
// Every slot of a list holds a valid index.  The caller waits (vmcnt) before
// reading L.
typedef __attribute__((address_space(3))) void lds_void_t;
__device__ __forceinline__ void list_to_lds(const RealArgs& a, int t, int c0, int32_t* L, int lane) {
  const int32_t* lst = a.nbr + (int64_t)t * a.kcap;
  const int nq = min(kListChunk, a.kcap - c0 + 255) / 256;     // 256 entries per instruction
#pragma unroll
  for (int q = 0; q < kListChunk / 256; ++q)
    if (q < nq) {
      const int e = min(c0 + q * 256 + 4 * lane, a.kcap - 4);
      __builtin_amdgcn_global_load_lds((const void*)(lst + e), (lds_void_t*)(L + q * 256), 16, 0, 0);
    }
}

// Pairs from the lists: a wave per particle t; its list entries 64 at a
// time, each lane's minimum-image separation tested against rc and the pair
// evaluated in place (no queue: the skin keeps the accepted share high).  The
// next batch's positions and the index batch after it are loaded while the
// current batch is evaluated; force sums are kept per lane and summed over
// the wave once per particle.  LJL: the Lennard-Jones table (at most
// kLjLds types) is read from LDS, which keeps its loads off the vector-memory
// counter the prefetched batch waits on.
template <bool P32, bool LJL, bool S>
__device__ __forceinline__ void pairs_list_body(const RealArgs& a, int bx, int nbx) {
  __shared__ int32_t lidx[kPairWaves][2][kListChunk];
  __shared__ double poly[kErfcxTerms];
  __shared__ double etab[64];
  __shared__ float poly32[kErfcxTerms32];
  __shared__ double ljs[LJL ? 2 * kLjLds * kLjLds : 1];
  __shared__ double sh[kPairWaves][8];
  __shared__ int sh_last;
  if (!(a.skin > 0.0)) return;
  if (short_series(a) != S) return;             // the other series' instance
  const int wave = uniform(threadIdx.x / 64), lane = threadIdx.x % 64;
  if (threadIdx.x < (S ? kErfcxTermsS : kErfcxTerms))
    poly[threadIdx.x] = S ? kErfcxPolyS[threadIdx.x] : kErfcxPoly[threadIdx.x];
  if (threadIdx.x < 64) etab[threadIdx.x] = kExpTab[threadIdx.x];
  if (threadIdx.x < kErfcxTerms32) poly32[threadIdx.x] = kErfcxPoly32[threadIdx.x];
  if (LJL)
    for (int q = threadIdx.x; q < 2 * a.ntypes * a.ntypes; q += blockDim.x) ljs[q] = a.lj[q];
  __syncthreads();
  double l[3];
  real_box(a, l);
  const double il[3] = {1.0 / l[0], 1.0 / l[1], 1.0 / l[2]};
  const double rc2 = a.rc * a.rc, sa = sqrt(a.alpha);
  const double two_sa_pi = 2.0 * sa / sqrt(M_PI);
  double u = 0, w[6] = {0, 0, 0, 0, 0, 0};
  float u32 = 0.0f, w32[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  constexpr int ppw = list_per_wave(P32);
  const int t0 = (int)((int64_t)bx * kPairWaves * ppw + wave * ppw);
  const int nt = uniform(max(0, min(ppw, (int)(a.n - t0))));   // the wave's particles
  // the header of the wave's next particle and the first chunk of its list
  // (copied straight to LDS) are requested while the current one is worked
  double4 vi_n = make_double4(0.0, 0.0, 0.0, 0.0);
  int ti_n = 0, tot_n = 0;
  if (nt > 0) {
    vi_n = a.xc[t0]; ti_n = a.ts[t0]; tot_n = a.ncount[t0];
    list_to_lds(a, t0, 0, lidx[wave][0], lane);
  }
  for (int k = 0; k < nt; ++k) {
    const int t = t0 + k, cur = k & 1;
    __builtin_amdgcn_s_waitcnt(0);              // header and list chunk of t in place
    wave_sync();
    const double4 vi = vi_n;
    const int ti = uniform(ti_n);
    const bool lj_i = P32 ? a.ntypes > 0 : lj_row_nonzero(a, LJL ? ljs : a.lj, ti);
    const int total = uniform(tot_n);
    if (k + 1 < nt) {
      vi_n = a.xc[t + 1]; ti_n = a.ts[t + 1]; tot_n = a.ncount[t + 1];
      list_to_lds(a, t + 1, 0, lidx[wave][cur ^ 1], lane);
    }
    int32_t* L = lidx[wave][cur];
    double fx = 0.0, fy = 0.0, fz = 0.0;
    float fx32 = 0.0f, fy32 = 0.0f, fz32 = 0.0f;
    for (int c0 = 0; c0 < total; c0 += kListChunk) {
      const int cnt = min(total - c0, kListChunk);
      if (c0 > 0) {                             // a list longer than one chunk
        wave_sync();
        list_to_lds(a, t, c0, L, lane);
        __builtin_amdgcn_s_waitcnt(0);
      }
      wave_sync();
      const int jmax = (int)a.n - 1;
      int jn = L[lane];
      double4 vn = a.xc[min(jn & kListIdxMask, jmax)];
      for (int base = 0; base < cnt; base += 64) {
        const int jc = jn;
        const double4 vc = vn;
        jn = L[min(base + 64 + lane, kListChunk - 1)];
        vn = a.xc[min(jn & kListIdxMask, jmax)];
        double ex = vc.x - vi.x, ey = vc.y - vi.y, ez = vc.z - vi.z;
        ex -= l[0] * rint(ex * il[0]);
        ey -= l[1] * rint(ey * il[1]);
        ez -= l[2] * rint(ez * il[2]);
        const bool valid = base + lane < cnt && ex * ex + ey * ey + ez * ez < rc2;
        PairLoad p;
        p.ex = ex; p.ey = ey; p.ez = ez;
        p.qj = vc.w;
        p.tj = jc >> kListTypeShift;
        if (P32) {
          float gx, gy, gz;
          pair_core32(a, p, valid, vi, ti, (float)sa, (float)two_sa_pi, (float)a.alpha, poly32,
                      LJL ? ljs : a.lj, lj_i, gx, gy, gz, u32, w32);
          fx32 += gx; fy32 += gy; fz32 += gz;
        } else {
          double gx, gy, gz;
          pair_core<S>(a, p, valid, vi, ti, sa, two_sa_pi, poly, etab, LJL ? ljs : a.lj, lj_i, gx, gy,
                       gz, u, w);
          fx += gx; fy += gy; fz += gz;
        }
      }
      wave_sync();
    }
    if (P32) { fx = (double)fx32; fy = (double)fy32; fz = (double)fz32; }
    fx = wsum(fx); fy = wsum(fy); fz = wsum(fz);
    if (lane == 0) {
      const int i = a.list[t];
      if (a.accumulate) { a.fx[i] += fx; a.fy[i] += fy; a.fz[i] += fz; }
      else { a.fx[i] = fx; a.fy[i] = fy; a.fz[i] = fz; }
    }
    if (P32) {
      u += (double)u32;
      u32 = 0.0f;
#pragma unroll
      for (int q = 0; q < 6; ++q) { w[q] += (double)w32[q]; w32[q] = 0.0f; }
    }
  }
  static_assert(sizeof(lidx) >= kRedScratch * sizeof(double), "reduction scratch");
  block_energy_virial(a, u, w, sh, sh_last, bx, nbx, wave, lane, reinterpret_cast<double*>(&lidx[0][0]));
}

// four waves per SIMD: the register budget that keeps the pair evaluation
// from spilling beyond a few registers
template <bool P32, bool S>
__global__ void __launch_bounds__(kPairWaves * 64) __attribute__((amdgpu_waves_per_eu(4)))
k_pairs(RealArgs a) {
  pairs_body<P32, S>(a, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(256) k_vcheck(RealArgs a) { vcheck_body(a, blockIdx.x, gridDim.x); }
__global__ void __launch_bounds__(kPairWaves * 64) k_build(RealArgs a) { build_body(a, blockIdx.x); }
template <bool P32, bool LJL, bool S>
__global__ void __launch_bounds__(kPairWaves * 64) __attribute__((amdgpu_waves_per_eu(3)))
k_pairs_list(RealArgs a) {
  pairs_list_body<P32, LJL, S>(a, blockIdx.x, gridDim.x);
}

static_assert(kErfcxRange == kErfcxShortX, "the range of the bounded erfcx series");

template <bool LJL, bool S>
void launch_pairs_list(const RealArgs& a, hipStream_t s) {
  const dim3 g((unsigned)list_blocks(a.n, a.prec32 != 0)), b(kPairWaves * 64);
  if (a.prec32) hipLaunchKernelGGL((k_pairs_list<true, LJL, S>), g, b, 0, s, a);
  else hipLaunchKernelGGL((k_pairs_list<false, LJL, S>), g, b, 0, s, a);
}

hipError_t launch_real_list(const RealArgs& a, int ncell_cap, hipStream_t s) {
  const unsigned vb = (unsigned)((a.n + 255) / 256), pb = (unsigned)bin_blocks(a.n);
  const unsigned qb = (unsigned)build_blocks(a.n);
  hipLaunchKernelGGL(k_vcheck, dim3(vb), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_bin, dim3(pb), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, a);
  hipLaunchKernelGGL(k_fill, dim3(pb), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_csort, dim3(ncell_cap), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_build, dim3(qb), dim3(kPairWaves * 64), 0, s, a);
  const bool sr = short_series(a);
  if (a.ntypes <= kLjLds) {
    if (sr) launch_pairs_list<true, true>(a, s); else launch_pairs_list<true, false>(a, s);
  } else {
    if (sr) launch_pairs_list<false, true>(a, s); else launch_pairs_list<false, false>(a, s);
  }
  return hipGetLastError();
}

hipError_t launch_real(const RealArgs& a, int ncell_cap, hipStream_t s) {
  if (a.skin > 0.0) return launch_real_list(a, ncell_cap, s);
  const unsigned pb = (unsigned)bin_blocks(a.n);
  hipLaunchKernelGGL(k_bin, dim3(pb), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, a);
  hipLaunchKernelGGL(k_fill, dim3(pb), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_csort, dim3(ncell_cap), dim3(256), 0, s, a);
  const dim3 g((unsigned)pair_blocks(a.n, a.prec32 != 0)), b(kPairWaves * 64);
  const bool sr = short_series(a);
  if (a.prec32) {
    if (sr) hipLaunchKernelGGL((k_pairs<true, true>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_pairs<true, false>), g, b, 0, s, a);
  } else {
    if (sr) hipLaunchKernelGGL((k_pairs<false, true>), g, b, 0, s, a);
    else hipLaunchKernelGGL((k_pairs<false, false>), g, b, 0, s, a);
  }
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
template <bool P32, bool S>
__global__ void __launch_bounds__(kPairWaves * 64) __attribute__((amdgpu_waves_per_eu(4)))
k_pairs_m(const RealArgs* tab, const int* bstart, int nsys) {
  REAL_MULTI_PROLOGUE
  pairs_body<P32, S>(sa, lb, nb);
}

__global__ void __launch_bounds__(256) k_vcheck_m(const RealArgs* tab, const int* bstart, int nsys) {
  REAL_MULTI_PROLOGUE
  vcheck_body(sa, lb, nb);
}
__global__ void __launch_bounds__(kPairWaves * 64) k_build_m(const RealArgs* tab, const int* bstart,
                                                             int nsys) {
  REAL_MULTI_PROLOGUE
  (void)nb;
  build_body(sa, lb);
}
template <bool P32, bool LJL, bool S>
__global__ void __launch_bounds__(kPairWaves * 64) __attribute__((amdgpu_waves_per_eu(3)))
k_pairs_list_m(const RealArgs* tab, const int* bstart, int nsys) {
  REAL_MULTI_PROLOGUE
  pairs_list_body<P32, LJL, S>(sa, lb, nb);
}

template <bool LJL, bool S>
void launch_pairs_list_m(int prec32, dim3 g, hipStream_t s, const RealArgs* d_tab,
                         const int* d_bstart_q, int nsys) {
  const dim3 b(kPairWaves * 64);
  if (prec32) hipLaunchKernelGGL((k_pairs_list_m<true, LJL, S>), g, b, 0, s, d_tab, d_bstart_q, nsys);
  else hipLaunchKernelGGL((k_pairs_list_m<false, LJL, S>), g, b, 0, s, d_tab, d_bstart_q, nsys);
}

template <bool S>
void launch_pairs_m(int prec32, dim3 g, hipStream_t s, const RealArgs* d_tab, const int* d_bstart_q,
                    int nsys) {
  const dim3 b(kPairWaves * 64);
  if (prec32) hipLaunchKernelGGL((k_pairs_m<true, S>), g, b, 0, s, d_tab, d_bstart_q, nsys);
  else hipLaunchKernelGGL((k_pairs_m<false, S>), g, b, 0, s, d_tab, d_bstart_q, nsys);
}

// bstart_p: binning blocks (bin_blocks(n) each); bstart_c: cell blocks;
// bstart_q: pair blocks (pair_blocks(n, prec32) each for a cell-list
// system, list_blocks(n, prec32) for a neighbour-list one); bstart_b:
// list-build blocks (build_blocks(n) each); series: bit 0 set if some
// system takes the bounded-range erfcx series, bit 1 if some takes the full
// one (each instance's blocks of the other kind's systems return at once, so
// a system's results do not depend on the others in the launch)
hipError_t launch_real_multi(const RealArgs* d_tab, const int* d_bstart_p, int total_p,
                             const int* d_bstart_c, int total_c, const int* d_bstart_q, int total_q,
                             const int* d_bstart_b, int total_b,
                             const int* d_bstart_v, int total_v, int any_list, int any_cells,
                             int max_types, int nsys, int prec32, int series, hipStream_t s) {
  if (any_list) hipLaunchKernelGGL(k_vcheck_m, dim3(total_v), dim3(256), 0, s, d_tab, d_bstart_v, nsys);
  hipLaunchKernelGGL(k_bin_m, dim3(total_p), dim3(256), 0, s, d_tab, d_bstart_p, nsys);
  hipLaunchKernelGGL(k_scan_m, dim3(nsys), dim3(1024), 0, s, d_tab, nsys);
  hipLaunchKernelGGL(k_fill_m, dim3(total_p), dim3(256), 0, s, d_tab, d_bstart_p, nsys);
  hipLaunchKernelGGL(k_csort_m, dim3(total_c), dim3(256), 0, s, d_tab, d_bstart_c, nsys);
  if (any_list) {
    hipLaunchKernelGGL(k_build_m, dim3(total_b), dim3(kPairWaves * 64), 0, s, d_tab, d_bstart_b, nsys);
    const dim3 g((unsigned)total_q);
    if (max_types <= kLjLds) {
      if (series & 1) launch_pairs_list_m<true, true>(prec32, g, s, d_tab, d_bstart_q, nsys);
      if (series & 2) launch_pairs_list_m<true, false>(prec32, g, s, d_tab, d_bstart_q, nsys);
    } else {
      if (series & 1) launch_pairs_list_m<false, true>(prec32, g, s, d_tab, d_bstart_q, nsys);
      if (series & 2) launch_pairs_list_m<false, false>(prec32, g, s, d_tab, d_bstart_q, nsys);
    }
  }
  if (any_cells) {
    if (series & 1) launch_pairs_m<true>(prec32, dim3(total_q), s, d_tab, d_bstart_q, nsys);
    if (series & 2) launch_pairs_m<false>(prec32, dim3(total_q), s, d_tab, d_bstart_q, nsys);
  }
  return hipGetLastError();
}

}  // namespace rbe
