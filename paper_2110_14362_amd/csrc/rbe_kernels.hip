// HIP kernels of the random batch Ewald Fourier-space step (gfx950).
//
// A step is two launches:
//   k_sfac   every block rebuilds the per-axis sampler tables and the cell
//            values in LDS (section 4.2 eq. (S), (psf); appendix C: the three
//            axes of a rectangular cell are independent), draws the
//            frequencies of its slice of the batch (eq. (probexpression)),
//            and sums rho(k) = sum_j q_j exp(i k.r_j) (eq. (U1fourier)) over
//            its particle chunk, one lane per frequency with the particles
//            broadcast from LDS.  Chunk partials are then combined in a fixed
//            order by the last-arriving blocks (two levels), which also form
//            the force coefficients of eq. (appforce) and the virial tensor
//            and energy of eq. (apppress) / (pressuretensorflexible).
//   k_force  one lane per particle, the batch split across the waves of a
//            block, frequency constants uniform across the wave (eq. (appforce)).
// Every sum has a fixed order, so results are bitwise reproducible and do not
// depend on which block arrives last or on what else runs on the GPU.
#include <hip/hip_ext.h>
#include "rbe_internal.h"
#include <math.h>
#include <type_traits>

namespace rbe {

// ---------------------------------------------------------------------------
// helpers

// Block barrier that orders LDS only: waits for this wave's LDS operations,
// not for its global loads and stores, which stay in flight across it (a
// __syncthreads waits for those too).  Global data exchanged between waves
// of a block goes through LDS after its loads returned, or is ordered by
// the explicit waits of arrive_last and publish.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ double wave_incl_scan(double v, int lane) {
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const double o = __shfl_up(v, off, kWave);
    if (lane >= off) v += o;
  }
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): multipliers and Weyl key
// increments of the 4x64 variant; ten rounds, key bumped between rounds.
__device__ __forceinline__ void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
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

constexpr uint64_t kTagKSample = 0x6B73616Dull;  // 'ksam': stream of the batch draws

// ceil(sqrt(53 ln2 alpha) l / pi): weights exp(-pi^2 m^2/(alpha l^2)) >= 2^-53
// Without branches, so that the three axes' chains (square root, division,
// ceiling) overlap: a non-finite or non-positive cell gives 1, an oversized
// one mcap, and both set err.
__device__ __forceinline__ int table_halfwidth(double alpha, double tail_ln, double l, int mcap,
                                               int& err) {
  const double mcd = ceil(sqrt(tail_ln * alpha * l * l) / M_PI);
  err |= (mcd >= 1.0 && mcd <= (double)mcap) ? 0 : 1;
  return (int)fmin(fmax(mcd, 1.0), (double)mcap);
}

__device__ __forceinline__ void table_offsets(const int mc[3], int off[3]) {
  off[0] = 0;
  off[1] = 4 * mc[0] + 1;
  off[2] = off[1] + 4 * mc[1] + 1;
}

constexpr int kTableTasks = 6;     // (axis, table) pairs of build_tables, one wave each

// Per-axis running sums of w_a(m) = exp(-pi^2 m^2 / (alpha l_a^2)) built by the
// whole block into `tab` (LDS or global).  Axis a occupies [off[a], off[a] +
// 4 mc_a + 1): the running sum over m = -mc..mc, then the running sum over the
// same m without m = 0.  One wave per (axis, table); a lane owns a contiguous
// segment, the lane totals are scanned across the wave.  Writes the cell
// values to *out (LDS).  Must be reached by every thread of the block.
// Without the closing barrier the cell values other than the sides, V and
// the half-widths (written before the tables' barrier when the block has a
// wave without a table task) are not yet visible to the other threads.
// The weights of the nonzero event split by its first nonzero axis, from the
// per-axis totals T = H - 1 of the m != 0 tables (one expression for every
// caller, so that all of them form the same values).
__device__ __forceinline__ void case_weights(const double* T, double cw[3]) {
  const double Hy = 1.0 + T[1], Hz = 1.0 + T[2];
  cw[0] = T[0] * Hy * Hz;
  cw[1] = T[1] * Hz;
  cw[2] = T[2];
}

__device__ void build_tables(const double l[3], const TriCell* tcp, double alpha, double tail_ln,
                             const int mcap[3], double* tab, BoxState* out, double* sh_T, int nt,
                             bool closing_barrier) {
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int nw = nt / kWave;
  int err = 0, mc[3], off[3];
  const bool tri = tcp != nullptr && tcp->on;
  const TriCell& tc = *tcp;          // read only when tri
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (tri) {
      // triclinic: the envelope's axis law exp(-d m^2), |m| <= ceil(sqrt(53 ln2 / d))
      const double mcd = ceil(sqrt(tail_ln / tc.d[a]));
      if (mcd >= 1.0 && mcd <= (double)mcap[a]) mc[a] = (int)mcd;
      else { err |= 1; mc[a] = mcd >= 1.0 ? mcap[a] : 1; }
    } else {
      mc[a] = table_halfwidth(alpha, tail_ln, l[a], mcap[a], err);
    }
  }
  table_offsets(mc, off);
  const double pi2 = M_PI * M_PI;
  for (int task = wave; task < kTableTasks; task += nw) {
    const int a = task >> 1, nz = task & 1;
    const int n = nz ? 2 * mc[a] : 2 * mc[a] + 1;
    double* t = tab + off[a] + (nz ? 2 * mc[a] + 1 : 0);
    const double c = -pi2 / (alpha * l[a] * l[a]);   // w(m) = exp(c m^2)
    const int seg = (n + kWave - 1) / kWave;
    const int b0 = min(n, lane * seg), b1 = min(n, b0 + seg);
    double loc = 0.0;
    for (int i = b0; i < b1; ++i) {
      const int m = nz ? (i < mc[a] ? i - mc[a] : i - mc[a] + 1) : i - mc[a];
      const double w = tri ? exp(-(tc.d[a] * ((double)m * (double)m)))
                           : exp(c * ((double)m * (double)m));
      t[i] = w;
      loc += w;
    }
    const double incl = wave_incl_scan(loc, lane);
    const double excl = incl - loc;
    double run = 0.0;
    for (int i = b0; i < b1; ++i) {
      run += t[i];
      t[i] = excl + run;
    }
    if (nz && lane == kWave - 1) sh_T[a] = incl;
  }
  // the cell values that do not need the tables (sides, their reciprocals,
  // half-widths, V): written before the barrier by the first lane of a wave
  // without a table task when the block has one, else after it by thread 0
  const int early = nw > kTableTasks ? kTableTasks * kWave : 0;
  auto sides = [&](BoxState& b) {
    for (int a = 0; a < 3; ++a) { b.l[a] = l[a]; b.inv_l[a] = 1.0 / l[a]; b.mcut[a] = mc[a]; }
    b.V = l[0] * l[1] * l[2];
  };
  if (early > 0 && (int)threadIdx.x == early) sides(*out);
  lds_barrier();
  if (threadIdx.x == 0) {
    const double Tx = sh_T[0], Ty = sh_T[1], Tz = sh_T[2];
    const double Hx = 1.0 + Tx, Hy = 1.0 + Ty, Hz = 1.0 + Tz;
    BoxState& b = *out;
    if (early == 0) sides(b);
    b.H[0] = Hx; b.H[1] = Hy; b.H[2] = Hz;
    case_weights(sh_T, b.case_w);
    b.S = b.case_w[0] + b.case_w[1] + b.case_w[2];
    b.err = err;
    if (tri) {
      b.tri = tc;
      b.S = tc.S;                // the estimator's normaliser; the tables are the envelope's
    } else {
      b.tri.on = 0;
    }
  }
  if (closing_barrier) lds_barrier();
}

__device__ __forceinline__ int first_greater(const double* c, int n, double t) {
  // smallest i with c[i] > t, or n-1 if none
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (c[mid] > t) hi = mid; else lo = mid + 1;
  }
  return lo;
}

// Draw frequency l of a step.  The nonzero event is split by its first
// nonzero axis (weights case_w, sum S); the pivot axis is drawn from its
// m != 0 table, later axes from their full tables, earlier axes are 0.
// Uniforms: the four Philox outputs of counter (step, l, 'ksam', 0), top 53
// bits.  A table draw is the first index whose running sum exceeds u times
// the table total; the three axes' binary searches run in lockstep.
// propose_from draws from the four Philox outputs c0..c3 given;
// propose_frequency forms them for attempt `attempt` first.
// cw: the case weights, if not b's
__device__ __forceinline__ void propose_from(const BoxState& b, const double* tab, uint64_t c0,
                                             uint64_t c1, uint64_t c2, uint64_t c3, int m[3],
                                             const double* cw = nullptr) {
  const double* w = cw ? cw : b.case_w;
  int off[3];
  table_offsets(b.mcut, off);
  const double u[4] = {(double)(c0 >> 11) * 0x1.0p-53, (double)(c1 >> 11) * 0x1.0p-53,
                       (double)(c2 >> 11) * 0x1.0p-53, (double)(c3 >> 11) * 0x1.0p-53};
  // both tables' totals of every axis are read before the pivot is known
  // (their addresses depend only on the half-widths): one LDS round trip
  double tot_full[3], tot_nz[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    tot_full[a] = tab[off[a] + 2 * b.mcut[a]];
    tot_nz[a] = tab[off[a] + 4 * b.mcut[a]];
  }
  const double t = u[0] * (w[0] + w[1] + w[2]);
  const int pivot = (t < w[0]) ? 0 : ((t < w[0] + w[1]) ? 1 : 2);
  const double* base[3];
  int lo[3], hi[3];
  double tgt[3];
  int nmax = 1;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int mc = b.mcut[a];
    const bool nz = (a == pivot);
    const int n = nz ? 2 * mc : 2 * mc + 1;
    base[a] = tab + off[a] + (nz ? 2 * mc + 1 : 0);
    lo[a] = 0;
    hi[a] = (a < pivot) ? 0 : n - 1;
    tgt[a] = u[a + 1] * (nz ? tot_nz[a] : tot_full[a]);
    nmax = max(nmax, n);
  }
  // each step reads the three axes' midpoints together (one LDS round trip
  // per step, not three) and updates them by selection; an axis whose range
  // has closed reads its own entry and keeps it
  const int iters = 32 - __clz(nmax);
  for (int it = 0; it < iters; ++it) {
    int mid[3];
    double v[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      mid[a] = (lo[a] + hi[a]) >> 1;
      v[a] = base[a][mid[a]];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const bool open = lo[a] < hi[a], gt = v[a] > tgt[a];
      hi[a] = open && gt ? mid[a] : hi[a];
      lo[a] = open && !gt ? mid[a] + 1 : lo[a];
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int mc = b.mcut[a];
    if (a < pivot) m[a] = 0;
    else if (a == pivot) m[a] = lo[a] < mc ? lo[a] - mc : lo[a] - mc + 1;
    else m[a] = lo[a] - mc;
  }
}

__device__ __forceinline__ void propose_frequency(const BoxState& b, const double* tab, uint64_t seed,
                                                  uint64_t sysid, uint64_t step, int l,
                                                  uint64_t attempt, int m[3],
                                                  const double* cw = nullptr) {
  uint64_t c[4] = {step, (uint64_t)l, kTagKSample, attempt};
  philox4x64_10(c, seed, sysid);
  propose_from(b, tab, c[0], c[1], c[2], c[3], m, cw);
}

constexpr uint64_t kTagKAccept = 0x6B616363ull;  // 'kacc': acceptance uniforms, triclinic draws
constexpr int kMaxAttempts = 256;

// Frequency l of a step.  Rectangular cell: the exact draw (attempt 0).
// Triclinic cell (appendix C): attempt a proposes from the separable
// envelope exp(-sum d_j m_j^2) with the uniforms of counter (step, l, 'ksam',
// a) and accepts with probability exp(-(Q(m) - sum d_j m_j^2)), the uniform
// from counter (step, l, 'kacc', a); the accepted m has law exp(-Q(m))/S.
// After kMaxAttempts rejections the last proposal is kept.  TRI selects the
// triclinic form at compile time (the cell values say which applies), so
// that kernels for rectangular cells carry none of the rejection loop's
// registers.
//
// pre (nullable): the Philox outputs of attempt 0, pre[j * pre_stride] for
// output j, formed ahead by slice_uniforms; identical to forming them here.
template <bool TRI>
__device__ __forceinline__ void draw_frequency(const BoxState& b, const double* tab, uint64_t seed,
                                               uint64_t sysid, uint64_t step, int l, int m[3],
                                               const uint64_t* pre = nullptr, int pre_stride = 0,
                                               const double* cw = nullptr) {
  for (int att = 0; att < kMaxAttempts; ++att) {
    if (att == 0 && pre)        // the same Philox outputs, formed ahead
      propose_from(b, tab, pre[0], pre[pre_stride], pre[2 * pre_stride], pre[3 * pre_stride], m,
                   cw);
    else
      propose_frequency(b, tab, seed, sysid, step, l, (uint64_t)att, m, cw);
    if (!TRI) return;
    const double x = m[0], y = m[1], z = m[2];
    const double* A = b.tri.A;
    const double Q = A[0] * x * x + A[1] * y * y + A[2] * z * z +
                     2.0 * (A[3] * x * y + A[4] * x * z + A[5] * y * z);
    const double excess = Q - (b.tri.d[0] * x * x + b.tri.d[1] * y * y + b.tri.d[2] * z * z);
    uint64_t c[4] = {step, (uint64_t)l, kTagKAccept, (uint64_t)att};
    philox4x64_10(c, seed, sysid);
    const double ua = (double)(c[0] >> 11) * 0x1.0p-53;
    if (ua < exp(-excess)) return;
  }
}

// The sides of a launch's cell (the arguments, device memory, or the
// committed cell values).
__device__ __forceinline__ void box_source(const StepArgs& a, double l[3]) {
  if (a.box_src == BOX_ARGS) {
    l[0] = a.box_arg[0]; l[1] = a.box_arg[1]; l[2] = a.box_arg[2];
  } else if (a.box_src == BOX_PTR) {
    l[0] = a.box_ptr[0]; l[1] = a.box_ptr[1]; l[2] = a.box_ptr[2];
  } else {
    l[0] = a.bs->l[0]; l[1] = a.bs->l[1]; l[2] = a.bs->l[2];
  }
}

// The launch's triclinic cell data copied to LDS (s), or NULL for a
// rectangular cell.  (A copy, not a pointer into the kernel arguments: a
// pointer that may address either the arguments or global memory makes the
// compiler copy all the arguments to scratch memory.)  Called once at the
// top of a kernel, so that no argument value stays live across the kernel.
// Reached by every thread; one barrier in triclinic contexts.
__device__ __forceinline__ const TriCell* stage_tri(const StepArgs& a, TriCell* s) {
  if (!a.tri_mode) return nullptr;           // a rectangular-cell context: nothing to stage
  if (threadIdx.x == 0) {
    if (a.box_src == BOX_ARGS) *s = a.tri_arg;
    else if (a.box_src == BOX_COMMITTED) *s = a.bs->tri;
    else s->on = 0;
  }
  lds_barrier();
  return s->on ? s : nullptr;
}

// Words of the cell values.  They are copied word by word by the block's
// first threads: a one-thread copy of the whole struct would hold all of it
// in registers at once.
constexpr int kBoxWords = sizeof(BoxState) / 8;
static_assert(sizeof(BoxState) % 8 == 0, "cell values copied as 8-byte words");

// The cell values of this launch become the committed ones (keeping any
// error flag already set), one 8-byte word per thread of the block's first
// kBoxWords threads.
__device__ __forceinline__ void commit_cell(const BoxState& b, BoxState* dst, int tid) {
  constexpr int ew = __builtin_offsetof(BoxState, err) / 8;
  static_assert(__builtin_offsetof(BoxState, err) == 8 * ew + 4, "err: high half of its word");
  if (tid >= kBoxWords) return;
  if (tid != ew) {
    reinterpret_cast<uint64_t*>(dst)[tid] = reinterpret_cast<const uint64_t*>(&b)[tid];
  } else {
    // the word's low half, then the error flags OR-ed in (no read of dst, so
    // the block does not wait for its loads in flight)
    reinterpret_cast<int32_t*>(dst)[2 * ew] = reinterpret_cast<const int32_t*>(&b)[2 * ew];
    if (b.err) __hip_atomic_fetch_or(&dst->err, b.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// A system's kernel arguments into LDS, 8 bytes per thread (a one-thread
// copy of the struct would hold all of it in registers).
__device__ __forceinline__ void copy_args(StepArgs* dst, const StepArgs* src) {
  static_assert(sizeof(StepArgs) % 8 == 0, "arguments copied as 8-byte words");
  constexpr int words = sizeof(StepArgs) / 8;
  for (int w = threadIdx.x; w < words; w += blockDim.x)
    reinterpret_cast<uint64_t*>(dst)[w] = reinterpret_cast<const uint64_t*>(src)[w];
}

// Cell values from global memory into LDS (dst), and from LDS to global
// memory, one 8-byte word per thread of the block's first kBoxWords threads;
// LDS results are read after a barrier.
__device__ __forceinline__ void load_box(BoxState& dst, const BoxState* src, int tid) {
  if (tid < kBoxWords)
    reinterpret_cast<uint64_t*>(&dst)[tid] = reinterpret_cast<const uint64_t*>(src)[tid];
}
__device__ __forceinline__ void copy_box(BoxState* dst, const BoxState& src, int tid) {
  if (tid < kBoxWords)
    reinterpret_cast<uint64_t*>(dst)[tid] = reinterpret_cast<const uint64_t*>(&src)[tid];
}

// Whether a batch drawn ahead for cell pb is the batch of this launch's cell.
__device__ __forceinline__ bool same_cell(const StepArgs& a, const BoxState& pb) {
  double l[3];
  box_source(a, l);
  int on = 0;
  double t0 = 0.0, t1 = 0.0, t2 = 0.0;
  if (a.box_src == BOX_ARGS) {
    on = a.tri_arg.on; t0 = a.tri_arg.tilt[0]; t1 = a.tri_arg.tilt[1]; t2 = a.tri_arg.tilt[2];
  } else if (a.box_src == BOX_COMMITTED) {
    on = a.bs->tri.on; t0 = a.bs->tri.tilt[0]; t1 = a.bs->tri.tilt[1]; t2 = a.bs->tri.tilt[2];
  }
  return l[0] == pb.l[0] && l[1] == pb.l[1] && l[2] == pb.l[2] && on == pb.tri.on &&
         (!on || (t0 == pb.tri.tilt[0] && t1 == pb.tri.tilt[1] && t2 == pb.tri.tilt[2]));
}

// Reduced coordinates s = h^-1 r wrapped into [0, 1): x/l per axis for a
// rectangular cell, back substitution through the upper-triangular h^-1 for
// a triclinic one (appendix C: k.r = 2 pi m.s).
__device__ __forceinline__ void reduce_pos(const BoxState& b, double x, double y, double z,
                                           double& sx, double& sy, double& sz) {
  if (b.tri.on) {
    const double* hi = b.tri.hinv;
    sx = hi[0] * x + hi[1] * y + hi[2] * z;
    sy = hi[3] * y + hi[4] * z;
    sz = hi[5] * z;
  } else {
    sx = x * b.inv_l[0]; sy = y * b.inv_l[1]; sz = z * b.inv_l[2];
  }
  sx -= floor(sx); sy -= floor(sy); sz -= floor(sz);
}

// Reduced coordinate s in [0,1) (reduce_pos), split as s = sh + sl with
// sh a multiple of 2^-11 (exact in FP32) and 0 <= sl < 2^-11.  For |m| <= 2048
// the product m.sh is a multiple of 2^-11 below 2^13 in magnitude: it and its
// fractional part are exact in FP32, so the integer part of the phase m.s is
// removed without rounding; m.sl is added after.
__device__ __forceinline__ void split_coord(double s, float& sh, float& sl) {
  const double h = floor(s * 2048.0) * (1.0 / 2048.0);
  sh = (float)h;
  sl = (float)(s - h);
}

// phase in revolutions of k = 2 pi m / l at the split coordinate, FP32 path
__device__ __forceinline__ float phase_rev(float mx, float my, float mz, float shx, float shy,
                                           float shz, float slx, float sly, float slz) {
  float th = mx * shx;
  th = fmaf(my, shy, th);
  th = fmaf(mz, shz, th);
  float f = __builtin_amdgcn_fractf(th);
  f = fmaf(mx, slx, f);
  f = fmaf(my, sly, f);
  return fmaf(mz, slz, f);
}

__device__ __forceinline__ void kahan_add(float& sum, float& comp, float v) {
  const float y = v - comp;
  const float t = sum + y;
  comp = (t - sum) - y;
  sum = t;
}

// FP64 cos and sin of 2 pi f for |f| <= 1/2: the nearest of kSinCosTab table
// angles 2 pi k/kSinCosTab (cos, sin in LDS) rotated by the remainder angle
// u = 2 pi (f - k/kSinCosTab), |u| <= pi/kSinCosTab, whose cos - 1 and sin
// are short Taylor series (next terms below 2e-20).  f - k/kSinCosTab is exact
// (Sterbenz), so the error is that of the table entries and a few roundings:
// a few 1e-16 absolute.
constexpr int kSinCosTab = 256;

__device__ __forceinline__ void fill_sincos_tab(double2* tab, int nt) {
  for (int k = threadIdx.x; k < kSinCosTab; k += nt) {
    double sn, cs;
    sincospi((double)k * (2.0 / kSinCosTab), &sn, &cs);
    tab[k] = make_double2(cs, sn);
  }
}

__device__ __forceinline__ void sincos2pi(double f, const double2* tab, double& sn, double& cs) {
  const double kf = rint(f * (double)kSinCosTab);
  const double2 e = tab[(int)kf & (kSinCosTab - 1)];
  const double u = (f - kf * (1.0 / kSinCosTab)) * (2.0 * M_PI);
  const double u2 = u * u;
  const double cm1 = u2 * fma(u2, fma(u2, -1.0 / 720.0, 1.0 / 24.0), -0.5);
  const double su = fma(u * u2, fma(u2, fma(u2, -1.0 / 5040.0, 1.0 / 120.0), -1.0 / 6.0), u);
  cs = fma(-e.y, su, fma(e.x, cm1, e.x));
  sn = fma(e.x, su, fma(e.y, cm1, e.y));
}

// ---------------------------------------------------------------------------
// charges: sums for the neutrality check and the self term, FP32 copy

__global__ void k_qsum(const double* __restrict__ q, float* __restrict__ qf,
                       double* __restrict__ out, int64_t n, uint32_t* __restrict__ zero,
                       int64_t nzero) {
  __shared__ double s0[1024], s1[1024], s2[1024];
  const int t = threadIdx.x;
  for (int64_t i = t; i < nzero; i += blockDim.x) zero[i] = 0u;   // words to clear, if any
  double a = 0.0, b = 0.0, c = 0.0;
  for (int64_t i = t; i < n; i += blockDim.x) {
    const double v = q[i];
    if (qf) qf[i] = (float)v;
    a += v; b += fabs(v); c += v * v;
  }
  s0[t] = a; s1[t] = b; s2[t] = c;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (t < w) { s0[t] += s0[t + w]; s1[t] += s1[t + w]; s2[t] += s2[t + w]; }
    __syncthreads();
  }
  if (t == 0) { out[0] = s0[0]; out[1] = s1[0]; out[2] = s2[0]; }
}

hipError_t launch_qsum(const double* d_q, float* d_qf, double* d_out3, int64_t n, hipStream_t s,
                       uint32_t* d_zero, int64_t nzero) {
  hipLaunchKernelGGL(k_qsum, dim3(1), dim3(1024), 0, s, d_q, d_qf, d_out3, n, d_zero, nzero);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// online Metropolis-Hastings sampler (section 4.3, online approach): chain l
// keeps its frequency from step to step and takes mh_iters independence
// moves per sampled step towards the law of the current cell.  Per axis the
// law is exp(-m^2/(2 sigma^2)), sigma = sqrt(alpha) l/(pi sqrt 2); the proposal
// rounds a continuous Gaussian of the same sigma to the integer whose
// [m - 1/2, m + 1/2) holds it, q(m) = Phi((m + 1/2)/sigma) - Phi((m - 1/2)/sigma);
// a move m -> m' is accepted with min(1, pi(m') q(m)/(pi(m) q(m'))), m' = 0
// never.  Move it of chain l at step s: counter (s, l, 'mhch', 2 it) gives
// the three normals (Box-Muller), (s, l, 'mhch', 2 it + 1) the acceptance
// uniform.

constexpr uint64_t kTagMH = 0x6D686368ull;  // 'mhch'

// q(m) for one axis, s = sigma sqrt 2, from erfc on the side away from the
// mode (no cancellation in the tails)
__device__ __forceinline__ double mh_qpmf(int m, double s) {
  if (m == 0) return erf(0.5 / s);
  const double a = (double)abs(m);
  return 0.5 * (erfc((a - 0.5) / s) - erfc((a + 0.5) / s));
}

__device__ void mh_frequency(const StepArgs& a, const BoxState& b, int l, int m[3]) {
  const double sq2 = 1.4142135623730951;
  double sig[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    sig[j] = sqrt(a.alpha) * b.l[j] / (M_PI * sq2);
    m[j] = a.mh_old[3 * l + j];
  }
  for (int it = 0; it < a.mh_iters; ++it) {
    uint64_t c[4] = {a.step, (uint64_t)l, kTagMH, 2ull * (uint64_t)it};
    philox4x64_10(c, a.seed, a.sysid);
    double u[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) u[j] = (double)(c[j] >> 11) * 0x1.0p-53;
    const double ra = sqrt(-2.0 * log(1.0 - u[0])), rb = sqrt(-2.0 * log(1.0 - u[2]));
    const double t1 = 2.0 * M_PI * u[1], t3 = 2.0 * M_PI * u[3];
    const double z[3] = {ra * cos(t1), ra * sin(t1), rb * cos(t3)};
    int mp[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) mp[j] = (int)floor(sig[j] * z[j] + 0.5);
    uint64_t c2[4] = {a.step, (uint64_t)l, kTagMH, 2ull * (uint64_t)it + 1ull};
    philox4x64_10(c2, a.seed, a.sysid);
    const double ua = (double)(c2[0] >> 11) * 0x1.0p-53;
    if (mp[0] == 0 && mp[1] == 0 && mp[2] == 0) continue;
    double e = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) e += (double)(mp[j] * mp[j] - m[j] * m[j]) / (2.0 * sig[j] * sig[j]);
    double r = exp(-e);
#pragma unroll
    for (int j = 0; j < 3; ++j) r *= mh_qpmf(m[j], sig[j] * sq2) / mh_qpmf(mp[j], sig[j] * sq2);
    if (ua < fmin(1.0, r)) { m[0] = mp[0]; m[1] = mp[1]; m[2] = mp[2]; }
  }
}

// The attempt-0 Philox outputs (counter (step, l, 'ksam', 0)) of the
// frequencies l = slice + s2 < p, s2 < FB, into su[j * FB + s2], formed by
// the waves that build_tables leaves idle (one wave per (axis, table): six),
// so that they run beside the table build instead of after it; the draw then
// only searches the tables.  Reached by every thread before build_tables,
// whose closing barrier makes su visible.  nt (the block's threads) > kTableTasks waves.
__device__ __forceinline__ void slice_uniforms(uint64_t* su, int FB, int64_t slice, int64_t p,
                                               uint64_t seed, uint64_t sysid, uint64_t step, int nt) {
  const int t = (int)threadIdx.x - kTableTasks * kWave;
  const int nu = nt - kTableTasks * kWave;
  if (t < 0) return;
  for (int s2 = t; s2 < FB && slice + s2 < p; s2 += nu) {
    uint64_t c[4] = {step, (uint64_t)(slice + s2), kTagKSample, 0ull};
    philox4x64_10(c, seed, sysid);
#pragma unroll
    for (int j = 0; j < 4; ++j) su[j * FB + s2] = c[j];
  }
}

// frequency l of the current step under the context's sampler (the chains
// move in the standalone draw kernel only: inlined into the structure-factor
// kernel, their FP64 transcendentals would raise its register budget)
__device__ __forceinline__ void sample_frequency(const StepArgs& a, const BoxState& b,
                                                 const double* tab, int l, int m[3]) {
  if (a.sampler == RBE_SAMPLER_MH && !a.mh_init) mh_frequency(a, b, l, m);
  else if (b.tri.on) draw_frequency<true>(b, tab, a.seed, a.sysid, a.step, l, m);
  else draw_frequency<false>(b, tab, a.seed, a.sysid, a.step, l, m);
}

// ---------------------------------------------------------------------------
// standalone tables / draw (when the batch or the cell is read on the host
// before a fused step has run)

__global__ void __launch_bounds__(256) k_tables(StepArgs a) {
  __shared__ BoxState sbs;
  __shared__ TriCell stc;
  __shared__ double sh_T[3];
  double l[3];
  const TriCell* tc = stage_tri(a, &stc);
  box_source(a, l);
  build_tables(l, tc, a.alpha, a.tail_ln, a.mcap, a.tab, &sbs, sh_T, 256, true);
  commit_cell(sbs, a.bs, threadIdx.x);
}

hipError_t launch_tables(const StepArgs& a, hipStream_t s, const LaunchEvents& ev) {
  void* args[] = {const_cast<StepArgs*>(&a)};
  return hipExtLaunchKernel(reinterpret_cast<const void*>(&k_tables), dim3(1), dim3(256), args, 0,
                            s, ev.start, ev.stop, 0);
}

__global__ void __launch_bounds__(256) k_sample(StepArgs a) {
  __shared__ BoxState sbs;
  load_box(sbs, a.bs, threadIdx.x);
  lds_barrier();
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= a.p) return;
  int m[3];
  sample_frequency(a, sbs, a.tab, l, m);
  a.m[3 * l] = m[0]; a.m[3 * l + 1] = m[1]; a.m[3 * l + 2] = m[2];
  if (a.sampler == RBE_SAMPLER_MH) { a.mh_new[3 * l] = m[0]; a.mh_new[3 * l + 1] = m[1]; a.mh_new[3 * l + 2] = m[2]; }
}

hipError_t launch_sample(const StepArgs& a, hipStream_t s, const LaunchEvents& ev) {
  void* args[] = {const_cast<StepArgs*>(&a)};
  return hipExtLaunchKernel(reinterpret_cast<const void*>(&k_sample), dim3((a.p + 255) / 256),
                            dim3(256), args, 0, s, ev.start, ev.stop, 0);
}

// ---------------------------------------------------------------------------
// k_sfac: tables, draw, structure factors, fixed-order reduction, virial
//
// Block = 8 waves.  A wave owns 64*R frequencies (R per lane: slot r*64 +
// lane), KB waves cover distinct frequency groups (FB = KB*64*R frequencies
// per block), SUB = 8/KB waves split the chunk's particles.  Several
// frequencies per lane amortise the LDS broadcast of each particle, whose
// return costs LDS bandwidth like any other read.

// Dynamic LDS of k_sfac, three regions:
//   R0 particle tiles (kTile x 32 B); after the main loop: reduction scratch
//   R1 the block's slice of the batch (3 ints per frequency)
//   R2 the sampler tables; after the draw: rho of the slice, then the 7 x
//      kSfacThreads virial summands
constexpr size_t kR0 = (size_t)kTile * 32;

__host__ __device__ static size_t sfac_r1(const StepArgs& a) { return (size_t)a.KB * kWave * a.R * 3 * sizeof(int); }
static size_t sfac_r2(const StepArgs& a) {
  const int cap = a.mcap[0] + a.mcap[1] + a.mcap[2];
  size_t r2 = (size_t)(4 * cap + 3) * sizeof(double);
  const size_t rho = (size_t)a.KB * kWave * a.R * sizeof(double2);
  const size_t vir = (size_t)7 * kSfacThreads * sizeof(double);
  if (rho > r2) r2 = rho;
  if (vir > r2) r2 = vir;
  return r2;
}
size_t sfac_lds_bytes(const StepArgs& a) { return kR0 + sfac_r1(a) + sfac_r2(a); }

// Data handed from block to block within a launch is stored and loaded with
// agent-scope atomic accesses (coherent across the XCDs' separate L2 caches)
// rather than plain accesses plus L2 write-back / invalidate fences, which
// cost microseconds per block on this chip.
__device__ __forceinline__ void st_coh(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coh2(double2* p, double2 v) {
  st_coh(&p->x, v.x);
  st_coh(&p->y, v.y);
}
__device__ __forceinline__ double ld_coh(const double* p) {
  return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double2 ld_coh2(const double2* p) {
  return make_double2(ld_coh(&p->x), ld_coh(&p->y));
}

// Last-arriving test.  Every block of a group increments the group counter
// once, after all its waves' coherent stores have completed (waitcnt, then
// barrier); the block that brings the counter to `total` gets true
// (block-uniform) and may read the others' coherent stores.
__device__ __forceinline__ bool arrive_last(uint32_t* counter, uint32_t total, int* sh_flag) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0)
    *sh_flag = (__hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
                total - 1u) ? 1 : 0;
  __syncthreads();
  return *sh_flag != 0;
}

// dst[i] = sum over r = 0..R-1 of src[r*stride + i] for i < W, in a fixed
// order, by the whole block (W and the block size powers of two).  If W <
// threads: thread t owns column t % W and rows t / W + RG*j (RG = threads /
// W), then the RG row-group sums are added in order through LDS.  Otherwise
// thread t owns columns t + threads*j and all rows.  Loads are issued kB
// (8 unless given) at a time.  src is read with coherent loads when SrcCoh (rows stored by other
// blocks of the same launch), else plainly (rows of an earlier launch, which
// the L2 may then serve to several blocks); dst is written with coherent
// stores when dst_coh, else plainly (LDS).  Reached by every thread;
// scratch holds nt entries (nt = the block's threads); scratch_free: no
// thread reads scratch any more (nothing has used it yet, or a barrier has
// passed since), so the barrier before it is written is skipped.
template <bool SrcCoh = true>
__device__ __forceinline__ double2 ld_row(const double2* p) {
  return SrcCoh ? ld_coh2(p) : *p;
}

template <bool SrcCoh = true, int kB = 8>
__device__ void block_sum_rows(const double2* src, int64_t stride, int R, int W, double2* dst,
                               bool dst_coh, double2* scratch, int nt, bool scratch_free = false) {
  // rows r0, r0 + step, ... (< R) of column col added in that order; loads
  // issued kB at a time (independent, all in flight) before the adds
  auto column_sum = [&](int col, int r0, int step) {
    double2 acc = make_double2(0.0, 0.0);
    for (int r = r0; r < R; r += kB * step) {
      double2 v[kB];
#pragma unroll
      for (int k = 0; k < kB; ++k)
        v[k] = (r + k * step < R) ? ld_row<SrcCoh>(src + (int64_t)(r + k * step) * stride + col)
                                  : make_double2(0.0, 0.0);
#pragma unroll
      for (int k = 0; k < kB; ++k)
        if (r + k * step < R) { acc.x += v[k].x; acc.y += v[k].y; }
    }
    return acc;
  };
  const int t = threadIdx.x;
  if (W >= nt) {
    for (int col = t; col < W; col += nt) {
      const double2 acc = column_sum(col, 0, 1);
      if (dst_coh) st_coh2(dst + col, acc); else dst[col] = acc;
    }
    lds_barrier();
    return;
  }
  const int RG = nt / W;
  const int col = t % W, rg = t / W;
  const double2 acc = column_sum(col, rg, RG);
  if (!scratch_free) lds_barrier();      // scratch's earlier readers are done
  scratch[t] = acc;
  lds_barrier();
  if (t < W) {
    double2 s2 = scratch[t];
    for (int g = 1; g < RG; ++g) { const double2 v = scratch[g * W + t]; s2.x += v.x; s2.y += v.y; }
    if (dst_coh) st_coh2(dst + t, s2); else dst[t] = s2;
  }
  lds_barrier();
}

// Per-frequency constants from rho_l and m_l (eq. (appforce), eq. (apppress)
// in tensor form, appendix C):
//   k = 2 pi m / l (triclinic: 2 pi h^-T m),  c = C (S/p_force) 4 pi / (V |k|^2)
//   ->  force coefficients (c Re rho, c Im rho);
//   the FP32 path keeps c |rho| and arg(rho) instead: Im(exp(-i theta) rho) =
//   |rho| sin(arg(rho) - theta) takes one sine per pair where the cos / sin
//   form takes two
//   tv = |rho|^2/|k|^2 [delta_ab - 2 (1/|k|^2 + 1/(4 alpha)) k_a k_b]  (xx yy zz xy xz yz) and
//   tv[6] = |rho|^2/|k|^2, to be scaled by C (2 pi / V)(S/p) after the batch sum.
__device__ __forceinline__ void freq_consts(const int mi[3], double2 r, const BoxState& b,
                                            double alpha, double coulomb, int p_force, FCoef64& f,
                                            FCoef32& h, double tv[7]) {
  // k = 2 pi h^-T m (appendix C; h^-1 upper triangular, diagonal 1/l for a
  // rectangular cell), selected per entry rather than by a branch so that
  // both cell kinds share one register budget
  double km[3], kk[3];
  for (int c = 0; c < 3; ++c) km[c] = (double)mi[c];
  {
    const bool tri = b.tri.on != 0;
    const double* hi = b.tri.hinv;
    const double t0 = tri ? hi[0] : b.inv_l[0], t3 = tri ? hi[3] : b.inv_l[1];
    const double t5 = tri ? hi[5] : b.inv_l[2];
    const double t1 = tri ? hi[1] : 0.0, t2 = tri ? hi[2] : 0.0, t4 = tri ? hi[4] : 0.0;
    kk[0] = 2.0 * M_PI * (t0 * km[0]);
    kk[1] = 2.0 * M_PI * (t1 * km[0] + t3 * km[1]);
    kk[2] = 2.0 * M_PI * (t2 * km[0] + t4 * km[1] + t5 * km[2]);
  }
  const double k2 = kk[0] * kk[0] + kk[1] * kk[1] + kk[2] * kk[2];
  const double ik2 = 1.0 / k2;
  const double cl = coulomb * (b.S / (double)p_force) * 4.0 * M_PI / b.V * ik2;
  const double fac = (r.x * r.x + r.y * r.y) * ik2;
  const double beta = 2.0 * (ik2 + 0.25 / alpha);
  tv[0] = fac * (1.0 - beta * kk[0] * kk[0]);
  tv[1] = fac * (1.0 - beta * kk[1] * kk[1]);
  tv[2] = fac * (1.0 - beta * kk[2] * kk[2]);
  tv[3] = -fac * beta * kk[0] * kk[1];
  tv[4] = -fac * beta * kk[0] * kk[2];
  tv[5] = -fac * beta * kk[1] * kk[2];
  tv[6] = fac;
  // the phase is kept in FP32, so its arctangent is taken in FP32 too
  const double amp = cl * sqrt(r.x * r.x + r.y * r.y);
  for (int c = 0; c < 3; ++c) {
    f.m[c] = km[c]; f.k[c] = kk[c];
    h.m[c] = (float)km[c]; h.ak[c] = (float)(amp * kk[c]);
  }
  h.pad = 0.0f;
  f.cA = cl * r.x; f.cB = cl * r.y;
  h.phi = atan2f((float)r.y, (float)r.x) * (float)(0.5 / M_PI);
}

// Batch sum of the virial summands held per thread (tv: the thread's own
// frequencies already summed in a fixed order, zero on idle threads), in a
// fixed order: 7 x 8 strided partial sums over the threads through LDS, then
// the 8 partials in order.  Writes the virial tensor and the energy.  Reached
// by every thread (nt of them); stv holds 7*nt doubles.
__device__ void virial_energy(const double tv[7], double* stv, double (*sh_vs)[8],
                              const BoxState& b, double coulomb, int p, double self_energy,
                              double* virial6, double* energy, int nt) {
  const int tid = threadIdx.x;
  lds_barrier();
  for (int c = 0; c < 7; ++c) stv[c * nt + tid] = tv[c];
  lds_barrier();
  if (tid < 56) {
    const int c = tid / 8, part_i = tid % 8;
    double v = 0.0;
    for (int l = part_i; l < nt; l += 8) v += stv[c * nt + l];
    sh_vs[c][part_i] = v;
  }
  lds_barrier();
  if (tid < 7) {
    double v = 0.0;
    for (int w = 0; w < 8; ++w) v += sh_vs[tid][w];
    const double pref = coulomb * (2.0 * M_PI / b.V) * (b.S / (double)p);
    if (tid < 6) { if (virial6) virial6[tid] = pref * v; }
    else if (energy) energy[0] = pref * v + self_energy;
  }
}

// rho sums over one LDS tile, FP32 path: lane frequencies (mx, my, mz)[r];
// the wave takes particles sub, sub + SUB, ... of the tile in runs of kKahan
// plain FP32 FMAs, each run folded into the per-lane Kahan pairs (SA, CA),
// (SB, CB).  The tile holds (sh.x, sh.y, sh.z, q) and (sl.x, sl.y, sl.z, 0)
// per particle, padded with zero charges to a multiple of SUB * kKahan.
template <int R>
__device__ __forceinline__ void sfac_tile32(const float4* tA, const float4* tB, int cntp, int sub,
                                            int SUB, const float (&mx)[R], const float (&my)[R],
                                            const float (&mz)[R], float (&SA)[R], float (&CA)[R],
                                            float (&SB)[R], float (&CB)[R]) {
  const int runlen = SUB * kKahan;
  for (int j0 = sub; j0 < cntp; j0 += runlen) {
    float ra[R], rb[R];
#pragma unroll
    for (int r = 0; r < R; ++r) { ra[r] = 0.f; rb[r] = 0.f; }
#pragma unroll
    for (int u = 0; u < kKahan; ++u) {
      const int j = j0 + u * SUB;
      const float4 pa = tA[j], pb = tB[j];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const float f = phase_rev(mx[r], my[r], mz[r], pa.x, pa.y, pa.z, pb.x, pb.y, pb.z);
        const float cs = __builtin_amdgcn_cosf(f);
        const float sn = __builtin_amdgcn_sinf(f);
        ra[r] = fmaf(pa.w, cs, ra[r]);
        rb[r] = fmaf(pa.w, sn, rb[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      kahan_add(SA[r], CA[r], ra[r]);
      kahan_add(SB[r], CB[r], rb[r]);
    }
  }
}

// rho sums over one LDS tile, FP64 path: the tile holds (s.x, s.y) and
// (s.z, q) per particle (reduced coordinates in [0, 1)), padded to a
// multiple of SUB with zero charges.
template <int R>
__device__ __forceinline__ void sfac_tile64(const double2* tA, const double2* tB, int cntp, int sub,
                                            int SUB, const double2* sctab, const double (&mx)[R],
                                            const double (&my)[R], const double (&mz)[R],
                                            double (&A)[R], double (&B)[R]) {
  for (int j = sub; j < cntp; j += SUB) {
    const double2 pa = tA[j], pb = tB[j];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const double t = mx[r] * pa.x + my[r] * pa.y + mz[r] * pb.x;
      const double f = t - rint(t);
      double sn, cs;
      sincos2pi(f, sctab, sn, cs);
      A[r] = fma(pb.y, cs, A[r]);
      B[r] = fma(pb.y, sn, B[r]);
    }
  }
}

// Block partial of rho: the SUB particle sub-slices of every frequency slot
// summed in order (through red, G x kSfacThreads entries of LDS: G of the R
// parts per pair of barriers) and stored with coherent stores to dst[slot]
// (slot = kg*64R + r*64 + lane).  Reached by every thread.
template <int R, int G = 1>
__device__ __forceinline__ void store_block_partial(const double2 (&part)[R], double2* red, int KB,
                                                    int SUB, double2* dst) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int r0 = 0; r0 < R; r0 += G) {
    lds_barrier();
#pragma unroll
    for (int r = r0; r < r0 + G && r < R; ++r) red[(r - r0) * kSfacThreads + tid] = part[r];
    lds_barrier();
    if (tid < KB * kWave) {                // (kg', lane') = (tid / 64, tid % 64)
#pragma unroll
      for (int r = r0; r < r0 + G && r < R; ++r) {
        const double2* rr = red + (r - r0) * kSfacThreads;
        double2 s2 = make_double2(0.0, 0.0);
        for (int sb = 0; sb < SUB; ++sb) { // wave = sb*KB + kg'  ->  index sb*KB*64 + tid
          const double2 v = rr[sb * KB * kWave + tid];
          s2.x += v.x; s2.y += v.y;
        }
        const int sl = (tid / kWave) * kWave * R + r * kWave + (tid % kWave);
        st_coh2(dst + sl, s2);
      }
    }
  }
}

template <bool F64, int R, bool TRI>
__device__ __forceinline__ void sfac_body(const StepArgs& a, const int x, const int y,
                                          unsigned char* lds_raw) {
  __shared__ BoxState sbs;
  __shared__ TriCell stc;
  __shared__ double sh_T[3];
  __shared__ int sh_flag;
  __shared__ double sh_vs[7][8];
  __shared__ double2 sctab[F64 ? kSinCosTab : 1];
  const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
  const int KB = a.KB, SUB = kSfacWaves / KB, FB = KB * kWave * R;
  if (F64) fill_sincos_tab(sctab, kSfacThreads);   // read after the barriers below
  const TriCell* tc = stage_tri(a, &stc);
  unsigned char* base = lds_raw;
  int* sm = reinterpret_cast<int*>(base + kR0);                     // batch slice, 3 ints each
  double* tabs = reinterpret_cast<double*>(base + kR0 + sfac_r1(a));  // R2

  // ---- the extra block: draw the batch of step + 1 for this launch's cell
  if (x == a.X) {
    if (y != 0) return;
    double l[3];
    box_source(a, l);
    build_tables(l, tc, a.alpha, a.tail_ln, a.mcap, tabs, &sbs, sh_T, kSfacThreads, true);
    const uint64_t next = a.step + 1;
    const int slot = (int)(next & 1);
    int32_t* mp = a.m_pre + (int64_t)slot * 3 * a.p;
    for (int l2 = tid; l2 < a.p; l2 += kSfacThreads) {
      int mv[3];
      draw_frequency<TRI>(sbs, tabs, a.seed, a.sysid, next, l2, mv);
      mp[3 * l2] = mv[0]; mp[3 * l2 + 1] = mv[1]; mp[3 * l2 + 2] = mv[2];
    }
    copy_box(&a.pre[slot].bs, sbs, tid);
    if (tid == 0) {
      a.pre[slot].step = next;
      a.pre[slot].valid = 1;
    }
    return;
  }

  // ---- the cell's sides first: they may be global loads (a device or the
  // committed cell), and a wait for a load also waits for every load issued
  // before it, so the particle loads go out after them and the table build
  // does not wait for the particles
  double lc[3];
  box_source(a, lc);
  __builtin_amdgcn_sched_barrier(0);

  // ---- first tile of particles: loads issued now, consumed after the tables
  const int64_t c0 = (int64_t)x * a.chunk;
  const int64_t c1 = min(a.n, c0 + (int64_t)a.chunk);
  const int first_cnt = (int)min((int64_t)kTile, c1 - c0);
  double px = 0.0, py = 0.0, pz = 0.0, pq = 0.0;
  if (tid < first_cnt) {
    px = a.x[c0 + tid]; py = a.y[c0 + tid]; pz = a.z[c0 + tid];
    pq = F64 ? a.q[c0 + tid] : (double)a.qf[c0 + tid];
  }

  // ---- batch drawn ahead: usable when its step and cell equal this call's
  const int pslot = (int)(a.step & 1);
  // (no check, and no barrier, when the host has ruled the batch out)
  bool pre = false;
  if (a.sample && a.use_pre) {
    if (tid == 0) {
      int ok = 0;
      if (a.pre[pslot].valid && a.pre[pslot].step == a.step) ok = same_cell(a, a.pre[pslot].bs) ? 1 : 0;
      sh_flag = ok;
    }
    lds_barrier();
    pre = sh_flag != 0;
  }
  if (pre) {
    load_box(sbs, &a.pre[pslot].bs, tid);
    lds_barrier();
  }
  const int32_t* m_pre = a.m_pre + (int64_t)pslot * 3 * a.p;

  // ---- cell values and tables; the slice's Philox outputs beside them, in
  // R0 (free until the tile is stored)
  const bool need_tables = !pre && (a.sample || a.box_src != BOX_COMMITTED);
  double cw[3] = {0.0, 0.0, 0.0};   // case weights for this block's draws
  const int64_t slice = (int64_t)y * FB;
  const bool su_on = a.sample && !pre && (size_t)FB * 4 * sizeof(uint64_t) <= kR0;
  uint64_t* su = reinterpret_cast<uint64_t*>(base);
  if (pre) {
    if (x == 0 && y == 0 && a.box_src != BOX_COMMITTED) commit_cell(sbs, a.bs, tid);
  } else if (need_tables) {
    if (su_on) slice_uniforms(su, FB, slice, a.p, a.seed, a.sysid, a.step, kSfacThreads);
    // the draw needs only the half-widths (visible after the tables'
    // barrier) and the case weights, formed here from the tables' totals, so
    // the block skips the closing barrier unless it commits the cell
    const bool commit = x == 0 && y == 0 && a.box_src != BOX_COMMITTED;
    const bool own_cw = !TRI && kSfacThreads / kWave > kTableTasks && !commit;
    build_tables(lc, tc, a.alpha, a.tail_ln, a.mcap, tabs, &sbs, sh_T, kSfacThreads, !own_cw);
    if (own_cw) case_weights(sh_T, cw);
    else { cw[0] = sbs.case_w[0]; cw[1] = sbs.case_w[1]; cw[2] = sbs.case_w[2]; }
    if (commit) commit_cell(sbs, a.bs, tid);
  } else {
    load_box(sbs, a.bs, tid);
    lds_barrier();
  }

  // ---- this block's slice of the batch: drawn here, or read (drawn ahead,
  // or stored); one loop per case, so that the drawing loop has no global
  // loads (whose waits would also wait for the particles)
  if (!pre && a.sample) {
    for (int s2 = tid; s2 < FB; s2 += kSfacThreads) {
      const int64_t l = slice + s2;
      int mv[3] = {0, 0, 0};
      if (l < a.p) {
        draw_frequency<TRI>(sbs, tabs, a.seed, a.sysid, a.step, (int)l, mv,
                            su_on ? su + s2 : nullptr, FB, cw);
        if (x == 0) { a.m[3 * l] = mv[0]; a.m[3 * l + 1] = mv[1]; a.m[3 * l + 2] = mv[2]; }
      }
      sm[3 * s2] = mv[0]; sm[3 * s2 + 1] = mv[1]; sm[3 * s2 + 2] = mv[2];
    }
  } else {
    const int32_t* msrc = pre ? m_pre : a.m;
    for (int s2 = tid; s2 < FB; s2 += kSfacThreads) {
      const int64_t l = slice + s2;
      int mv[3] = {0, 0, 0};
      if (l < a.p) {
        mv[0] = msrc[3 * l]; mv[1] = msrc[3 * l + 1]; mv[2] = msrc[3 * l + 2];
        if (pre && x == 0) { a.m[3 * l] = mv[0]; a.m[3 * l + 1] = mv[1]; a.m[3 * l + 2] = mv[2]; }
      }
      sm[3 * s2] = mv[0]; sm[3 * s2 + 1] = mv[1]; sm[3 * s2 + 2] = mv[2];
    }
  }
  lds_barrier();

  // ---- structure factors over the chunk: lane owns frequencies
  // kg*64R + r*64 + lane (r < R); wave = sub*KB + kg
  const int kg = wave % KB, sub = wave / KB;
  const double ix = sbs.inv_l[0], iy = sbs.inv_l[1], iz = sbs.inv_l[2];
  double2 part[R];
  if (!F64) {
    // plain FP32 runs of kKahan terms between compensated folds: for random
    // rounding errors the total over N particles grows like sqrt(N) eps |q|
    // whatever the run length, and longer runs issue fewer fold operations
    constexpr int kRun = kKahan;
    const int runlen = SUB * kRun;
    float4* tA = reinterpret_cast<float4*>(base);           // sh.x sh.y sh.z q
    float4* tB = tA + kTile;                                // sl.x sl.y sl.z 0
    float mx[R], my[R], mz[R], SA[R], CA[R], SB[R], CB[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int sl = kg * kWave * R + r * kWave + lane;
      mx[r] = (float)sm[3 * sl]; my[r] = (float)sm[3 * sl + 1]; mz[r] = (float)sm[3 * sl + 2];
      SA[r] = CA[r] = SB[r] = CB[r] = 0.f;
    }
    for (int64_t t0 = c0; t0 < c1; t0 += kTile) {
      const int cnt = (int)min((int64_t)kTile, c1 - t0);
      const int cntp = (cnt + runlen - 1) / runlen * runlen;
      if (t0 != c0) lds_barrier();     // the first tile: the barrier after the draw
      for (int j = tid; j < cntp; j += kSfacThreads) {
        float4 u = make_float4(0.f, 0.f, 0.f, 0.f), v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (j < cnt) {
          const int64_t i = t0 + j;
          const bool first = (t0 == c0);     // j == tid here: prefetched above
          double sx, sy, sz;
          reduce_pos(sbs, first ? px : a.x[i], first ? py : a.y[i], first ? pz : a.z[i], sx, sy,
                     sz);
          split_coord(sx, u.x, v.x);
          split_coord(sy, u.y, v.y);
          split_coord(sz, u.z, v.z);
          u.w = first ? (float)pq : a.qf[i];
        }
        tA[j] = u; tB[j] = v;
      }
      lds_barrier();
      sfac_tile32<R>(tA, tB, cntp, sub, SUB, mx, my, mz, SA, CA, SB, CB);
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
      part[r] = make_double2((double)SA[r] - (double)CA[r], (double)SB[r] - (double)CB[r]);
  } else {
    double2* tA = reinterpret_cast<double2*>(base);         // s.x s.y
    double2* tB = tA + kTile;                               // s.z q
    double mx[R], my[R], mz[R], A[R], B[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int sl = kg * kWave * R + r * kWave + lane;
      mx[r] = (double)sm[3 * sl]; my[r] = (double)sm[3 * sl + 1]; mz[r] = (double)sm[3 * sl + 2];
      A[r] = B[r] = 0.0;
    }
    for (int64_t t0 = c0; t0 < c1; t0 += kTile) {
      const int cnt = (int)min((int64_t)kTile, c1 - t0);
      const int cntp = (cnt + SUB - 1) / SUB * SUB;
      if (t0 != c0) lds_barrier();     // the first tile: the barrier after the draw
      for (int j = tid; j < cntp; j += kSfacThreads) {
        double2 u = make_double2(0.0, 0.0), v = make_double2(0.0, 0.0);
        if (j < cnt) {
          const int64_t i = t0 + j;
          const bool first = (t0 == c0);     // j == tid here: prefetched above
          double sx, sy, sz;
          reduce_pos(sbs, first ? px : a.x[i], first ? py : a.y[i], first ? pz : a.z[i], sx, sy,
                     sz);
          u = make_double2(sx, sy);
          v = make_double2(sz, first ? pq : a.q[i]);
        }
        tA[j] = u; tB[j] = v;
      }
      lds_barrier();
      sfac_tile64<R>(tA, tB, cntp, sub, SUB, sctab, mx, my, mz, A, B);
    }
#pragma unroll
    for (int r = 0; r < R; ++r) part[r] = make_double2(A[r], B[r]);
  }

  // ---- block partial: sum the SUB particle sub-slices, in order, per slot
  double2* red = reinterpret_cast<double2*>(base);          // kSfacThreads entries (R0)
  static_assert(2 * kSfacThreads * sizeof(double2) <= kR0, "two parts per pass in R0");
  store_block_partial<R, 2>(part, red, KB, SUB, a.partial + (int64_t)x * a.Ppad + slice);

  // ---- level 1: the last block of each chunk group sums the group's partials
  const int g = x / a.GX;
  const int gsize = min(a.GX, a.X - g * a.GX);
  if (a.NG > 1) {
    if (!arrive_last(a.cnt + cnt_index(a, CNT_GROUP, y * a.NG + g), (uint32_t)gsize, &sh_flag))
      return;
    block_sum_rows(a.partial + (int64_t)g * a.GX * a.Ppad + slice, a.Ppad, gsize, FB,
                   a.gpart + (int64_t)g * a.Ppad + slice, true, red, kSfacThreads, true);
    if (tid == 0) a.cnt[cnt_index(a, CNT_GROUP, y * a.NG + g)] = 0u;
  }

  // the force kernel takes it from here (small batches: every force block
  // sums the NG group partials itself)
  if (a.k2reduce) return;

  // ---- level 2: the last group of the slice forms rho, the force
  // coefficients and the per-frequency virial summands
  if (!arrive_last(a.cnt + cnt_index(a, CNT_SLICE, y), (uint32_t)a.NG, &sh_flag)) return;
  double2* srho = reinterpret_cast<double2*>(tabs);          // R2 (tables are dead)
  if (a.NG > 1)
    block_sum_rows(a.gpart + slice, a.Ppad, a.NG, FB, srho, false, red, kSfacThreads);
  else
    block_sum_rows(a.partial + slice, a.Ppad, a.X, FB, srho, false, red, kSfacThreads);
  double tv[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int s2 = tid; s2 < FB; s2 += kSfacThreads) {
    if (slice + s2 >= a.p) break;
    const int l = (int)(slice + s2);
    const double2 r = srho[s2];
    a.rho[l] = r;
    const int mi[3] = {sm[3 * s2], sm[3 * s2 + 1], sm[3 * s2 + 2]};
    FCoef64 f;
    FCoef32 h;
    double tl[7];
    freq_consts(mi, r, sbs, a.alpha, a.coulomb, a.pf, f, h, tl);
    if (a.Y > 1) {
      double* tr = a.terms + (int64_t)l * 8;
      for (int c = 0; c < 7; ++c) st_coh(tr + c, tl[c]);
    }
    for (int c = 0; c < 7; ++c) tv[c] += tl[c];
    a.fc64[l] = f;
    a.fc32[l] = h;
  }
  if (tid == 0) a.cnt[cnt_index(a, CNT_SLICE, y)] = 0u;

  // ---- level 3: the batch sum -> virial tensor and energy.  With one slice
  // the level-2 block holds every summand; otherwise the last slice loads
  // them back, thread t taking frequencies t, t + kSfacThreads, ...
  if (a.Y > 1) {
    if (!arrive_last(a.cnt + cnt_index(a, CNT_BATCH), (uint32_t)a.Y, &sh_flag)) return;
    for (int c = 0; c < 7; ++c) tv[c] = 0.0;
    for (int l = tid; l < a.p; l += kSfacThreads)
      for (int c = 0; c < 7; ++c) tv[c] += ld_coh(a.terms + (int64_t)l * 8 + c);
  }
  virial_energy(tv, tabs, sh_vs, sbs, a.coulomb, a.p, a.self_energy, a.virial6, a.energy,
                kSfacThreads);
  if (tid == 0 && a.Y > 1) a.cnt[cnt_index(a, CNT_BATCH)] = 0u;
}

template <bool F64, int R, bool TRI>
__global__ void __launch_bounds__(kSfacThreads) k_sfac(StepArgs a) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  sfac_body<F64, R, TRI>(a, blockIdx.x, blockIdx.y, lds_raw);
}

// Many systems in one launch: block b belongs to system s with
// bstart[s] <= b < bstart[s+1]; its local index runs over that system's
// (X + predraw) x Y grid.  The system's arguments are copied to LDS.
__device__ __forceinline__ int find_system(const int* bstart, int nsys, int b) {
  int lo = 0, hi = nsys - 1;
  while (lo < hi) {                          // last s with bstart[s] <= b
    const int mid = (lo + hi + 1) >> 1;
    if (bstart[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <bool F64, int R>
__global__ void __launch_bounds__(kSfacThreads) k_sfac_multi(const StepArgs* tab, const int* bstart,
                                                             int nsys) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ StepArgs sa;
  const int b = blockIdx.x;
  const int sys = find_system(bstart, nsys, b);
  copy_args(&sa, tab + sys);
  lds_barrier();
  const int local = b - bstart[sys];
  const int xs = sa.X + (sa.predraw ? 1 : 0);
  sfac_body<F64, R, false>(sa, local % xs, local / xs, lds_raw);   // no triclinic systems
}

// the kernel instance for a precision, lane width R and cell kind
template <bool TRI>
static const void* sfac_kernel(int precision, int R) {
  if (precision == RBE_PREC_FP64) return reinterpret_cast<const void*>(&k_sfac<true, 1, TRI>);
  if (R == 4) return reinterpret_cast<const void*>(&k_sfac<false, 4, TRI>);
  if (R == 2) return reinterpret_cast<const void*>(&k_sfac<false, 2, TRI>);
  return reinterpret_cast<const void*>(&k_sfac<false, 1, TRI>);
}

hipError_t launch_sfac(int precision, const StepArgs& a, hipStream_t s, const LaunchEvents& ev) {
  const dim3 grid(a.X + (a.predraw ? 1 : 0), a.Y);
  const size_t lds = sfac_lds_bytes(a);
  const void* fn = a.tri_mode ? sfac_kernel<true>(precision, a.R) : sfac_kernel<false>(precision, a.R);
  void* args[] = {const_cast<StepArgs*>(&a)};
  return hipExtLaunchKernel(fn, grid, dim3(kSfacThreads), args, lds, s, ev.start, ev.stop, 0);
}

int sfac_blocks(const StepArgs& a) { return (a.X + (a.predraw ? 1 : 0)) * a.Y; }

hipError_t launch_sfac_multi(int precision, int R, const StepArgs* d_tab, const int* d_bstart,
                             int nsys, int total_blocks, size_t lds, hipStream_t s) {
  const dim3 grid(total_blocks), block(kSfacThreads);
  if (precision == RBE_PREC_FP64)
    hipLaunchKernelGGL((k_sfac_multi<true, 1>), grid, block, lds, s, d_tab, d_bstart, nsys);
  else if (R == 4)
    hipLaunchKernelGGL((k_sfac_multi<false, 4>), grid, block, lds, s, d_tab, d_bstart, nsys);
  else if (R == 2)
    hipLaunchKernelGGL((k_sfac_multi<false, 2>), grid, block, lds, s, d_tab, d_bstart, nsys);
  else
    hipLaunchKernelGGL((k_sfac_multi<false, 1>), grid, block, lds, s, d_tab, d_bstart, nsys);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// k_force: the batch split over KS waves; PW particle waves per block, each
// lane holding RP particles, so every frequency's constants (read by all
// lanes at one LDS address) serve RP particles.  Constants are staged in LDS
// in chunks of up to 32 KB.  Small batches (k2reduce): every block first sums
// the group partials of rho itself, in one fixed order, and forms the
// constants in LDS; one extra block (the last) then does the batch-wide work
// instead of forces: rho, the virial tensor and the energy.

// Force constants staged per chunk: 512 of them in either precision (FP32
// 32 B, FP64 64 B each), so that the small-batch mode's p <= 512 constants
// fit one chunk; the FP32 kernel's 16 KB leave room for more blocks per CU
// (10^6 charges, P = 2000: 2.5 % faster than 32 KB).
template <bool F64>
constexpr int force_stage_bytes() { return F64 ? 32768 : 16384; }
// red_raw holds, in turn: the small-batch row sums (scratch of nt
// double2, then rho of Ppad <= 512 double2) and the cross-wave sums (at most
// 8 waves x 64 lanes x RP particles x 3 components, FP32 with RP = 2 or FP64
// with RP = 1: 12 KB).  Blocks have at most 8 waves (KS <= 8, PW = 8 only with
// KS = 1; checked at launch).  Kept this small so that more blocks share a CU.
constexpr int kForceMaxWaves = 8;
constexpr int kForceRedBytes = kForceMaxWaves * kWave * 16 + 512 * 16;
static_assert(kForceRedBytes >= kForceMaxWaves * kWave * 3 * 8, "cross-wave sums must fit");

// Force sums of RP particles per lane over the frequencies [l0, l1) of the
// constants in LDS, FP32 path: h += sin(2 pi (arg(rho)/(2 pi) - f)) c |rho| k,
// which is c Im(exp(-i 2 pi f) rho) k (eq. (appforce)), one sine per pair.
template <int RP>
__device__ __forceinline__ void force_slice32(const FCoef32* sc, int l0, int l1,
                                              const float (&shx)[RP], const float (&shy)[RP],
                                              const float (&shz)[RP], const float (&slx)[RP],
                                              const float (&sly)[RP], const float (&slz)[RP],
                                              float (&hx)[RP], float (&hy)[RP], float (&hz)[RP]) {
#pragma unroll 2
  for (int l = l0; l < l1; ++l) {
    const FCoef32 c = sc[l];
#pragma unroll
    for (int r = 0; r < RP; ++r) {
      const float f = phase_rev(c.m[0], c.m[1], c.m[2], shx[r], shy[r], shz[r], slx[r], sly[r],
                                slz[r]);
      const float sg = __builtin_amdgcn_sinf(c.phi - f);
      hx[r] = fmaf(sg, c.ak[0], hx[r]);
      hy[r] = fmaf(sg, c.ak[1], hy[r]);
      hz[r] = fmaf(sg, c.ak[2], hz[r]);
    }
  }
}

// FP64 path: g += (cos(k.r) c Im rho - sin(k.r) c Re rho) k.
template <int RP>
__device__ __forceinline__ void force_slice64(const FCoef64* sc, int l0, int l1, const double2* sctab,
                                              const double (&sx)[RP], const double (&sy)[RP],
                                              const double (&sz)[RP], double (&gx)[RP],
                                              double (&gy)[RP], double (&gz)[RP]) {
  for (int l = l0; l < l1; ++l) {
    const FCoef64 c = sc[l];
#pragma unroll
    for (int r = 0; r < RP; ++r) {
      const double t = c.m[0] * sx[r] + c.m[1] * sy[r] + c.m[2] * sz[r];
      const double f = t - rint(t);
      double sn, cs;
      sincos2pi(f, sctab, sn, cs);
      const double gg = cs * c.cB - sn * c.cA;
      gx[r] = fma(gg, c.k[0], gx[r]);
      gy[r] = fma(gg, c.k[1], gy[r]);
      gz[r] = fma(gg, c.k[2], gz[r]);
    }
  }
}

// K2: 1 = the block sums the group partials of rho itself (small batches,
// a.k2reduce), 0 = it reads the force constants the structure-factor kernel
// stored, -1 = as a.k2reduce says (multi-system launches, where systems of
// both kinds share a launch).  The fixed modes keep the other mode's code,
// and its registers, out of the kernel.
template <bool F64, int RP, int K2>
__device__ __forceinline__ void force_body(const StepArgs& a, const int bx, const int nbx) {
  const bool k2red = K2 < 0 ? a.k2reduce != 0 : K2 == 1;
  using Coef = typename std::conditional<F64, FCoef64, FCoef32>::type;
  constexpr int kChunk = force_stage_bytes<F64>() / (int)sizeof(Coef);
  static_assert(kChunk >= 512, "the small-batch mode keeps up to 512 constants");
  __shared__ __align__(16) unsigned char red_raw[kForceRedBytes];
  __shared__ __align__(16) Coef scoef[kChunk];
  __shared__ BoxState sbs;
  __shared__ double sh_vs[7][8];
  __shared__ double2 sctab[F64 ? kSinCosTab : 1];
  const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
  // the block's threads from the plan (KS x PW waves, as launched): blockDim
  // is a load from the dispatch packet, whose wait would also wait for the
  // particle loads in flight
  const int PW = a.PW, KS = a.KS, nt = KS * PW * kWave;
  const bool extra = k2red && bx == nbx - 1;
  if (F64 && !extra) fill_sincos_tab(sctab, nt);   // read after the barriers below
  // rows of rho partials left by k_sfac in k2reduce mode
  const double2* rows = a.NG > 1 ? a.gpart : a.partial;
  const int Rr = a.NG > 1 ? a.NG : a.X;
  double2* scratch = reinterpret_cast<double2*>(red_raw);   // nt entries
  double2* srho = scratch + nt;                               // Ppad <= 512 entries

  // Loads issued before the rows are summed, consumed after: this thread's
  // word of the cell values and, in the small-batch mode, the first frequency
  // it forms constants for (a wait for a load also waits for every older one,
  // so loads whose results are needed late go out first)
  const uint64_t bw = tid < kBoxWords ? reinterpret_cast<const uint64_t*>(a.bs)[tid] : 0ull;
  int mf[3] = {0, 0, 0};
  if (k2red && tid < a.p) { mf[0] = a.m[3 * tid]; mf[1] = a.m[3 * tid + 1]; mf[2] = a.m[3 * tid + 2]; }

  if (extra) {
    block_sum_rows<false>(rows, a.Ppad, Rr, a.Ppad, srho, false, scratch, nt, true);
    if (tid < kBoxWords) reinterpret_cast<uint64_t*>(&sbs)[tid] = bw;
    lds_barrier();
    double tv[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int l = tid; l < a.p; l += nt) {
      int mi[3] = {mf[0], mf[1], mf[2]};
      if (l != tid) { mi[0] = a.m[3 * l]; mi[1] = a.m[3 * l + 1]; mi[2] = a.m[3 * l + 2]; }
      const double2 r = srho[l];
      a.rho[l] = r;
      FCoef64 f;
      FCoef32 h;
      double tl[7];
      freq_consts(mi, r, sbs, a.alpha, a.coulomb, a.pf, f, h, tl);
      for (int c = 0; c < 7; ++c) tv[c] += tl[c];
    }
    virial_energy(tv, reinterpret_cast<double*>(scoef), sh_vs, sbs, a.coulomb, a.p,
                  a.self_energy, a.virial6, a.energy, nt);
    return;
  }

  const int pw = wave % PW, ks = wave / PW;
  const int64_t pbase = (int64_t)bx * (kWave * RP * PW) + pw * kWave * RP + lane;
  double xi[RP], yi[RP], zi[RP];
#pragma unroll
  for (int r = 0; r < RP; ++r) {
    const int64_t i = pbase + r * kWave;
    xi[r] = yi[r] = zi[r] = 0.0;
    if (i < a.n) { xi[r] = a.x[i]; yi[r] = a.y[i]; zi[r] = a.z[i]; }
  }
  if (k2red) {
    block_sum_rows<false>(rows, a.Ppad, Rr, a.Ppad, srho, false, scratch, nt, true);
    if (tid < kBoxWords) reinterpret_cast<uint64_t*>(&sbs)[tid] = bw;
    lds_barrier();
    for (int l = tid; l < a.p; l += nt) {
      int mi[3] = {mf[0], mf[1], mf[2]};
      if (l != tid) { mi[0] = a.m[3 * l]; mi[1] = a.m[3 * l + 1]; mi[2] = a.m[3 * l + 2]; }
      FCoef64 f;
      FCoef32 h;
      double tl[7];
      freq_consts(mi, srho[l], sbs, a.alpha, a.coulomb, a.pf, f, h, tl);
      if (F64) reinterpret_cast<FCoef64*>(scoef)[l] = f;
      else reinterpret_cast<FCoef32*>(scoef)[l] = h;
    }
  } else {
    if (tid < kBoxWords) reinterpret_cast<uint64_t*>(&sbs)[tid] = bw;
  }
  lds_barrier();
  const Coef* gcoef = F64 ? reinterpret_cast<const Coef*>(a.fc64)
                          : reinterpret_cast<const Coef*>(a.fc32);
  double gx[RP], gy[RP], gz[RP];
  float shx[RP], shy[RP], shz[RP], slx[RP], sly[RP], slz[RP];
  double sx[RP], sy[RP], sz[RP];
#pragma unroll
  for (int r = 0; r < RP; ++r) {
    gx[r] = gy[r] = gz[r] = 0.0;
    reduce_pos(sbs, xi[r], yi[r], zi[r], sx[r], sy[r], sz[r]);
    if (!F64) {
      split_coord(sx[r], shx[r], slx[r]);
      split_coord(sy[r], shy[r], sly[r]);
      split_coord(sz[r], shz[r], slz[r]);
    }
  }
  float hx[RP], hy[RP], hz[RP];
#pragma unroll
  for (int r = 0; r < RP; ++r) hx[r] = hy[r] = hz[r] = 0.f;
  const int nchunk = k2red ? 1 : (a.pf + kChunk - 1) / kChunk;
  for (int ch = 0; ch < nchunk; ++ch) {
    const int cb = ch * kChunk;
    const int cnt = min(kChunk, a.pf - cb);
    if (!k2red) {
      lds_barrier();
      const int nvec = (int)((size_t)cnt * sizeof(Coef) / 16);
      const uint4* src = reinterpret_cast<const uint4*>(gcoef + cb);
      uint4* dst = reinterpret_cast<uint4*>(scoef);
      for (int v = tid; v < nvec; v += nt) dst[v] = src[v];
      lds_barrier();
    }
    const int per = (cnt + KS - 1) / KS;
    const int l0 = min(cnt, ks * per), l1 = min(cnt, l0 + per);
    if (!F64)
      force_slice32<RP>(reinterpret_cast<const FCoef32*>(scoef), l0, l1, shx, shy, shz, slx, sly,
                        slz, hx, hy, hz);
    else
      force_slice64<RP>(reinterpret_cast<const FCoef64*>(scoef), l0, l1, sctab, sx, sy, sz, gx,
                        gy, gz);
    if (!F64) {
      // fold the chunk's FP32 sums into FP64 (chunks of up to 1024 terms)
#pragma unroll
      for (int r = 0; r < RP; ++r) {
        gx[r] += (double)hx[r]; gy[r] += (double)hy[r]; gz[r] += (double)hz[r];
        hx[r] = hy[r] = hz[r] = 0.f;
      }
    }
  }
  // cross-wave (k-slice) sums, fixed order, then -q_i times the sum.  With the
  // rows summed here, scratch and srho (in red_raw) were last read before the
  // barrier that published the constants; otherwise wait until they are dead.
  if (!k2red) lds_barrier();
  float* redf = reinterpret_cast<float*>(red_raw);
  double* redd = reinterpret_cast<double*>(red_raw);
#pragma unroll
  for (int r = 0; r < RP; ++r) {
    const int idx = (wave * RP + r) * kWave + lane;
    if (F64) { redd[3 * idx] = gx[r]; redd[3 * idx + 1] = gy[r]; redd[3 * idx + 2] = gz[r]; }
    else { redf[3 * idx] = (float)gx[r]; redf[3 * idx + 1] = (float)gy[r]; redf[3 * idx + 2] = (float)gz[r]; }
  }
  lds_barrier();
  if (ks == 0) {
#pragma unroll
    for (int r = 0; r < RP; ++r) {
      const int64_t i = pbase + r * kWave;
      if (i >= a.n) continue;
      double sx2 = 0.0, sy2 = 0.0, sz2 = 0.0;
      for (int k2 = 0; k2 < KS; ++k2) {
        const int idx = ((k2 * PW + pw) * RP + r) * kWave + lane;
        if (F64) { sx2 += redd[3 * idx]; sy2 += redd[3 * idx + 1]; sz2 += redd[3 * idx + 2]; }
        else { sx2 += redf[3 * idx]; sy2 += redf[3 * idx + 1]; sz2 += redf[3 * idx + 2]; }
      }
      const double qi = -a.q[i];
      if (a.accumulate) { a.fx[i] += qi * sx2; a.fy[i] += qi * sy2; a.fz[i] += qi * sz2; }
      else { a.fx[i] = qi * sx2; a.fy[i] = qi * sy2; a.fz[i] = qi * sz2; }
    }
  }
}

template <bool F64, int RP, int K2>
__global__ void __launch_bounds__(1024) k_force(StepArgs a) {
  force_body<F64, RP, K2>(a, blockIdx.x, gridDim.x);
}

template <bool F64, int RP>
__global__ void __launch_bounds__(1024) k_force_multi(const StepArgs* tab, const int* bstart,
                                                      int nsys) {
  __shared__ StepArgs sa;
  const int b = blockIdx.x;
  const int sys = find_system(bstart, nsys, b);
  copy_args(&sa, tab + sys);
  lds_barrier();
  force_body<F64, RP, -1>(sa, b - bstart[sys], bstart[sys + 1] - bstart[sys]);
}

int force_blocks(int precision, const StepArgs& a) {
  const int RP = precision == RBE_PREC_FP64 ? 1 : 2;
  const int64_t per_block = (int64_t)kWave * RP * a.PW;
  return (int)((a.n + per_block - 1) / per_block + (a.k2reduce ? 1 : 0));
}

hipError_t launch_force(int precision, const StepArgs& a, hipStream_t s, const LaunchEvents& ev) {
  if (a.KS * a.PW > kForceMaxWaves) return hipErrorInvalidConfiguration;
  const dim3 block(a.KS * a.PW * kWave);
  const dim3 grid((unsigned)force_blocks(precision, a));
  const void* fn;
  if (precision == RBE_PREC_FP64)
    fn = a.k2reduce ? reinterpret_cast<const void*>(&k_force<true, 1, 1>)
                    : reinterpret_cast<const void*>(&k_force<true, 1, 0>);
  else
    fn = a.k2reduce ? reinterpret_cast<const void*>(&k_force<false, 2, 1>)
                    : reinterpret_cast<const void*>(&k_force<false, 2, 0>);
  void* args[] = {const_cast<StepArgs*>(&a)};
  return hipExtLaunchKernel(fn, grid, block, args, 0, s, ev.start, ev.stop, 0);
}

// every system of a multi launch must use the same force block shape (KS, PW)
hipError_t launch_force_multi(int precision, int threads, const StepArgs* d_tab,
                              const int* d_bstart, int nsys, int total_blocks, hipStream_t s) {
  if (threads > kForceMaxWaves * kWave) return hipErrorInvalidConfiguration;
  const dim3 grid(total_blocks), block(threads);
  if (precision == RBE_PREC_FP64)
    hipLaunchKernelGGL((k_force_multi<true, 1>), grid, block, 0, s, d_tab, d_bstart, nsys);
  else
    hipLaunchKernelGGL((k_force_multi<false, 2>), grid, block, 0, s, d_tab, d_bstart, nsys);
  return hipGetLastError();
}


// ---------------------------------------------------------------------------
// k_step: the whole Fourier-space step of one system in ONE launch, for
// systems whose particle chunks fit one LDS tile and whose batch fits one
// block (every block of the grid must be resident at once, see below).  Its
// plan has its own chunks: up to 512 particles, about 64 of them.  Per block:
//   1. its chunk's particles in LDS (split or reduced coordinates and FP64
//      charges, kept to the end), the cell tables and the batch in LDS, as
//      k_sfac builds them (section 4.2 eq. (S), (psf), (probexpression));
//   2. the chunk's rho partial (eq. (U1fourier)) -> partial[x], then one
//      count on the ready word;
//   3. once all X partials are in, every block sums the X rows in chunk
//      order (so every block holds the same rho, bit for bit) and forms the
//      force constants in LDS; block 0 also writes rho, the batch, the
//      constants, the virial tensor and the energy (eq. (apppress));
//   4. the forces of its particles (eq. (appforce)) from the LDS copies: no
//      second launch, no reload of positions, one grid-wide wait.
// Counters (zero between launches, each on its own line, cnt_index): ready
// (one count per block), done (blocks past the wait; the last one resets
// ready and itself), and the error word of the bounded wait (a block that
// gives up sets it and skips its forces).
// Residency: the grid is at most the number of blocks the device holds at
// once (checked by the host against the occupancy of this kernel); a plain
// launch is used (a cooperative launch measured ~20 us of runtime overhead
// per step here).  Blocks that would not get a compute unit while others
// wait (another application holding the device) make the waits give up:
// an error, not a hang.

constexpr uint32_t kSpinCap = 1u << 22;      // polls (~0.2 s) before a wait gives up

// LDS of k_step: particle tile | FP64 charges | batch | tables, then rho and
// the force constants | scratch (block partial, row sums, virial summands,
// cross-wave force sums)
constexpr size_t kStepTile = (size_t)kTile * 32;
constexpr size_t kStepQ = (size_t)kTile * 8;
constexpr size_t kStepRed = (size_t)7 * kSfacThreads * 8;
__host__ __device__ static size_t step_sm_bytes(const StepArgs& a) {
  return ((size_t)a.Ppad * 3 * sizeof(int) + 15) / 16 * 16;
}
__host__ __device__ static size_t step_r2_bytes(const StepArgs& a) {
  const int cap = a.mcap[0] + a.mcap[1] + a.mcap[2];
  const size_t tab = ((size_t)(4 * cap + 3) * sizeof(double) + 15) / 16 * 16;
  const size_t rc = (size_t)a.Ppad * sizeof(double2) + (size_t)a.Ppad * sizeof(FCoef64);
  return tab > rc ? tab : rc;
}
size_t step_lds_bytes(const StepArgs& a) {
  return kStepTile + kStepQ + step_sm_bytes(a) + step_r2_bytes(a) + kStepRed;
}

// Thread 0 polls *c (coherent loads) until it reaches target; false if the
// bounded wait gave up.  Block-uniform result; reached by every thread.
__device__ __forceinline__ bool wait_count(uint32_t* c, uint32_t target, int* sh_flag) {
  if (threadIdx.x == 0) {
    int ok = 0;
    for (uint32_t it = 0; it < kSpinCap; ++it) {
      if (__hip_atomic_load(c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) {
        ok = 1;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    *sh_flag = ok;
  }
  lds_barrier();
  return *sh_flag != 0;
}

// Every thread's coherent stores complete (waitcnt), then one increment of
// *c: whoever sees the new count may read them.
__device__ __forceinline__ void publish(uint32_t* c) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0)
    (void)__hip_atomic_fetch_add(c, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool F64, int R, bool TRI>
__global__ void __launch_bounds__(kSfacThreads) k_step(StepArgs a) {
  using Coef = typename std::conditional<F64, FCoef64, FCoef32>::type;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  __shared__ BoxState sbs;
  __shared__ TriCell stc;
  __shared__ double sh_T[3];
  __shared__ int sh_flag;
  __shared__ double sh_vs[7][8];
  __shared__ double2 sctab[F64 ? kSinCosTab : 1];
  const int tid = threadIdx.x, wave = tid / kWave, lane = tid % kWave;
  const int x = blockIdx.x;
  const int KB = a.KB, SUB = kSfacWaves / KB, FB = KB * kWave * R;   // FB = Ppad >= p
  if (F64) fill_sincos_tab(sctab, kSfacThreads);   // read after the barriers below
  const TriCell* tc = stage_tri(a, &stc);
  unsigned char* tile = lds_raw;
  double* qd = reinterpret_cast<double*>(lds_raw + kStepTile);
  int* sm = reinterpret_cast<int*>(lds_raw + kStepTile + kStepQ);
  unsigned char* r2 = lds_raw + kStepTile + kStepQ + step_sm_bytes(a);
  double* tabs = reinterpret_cast<double*>(r2);
  double2* srho = reinterpret_cast<double2*>(r2);
  Coef* scoef = reinterpret_cast<Coef*>(r2 + (size_t)a.Ppad * sizeof(double2));
  unsigned char* red_raw = r2 + step_r2_bytes(a);
  double2* red2 = reinterpret_cast<double2*>(red_raw);
  double* redd = reinterpret_cast<double*>(red_raw);
  float* redf = reinterpret_cast<float*>(red_raw);

  // ---- 1. the cell's sides, then the chunk's particles (loads issued now,
  // used after the tables): the sides may be global loads, and a wait for a
  // load also waits for every older one, so they go out first
  double lc[3];
  box_source(a, lc);
  __builtin_amdgcn_sched_barrier(0);
  const int64_t c0 = (int64_t)x * a.chunk;
  const int cnt = (int)min((int64_t)a.chunk, a.n - c0);        // 1 .. kTile (plan)
  double px = 0.0, py = 0.0, pz = 0.0, pq = 0.0;
  if (tid < cnt) {
    px = a.x[c0 + tid]; py = a.y[c0 + tid]; pz = a.z[c0 + tid]; pq = a.q[c0 + tid];
  }
  // the batch's Philox outputs beside the table build, in the tile region
  // (written only after the draw)
  const bool su_on = a.sample && (size_t)FB * 4 * sizeof(uint64_t) <= kStepTile;
  uint64_t* su = reinterpret_cast<uint64_t*>(tile);
  if (a.sample || a.box_src != BOX_COMMITTED) {
    if (su_on) slice_uniforms(su, FB, 0, a.p, a.seed, a.sysid, a.step, kSfacThreads);
    build_tables(lc, tc, a.alpha, a.tail_ln, a.mcap, tabs, &sbs, sh_T, kSfacThreads, true);
    if (x == 0 && a.box_src != BOX_COMMITTED) commit_cell(sbs, a.bs, tid);
  } else {
    load_box(sbs, a.bs, tid);
    lds_barrier();
  }
  for (int l = tid; l < FB; l += kSfacThreads) {
    int mv[3] = {0, 0, 0};
    if (l < a.p) {
      if (a.sample) {
        draw_frequency<TRI>(sbs, tabs, a.seed, a.sysid, a.step, l, mv, su_on ? su + l : nullptr,
                            FB);
        if (x == 0) { a.m[3 * l] = mv[0]; a.m[3 * l + 1] = mv[1]; a.m[3 * l + 2] = mv[2]; }
      } else {
        mv[0] = a.m[3 * l]; mv[1] = a.m[3 * l + 1]; mv[2] = a.m[3 * l + 2];
      }
    }
    sm[3 * l] = mv[0]; sm[3 * l + 1] = mv[1]; sm[3 * l + 2] = mv[2];
  }
  if (su_on) lds_barrier();                 // su is read before the tile overwrites it
  // the whole tile, zero beyond the chunk (thread j owns entry j: blockDim
  // = kTile); the structure-factor loop reads the first cntp entries
  const int cntp = F64 ? (cnt + SUB - 1) / SUB * SUB
                       : (cnt + SUB * kKahan - 1) / (SUB * kKahan) * (SUB * kKahan);
  static_assert(kSfacThreads == kTile, "one tile entry per thread");
  {
    if (!F64) {
      float4 u = make_float4(0.f, 0.f, 0.f, 0.f), v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (tid < cnt) {
        double sx, sy, sz;
        reduce_pos(sbs, px, py, pz, sx, sy, sz);
        split_coord(sx, u.x, v.x);
        split_coord(sy, u.y, v.y);
        split_coord(sz, u.z, v.z);
        u.w = (float)pq;
      }
      reinterpret_cast<float4*>(tile)[tid] = u;
      reinterpret_cast<float4*>(tile)[kTile + tid] = v;
    } else {
      double2 u = make_double2(0.0, 0.0), v = make_double2(0.0, 0.0);
      if (tid < cnt) {
        double sx, sy, sz;
        reduce_pos(sbs, px, py, pz, sx, sy, sz);
        u = make_double2(sx, sy);
        v = make_double2(sz, pq);
      }
      reinterpret_cast<double2*>(tile)[tid] = u;
      reinterpret_cast<double2*>(tile)[kTile + tid] = v;
    }
    qd[tid] = tid < cnt ? pq : 0.0;
  }
  lds_barrier();

  // ---- 2. rho partial of the chunk: lane owns frequencies kg*64R + r*64 + lane
  const int kg = wave % KB, sub = wave / KB;
  double2 part[R];
  if (!F64) {
    float mx[R], my[R], mz[R], SA[R], CA[R], SB[R], CB[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int sl = kg * kWave * R + r * kWave + lane;
      mx[r] = (float)sm[3 * sl]; my[r] = (float)sm[3 * sl + 1]; mz[r] = (float)sm[3 * sl + 2];
      SA[r] = CA[r] = SB[r] = CB[r] = 0.f;
    }
    const float4* tA = reinterpret_cast<const float4*>(tile);
    sfac_tile32<R>(tA, tA + kTile, cntp, sub, SUB, mx, my, mz, SA, CA, SB, CB);
#pragma unroll
    for (int r = 0; r < R; ++r)
      part[r] = make_double2((double)SA[r] - (double)CA[r], (double)SB[r] - (double)CB[r]);
  } else {
    double mx[R], my[R], mz[R], A[R], B[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int sl = kg * kWave * R + r * kWave + lane;
      mx[r] = (double)sm[3 * sl]; my[r] = (double)sm[3 * sl + 1]; mz[r] = (double)sm[3 * sl + 2];
      A[r] = B[r] = 0.0;
    }
    const double2* tA = reinterpret_cast<const double2*>(tile);
    sfac_tile64<R>(tA, tA + kTile, cntp, sub, SUB, sctab, mx, my, mz, A, B);
#pragma unroll
    for (int r = 0; r < R; ++r) part[r] = make_double2(A[r], B[r]);
  }
  store_block_partial<R>(part, red2, KB, SUB, a.partial + (int64_t)x * a.Ppad);

  // ---- 3. every block's partial stored: one count per block; then every
  // block sums all X chunk rows itself, in chunk order (each block gets the
  // same rho, bit for bit), and forms the force constants in LDS
  uint32_t* ready = a.cnt + cnt_index(a, CNT_READY);
  uint32_t* done = a.cnt + cnt_index(a, CNT_DONE);
  uint32_t* errw = a.cnt + cnt_index(a, CNT_ERR);
  publish(ready);
  const bool ok = wait_count(ready, (uint32_t)a.X, &sh_flag);
  if (tid == 0) {
    if (!ok) __hip_atomic_fetch_or(errw, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (__hip_atomic_fetch_add(done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ==
        (uint32_t)a.X - 1u) {
      __hip_atomic_store(ready, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (!ok) return;
  block_sum_rows<true, 16>(a.partial, a.Ppad, a.X, a.Ppad, srho, false, red2, kSfacThreads);
  double tv[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int l = tid; l < a.p; l += kSfacThreads) {
    const int mi[3] = {sm[3 * l], sm[3 * l + 1], sm[3 * l + 2]};
    const double2 r = srho[l];
    FCoef64 f;
    FCoef32 h;
    double tl[7];
    freq_consts(mi, r, sbs, a.alpha, a.coulomb, a.pf, f, h, tl);
    if (F64) reinterpret_cast<FCoef64*>(scoef)[l] = f;
    else reinterpret_cast<FCoef32*>(scoef)[l] = h;
    if (x == 0) {
      a.rho[l] = r;
      a.fc64[l] = f;
      a.fc32[l] = h;
      for (int c = 0; c < 7; ++c) tv[c] += tl[c];
    }
  }
  // ---- 4. block 0: the virial tensor and the energy (the self term from the
  // host, or from the charge sums on the device)
  if (x == 0) {
    const double self = a.qsum_dev ? -a.coulomb * a.qsum_dev[2] * sqrt(a.alpha / M_PI)
                                   : a.self_energy;
    virial_energy(tv, redd, sh_vs, sbs, a.coulomb, a.p, self, a.virial6, a.energy, kSfacThreads);
  }
  lds_barrier();

  // ---- 5. forces: KS waves split the batch, 8/KS particle waves side by
  // side, rounds of (8/KS) x 64 x RP particles (one round when the plan's KS
  // is chosen for the chunk)
  constexpr int RP = F64 ? 1 : 2;
  const int KS = a.KS, PWp = kSfacWaves / KS;
  const int ks = wave / PWp, pw = wave % PWp;
  const int per = (a.pf + KS - 1) / KS;
  const int l0 = min(a.pf, ks * per), l1 = min(a.pf, l0 + per);
  const int rounds = (cnt + PWp * kWave * RP - 1) / (PWp * kWave * RP);
  for (int rd = 0; rd < rounds; ++rd) {
    const int jbase = (rd * PWp + pw) * kWave * RP + lane;
    double gx[RP], gy[RP], gz[RP];
    float shx[RP], shy[RP], shz[RP], slx[RP], sly[RP], slz[RP];
    double sx[RP], sy[RP], sz[RP];
#pragma unroll
    for (int r = 0; r < RP; ++r) {
      const int j = min(jbase + r * kWave, kTile - 1);     // beyond cnt: a padding entry, not stored
      gx[r] = gy[r] = gz[r] = 0.0;
      if (!F64) {
        const float4 u = reinterpret_cast<const float4*>(tile)[j];
        const float4 v = reinterpret_cast<const float4*>(tile)[kTile + j];
        shx[r] = u.x; shy[r] = u.y; shz[r] = u.z; slx[r] = v.x; sly[r] = v.y; slz[r] = v.z;
      } else {
        const double2 u = reinterpret_cast<const double2*>(tile)[j];
        const double2 v = reinterpret_cast<const double2*>(tile)[kTile + j];
        sx[r] = u.x; sy[r] = u.y; sz[r] = v.x;
      }
    }
    if (!F64) {
      float hx[RP], hy[RP], hz[RP];
#pragma unroll
      for (int r = 0; r < RP; ++r) hx[r] = hy[r] = hz[r] = 0.f;
      force_slice32<RP>(reinterpret_cast<const FCoef32*>(scoef), l0, l1, shx, shy, shz, slx, sly,
                        slz, hx, hy, hz);
#pragma unroll
      for (int r = 0; r < RP; ++r) {
        gx[r] += (double)hx[r]; gy[r] += (double)hy[r]; gz[r] += (double)hz[r];
      }
    } else {
      force_slice64<RP>(reinterpret_cast<const FCoef64*>(scoef), l0, l1, sctab, sx, sy, sz, gx, gy,
                        gz);
    }
    // cross-wave sums in slice order, then -q_i times the sum
    lds_barrier();                          // red is free (virial summands, last round)
#pragma unroll
    for (int r = 0; r < RP; ++r) {
      const int idx = (wave * RP + r) * kWave + lane;
      if (F64) { redd[3 * idx] = gx[r]; redd[3 * idx + 1] = gy[r]; redd[3 * idx + 2] = gz[r]; }
      else { redf[3 * idx] = (float)gx[r]; redf[3 * idx + 1] = (float)gy[r]; redf[3 * idx + 2] = (float)gz[r]; }
    }
    lds_barrier();
    if (ks == 0) {
#pragma unroll
      for (int r = 0; r < RP; ++r) {
        const int j = jbase + r * kWave;
        if (j >= cnt) continue;
        double sx2 = 0.0, sy2 = 0.0, sz2 = 0.0;
        for (int k2 = 0; k2 < KS; ++k2) {
          const int idx = ((k2 * PWp + pw) * RP + r) * kWave + lane;
          if (F64) { sx2 += redd[3 * idx]; sy2 += redd[3 * idx + 1]; sz2 += redd[3 * idx + 2]; }
          else { sx2 += redf[3 * idx]; sy2 += redf[3 * idx + 1]; sz2 += redf[3 * idx + 2]; }
        }
        const int64_t i = c0 + j;
        const double qi = -qd[j];
        if (a.accumulate) { a.fx[i] += qi * sx2; a.fy[i] += qi * sy2; a.fz[i] += qi * sz2; }
        else { a.fx[i] = qi * sx2; a.fy[i] = qi * sy2; a.fz[i] = qi * sz2; }
      }
    }
  }
}

bool step_supported(int precision, const StepArgs& a) {
  return a.Y == 1 && a.Ppad <= 512 && a.chunk <= kTile && a.KS * a.PW == kSfacWaves &&
         (precision == RBE_PREC_FP64 ? a.R == 1 : (a.R == 1 || a.R == 2 || a.R == 4));
}

template <bool TRI>
static const void* step_kernel(int precision, int R) {
  if (precision == RBE_PREC_FP64) return reinterpret_cast<const void*>(&k_step<true, 1, TRI>);
  if (R == 4) return reinterpret_cast<const void*>(&k_step<false, 4, TRI>);
  if (R == 2) return reinterpret_cast<const void*>(&k_step<false, 2, TRI>);
  return reinterpret_cast<const void*>(&k_step<false, 1, TRI>);
}
static const void* step_kernel(int precision, const StepArgs& a) {
  return a.tri_mode ? step_kernel<true>(precision, a.R) : step_kernel<false>(precision, a.R);
}

hipError_t step_max_blocks(int precision, const StepArgs& a, int* max_blocks) {
  int dev = 0, cus = 0, per = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, step_kernel(precision, a), kSfacThreads,
                                                   step_lds_bytes(a));
  *max_blocks = cus * per;
  return e;
}

hipError_t launch_step(int precision, const StepArgs& a, hipStream_t s, const LaunchEvents& ev) {
  void* args[] = {const_cast<StepArgs*>(&a)};
  const dim3 grid(a.X), block(kSfacThreads);
  const size_t lds = step_lds_bytes(a);
  return hipExtLaunchKernel(step_kernel(precision, a), grid, block, args, lds, s, ev.start, ev.stop,
                            0);
}


// ---------------------------------------------------------------------------
// batch moments of the estimator (Proposition 1 on the device): per particle
// and component the running sums of F* and F*^2 over batches, and of the
// isotropic P2* = tr W/(3V) and its square (thread 0)

__global__ void k_moments(const double* __restrict__ fx, const double* __restrict__ fy,
                          const double* __restrict__ fz, const double* __restrict__ vir, double V,
                          int64_t n, double* __restrict__ sum, double* __restrict__ sq,
                          double* __restrict__ psum) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const double f[3] = {fx[i], fy[i], fz[i]};
    for (int c = 0; c < 3; ++c) {
      sum[c * n + i] += f[c];
      sq[c * n + i] += f[c] * f[c];
    }
  }
  if (i == 0) {
    const double P2 = (vir[0] + vir[1] + vir[2]) / (3.0 * V);
    psum[0] += P2;
    psum[1] += P2 * P2;
  }
}

hipError_t launch_moments(const double* fx, const double* fy, const double* fz, const double* vir,
                          double V, int64_t n, double* sum, double* sq, double* psum,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_moments, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, fx, fy, fz, vir,
                     V, n, sum, sq, psum);
  return hipGetLastError();
}

}  // namespace rbe
