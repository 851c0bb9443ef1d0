// Internal declarations shared by the C ABI layer and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "../../include/rbe.h"

namespace rbe {

// Largest |m| per axis the sampler tables may hold: keeps the three axes'
// running-sum tables (4*mcap+1 doubles each, 31 KB in all) in LDS next to the
// particle tiles, and |m| <= 2048 as the FP32 two-part phase product needs.
constexpr int kMaxMcut = 320;
constexpr int kWave = 64;
constexpr int kSfacThreads = 512;     // structure-factor kernel: 8 waves
constexpr int kSfacWaves = kSfacThreads / 64;
constexpr int kTile = 512;            // particles per LDS tile
constexpr int kKahan = 16;            // plain FP32 run between compensated folds

// A triclinic cell (appendix C), as the host prepares it from (lx, ly, lz,
// xy, xz, yz): h = [[lx, xy, xz], [0, ly, yz], [0, 0, lz]] (columns a, b, c).
struct TriCell {
  int32_t on;        // 1: this cell is triclinic
  int32_t pad;
  double tilt[3];    // xy, xz, yz
  double hinv[6];    // h^-1 (upper triangular): xx, xy, xz, yy, yz, zz
  double A[6];       // Q(m) = |2 pi h^-T m|^2/(4 alpha) = m^T A m: xx, yy, zz, xy, xz, yz
  double d[3];       // separable envelope exp(-sum d_j m_j^2) <= exp(-Q(m))
  double S;          // normaliser: sum over m != 0 of exp(-Q(m))
};

// Cell-derived values (section 4.2 eq. (S), (psf); appendix C sampling).
struct BoxState {
  double l[3];       // side lengths
  double inv_l[3];   // 1/l
  double V;          // volume
  double S;          // normaliser: sum over k != 0 of exp(-k^2/(4 alpha))
  double H[3];       // one-axis sums (m = 0 term included) of the sampler tables
  double case_w[3];  // weights of the first-nonzero-axis cases (rectangular: sum = S;
                     // triclinic: the envelope's law)
  int32_t mcut[3];   // table half-widths in use
  int32_t err;       // bit 0: cell outside the table capacity
  TriCell tri;       // triclinic cells (tri.on), else zero
};

// Force-pass constants of one frequency, FP32 path (32 B: one scalar load).
struct alignas(32) FCoef32 {
  float m[3];        // m (exact small integers)
  float phi;         // arg(rho) / (2 pi), revolutions in [-1/2, 1/2]
  float ak[3];       // c |rho| k with c = C (S/p) 4 pi / (V k^2), k = 2 pi m / l
  float pad;
};
// FP64 path.
struct alignas(64) FCoef64 {
  double m[3];
  double cA, cB;
  double k[3];
};

enum BoxSource : int32_t { BOX_COMMITTED = 0, BOX_ARGS = 1, BOX_PTR = 2 };

// A batch drawn ahead of time by an extra block of the structure-factor
// kernel: the draw of step `step` for the cell `bs` (that launch's cell).  The
// next launch uses it instead of redrawing when its step and cell match
// exactly, which gives the identical batch.  Two slots, by step parity, so a
// launch reads one while its extra block fills the other.
struct PreDraw {
  BoxState bs;
  uint64_t step;
  int32_t valid;
  int32_t pad;
};

// Everything one Fourier-space evaluation of one system needs (passed by value
// as the kernel argument).
struct StepArgs {
  const double* x; const double* y; const double* z;
  const double* q; const float* qf;
  double* fx; double* fy; double* fz;
  double* virial6; double* energy;
  int32_t box_src;      // BoxSource
  int32_t sample;       // 1: draw the batch of `step`; 0: use m as stored
  int32_t accumulate;   // forces: add instead of overwrite
  int32_t p;            // frequencies drawn per step (rho, virial and energy: weight S/p)
  int32_t pf;           // the first pf of them serve the forces (weight S/pf), pf <= p
  int64_t n;
  double box_arg[3];
  int32_t tri_mode;     // 1: a triclinic-cell context
  TriCell tri_arg;      // with BOX_ARGS: the triclinic cell (tri_arg.on), box_arg its sides
  const double* box_ptr;
  double alpha, coulomb, self_energy, tail_ln;
  const double* qsum_dev;   // non-NULL: the self term from these charge sums (sum q^2 at [2])
  uint64_t seed, sysid, step;
  int32_t mcap[3];
  int32_t tab_stride;
  // launch plan
  int32_t X, Y, KB, GX, NG, chunk, Ppad, KS;
  int32_t R;            // frequencies per lane in k_sfac (FP32: 1, 2 or 4)
  int32_t PW;           // particle waves per k_force block
  int32_t k2reduce;     // 1: the force kernel sums the NG group partials itself
  int32_t predraw;      // 1: an extra k_sfac block draws the batch of step + 1 ahead
  int32_t use_pre;      // 1: k_sfac may take the batch drawn ahead
  // context-owned state and scratch
  BoxState* bs; double* tab;
  int32_t* m;
  double2* partial;     // [X][Ppad]
  double2* gpart;       // [NG][Ppad]
  double2* rho;         // [p]
  double* terms;        // [p][8]
  FCoef32* fc32; FCoef64* fc64;
  uint32_t* cnt;        // arrival counters, zero between launches, one per
                        // kCntStride words (cnt_index): [Y*NG] group arrivals,
                        // [Y] slice arrivals, [1] batch arrivals, and the
                        // single launch's ready / done / error words
  PreDraw* pre;         // [2] batches drawn ahead: step and cell, by step parity
  int32_t* m_pre;       // [2][3p]
  // online Metropolis-Hastings sampler (sampler == RBE_SAMPLER_MH): the
  // chains' states at the previous sampled step (read) and at this one
  // (written); mh_init: no state yet, the chains start from an exact draw
  int32_t sampler, mh_iters, mh_init;
  const int32_t* mh_old;
  int32_t* mh_new;
};

// Every arrival counter sits on its own 256-byte line (64 words), so that
// blocks arriving at different counters at the same moment do not queue on
// one line.  Counter k of the list above is word k * kCntStride.
constexpr int kCntStride = 64;
enum CntKind { CNT_GROUP = 0, CNT_SLICE, CNT_BATCH, CNT_READY, CNT_DONE, CNT_ERR };
__host__ __device__ inline int64_t cnt_index(const StepArgs& a, CntKind k, int i = 0) {
  const int64_t base = k == CNT_GROUP ? 0 : (k == CNT_SLICE ? (int64_t)a.Y * a.NG
                                                            : (int64_t)a.Y * a.NG + a.Y + (k - CNT_BATCH));
  return (base + i) * kCntStride;
}
// words of the counter array for a plan
inline int64_t cnt_words(int Y, int NG) { return ((int64_t)Y * NG + Y + 4) * kCntStride; }

size_t sfac_lds_bytes(const StepArgs& a);

// Start and stop events of one launch for kernel timing: the launch itself
// timestamps them (hipExtLaunchKernel), so they bracket the kernel's own
// execution and not the queue around it.  Null when timing is off.
struct LaunchEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};

// charge sums (sum q, sum |q|, sum q^2) into d_out3, the FP32 copy of the
// charges (d_qf, nullable), and nzero words of d_zero cleared first
hipError_t launch_qsum(const double* d_q, float* d_qf, double* d_out3, int64_t n, hipStream_t s,
                       uint32_t* d_zero = nullptr, int64_t nzero = 0);
// standalone table and draw kernels (used when a result is read before the
// fused kernel has run)
hipError_t launch_tables(const StepArgs& a, hipStream_t s, const LaunchEvents& ev = {});
hipError_t launch_sample(const StepArgs& a, hipStream_t s, const LaunchEvents& ev = {});
// the two kernels of a step
hipError_t launch_sfac(int precision, const StepArgs& a, hipStream_t s,
                       const LaunchEvents& ev = {});
hipError_t launch_force(int precision, const StepArgs& a, hipStream_t s,
                        const LaunchEvents& ev = {});
// the whole step in one launch (k_step): whether the plan allows
// it (particle chunks within one LDS tile, the batch within one block, the
// force layout of 8 waves), how many of its blocks fit the device at once,
// its LDS bytes, the launch
bool step_supported(int precision, const StepArgs& a);
hipError_t step_max_blocks(int precision, const StepArgs& a, int* max_blocks);
size_t step_lds_bytes(const StepArgs& a);
hipError_t launch_step(int precision, const StepArgs& a, hipStream_t s,
                       const LaunchEvents& ev = {});
// running sums of F*, F*^2 (per particle and component) and of P2*, P2*^2
hipError_t launch_moments(const double* fx, const double* fy, const double* fz, const double* vir,
                          double V, int64_t n, double* sum, double* sq, double* psum,
                          hipStream_t s);
// many systems per launch (served batching)
int sfac_blocks(const StepArgs& a);
int force_blocks(int precision, const StepArgs& a);
hipError_t launch_sfac_multi(int precision, int R, const StepArgs* d_tab, const int* d_bstart,
                             int nsys, int total_blocks, size_t lds, hipStream_t s);
hipError_t launch_force_multi(int precision, int threads, const StepArgs* d_tab,
                              const int* d_bstart, int nsys, int total_blocks, hipStream_t s);

// Standalone table / draw launches that must precede a step's kernels (the
// Metropolis-Hastings chains, draws from a frozen cell under sample reuse).
struct PendingLaunch {
  int32_t frozen = 0, tables = 0, sample = 0;
  StepArgs frozen_args{}, table_args{}, sample_args{};
};

// host side of rbe_forces_pressure without the step's own launches: the
// arguments of its kernels, with the pending cell and draw folded in (the
// context's pending state is consumed as by a launch).  Standalone table and
// draw work the step needs first is launched at once when pre is NULL, else
// recorded in *pre for kspace_run_pending, which the caller must launch on
// the context's stream before the step's kernels (after whatever writes the
// cell they read).
rbe_status kspace_step_args(rbe_ctx c, const double* d_x, const double* d_y, const double* d_z,
                            double* d_fx, double* d_fy, double* d_fz, int accumulate,
                            double* d_virial6, double* d_energy, StepArgs* out,
                            PendingLaunch* pre, bool single_launch = false);
rbe_status kspace_run_pending(rbe_ctx c, const PendingLaunch& pre);
int kspace_precision(rbe_ctx c);
// device bytes rbe_init allocates for this configuration (each buffer rounded
// up to 256 bytes)
int64_t kspace_footprint(const rbe_config* cfg, const double* box);
// The triclinic cell of h6 = (lx, ly, lz, xy, xz, yz): h^-1, the quadratic
// form A of Q(m), the envelope d and the normaliser S (its Poisson-summed
// form over real-space cell vectors); false for a degenerate cell.
bool triclinic_cell(double alpha, const double* h6, TriCell* t);
// rbe_init's checks of cfg and box (all but neutrality, which needs the
// charges) and its launch plan and constants in *a (pointers left NULL);
// *single: whether the single-launch step applies.  No device memory.
rbe_status kspace_plan(const rbe_config* cfg, const double* box, StepArgs* a, bool* single);

}  // namespace rbe
