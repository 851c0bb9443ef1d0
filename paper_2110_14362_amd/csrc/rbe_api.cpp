// C ABI of the random batch Ewald Fourier-space step: argument checks,
// context ownership and the launch sequence.  Declarations and contracts are
// in include/rbe.h.
#include "rbe_internal.h"
#include <cstddef>

#include <algorithm>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

using namespace rbe;

struct rbe_ctx_s {
  rbe_config cfg;
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t n = 0;
  int p = 0;                // frequencies drawn per step: max(cfg.p, cfg.p_pressure)
  int pf = 0;               // the first pf of them serve the forces: cfg.p
  int mcap[3] = {0, 0, 0};
  int tab_stride = 0;
  double tail_ln = 0.0;
  double self_energy = 0.0;
  bool have_k = false;
  // work recorded by rbe_rescale_box* / rbe_sample_k, executed by the next
  // kernel that needs it (the fused step, or the standalone table/draw
  // kernels when a result is read first)
  int32_t pend_box = BOX_COMMITTED;
  double pend_box_val[3] = {0, 0, 0};
  TriCell pend_tri{};        // with BOX_ARGS in triclinic mode: the cell
  int mcap_tri[3] = {0, 0, 0};
  const double* pend_box_ptr = nullptr;
  bool pend_sample = false;
  uint64_t pend_step = 0;
  StepArgs a{};             // launch plan, scratch pointers and constants
  // device memory (owned)
  double* d_q = nullptr;
  float* d_qf = nullptr;
  double* d_qsum = nullptr;      // 3 doubles
  BoxState* d_bs = nullptr;
  double* d_tab = nullptr;
  int32_t* d_m = nullptr;        // 3p
  double2* d_partial = nullptr;  // X * Ppad
  double2* d_gpart = nullptr;    // NG * Ppad
  double2* d_rho = nullptr;      // p
  double* d_terms = nullptr;     // 8p
  FCoef32* d_fc32 = nullptr;     // p
  FCoef64* d_fc64 = nullptr;     // p
  uint32_t* d_cnt = nullptr;     // Y*NG + Y + 1
  PreDraw* d_pre = nullptr;
  int32_t* d_m_pre = nullptr;    // 3p
  bool pre_valid = false;        // a batch for step pre_step was drawn ahead (device checks the cell)
  uint64_t pre_step = 0;
  // the cell of the last launch as the host knows it (passed by value), so
  // that a changed cell skips the drawn-ahead batch without a device check
  bool last_cell_known = false;
  double last_cell[6] = {0, 0, 0, 0, 0, 0};
  // online Metropolis-Hastings sampler: chain states [2][3p], the buffer
  // holding the latest state, and whether the chains have started
  int32_t sampler = RBE_SAMPLER_EXACT;
  int32_t mh_iters = 1;
  int32_t* d_chain = nullptr;
  int mh_cur = 0;
  bool mh_started = false;
  // sample reuse (section 4.3, parallel strategy): draws of the steps of one
  // block [kM, (k+1)M) all use the cell of the block's first sampled step
  int32_t reuse = 1;
  // the whole step in one launch (k_step) where the plan and the device allow
  // it (fused_ok), unless switched off (rbe_set_fused)
  bool fused_ok = false;
  bool fused_on = false;
  // the single launch's own plan: chunks (fX of them, fchunk particles each)
  // and force layout (fKS frequency slices)
  int fX = 0, fchunk = 0, fKS = 0, fPW = 0;
  bool frozen_valid = false;
  uint64_t frozen_block = 0;
  BoxState* d_bs_frozen = nullptr;   // that cell's values and tables
  double* d_tab_frozen = nullptr;
  // kernel timing (rbe_timing_enable)
  static constexpr int kKinds = 5;
  int timing_cap = 0;
  std::vector<hipEvent_t> ev[kKinds];
  int ev_used[kKinds] = {0, 0, 0, 0, 0};
};

namespace {

thread_local std::string g_err;

}  // namespace

namespace rbe {
rbe_status set_error(rbe_status st, const char* msg) {
  g_err = msg;
  return st;
}
}  // namespace rbe

namespace {

rbe_status fail(rbe_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
rbe_status fail(rbe_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

rbe_status hip_fail(hipError_t e, const char* what) {
  return fail(RBE_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(call, what)                        \
  do {                                             \
    hipError_t e_ = (call);                        \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// ceil(sqrt(53 ln2 * alpha) * l / pi): the half-width of a one-axis table
double axis_mcut(double tail_ln, double alpha, double l) {
  return std::ceil(std::sqrt(tail_ln * alpha * l * l) / M_PI);
}

// The triclinic cell of a host box (6 values), checked: sides positive and
// finite, tilts bounded, envelope tables within the capacity set at init
// (capacity 0: no check).
rbe_status check_triclinic(double alpha, double tail_ln, const double* box, const int* cap,
                           TriCell* t, int mc_out[3]) {
  for (int a = 0; a < 3; ++a)
    if (!finite_pos(box[a])) return fail(RBE_ERR_ARG, "box[%d] = %g is not a positive finite length", a, box[a]);
  for (int a = 3; a < 6; ++a)
    if (!std::isfinite(box[a])) return fail(RBE_ERR_ARG, "tilt box[%d] = %g is not finite", a, box[a]);
  if (std::fabs(box[3]) > box[0] || std::fabs(box[4]) > box[0] || std::fabs(box[5]) > box[1])
    return fail(RBE_ERR_ARG, "tilts (xy %g, xz %g, yz %g) must satisfy |xy|, |xz| <= lx, |yz| <= ly",
                box[3], box[4], box[5]);
  if (!triclinic_cell(alpha, box, t)) return fail(RBE_ERR_ARG, "degenerate triclinic cell");
  for (int a = 0; a < 3; ++a) {
    const double mc = std::ceil(std::sqrt(tail_ln / t->d[a]));
    if (cap && mc > cap[a])
      return fail(RBE_ERR_CAPACITY, "the triclinic cell needs %g sampler entries per side on axis %d, "
                                    "capacity %d (cells up to 2x the initial one)", mc, a, cap[a]);
    if (mc_out) mc_out[a] = (int)mc;
  }
  return RBE_OK;
}

rbe_status check_box(const rbe_ctx_s* c, const double* box) {
  if (!box) return fail(RBE_ERR_ARG, "box pointer is NULL");
  if (c->cfg.box_mode == RBE_BOX_TRICLINIC) {
    TriCell t;
    return check_triclinic(c->cfg.alpha, c->tail_ln, box, c->mcap, &t, nullptr);
  }
  for (int a = 0; a < 3; ++a)
    if (!finite_pos(box[a])) return fail(RBE_ERR_ARG, "box[%d] = %g is not a positive finite length", a, box[a]);
  const int mode = c->cfg.box_mode;
  const double tol = 1e-12 * box[0];
  if (mode == RBE_BOX_ISO && (std::fabs(box[1] - box[0]) > tol || std::fabs(box[2] - box[0]) > tol))
    return fail(RBE_ERR_ARG, "isotropic mode needs a cubic box (got %.17g %.17g %.17g)", box[0], box[1], box[2]);
  if (mode == RBE_BOX_SEMIISO && std::fabs(box[1] - box[0]) > tol)
    return fail(RBE_ERR_ARG, "semi-isotropic mode needs lx == ly (got %.17g %.17g)", box[0], box[1]);
  for (int a = 0; a < 3; ++a) {
    const double mc = axis_mcut(c->tail_ln, c->cfg.alpha, box[a]);
    if (mc > c->mcap[a])
      return fail(RBE_ERR_CAPACITY, "box[%d] = %g needs %g sampler entries per side, capacity %d (2x the initial box)",
                  a, box[a], mc, c->mcap[a]);
  }
  return RBE_OK;
}

// Launch geometry.  Structure factors: 8-wave blocks; a lane owns R
// frequencies (FP32: more per lane for larger batches, so each particle read
// from LDS serves more pairs), KB waves cover distinct frequency groups
// (FB = KB*64*R per block, a power of two), 8/KB waves split the particles;
// X particle chunks x Y frequency slices, about one block per CU.  Chunk
// partials are summed in groups of GX.  Forces: lanes hold 2 particles
// (FP32) or 1 (FP64); KS waves split the batch, PW particle waves share the
// staged constants; about 16 waves per CU.
void plan_launch(rbe_ctx_s* c) {
  StepArgs& a = c->a;
  const bool f64 = c->cfg.precision == RBE_PREC_FP64;
  a.R = f64 ? 1 : (c->p <= 64 ? 1 : (c->p <= 256 ? 2 : 4));
  const int per_wave = kWave * a.R;
  const int kgroups = (c->p + per_wave - 1) / per_wave;
  int KB = 1;
  while (KB < kgroups && KB < kSfacWaves) KB <<= 1;
  a.KB = KB;
  a.Y = (kgroups + KB - 1) / KB;
  a.Ppad = a.Y * KB * per_wave;
  // about one block per CU; two for large batches over many particles, where
  // the second block's waves hide latency (10^6 charges, P = 500 or 2000:
  // 4 % faster; 30k charges, P = 100: slower, the extra partials cost more)
  const double work = (double)c->n * (double)a.Ppad;
  const long target_blocks = work >= 134217728.0 ? 512 : 256;
  long X = (target_blocks + a.Y - 1) / a.Y;
  const long max_x = (c->n + 15) / 16;          // at least 16 particles per chunk
  if (X > max_x) X = max_x;
  if (X < 1) X = 1;
  long chunk = (long)((c->n + X - 1) / X);
  X = (long)((c->n + chunk - 1) / chunk);
  a.X = (int)X;
  a.chunk = (int)chunk;
  // groups of about sqrt(X) chunks: the last-arriving block of a group sums
  // its GX partials, the group partials are summed next
  int GX = 1;
  while ((long)GX * GX < X) ++GX;
  // small batches: every force block sums the group partials of rho itself
  // (read through L2, from the previous launch) if there are at most 4096
  // of them.  Halving the groups then pays: each group's arrival counter
  // takes half as many same-address atomics, and the force blocks read
  // twice as many (cached) rows.
  auto rows_of = [&](int gx) { const long ng = (X + gx - 1) / gx; return ng > 1 ? ng : X; };
  const bool k2 = a.Y == 1 && a.Ppad <= 512;
  const int GXh = (GX + 1) / 2;
  if (k2 && GXh >= 2 && GXh < GX && rows_of(GXh) * a.Ppad <= 4096) GX = GXh;
  a.GX = GX;
  a.NG = (int)((X + GX - 1) / GX);
  a.k2reduce = (k2 && rows_of(GX) * a.Ppad <= 4096) ? 1 : 0;
  const int RP = f64 ? 1 : 2;
  const long groups = (c->n + (long)kWave * RP - 1) / ((long)kWave * RP);
  const long target_waves = 4096;
  int KS = 1;
  while (KS < 8 && (long)(KS * 2) * groups <= target_waves && KS * 2 <= c->pf) KS <<= 1;
  a.KS = KS;
  // many particles: 8 particle waves per block (10^6 charges, P = 2000:
  // 1.4 % faster than 4, and 2 waves are 1.6x slower)
  a.PW = (KS == 1 && groups >= 1024) ? 8 : 1;
}

// The single launch (k_step): every block sums all chunk partials itself
// after one grid-wide wait, so it takes few, large chunks: up to 512
// particles (one LDS tile), about kStepBlocks of them; the force layout puts
// as many particle waves side by side as the chunk fills, so one round
// covers it.
constexpr long kStepBlocks = 64;

void plan_single(rbe_ctx_s* c) {
  long X = std::min(kStepBlocks, (long)((c->n + 15) / 16));
  X = std::max(X, (long)((c->n + kTile - 1) / kTile));
  const long chunk = (c->n + X - 1) / X;
  X = (c->n + chunk - 1) / chunk;
  const int per_wave = kWave * (c->cfg.precision == RBE_PREC_FP64 ? 1 : 2);
  int pw = 1;
  while (pw < kSfacWaves && (long)pw * per_wave < chunk) pw <<= 1;
  c->fX = (int)X;
  c->fchunk = (int)chunk;
  c->fPW = pw;
  c->fKS = kSfacWaves / pw;
}

// StepArgs of the single launch from those of the two-launch plan.
StepArgs single_args(const rbe_ctx_s* c, StepArgs a) {
  a.X = c->fX;
  a.chunk = c->fchunk;
  a.KS = c->fKS;
  a.PW = c->fPW;
  return a;
}

enum Kind { K_TABLES = 0, K_SAMPLE, K_SFAC, K_FORCE, K_STEP };

// The start and stop events for the next launch of kind k if timing is on
// (the launch records them), else none.
LaunchEvents timed(rbe_ctx_s* c, int k) {
  if (c->timing_cap == 0 || c->ev_used[k] >= c->timing_cap) return {};
  const int slot = c->ev_used[k]++;
  LaunchEvents ev;
  ev.start = c->ev[k][2 * slot];
  ev.stop = c->ev[k][2 * slot + 1];
  return ev;
}

void destroy_events(rbe_ctx_s* c) {
  for (int k = 0; k < rbe_ctx_s::kKinds; ++k) {
    for (hipEvent_t e : c->ev[k])
      if (e) (void)hipEventDestroy(e);
    c->ev[k].clear();
    c->ev_used[k] = 0;
  }
  c->timing_cap = 0;
}

void free_all(rbe_ctx_s* c) {
  void* bufs[] = {c->d_q, c->d_qf, c->d_qsum, c->d_bs, c->d_tab, c->d_m, c->d_partial,
                  c->d_gpart, c->d_rho, c->d_terms, c->d_fc32, c->d_fc64, c->d_cnt,
                  c->d_pre, c->d_m_pre, c->d_chain, c->d_bs_frozen, c->d_tab_frozen};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
}

// StepArgs for the current call: pending cell and draw folded in.
StepArgs step_args(rbe_ctx_s* c) {
  StepArgs a = c->a;
  a.box_src = c->pend_box;
  a.box_arg[0] = c->pend_box_val[0]; a.box_arg[1] = c->pend_box_val[1]; a.box_arg[2] = c->pend_box_val[2];
  a.tri_arg = c->pend_box == BOX_ARGS ? c->pend_tri : TriCell{};
  a.box_ptr = c->pend_box_ptr;
  a.sample = c->pend_sample ? 1 : 0;
  a.step = c->pend_step;
  a.use_pre = (c->pend_sample && c->sampler == RBE_SAMPLER_EXACT && c->pre_valid &&
               c->pre_step == c->pend_step) ? 1 : 0;
  a.predraw = 0;
  a.sampler = c->sampler;
  a.mh_iters = c->mh_iters;
  a.mh_init = 0;
  a.mh_old = nullptr;
  a.mh_new = nullptr;
  if (a.sample && c->sampler == RBE_SAMPLER_MH) {
    // this call's launch moves the chains: read the latest state, write the other buffer
    const size_t w = 3 * (size_t)c->p;
    a.mh_init = c->mh_started ? 0 : 1;
    a.mh_old = c->d_chain + (size_t)c->mh_cur * w;
    a.mh_new = c->d_chain + (size_t)(1 - c->mh_cur) * w;
    c->mh_cur = 1 - c->mh_cur;
    c->mh_started = true;
  }
  return a;
}

void clear_pending(rbe_ctx_s* c) {
  c->pend_box = BOX_COMMITTED;
  c->pend_box_ptr = nullptr;
  c->pend_sample = false;
}

// Pending table / draw work as standalone launches, recorded without
// launching (plan_flush) and launched later in stream order (run_flush).
// The host-side state (frozen block, chain buffer flip, pending flags) is
// advanced by plan_flush.
rbe_status plan_flush(rbe_ctx_s* c, PendingLaunch* pl) {
  *pl = PendingLaunch{};
  if (c->pend_box == BOX_COMMITTED && !c->pend_sample) return RBE_OK;
  const StepArgs a = step_args(c);
  const bool reuse = c->pend_sample && c->reuse > 1;
  if (reuse) {
    // first sampled step of a new block: freeze this step's cell (the pending
    // one, else the committed one) for the block's draws
    const uint64_t block = c->pend_step / (uint64_t)c->reuse;
    if (!c->frozen_valid || block != c->frozen_block) {
      StepArgs f = a;
      f.bs = c->d_bs_frozen;
      f.tab = c->d_tab_frozen;
      if (a.box_src == BOX_COMMITTED) {   // the committed cell: BoxState::l on the device
        f.box_src = BOX_PTR;
        f.box_ptr = reinterpret_cast<const double*>(reinterpret_cast<const char*>(c->a.bs) +
                                                    offsetof(BoxState, l));
      }
      pl->frozen = 1;
      pl->frozen_args = f;
      c->frozen_block = block;
      c->frozen_valid = true;
    }
  }
  pl->tables = 1;
  pl->table_args = a;
  // the table kernel commits this cell: what the host knows of it
  c->last_cell_known = a.box_src == BOX_ARGS || (a.box_src == BOX_COMMITTED && c->last_cell_known);
  if (a.box_src == BOX_ARGS) {
    for (int k = 0; k < 3; ++k) c->last_cell[k] = a.box_arg[k];
    for (int k = 0; k < 3; ++k) c->last_cell[3 + k] = a.tri_arg.on ? a.tri_arg.tilt[k] : 0.0;
  }
  if (c->pend_sample) {
    StepArgs d = a;
    if (reuse) { d.bs = c->d_bs_frozen; d.tab = c->d_tab_frozen; }
    pl->sample = 1;
    pl->sample_args = d;
  }
  clear_pending(c);
  return RBE_OK;
}

rbe_status run_flush(rbe_ctx_s* c, const PendingLaunch& pl) {
  hipError_t e;
  if (pl.frozen && (e = launch_tables(pl.frozen_args, c->stream)) != hipSuccess)
    return hip_fail(e, "table kernel");
  if (pl.tables) {
    e = launch_tables(pl.table_args, c->stream, timed(c, K_TABLES));
    if (e != hipSuccess) return hip_fail(e, "table kernel");
  }
  if (pl.sample) {
    e = launch_sample(pl.sample_args, c->stream, timed(c, K_SAMPLE));
    if (e != hipSuccess) return hip_fail(e, "sample kernel");
  }
  return RBE_OK;
}

// Run pending table / draw work with the standalone kernels now.
rbe_status flush(rbe_ctx_s* c) {
  PendingLaunch pl;
  rbe_status st = plan_flush(c, &pl);
  if (st != RBE_OK) return st;
  return run_flush(c, pl);
}

// rbe_init's checks of the configuration and the cell (all but neutrality),
// the sampler-table capacity, the launch plan and whether the single-launch
// step applies; fills c (no device memory).
rbe_status configure(const rbe_config* cfg, const double* box_host, rbe_ctx_s* c) {
  if (cfg->n < 1) return fail(RBE_ERR_ARG, "n = %lld must be >= 1", (long long)cfg->n);
  if (cfg->p < 1 || cfg->p > 65536) return fail(RBE_ERR_ARG, "p = %d must be in 1..65536", cfg->p);
  if (cfg->p_pressure != 0 && (cfg->p_pressure < cfg->p || cfg->p_pressure > 65536))
    return fail(RBE_ERR_ARG, "p_pressure = %d must be 0 or in p..65536 (p = %d)", cfg->p_pressure, cfg->p);
  if (cfg->box_mode < 0 || cfg->box_mode > 3) return fail(RBE_ERR_ARG, "unknown box_mode %d", cfg->box_mode);
  if (cfg->precision < 0 || cfg->precision > 1) return fail(RBE_ERR_ARG, "unknown precision %d", cfg->precision);
  if (!finite_pos(cfg->alpha)) return fail(RBE_ERR_ARG, "alpha = %g must be positive and finite", cfg->alpha);
  if (!finite_pos(cfg->coulomb)) return fail(RBE_ERR_ARG, "coulomb = %g must be positive and finite", cfg->coulomb);
  c->cfg = *cfg;
  c->n = cfg->n;
  c->pf = cfg->p;
  c->p = cfg->p_pressure > cfg->p ? cfg->p_pressure : cfg->p;
  c->tail_ln = 53.0 * std::log(2.0);
  if (cfg->box_mode == RBE_BOX_TRICLINIC) {
    // capacity: the envelope tables of cells up to 2x the initial one
    TriCell t;
    int mc[3];
    rbe_status st = check_triclinic(cfg->alpha, c->tail_ln, box_host, nullptr, &t, mc);
    if (st != RBE_OK) return st;
    for (int a = 0; a < 3; ++a) {
      const double cap = std::ceil(2.0 * std::sqrt(c->tail_ln / t.d[a]));
      if (cap > kMaxMcut)
        return fail(RBE_ERR_ARG, "alpha*l^2 too large: axis %d needs %g sampler entries per side (limit %d)", a, cap, kMaxMcut);
      c->mcap[a] = (int)cap;
    }
  } else {
    for (int a = 0; a < 3; ++a) {
      if (!finite_pos(box_host[a]))
        return fail(RBE_ERR_ARG, "box[%d] = %g is not a positive finite length", a, box_host[a]);
      const double mc = axis_mcut(c->tail_ln, cfg->alpha, 2.0 * box_host[a]);
      if (mc > kMaxMcut)
        return fail(RBE_ERR_ARG, "alpha*l^2 too large: axis %d needs %g sampler entries per side (limit %d)", a, mc, kMaxMcut);
      c->mcap[a] = (int)mc;
    }
  }
  c->tab_stride = 4 * (c->mcap[0] + c->mcap[1] + c->mcap[2]) + 3;
  rbe_status st = check_box(c, box_host);
  if (st != RBE_OK) return st;
  hipError_t e = hipGetDevice(&c->device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  plan_launch(c);
  plan_single(c);
  StepArgs& A = c->a;
  c->fused_ok = false;
  const StepArgs F = single_args(c, A);
  if (step_supported(cfg->precision, F)) {
    // the single launch needs every block resident at once: at most the
    // blocks the device holds together at this kernel's occupancy
    int maxb = 0;
    e = step_max_blocks(cfg->precision, F, &maxb);
    if (e != hipSuccess) return hip_fail(e, "occupancy query");
    c->fused_ok = F.X <= maxb;
  }
  A.p = c->p; A.pf = c->pf; A.n = c->n;
  A.tri_mode = cfg->box_mode == RBE_BOX_TRICLINIC ? 1 : 0;
  A.alpha = cfg->alpha; A.coulomb = cfg->coulomb; A.tail_ln = c->tail_ln;
  A.seed = cfg->seed; A.sysid = cfg->system_id;
  for (int k = 0; k < 3; ++k) A.mcap[k] = c->mcap[k];
  A.tab_stride = c->tab_stride;
  return RBE_OK;
}

}  // namespace

namespace rbe {

rbe_status kspace_step_args(rbe_ctx c, const double* d_x, const double* d_y, const double* d_z,
                            double* d_fx, double* d_fy, double* d_fz, int accumulate,
                            double* d_virial6, double* d_energy, StepArgs* out,
                            PendingLaunch* pre, bool single_launch) {
  if (pre) *pre = PendingLaunch{};
  if (!c) return fail(RBE_ERR_ARG, "NULL context");
  if (!d_x || !d_y || !d_z || !d_fx || !d_fy || !d_fz) return fail(RBE_ERR_ARG, "NULL particle array");
  if (!c->have_k) return fail(RBE_ERR_STATE, "rbe_forces_pressure before rbe_sample_k / rbe_set_k");
  if (c->pend_sample && (c->sampler == RBE_SAMPLER_MH || c->reuse > 1)) {
    // the chains move, and draws from a frozen cell run, in the standalone
    // table and draw kernels: launched now, or by the caller (pre) just
    // before the step's own kernels, once the cell they read is final
    rbe_status st = pre ? plan_flush(c, pre) : flush(c);
    if (st != RBE_OK) return st;
  }
  StepArgs a = step_args(c);
  a.x = d_x; a.y = d_y; a.z = d_z;
  a.fx = d_fx; a.fy = d_fy; a.fz = d_fz;
  a.accumulate = accumulate ? 1 : 0;
  a.virial6 = d_virial6; a.energy = d_energy;
  // The cell of this launch as far as the host knows it: given by value, or
  // the committed one (that of the last launch); a device pointer is not
  // known here.  A batch drawn ahead was drawn for the last launch's cell, so
  // a known change of cell rules it out without the device's check (a
  // dependent global read at the start of every block), and a sampled step
  // of the two-launch path draws the next step's batch ahead only while the
  // cell stays the same (under a barostat it changes every step and the
  // batch drawn ahead would never be used).  The single launch has no spare
  // block for it.
  bool known = false;
  double cell[6] = {0, 0, 0, 0, 0, 0};
  if (a.box_src == BOX_ARGS) {
    known = true;
    for (int k = 0; k < 3; ++k) cell[k] = a.box_arg[k];
    if (a.tri_arg.on)
      for (int k = 0; k < 3; ++k) cell[3 + k] = a.tri_arg.tilt[k];
  } else if (a.box_src == BOX_COMMITTED && c->last_cell_known) {
    known = true;
    for (int k = 0; k < 6; ++k) cell[k] = c->last_cell[k];
  }
  bool same = known && c->last_cell_known;
  for (int k = 0; k < 6 && same; ++k) same = cell[k] == c->last_cell[k];
  const bool changed = known && c->last_cell_known && !same;
  if (changed || single_launch) a.use_pre = 0;
  a.predraw = a.sample && c->sampler == RBE_SAMPLER_EXACT && !single_launch && !changed ? 1 : 0;
  c->pre_valid = a.predraw != 0;
  if (a.predraw) c->pre_step = a.step + 1;
  c->last_cell_known = known;
  for (int k = 0; k < 6; ++k) c->last_cell[k] = cell[k];
  clear_pending(c);
  *out = a;
  return RBE_OK;
}

int kspace_precision(rbe_ctx c) { return c->cfg.precision; }

rbe_status kspace_plan(const rbe_config* cfg, const double* box, StepArgs* a, bool* single) {
  if (!cfg || !box || !a || !single) return fail(RBE_ERR_ARG, "NULL argument");
  rbe_ctx_s c;
  const rbe_status st = configure(cfg, box, &c);
  if (st != RBE_OK) return st;
  *a = single_args(&c, c.a);
  *single = c.fused_ok;
  return RBE_OK;
}

rbe_status kspace_run_pending(rbe_ctx c, const PendingLaunch& pre) { return run_flush(c, pre); }

bool triclinic_cell(double alpha, const double* b, TriCell* t) {
  const double lx = b[0], ly = b[1], lz = b[2], xy = b[3], xz = b[4], yz = b[5];
  *t = TriCell{};
  t->on = 1;
  t->tilt[0] = xy; t->tilt[1] = xz; t->tilt[2] = yz;
  double* hi = t->hinv;          // h^-1 of the upper-triangular h
  hi[0] = 1.0 / lx;
  hi[1] = -xy / (lx * ly);
  hi[2] = (xy * yz - ly * xz) / (lx * ly * lz);
  hi[3] = 1.0 / ly;
  hi[4] = -yz / (ly * lz);
  hi[5] = 1.0 / lz;
  // A = (pi^2/alpha) h^-1 h^-T: xx, yy, zz, xy, xz, yz
  const double f = M_PI * M_PI / alpha;
  double* A = t->A;
  A[0] = f * (hi[0] * hi[0] + hi[1] * hi[1] + hi[2] * hi[2]);
  A[1] = f * (hi[3] * hi[3] + hi[4] * hi[4]);
  A[2] = f * (hi[5] * hi[5]);
  A[3] = f * (hi[1] * hi[3] + hi[2] * hi[4]);
  A[4] = f * (hi[2] * hi[5]);
  A[5] = f * (hi[4] * hi[5]);
  if (A[3] == 0.0 && A[4] == 0.0 && A[5] == 0.0) {
    t->d[0] = A[0]; t->d[1] = A[1]; t->d[2] = A[2];    // rectangular: the law itself
  } else {
    // smallest eigenvalue of C = D^-1/2 A D^-1/2 = I + E (unit diagonal):
    // the eigenvalues of E solve x^3 - (a^2 + b^2 + c^2) x - 2abc = 0
    const double a = A[3] / std::sqrt(A[0] * A[1]), bb = A[4] / std::sqrt(A[0] * A[2]),
                 cc = A[5] / std::sqrt(A[1] * A[2]);
    const double pp = a * a + bb * bb + cc * cc, qq = 2.0 * a * bb * cc;
    double arg = (1.5 * qq / pp) * std::sqrt(3.0 / pp);
    arg = std::max(-1.0, std::min(1.0, arg));
    const double th = std::acos(arg);
    const double lmin = 1.0 + 2.0 * std::sqrt(pp / 3.0) * std::cos(th / 3.0 + 2.0 * M_PI / 3.0);
    if (!(lmin > 0.0)) return false;
    const double tf = (1.0 - 1e-9) * lmin;
    t->d[0] = tf * A[0]; t->d[1] = tf * A[1]; t->d[2] = tf * A[2];
  }
  // S + 1 = (alpha/pi)^(3/2) V sum_n exp(-alpha |h n|^2) (Poisson-summed lattice sum)
  const double V = lx * ly * lz;
  const double G[3] = {A[0] / f, A[1] / f, A[2] / f};
  int nb[3];
  for (int k = 0; k < 3; ++k) nb[k] = (int)std::floor(std::sqrt(60.0 * G[k] / alpha));
  double sum = 0.0;
  for (int n0 = -nb[0]; n0 <= nb[0]; ++n0)
    for (int n1 = -nb[1]; n1 <= nb[1]; ++n1)
      for (int n2 = -nb[2]; n2 <= nb[2]; ++n2) {
        const double rx = lx * n0 + xy * n1 + xz * n2, ry = ly * n1 + yz * n2, rz = lz * n2;
        const double e = alpha * (rx * rx + ry * ry + rz * rz);
        if (e <= 60.0) sum += std::exp(-e);
      }
  t->S = std::pow(alpha / M_PI, 1.5) * V * sum - 1.0;
  return std::isfinite(t->S) && t->S > 0.0;
}

int64_t kspace_footprint(const rbe_config* cfg, const double* box) {
  rbe_ctx_s c;
  c.cfg = *cfg;
  c.n = cfg->n;
  c.pf = cfg->p;
  c.p = cfg->p_pressure > cfg->p ? cfg->p_pressure : cfg->p;
  c.tail_ln = 53.0 * std::log(2.0);
  for (int k = 0; k < 3; ++k) c.mcap[k] = (int)axis_mcut(c.tail_ln, cfg->alpha, 2.0 * box[k]);
  c.tab_stride = 4 * (c.mcap[0] + c.mcap[1] + c.mcap[2]) + 3;
  plan_launch(&c);
  plan_single(&c);
  const StepArgs& A = c.a;
  const int64_t n = c.n, p = c.p;
  auto r = [](int64_t b) { return (b + 255) / 256 * 256; };
  return r(n * 8) + r(n * 4) + r(24) + r(sizeof(BoxState)) + r((int64_t)c.tab_stride * 8) + r(12 * p) +
         r((int64_t)std::max(A.X, c.fX) * A.Ppad * 16) + r((int64_t)A.NG * A.Ppad * 16) + r(16 * p) + r(64 * p) +
         r(p * (int64_t)sizeof(FCoef32)) + r(p * (int64_t)sizeof(FCoef64)) +
         r(4 * cnt_words(A.Y, A.NG)) + r(2 * sizeof(PreDraw)) + r(24 * p);
}

}  // namespace rbe

extern "C" {

const char* rbe_last_error(void) { return g_err.c_str(); }

const char* rbe_version(void) { return "rbe-gfx950 0.2"; }

rbe_status rbe_init(const rbe_config* cfg, const double* d_q, const double* box_host,
                    void* stream, rbe_ctx* out) {
  g_err.clear();
  if (!cfg || !d_q || !box_host || !out) return fail(RBE_ERR_ARG, "NULL argument to rbe_init");
  *out = nullptr;
  rbe_ctx_s* c = new (std::nothrow) rbe_ctx_s();
  if (!c) return fail(RBE_ERR_ALLOC, "host allocation failed");
  c->stream = (hipStream_t)stream;
  {
    const rbe_status st = configure(cfg, box_host, c);
    if (st != RBE_OK) { delete c; return st; }
  }
  hipError_t e = hipSuccess;
  StepArgs& A = c->a;

  const size_t n = (size_t)c->n, p = (size_t)c->p;
  const size_t ncnt = (size_t)cnt_words(A.Y, A.NG);
  bool ok = true;
  ok = ok && hipMalloc(&c->d_q, n * sizeof(double)) == hipSuccess;
  ok = ok && hipMalloc(&c->d_qf, n * sizeof(float)) == hipSuccess;
  ok = ok && hipMalloc(&c->d_qsum, 3 * sizeof(double)) == hipSuccess;
  ok = ok && hipMalloc(&c->d_bs, sizeof(BoxState)) == hipSuccess;
  ok = ok && hipMalloc(&c->d_tab, (size_t)c->tab_stride * sizeof(double)) == hipSuccess;
  ok = ok && hipMalloc(&c->d_m, 3 * p * sizeof(int32_t)) == hipSuccess;
  ok = ok && hipMalloc(&c->d_partial, (size_t)std::max(A.X, c->fX) * A.Ppad * sizeof(double2)) == hipSuccess;
  ok = ok && hipMalloc(&c->d_gpart, (size_t)A.NG * A.Ppad * sizeof(double2)) == hipSuccess;
  ok = ok && hipMalloc(&c->d_rho, p * sizeof(double2)) == hipSuccess;
  ok = ok && hipMalloc(&c->d_terms, 8 * p * sizeof(double)) == hipSuccess;
  ok = ok && hipMalloc(&c->d_fc32, p * sizeof(FCoef32)) == hipSuccess;
  ok = ok && hipMalloc(&c->d_fc64, p * sizeof(FCoef64)) == hipSuccess;
  ok = ok && hipMalloc(&c->d_cnt, ncnt * sizeof(uint32_t)) == hipSuccess;
  ok = ok && hipMalloc(&c->d_pre, 2 * sizeof(PreDraw)) == hipSuccess;
  ok = ok && hipMalloc(&c->d_m_pre, 2 * 3 * p * sizeof(int32_t)) == hipSuccess;
  if (!ok) { free_all(c); delete c; return fail(RBE_ERR_ALLOC, "device allocation failed"); }

  A.q = c->d_q; A.qf = c->d_qf;
  A.seed = cfg->seed; A.sysid = cfg->system_id;
  for (int k = 0; k < 3; ++k) A.mcap[k] = c->mcap[k];
  A.tab_stride = c->tab_stride;
  A.bs = c->d_bs; A.tab = c->d_tab; A.m = c->d_m;
  A.partial = c->d_partial; A.gpart = c->d_gpart; A.rho = c->d_rho; A.terms = c->d_terms;
  A.fc32 = c->d_fc32; A.fc64 = c->d_fc64; A.cnt = c->d_cnt;
  A.pre = c->d_pre; A.m_pre = c->d_m_pre;

  rbe_status st = RBE_OK;
  double qs[3] = {0, 0, 0};
  do {
    if ((e = hipMemsetAsync(c->d_bs, 0, sizeof(BoxState), c->stream)) != hipSuccess) { st = hip_fail(e, "hipMemsetAsync"); break; }
    if ((e = hipMemsetAsync(c->d_cnt, 0, ncnt * sizeof(uint32_t), c->stream)) != hipSuccess) { st = hip_fail(e, "hipMemsetAsync"); break; }
    if ((e = hipMemsetAsync(c->d_m, 0, 3 * p * sizeof(int32_t), c->stream)) != hipSuccess) { st = hip_fail(e, "hipMemsetAsync"); break; }
    if ((e = hipMemsetAsync(c->d_pre, 0, 2 * sizeof(PreDraw), c->stream)) != hipSuccess) { st = hip_fail(e, "hipMemsetAsync"); break; }
    if ((e = hipMemcpyAsync(c->d_q, d_q, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream)) != hipSuccess) { st = hip_fail(e, "copy charges"); break; }
    if ((e = launch_qsum(c->d_q, c->d_qf, c->d_qsum, c->n, c->stream)) != hipSuccess) { st = hip_fail(e, "charge sums"); break; }
    if ((e = hipMemcpyAsync(qs, c->d_qsum, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream)) != hipSuccess) { st = hip_fail(e, "copy charge sums"); break; }
    if ((e = hipStreamSynchronize(c->stream)) != hipSuccess) { st = hip_fail(e, "hipStreamSynchronize"); break; }
    if (!std::isfinite(qs[0]) || !std::isfinite(qs[1])) { st = fail(RBE_ERR_ARG, "charges are not finite"); break; }
    if (std::fabs(qs[0]) > 1e-10 * qs[1]) { st = fail(RBE_ERR_NONNEUTRAL, "system is not neutral: sum q = %g, sum |q| = %g", qs[0], qs[1]); break; }
  } while (0);
  if (st != RBE_OK) { free_all(c); delete c; return st; }
  c->self_energy = -cfg->coulomb * qs[2] * std::sqrt(cfg->alpha / M_PI);
  A.self_energy = c->self_energy;
  st = rbe_rescale_box(c, box_host);
  if (st == RBE_OK) st = flush(c);     // commit the initial cell
  if (st != RBE_OK) { free_all(c); delete c; return st; }
  *out = c;
  return RBE_OK;
}

rbe_status rbe_set_stream(rbe_ctx c, void* stream) {
  if (!c) return fail(RBE_ERR_ARG, "NULL context");
  c->stream = (hipStream_t)stream;
  return RBE_OK;
}

rbe_status rbe_rescale_box(rbe_ctx c, const double* box_host) {
  if (!c) return fail(RBE_ERR_ARG, "NULL context");
  rbe_status st = check_box(c, box_host);
  if (st != RBE_OK) return st;
  c->pend_tri = TriCell{};
  if (c->cfg.box_mode == RBE_BOX_TRICLINIC &&
      (st = check_triclinic(c->cfg.alpha, c->tail_ln, box_host, c->mcap, &c->pend_tri, nullptr)) != RBE_OK)
    return st;
  c->pend_box = BOX_ARGS;
  for (int k = 0; k < 3; ++k) c->pend_box_val[k] = box_host[k];
  c->pend_box_ptr = nullptr;
  return RBE_OK;
}

rbe_status rbe_rescale_box_dev(rbe_ctx c, const double* d_box) {
  if (!c) return fail(RBE_ERR_ARG, "NULL context");
  if (!d_box) return fail(RBE_ERR_ARG, "NULL device box");
  if (c->cfg.box_mode == RBE_BOX_TRICLINIC)
    return fail(RBE_ERR_ARG, "a triclinic cell is given from the host (rbe_rescale_box)");
  c->pend_box = BOX_PTR;
  c->pend_box_ptr = d_box;
  return RBE_OK;
}

rbe_status rbe_sample_k(rbe_ctx c, uint64_t step) {
  if (!c) return fail(RBE_ERR_ARG, "NULL context");
  c->pend_sample = true;
  c->pend_step = step;
  c->have_k = true;
  return RBE_OK;
}

rbe_status rbe_set_sampler(rbe_ctx c, int32_t sampler, int32_t iters) {
  if (!c) return fail(RBE_ERR_ARG, "NULL context");
  if (sampler != RBE_SAMPLER_EXACT && sampler != RBE_SAMPLER_MH)
    return fail(RBE_ERR_ARG, "unknown sampler %d", sampler);
  if (sampler == RBE_SAMPLER_MH && (iters < 1 || iters > 64))
    return fail(RBE_ERR_ARG, "iters = %d must be in 1..64", iters);
  if (sampler == RBE_SAMPLER_MH && c->reuse > 1)
    return fail(RBE_ERR_ARG, "sample reuse (period %d) goes with the exact sampler", c->reuse);
  if (sampler == RBE_SAMPLER_MH && c->cfg.box_mode == RBE_BOX_TRICLINIC)
    return fail(RBE_ERR_ARG, "the Metropolis-Hastings chains need a rectangular cell");
  rbe_status st = flush(c);                // a pending draw belongs to the old sampler
  if (st != RBE_OK) return st;
  if (sampler == RBE_SAMPLER_MH && !c->d_chain)
    HIP_TRY(hipMalloc(&c->d_chain, 6 * (size_t)c->p * sizeof(int32_t)), "chain state");
  HIP_TRY(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  c->sampler = sampler;
  c->mh_iters = sampler == RBE_SAMPLER_MH ? iters : 1;
  c->mh_started = false;
  c->mh_cur = 0;
  c->pre_valid = false;
  return RBE_OK;
}

rbe_status rbe_set_sample_reuse(rbe_ctx c, int32_t period) {
  if (!c) return fail(RBE_ERR_ARG, "NULL context");
  if (period < 1 || period > 1000000) return fail(RBE_ERR_ARG, "period = %d must be in 1..1000000", period);
  if (period > 1 && c->sampler != RBE_SAMPLER_EXACT)
    return fail(RBE_ERR_ARG, "sample reuse goes with the exact sampler");
  if (period > 1 && c->cfg.box_mode == RBE_BOX_TRICLINIC)
    return fail(RBE_ERR_ARG, "sample reuse needs a rectangular cell");
  rbe_status st = flush(c);                // a pending draw belongs to the old setting
  if (st != RBE_OK) return st;
  if (period > 1 && !c->d_bs_frozen) {
    HIP_TRY(hipMalloc(&c->d_bs_frozen, sizeof(BoxState)), "frozen cell");
    HIP_TRY(hipMalloc(&c->d_tab_frozen, (size_t)c->tab_stride * sizeof(double)), "frozen tables");
    HIP_TRY(hipMemsetAsync(c->d_bs_frozen, 0, sizeof(BoxState), c->stream), "hipMemsetAsync");
  }
  HIP_TRY(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  c->reuse = period;
  c->frozen_valid = false;
  c->pre_valid = false;
  return RBE_OK;
}

rbe_status rbe_set_k(rbe_ctx c, const int32_t* h_m, int32_t p_in) {
  if (!c) return fail(RBE_ERR_ARG, "NULL context");
  if (!h_m) return fail(RBE_ERR_ARG, "NULL batch");
  if (p_in != c->p)
    return fail(RBE_ERR_ARG, "batch size %d differs from the configured batch max(p, p_pressure) = %d", p_in, c->p);
  for (int l = 0; l < p_in; ++l) {
    const int32_t* m = h_m + 3 * l;
    if (m[0] == 0 && m[1] == 0 && m[2] == 0) return fail(RBE_ERR_ARG, "row %d of the batch is the zero vector", l);
    for (int a = 0; a < 3; ++a)
      if (m[a] > 2048 || m[a] < -2048) return fail(RBE_ERR_ARG, "row %d: |m| = %d exceeds 2048", l, m[a]);
  }
  c->pend_sample = false;               // an explicit batch replaces a pending draw
  HIP_TRY(hipMemcpyAsync(c->d_m, h_m, 3 * (size_t)p_in * sizeof(int32_t), hipMemcpyHostToDevice, c->stream), "copy batch");
  HIP_TRY(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  c->have_k = true;
  return RBE_OK;
}

rbe_status rbe_get_k(rbe_ctx c, int32_t* h_m) {
  if (!c || !h_m) return fail(RBE_ERR_ARG, "NULL argument");
  if (!c->have_k) return fail(RBE_ERR_STATE, "no batch drawn or set yet");
  rbe_status st = flush(c);
  if (st != RBE_OK) return st;
  HIP_TRY(hipMemcpyAsync(h_m, c->d_m, 3 * (size_t)c->p * sizeof(int32_t), hipMemcpyDeviceToHost, c->stream), "copy batch");
  HIP_TRY(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  return RBE_OK;
}

rbe_status rbe_forces_pressure(rbe_ctx c, const double* d_x, const double* d_y, const double* d_z,
                               double* d_fx, double* d_fy, double* d_fz, int accumulate,
                               double* d_virial6, double* d_energy) {
  StepArgs a;
  const bool single = c && c->fused_ok && c->fused_on;
  rbe_status st = rbe::kspace_step_args(c, d_x, d_y, d_z, d_fx, d_fy, d_fz, accumulate, d_virial6,
                                        d_energy, &a, nullptr, single);
  if (st != RBE_OK) return st;
  const int prec = c->cfg.precision;
  if (single) {
    const hipError_t e = launch_step(prec, single_args(c, a), c->stream, timed(c, K_STEP));
    if (e != hipSuccess) return hip_fail(e, "single-launch step kernel");
    return RBE_OK;
  }
  hipError_t e = launch_sfac(prec, a, c->stream, timed(c, K_SFAC));
  if (e != hipSuccess) return hip_fail(e, "structure-factor kernel");
  e = launch_force(prec, a, c->stream, timed(c, K_FORCE));
  if (e != hipSuccess) return hip_fail(e, "force kernel");
  return RBE_OK;
}

rbe_status rbe_get_rho(rbe_ctx c, double* h_rho) {
  if (!c || !h_rho) return fail(RBE_ERR_ARG, "NULL argument");
  HIP_TRY(hipMemcpyAsync(h_rho, c->d_rho, (size_t)c->p * sizeof(double2), hipMemcpyDeviceToHost, c->stream), "copy rho");
  HIP_TRY(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  return RBE_OK;
}

rbe_status rbe_get_box_info(rbe_ctx c, double* h_info) {
  if (!c || !h_info) return fail(RBE_ERR_ARG, "NULL argument");
  rbe_status st = flush(c);
  if (st != RBE_OK) return st;
  BoxState b;
  HIP_TRY(hipMemcpyAsync(&b, c->d_bs, sizeof b, hipMemcpyDeviceToHost, c->stream), "copy box state");
  HIP_TRY(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  h_info[0] = b.V; h_info[1] = b.S;
  h_info[2] = b.H[0]; h_info[3] = b.H[1]; h_info[4] = b.H[2];
  h_info[5] = b.l[0]; h_info[6] = b.l[1]; h_info[7] = b.l[2];
  h_info[8] = b.mcut[0]; h_info[9] = b.mcut[1]; h_info[10] = b.mcut[2];
  h_info[11] = b.err;
  return RBE_OK;
}

rbe_status rbe_get_plan(rbe_ctx c, int32_t* h) {
  if (!c || !h) return fail(RBE_ERR_ARG, "NULL argument");
  const StepArgs& a = c->a;
  const int32_t v[16] = {a.X, a.Y, a.KB, a.R, a.GX, a.NG, a.chunk, a.Ppad, a.KS, a.PW, a.k2reduce,
                         (c->fused_ok && c->fused_on) ? 1 : 0, c->fX, c->fchunk, c->fKS, 0};
  for (int i = 0; i < 16; ++i) h[i] = v[i];
  return RBE_OK;
}

rbe_status rbe_check(rbe_ctx c) {
  if (!c) return fail(RBE_ERR_ARG, "NULL context");
  rbe_status st = flush(c);
  if (st != RBE_OK) return st;
  HIP_TRY(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  int32_t err = 0;
  HIP_TRY(hipMemcpy(&err, &c->d_bs->err, sizeof err, hipMemcpyDeviceToHost), "read error flags");
  if (c->fused_ok) {
    // the single launch's bounded wait for the force constants gave up (it
    // never does while every block is resident): the counters are cleared
    const StepArgs& A = c->a;
    uint32_t wait_err = 0;
    uint32_t* errw = c->d_cnt + cnt_index(A, CNT_ERR);
    HIP_TRY(hipMemcpy(&wait_err, errw, sizeof wait_err, hipMemcpyDeviceToHost), "read error flags");
    if (wait_err) {
      const size_t ncnt = (size_t)cnt_words(A.Y, A.NG);
      HIP_TRY(hipMemset(c->d_cnt, 0, ncnt * sizeof(uint32_t)), "clear counters");
      return fail(RBE_ERR_DEVICE, "a single-launch step gave up waiting for the rho partials of "
                                  "other blocks; its forces were not written");
    }
  }
  if (err) {
    const int32_t zero = 0;
    HIP_TRY(hipMemcpy(&c->d_bs->err, &zero, sizeof zero, hipMemcpyHostToDevice), "clear error flags");
    return fail(RBE_ERR_CAPACITY, "a device-side rescale met a cell outside the sampler-table capacity (flags %d)", err);
  }
  return RBE_OK;
}

rbe_status rbe_variance_probe(rbe_ctx c, const double* d_x, const double* d_y, const double* d_z,
                              int32_t batches, uint64_t first_step, double* h_out,
                              double* h_var) {
  if (!c || !d_x || !d_y || !d_z || !h_out) return fail(RBE_ERR_ARG, "NULL argument");
  if (batches < 2 || batches > 1000000)
    return fail(RBE_ERR_ARG, "batches = %d must be in 2..1000000", batches);
  const int64_t n = c->n;
  double* mem = nullptr;
  // forces (3n), sums (3n), squares (3n), virial (6), P2 sums (2)
  const size_t count = 9 * (size_t)n + 8;
  HIP_TRY(hipMalloc(&mem, count * sizeof(double)), "probe scratch");
  double *f = mem, *sum = mem + 3 * n, *sq = mem + 6 * n, *vir = mem + 9 * n, *ps = vir + 6;
  rbe_status st = RBE_OK;
  hipError_t e = hipMemsetAsync(mem, 0, count * sizeof(double), c->stream);
  if (e != hipSuccess) st = hip_fail(e, "hipMemsetAsync");
  BoxState b{};
  for (int32_t k = 0; k < batches && st == RBE_OK; ++k) {
    st = rbe_sample_k(c, first_step + (uint64_t)k);
    if (st == RBE_OK)
      st = rbe_forces_pressure(c, d_x, d_y, d_z, f, f + n, f + 2 * n, 0, vir, nullptr);
    if (st == RBE_OK && k == 0) {
      // the cell of the evaluations (committed by the first one)
      e = hipMemcpyAsync(&b, c->d_bs, sizeof b, hipMemcpyDeviceToHost, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      if (e != hipSuccess) st = hip_fail(e, "read cell");
    }
    if (st == RBE_OK && (e = launch_moments(f, f + n, f + 2 * n, vir, b.V, n, sum, sq, ps,
                                            c->stream)) != hipSuccess)
      st = hip_fail(e, "moments kernel");
  }
  std::vector<double> h((size_t)6 * n + 2);
  if (st == RBE_OK) {
    e = hipMemcpyAsync(h.data(), sum, 6 * (size_t)n * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(h.data() + 6 * n, ps, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) st = hip_fail(e, "read moments");
  }
  (void)hipStreamSynchronize(c->stream);
  (void)hipFree(mem);
  if (st != RBE_OK) return st;
  const double B = (double)batches;
  double tot = 0.0, mean2 = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double vi = 0.0;
    for (int a = 0; a < 3; ++a) {
      const double m = h[(size_t)a * n + i] / B;
      vi += (h[(size_t)(3 + a) * n + i] / B - m * m) * (B / (B - 1.0));
      mean2 += m * m;
    }
    if (h_var) h_var[i] = vi;
    tot += vi;
  }
  const double pm = h[6 * n] / B;
  h_out[0] = tot;
  h_out[1] = (h[6 * n + 1] / B - pm * pm) * (B / (B - 1.0));
  h_out[2] = mean2;
  h_out[3] = pm;
  return RBE_OK;
}

rbe_status rbe_batch_size_for_variance(int32_t p, double var, double target, int32_t* p_out) {
  if (!p_out) return fail(RBE_ERR_ARG, "NULL argument");
  if (p < 1 || !(var >= 0.0) || !std::isfinite(var) || !(target > 0.0) || !std::isfinite(target))
    return fail(RBE_ERR_ARG, "need p >= 1, a finite variance >= 0 and a finite target > 0");
  const double want = std::ceil((double)p * var / target);
  *p_out = want < 1.0 ? 1 : (want > 65536.0 ? 65536 : (int32_t)want);
  return RBE_OK;
}

rbe_status rbe_set_fused(rbe_ctx c, int32_t enable) {
  if (!c) return fail(RBE_ERR_ARG, "NULL context");
  if (enable != 0 && enable != 1) return fail(RBE_ERR_ARG, "enable = %d must be 0 or 1", enable);
  c->fused_on = enable != 0;
  return RBE_OK;
}

rbe_status rbe_timing_enable(rbe_ctx c, int32_t max_launches) {
  if (!c) return fail(RBE_ERR_ARG, "NULL context");
  if (max_launches < 0) return fail(RBE_ERR_ARG, "max_launches = %d must be >= 0", max_launches);
  HIP_TRY(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  destroy_events(c);
  if (max_launches == 0) return RBE_OK;
  for (int k = 0; k < rbe_ctx_s::kKinds; ++k) {
    c->ev[k].assign(2 * (size_t)max_launches, nullptr);
    for (auto& e : c->ev[k]) {
      if (hipEventCreate(&e) != hipSuccess) {
        e = nullptr;
        destroy_events(c);
        return fail(RBE_ERR_DEVICE, "hipEventCreate failed");
      }
    }
  }
  c->timing_cap = max_launches;
  return RBE_OK;
}

rbe_status rbe_timing_read(rbe_ctx c, double* h_ms, int32_t* h_count) {
  if (!c || !h_ms || !h_count) return fail(RBE_ERR_ARG, "NULL argument");
  HIP_TRY(hipStreamSynchronize(c->stream), "hipStreamSynchronize");
  for (int k = 0; k < rbe_ctx_s::kKinds; ++k) {
    double tot = 0.0;
    for (int i = 0; i < c->ev_used[k]; ++i) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, c->ev[k][2 * i], c->ev[k][2 * i + 1]), "hipEventElapsedTime");
      tot += ms;
    }
    h_ms[k] = tot;
    h_count[k] = c->ev_used[k];
    c->ev_used[k] = 0;
  }
  return RBE_OK;
}

void rbe_destroy(rbe_ctx c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  destroy_events(c);
  free_all(c);
  delete c;
}

}  // extern "C"
