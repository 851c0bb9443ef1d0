// Served batching: many independent NPT systems resident on one GPU, every
// kernel of a step launched once for all of them (declarations and contracts
// in include/rbe.h).
//
// Each system keeps its own three contexts (Fourier part, real-space pairs,
// integrator) and its own launch plan, so the arithmetic, tiling and
// reduction order of a system are the ones it has alone; a fused launch only
// concatenates the systems' block ranges.  Per step the host gathers every
// active system's kernel arguments into a pinned table, copies it to the
// device in one transfer, and launches
//   md first half | structure factors (one launch per lane width R) |
//   forces (one launch per block shape) | cell list + pairs (5) | md second half
// where a block finds its system by a binary search over the table's block
// offsets.
#include "rbe_internal.h"
#include "rbe_md_internal.h"
#include "rbe_real_internal.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <vector>

using namespace rbe;

namespace rbe {
rbe_status set_error(rbe_status st, const char* msg);
}

namespace {

struct Slot {
  bool active = false;
  rbe_system_desc desc{};
  int64_t bytes = 0;
  uint64_t step = 0;
  rbe_ctx k = nullptr;
  rbe_real_ctx r = nullptr;
  rbe_md_ctx m = nullptr;
  void* mem = nullptr;          // one allocation: the state arrays below
  double *x, *y, *z, *px, *py, *pz, *fx, *fy, *fz, *q, *mass, *vk, *vr, *ek, *er;
  int32_t* type;
  const double* box_dev = nullptr;
};

// staging for the per-step argument tables (pinned host + device copy)
struct Stage {
  char* host = nullptr;
  char* dev = nullptr;
  hipEvent_t done = nullptr;    // the copy out of `host` has completed
  size_t used = 0;
  bool overflow = false;
};

}  // namespace

struct rbe_batch_s {
  rbe_batch_config cfg{};
  hipStream_t stream = nullptr;
  std::vector<Slot> slots;
  int64_t bytes_in_use = 0;
  int64_t steps_launched = 0;
  size_t stage_cap = 0;
  Stage stage[2];
  int cur = 0;
  // kernel timing of fused steps: events around each kernel family
  static constexpr int kKinds = 5;   // md first half, structure factors, forces, real space, md second half
  int timing_cap = 0, timed = 0;
  std::vector<hipEvent_t> ev;        // [timing_cap][kKinds + 1]
  double timed_np = 0.0;             // sum of N p over the timed steps
  // a step failed after some systems' host state had advanced (step
  // counters, Metropolis-Hastings chain buffers): the systems no longer agree
  // with what ran on the device, so every later step is refused
  bool broken = false;
};

namespace {

rbe_status bfail(rbe_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
rbe_status bfail(rbe_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return rbe::set_error(st, buf);
}

bool fin(double v) { return std::isfinite(v); }

rbe_status check_desc(const rbe_system_desc* d, const double* box) {
  if (!d || !box) return bfail(RBE_ERR_ARG, "NULL system description or box");
  if (d->n < 1) return bfail(RBE_ERR_ARG, "n = %lld must be >= 1", (long long)d->n);
  if (d->p < 1 || d->p > 65536) return bfail(RBE_ERR_ARG, "p = %d must be in 1..65536", d->p);
  if (d->box_mode != RBE_BOX_ISO && d->box_mode != RBE_BOX_SEMIISO && d->box_mode != RBE_BOX_ANISO)
    return bfail(RBE_ERR_ARG, "box_mode must be RBE_BOX_ISO, RBE_BOX_SEMIISO or RBE_BOX_ANISO");
  if (d->sampler != RBE_SAMPLER_EXACT && d->sampler != RBE_SAMPLER_MH)
    return bfail(RBE_ERR_ARG, "sampler = %d is not a known rbe_sampler", d->sampler);
  if (d->ntypes < 0 || d->ntypes > 64) return bfail(RBE_ERR_ARG, "ntypes = %d must be in 0..64", d->ntypes);
  if (!(d->skin >= 0.0 && fin(d->skin))) return bfail(RBE_ERR_ARG, "skin = %g must be >= 0", d->skin);
  if (!(d->alpha > 0 && fin(d->alpha)) || !(d->rc > 0 && fin(d->rc)) || !(d->coulomb > 0 && fin(d->coulomb)))
    return bfail(RBE_ERR_ARG, "alpha, rc and coulomb must be positive and finite");
  for (int a = 0; a < 3; ++a)
    if (!(box[a] > 0 && fin(box[a]))) return bfail(RBE_ERR_ARG, "box[%d] = %g is not a positive finite length", a, box[a]);
  return RBE_OK;
}

rbe_config kspace_cfg(const rbe_batch_s* b, const rbe_system_desc* d, const double* box) {
  rbe_config c{};
  c.n = d->n;
  c.p = d->p;
  // the Fourier part checks only the cell's shape; isotropic coupling of a
  // non-cubic cell keeps a general rectangular cell
  const bool cubic = box[0] == box[1] && box[0] == box[2];
  c.box_mode = d->box_mode == RBE_BOX_SEMIISO ? RBE_BOX_SEMIISO
               : (cubic && d->box_mode == RBE_BOX_ISO ? RBE_BOX_ISO : RBE_BOX_ANISO);
  c.precision = b ? b->cfg.precision : RBE_PREC_FP32;
  c.alpha = d->alpha;
  c.coulomb = d->coulomb;
  c.seed = d->seed;
  c.system_id = d->system_id;
  return c;
}

rbe_real_config real_cfg(const rbe_batch_s* b, const rbe_system_desc* d) {
  rbe_real_config c{};
  c.n = d->n;
  c.precision = b ? b->cfg.real_precision : RBE_PREC_FP64;
  c.ntypes = d->ntypes;
  c.alpha = d->alpha;
  c.rc = d->rc;
  c.coulomb = d->coulomb;
  return c;
}

rbe_md_config md_cfg(const rbe_system_desc* d) {
  rbe_md_config c{};
  c.n = d->n;
  c.box_mode = d->box_mode;
  c.dt = d->dt; c.kT = d->kT; c.p_ext = d->p_ext;
  c.gamma_p = d->gamma_p; c.gamma_cell = d->gamma_cell;
  c.mass_cell = d->mass_cell; c.mass_cell_z = d->mass_cell_z;
  c.ftm = d->ftm;
  c.seed = d->seed;
  c.system_id = d->system_id;
  return c;
}

int64_t round256(int64_t b) { return (b + 255) / 256 * 256; }

// state arrays of one system: x y z px py pz fx fy fz q mass (n doubles
// each), virials (2 x 6), energies (2), types (n int32)
int64_t state_bytes(int64_t n) { return round256(11 * 8 * n + 14 * 8 + 4 * n); }

int64_t footprint(const rbe_batch_s* b, const rbe_system_desc* d, const double* box) {
  const rbe_config kc = kspace_cfg(b, d, box);
  const rbe_real_config rc = real_cfg(b, d);
  return state_bytes(d->n) + kspace_footprint(&kc, box) + real_footprint(&rc, box, d->skin) +
         md_footprint(d->n);
}

void release_slot(Slot& s) {
  if (s.k) rbe_destroy(s.k);
  if (s.r) rbe_real_destroy(s.r);
  if (s.m) rbe_md_destroy(s.m);
  if (s.mem) (void)hipFree(s.mem);
  s = Slot{};
}

size_t align64(size_t v) { return (v + 63) & ~size_t(63); }

// append `bytes` from `src` to the host stage; returns the device address
template <typename T>
const T* put(rbe_batch_s* b, const T* src, size_t count) {
  Stage& st = b->stage[b->cur];
  const size_t off = align64(st.used);
  if (off + count * sizeof(T) > b->stage_cap) { st.overflow = true; return nullptr; }
  std::memcpy(st.host + off, src, count * sizeof(T));
  st.used = off + count * sizeof(T);
  return reinterpret_cast<const T*>(st.dev + off);
}

size_t stage_bytes_per_system() {
  return 2 * sizeof(StepArgs) + sizeof(RealArgs) + 2 * sizeof(MDArgs) + 10 * sizeof(int) + 10 * 64;
}

}  // namespace

extern "C" {

rbe_status rbe_batch_create(const rbe_batch_config* cfg, void* stream, rbe_batch* out) {
  if (!cfg || !out) return bfail(RBE_ERR_ARG, "NULL argument to rbe_batch_create");
  *out = nullptr;
  if (cfg->precision != RBE_PREC_FP32 && cfg->precision != RBE_PREC_FP64)
    return bfail(RBE_ERR_ARG, "unknown precision %d", cfg->precision);
  if (cfg->max_systems < 1 || cfg->max_systems > 4096)
    return bfail(RBE_ERR_ARG, "max_systems = %d must be in 1..4096", cfg->max_systems);
  if (cfg->hbm_budget <= 0) return bfail(RBE_ERR_ARG, "hbm_budget must be positive");
  if (cfg->real_precision != RBE_PREC_FP32 && cfg->real_precision != RBE_PREC_FP64)
    return bfail(RBE_ERR_ARG, "unknown real_precision %d", cfg->real_precision);
  if (cfg->reserved != 0) return bfail(RBE_ERR_ARG, "reserved field must be 0");
  rbe_batch_s* b = new (std::nothrow) rbe_batch_s();
  if (!b) return bfail(RBE_ERR_ALLOC, "host allocation failed");
  b->cfg = *cfg;
  b->stream = (hipStream_t)stream;
  b->slots.resize(cfg->max_systems);
  // tables of one step: every system once per kernel family, plus one
  // 64-byte alignment per group (at most 3 lane widths + 4 block shapes)
  b->stage_cap = (size_t)cfg->max_systems * stage_bytes_per_system() + 64 * 1024;
  for (Stage& st : b->stage) {
    hipError_t e = hipHostMalloc((void**)&st.host, b->stage_cap, hipHostMallocDefault);
    const char* what = "hipHostMalloc";
    if (e == hipSuccess) { what = "hipMalloc"; e = hipMalloc((void**)&st.dev, b->stage_cap); }
    if (e == hipSuccess) { what = "hipEventCreate"; e = hipEventCreateWithFlags(&st.done, hipEventDisableTiming); }
    if (e != hipSuccess) {
      const size_t cap = b->stage_cap;
      rbe_batch_destroy(b);
      return bfail(RBE_ERR_ALLOC, "staging (%zu bytes): %s: %s", cap, what, hipGetErrorString(e));
    }
  }
  *out = b;
  return RBE_OK;
}

rbe_status rbe_batch_footprint(const rbe_system_desc* d, const double* box_host, int64_t* bytes) {
  if (!bytes) return bfail(RBE_ERR_ARG, "NULL output");
  rbe_status st = check_desc(d, box_host);
  if (st != RBE_OK) return st;
  *bytes = footprint(nullptr, d, box_host);
  return RBE_OK;
}

rbe_status rbe_batch_admit(rbe_batch b, const rbe_system_desc* d, const double* h_pos,
                           const double* h_mom, const double* h_q, const double* h_mass,
                           const int32_t* h_type, const double* h_lj, const double* box_host,
                           int32_t* slot_out) {
  if (!b || !h_pos || !h_q || !h_mass || !slot_out) return bfail(RBE_ERR_ARG, "NULL argument to rbe_batch_admit");
  *slot_out = -1;
  rbe_status st = check_desc(d, box_host);
  if (st != RBE_OK) return st;
  if (d->ntypes > 0 && (!h_type || !h_lj)) return bfail(RBE_ERR_ARG, "ntypes > 0 needs types and LJ coefficients");
  int sl = -1;
  for (int i = 0; i < (int)b->slots.size(); ++i)
    if (!b->slots[i].active) { sl = i; break; }
  if (sl < 0) return bfail(RBE_ERR_CAPACITY, "all %d slots are in use", b->cfg.max_systems);
  const int64_t need = footprint(b, d, box_host);
  if (b->bytes_in_use + need > b->cfg.hbm_budget)
    return bfail(RBE_ERR_CAPACITY, "system needs %lld bytes, %lld of %lld in use", (long long)need,
                 (long long)b->bytes_in_use, (long long)b->cfg.hbm_budget);

  Slot& s = b->slots[sl];
  s = Slot{};
  s.desc = *d;
  const int64_t n = d->n;
  if (hipMalloc(&s.mem, (size_t)state_bytes(n)) != hipSuccess) {
    s = Slot{};
    return bfail(RBE_ERR_ALLOC, "device allocation of %lld bytes failed", (long long)state_bytes(n));
  }
  double* base = (double*)s.mem;
  double** arr[] = {&s.x, &s.y, &s.z, &s.px, &s.py, &s.pz, &s.fx, &s.fy, &s.fz, &s.q, &s.mass};
  for (int i = 0; i < 11; ++i) *arr[i] = base + (size_t)i * n;
  s.vk = base + 11 * n; s.vr = s.vk + 6; s.ek = s.vr + 6; s.er = s.ek + 1;
  s.type = (int32_t*)(s.er + 1);

  // host layout [n][3] -> device SoA
  std::vector<double> h((size_t)11 * n + 14, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      h[(size_t)a * n + i] = h_pos[3 * i + a];
      h[(size_t)(3 + a) * n + i] = h_mom ? h_mom[3 * i + a] : 0.0;
    }
  std::memcpy(&h[(size_t)9 * n], h_q, (size_t)n * 8);
  std::memcpy(&h[(size_t)10 * n], h_mass, (size_t)n * 8);
  hipError_t e = hipMemcpyAsync(s.mem, h.data(), h.size() * 8, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess && d->ntypes > 0)
    e = hipMemcpyAsync(s.type, h_type, (size_t)n * 4, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) {
    release_slot(s);
    return bfail(RBE_ERR_DEVICE, "admission copies: %s", hipGetErrorString(e));
  }
  const rbe_config kc = kspace_cfg(b, d, box_host);
  const rbe_real_config rc = real_cfg(b, d);
  const rbe_md_config mc = md_cfg(d);
  st = rbe_init(&kc, s.q, box_host, b->stream, &s.k);
  if (st == RBE_OK && d->sampler == RBE_SAMPLER_MH) st = rbe_set_sampler(s.k, RBE_SAMPLER_MH, 1);
  if (st == RBE_OK) st = rbe_real_init(&rc, s.q, d->ntypes > 0 ? s.type : nullptr, h_lj, box_host, b->stream, &s.r);
  if (st == RBE_OK && d->skin > 0.0) st = rbe_real_set_skin(s.r, d->skin);
  if (st == RBE_OK) st = rbe_md_init(&mc, s.mass, box_host, b->stream, &s.m);
  if (st == RBE_OK && d->rigid_count > 0)
    st = rbe_md_set_rigid(s.m, d->rigid_first, d->rigid_count, d->d_oh, d->d_hh);
  // initial forces and pressure (the batch of the opening evaluation uses
  // step 2^63, outside the range of step indices)
  if (st == RBE_OK) st = rbe_sample_k(s.k, 1ull << 63);
  if (st == RBE_OK) st = rbe_forces_pressure(s.k, s.x, s.y, s.z, s.fx, s.fy, s.fz, 0, s.vk, s.ek);
  if (st == RBE_OK) st = rbe_real_forces(s.r, s.x, s.y, s.z, s.fx, s.fy, s.fz, 1, s.vr, s.er);
  if (st == RBE_OK)
    st = rbe_md_pressure(s.m, s.x, s.y, s.z, s.px, s.py, s.pz, s.fx, s.fy, s.fz, s.vk, s.vr);
  if (st == RBE_OK) {
    // the integrator's mid-step cell drives both force evaluations
    s.box_dev = rbe_md_box_dev(s.m);
    st = rbe_real_set_box_dev(s.r, s.box_dev);
  }
  if (st == RBE_OK && hipStreamSynchronize(b->stream) != hipSuccess)
    st = bfail(RBE_ERR_DEVICE, "admission: initial evaluation failed");
  if (st != RBE_OK) {
    release_slot(s);
    return st;
  }
  s.active = true;
  s.bytes = need;
  b->bytes_in_use += need;
  *slot_out = sl;
  return RBE_OK;
}

namespace {

// One step of every active system: the whole NPT step, or (fourier_only)
// the Fourier-space forces, virial and energy at the current positions and
// cell (the batch of the system's current step).
rbe_status batch_step_impl(rbe_batch b, int32_t fused, bool fourier_only);

rbe_status batch_step(rbe_batch b, int32_t fused, bool fourier_only) {
  if (!b) return bfail(RBE_ERR_ARG, "NULL batch");
  if (b->broken)
    return bfail(RBE_ERR_STATE, "an earlier step failed part way; the batch refuses further steps "
                                "(release or destroy it)");
  const rbe_status st = batch_step_impl(b, fused, fourier_only);
  if (st != RBE_OK) b->broken = true;
  return st;
}

rbe_status batch_step_impl(rbe_batch b, int32_t fused, bool fourier_only) {
  std::vector<int> act;
  for (int i = 0; i < (int)b->slots.size(); ++i)
    if (b->slots[i].active) act.push_back(i);
  if (act.empty()) return RBE_OK;
  const int nsys = (int)act.size();
  const int prec = b->cfg.precision;
  std::vector<MDArgs> md1(nsys), md2(nsys);
  std::vector<StepArgs> ka(nsys);
  std::vector<PendingLaunch> pend(nsys);   // Metropolis-Hastings / frozen-cell draws
  std::vector<RealArgs> ra(nsys);
  std::vector<int> ncap(nsys);
  for (int j = 0; j < nsys; ++j) {
    Slot& s = b->slots[act[j]];
    rbe_status st = RBE_OK;
    if (!fourier_only) {
      st = md_first_args(s.m, s.step, s.x, s.y, s.z, s.px, s.py, s.pz, s.fx, s.fy, s.fz, &md1[j]);
      if (st == RBE_OK) st = rbe_rescale_box_dev(s.k, s.box_dev);
    }
    if (st == RBE_OK) st = rbe_sample_k(s.k, s.step);
    // draws that need standalone kernels are launched after the integrator's
    // first half, which writes the cell they read
    if (st == RBE_OK)
      st = kspace_step_args(s.k, s.x, s.y, s.z, s.fx, s.fy, s.fz, 0, s.vk, s.ek, &ka[j], &pend[j]);
    if (!fourier_only) {
      if (st == RBE_OK) st = real_step_args(s.r, s.x, s.y, s.z, s.fx, s.fy, s.fz, 1, s.vr, s.er, &ra[j], &ncap[j]);
      if (st == RBE_OK)
        st = md_second_args(s.m, s.x, s.y, s.z, s.px, s.py, s.pz, s.fx, s.fy, s.fz, s.vk, s.vr, &md2[j]);
    }
    if (st != RBE_OK) return st;
    s.step++;
  }
  hipError_t e = hipSuccess;
  if (!fused) {
    // every system's kernels launched by themselves, one system after another
    for (int j = 0; j < nsys && e == hipSuccess; ++j) {
      if (!fourier_only) e = launch_md_first(md1[j], b->stream);
      if (e == hipSuccess && kspace_run_pending(b->slots[act[j]].k, pend[j]) != RBE_OK)
        e = hipErrorLaunchFailure;
      if (e == hipSuccess) e = launch_sfac(prec, ka[j], b->stream);
      if (e == hipSuccess) e = launch_force(prec, ka[j], b->stream);
      if (!fourier_only) {
        if (e == hipSuccess) e = launch_real(ra[j], ncap[j], b->stream);
        if (e == hipSuccess) e = launch_md_second(md2[j], 0, b->stream);
      }
    }
    b->steps_launched++;
    if (e != hipSuccess) return bfail(RBE_ERR_DEVICE, "step launches: %s", hipGetErrorString(e));
    return RBE_OK;
  }

  Stage& stg = b->stage[b->cur];
  // the previous copy out of this buffer must be done before it is rewritten
  e = hipEventSynchronize(stg.done);
  if (e != hipSuccess) return bfail(RBE_ERR_DEVICE, "stage event: %s", hipGetErrorString(e));
  stg.used = 0;
  stg.overflow = false;

  auto prefix = [](const std::vector<int>& cnt) {
    std::vector<int> o(cnt.size() + 1, 0);
    for (size_t i = 0; i < cnt.size(); ++i) o[i + 1] = o[i] + cnt[i];
    return o;
  };
  // binning kernels: bin_blocks(n); pairs: pair_blocks(n); integrator: kMdThreads units (rigid
  // molecules or free atoms) per block; cell sort: one block per cell of
  // the capacity
  std::vector<int> pb(nsys), ub(nsys), cb(nsys), qb(nsys), vb(nsys), bb(nsys);
  const bool p32 = b->cfg.real_precision == RBE_PREC_FP32;
  int any_list = 0, any_cells = 0, max_types = 0, series = 0;
  for (int j = 0; j < nsys && !fourier_only; ++j) {
    vb[j] = (int)((b->slots[act[j]].desc.n + 255) / 256);
    if (ra[j].skin > 0.0) any_list = 1; else any_cells = 1;
    max_types = std::max(max_types, ra[j].ntypes);
    series |= short_series(ra[j]) ? 1 : 2;
    pb[j] = (int)bin_blocks(b->slots[act[j]].desc.n);
    ub[j] = (int)md_blocks(md_units(md1[j]));
    cb[j] = ncap[j];
    qb[j] = (int)(ra[j].skin > 0.0 ? list_blocks(b->slots[act[j]].desc.n, p32)
                                    : pair_blocks(b->slots[act[j]].desc.n, p32));
    bb[j] = (int)build_blocks(b->slots[act[j]].desc.n);
  }
  const std::vector<int> pstart = prefix(pb), ustart = prefix(ub), cstart = prefix(cb),
                         qstart = prefix(qb), vstart = prefix(vb), bstart = prefix(bb);
  const MDArgs* d_md1 = nullptr; const MDArgs* d_md2 = nullptr; const RealArgs* d_ra = nullptr;
  const int *d_pstart = nullptr, *d_ustart = nullptr, *d_qstart = nullptr, *d_vstart = nullptr,
            *d_bstart_b = nullptr, *d_cstart = nullptr;
  if (!fourier_only) {
    d_md1 = put(b, md1.data(), nsys);
    d_md2 = put(b, md2.data(), nsys);
    d_ra = put(b, ra.data(), nsys);
    d_pstart = put(b, pstart.data(), nsys + 1);
    d_ustart = put(b, ustart.data(), nsys + 1);
    d_qstart = put(b, qstart.data(), nsys + 1);
    d_vstart = put(b, vstart.data(), nsys + 1);
    d_bstart_b = put(b, bstart.data(), nsys + 1);
    d_cstart = put(b, cstart.data(), nsys + 1);
  }
  // structure factors grouped by lane width, forces by block shape
  struct Group { std::vector<int> idx; const StepArgs* tab; const int* start; int total; size_t lds; };
  std::map<int, Group> sg, fg;
  for (int j = 0; j < nsys; ++j) {
    sg[ka[j].R].idx.push_back(j);
    fg[ka[j].KS * ka[j].PW * kWave].idx.push_back(j);
  }
  for (auto* groups : {&sg, &fg}) {
    const bool sf = groups == &sg;
    for (auto& kv : *groups) {
      Group& g = kv.second;
      std::vector<StepArgs> tab;
      std::vector<int> cnt;
      g.lds = 0;
      for (int j : g.idx) {
        tab.push_back(ka[j]);
        cnt.push_back(sf ? sfac_blocks(ka[j]) : force_blocks(prec, ka[j]));
        if (sf) g.lds = std::max(g.lds, sfac_lds_bytes(ka[j]));
      }
      const std::vector<int> st = prefix(cnt);
      g.total = st.back();
      g.tab = put(b, tab.data(), tab.size());
      g.start = put(b, st.data(), st.size());
    }
  }
  if (stg.overflow) return bfail(RBE_ERR_STATE, "argument table overflow");
  e = hipMemcpyAsync(stg.dev, stg.host, stg.used, hipMemcpyHostToDevice, b->stream);
  if (e == hipSuccess) e = hipEventRecord(stg.done, b->stream);
  // timing: an event before each kernel family and one after the last
  hipEvent_t* tev = nullptr;
  if (b->timed < b->timing_cap) {
    tev = &b->ev[(size_t)b->timed * (rbe_batch_s::kKinds + 1)];
    b->timed++;
    for (int j = 0; j < nsys; ++j) b->timed_np += (double)ka[j].n * (double)ka[j].p;
  }
  auto mark = [&](int k) {
    if (tev && e == hipSuccess) e = hipEventRecord(tev[k], b->stream);
  };
  mark(0);
  if (e == hipSuccess && !fourier_only) e = launch_md_first_multi(d_md1, d_ustart, nsys, ustart.back(), b->stream);
  mark(1);
  for (int j = 0; j < nsys && e == hipSuccess; ++j)
    if (kspace_run_pending(b->slots[act[j]].k, pend[j]) != RBE_OK) e = hipErrorLaunchFailure;
  for (auto& kv : sg)
    if (e == hipSuccess)
      e = launch_sfac_multi(prec, kv.first, kv.second.tab, kv.second.start, (int)kv.second.idx.size(),
                            kv.second.total, kv.second.lds, b->stream);
  mark(2);
  for (auto& kv : fg)
    if (e == hipSuccess)
      e = launch_force_multi(prec, kv.first, kv.second.tab, kv.second.start, (int)kv.second.idx.size(),
                             kv.second.total, b->stream);
  mark(3);
  if (e == hipSuccess && !fourier_only)
    e = launch_real_multi(d_ra, d_pstart, pstart.back(), d_cstart, cstart.back(), d_qstart,
                          qstart.back(), d_bstart_b, bstart.back(), d_vstart, vstart.back(), any_list,
                          any_cells, max_types, nsys,
                          b->cfg.real_precision == RBE_PREC_FP32, series, b->stream);
  mark(4);
  if (e == hipSuccess && !fourier_only)
    e = launch_md_second_multi(d_md2, d_ustart, nsys, ustart.back(), 0, b->stream);
  mark(5);
  b->cur ^= 1;
  b->steps_launched++;
  if (e != hipSuccess) return bfail(RBE_ERR_DEVICE, "fused step launches: %s", hipGetErrorString(e));
  return RBE_OK;
}

}  // namespace

rbe_status rbe_batch_step(rbe_batch b, int32_t fused) { return batch_step(b, fused, false); }

rbe_status rbe_batch_step_fourier(rbe_batch b, int32_t fused) { return batch_step(b, fused, true); }

rbe_status rbe_batch_sync(rbe_batch b) {
  if (!b) return bfail(RBE_ERR_ARG, "NULL batch");
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bfail(RBE_ERR_DEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
  return RBE_OK;
}

rbe_status rbe_batch_read(rbe_batch b, int32_t slot, double* h_pos, double* h_mom, double* h_frc,
                          double* h_state) {
  if (!b) return bfail(RBE_ERR_ARG, "NULL batch");
  if (slot < 0 || slot >= (int)b->slots.size() || !b->slots[slot].active)
    return bfail(RBE_ERR_ARG, "slot %d is not admitted", slot);
  Slot& s = b->slots[slot];
  const int64_t n = s.desc.n;
  std::vector<double> h((size_t)9 * n);
  hipError_t e = hipMemcpyAsync(h.data(), s.mem, h.size() * 8, hipMemcpyDeviceToHost, b->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bfail(RBE_ERR_DEVICE, "read state: %s", hipGetErrorString(e));
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      if (h_pos) h_pos[3 * i + a] = h[(size_t)a * n + i];
      if (h_mom) h_mom[3 * i + a] = h[(size_t)(3 + a) * n + i];
      if (h_frc) h_frc[3 * i + a] = h[(size_t)(6 + a) * n + i];
    }
  if (h_state) return rbe_md_get_state(s.m, h_state);
  return RBE_OK;
}

rbe_status rbe_batch_list_stats(rbe_batch b, int32_t slot, int64_t* h_stats) {
  if (!b) return bfail(RBE_ERR_ARG, "NULL batch");
  if (slot < 0 || slot >= (int)b->slots.size() || !b->slots[slot].active)
    return bfail(RBE_ERR_ARG, "slot %d is not admitted", slot);
  return rbe_real_list_stats(b->slots[slot].r, h_stats);
}

rbe_status rbe_batch_check(rbe_batch b, int32_t slot) {
  if (!b) return bfail(RBE_ERR_ARG, "NULL batch");
  if (slot < 0 || slot >= (int)b->slots.size() || !b->slots[slot].active)
    return bfail(RBE_ERR_ARG, "slot %d is not admitted", slot);
  Slot& s = b->slots[slot];
  rbe_status st = rbe_check(s.k);
  if (st == RBE_OK) st = rbe_real_check(s.r);
  if (st == RBE_OK) st = rbe_md_check(s.m);
  return st;
}

rbe_status rbe_batch_release(rbe_batch b, int32_t slot) {
  if (!b) return bfail(RBE_ERR_ARG, "NULL batch");
  if (slot < 0 || slot >= (int)b->slots.size() || !b->slots[slot].active)
    return bfail(RBE_ERR_ARG, "slot %d is not admitted", slot);
  Slot& s = b->slots[slot];
  // kernels of launched steps may still read the slot's memory
  hipError_t e = hipStreamSynchronize(b->stream);
  b->bytes_in_use -= s.bytes;
  release_slot(s);
  if (e != hipSuccess) return bfail(RBE_ERR_DEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
  return RBE_OK;
}

rbe_status rbe_batch_info(rbe_batch b, int64_t* h) {
  if (!b || !h) return bfail(RBE_ERR_ARG, "NULL argument");
  int64_t act = 0;
  for (const Slot& s : b->slots) act += s.active ? 1 : 0;
  h[0] = act;
  h[1] = b->bytes_in_use;
  h[2] = b->cfg.hbm_budget;
  h[3] = b->steps_launched;
  return RBE_OK;
}

rbe_status rbe_batch_slot_step(rbe_batch b, int32_t slot, int64_t* step) {
  if (!b || !step) return bfail(RBE_ERR_ARG, "NULL argument");
  if (slot < 0 || slot >= (int)b->slots.size() || !b->slots[slot].active)
    return bfail(RBE_ERR_ARG, "slot %d is not admitted", slot);
  *step = (int64_t)b->slots[slot].step;
  return RBE_OK;
}

rbe_status rbe_batch_timing_enable(rbe_batch b, int32_t max_steps) {
  if (!b) return bfail(RBE_ERR_ARG, "NULL batch");
  if (max_steps < 0) return bfail(RBE_ERR_ARG, "max_steps = %d must be >= 0", max_steps);
  (void)hipStreamSynchronize(b->stream);
  for (hipEvent_t e : b->ev)
    if (e) (void)hipEventDestroy(e);
  b->ev.clear();
  b->timing_cap = b->timed = 0;
  b->timed_np = 0.0;
  if (max_steps == 0) return RBE_OK;
  b->ev.assign((size_t)max_steps * (rbe_batch_s::kKinds + 1), nullptr);
  for (hipEvent_t& e : b->ev)
    if (hipEventCreate(&e) != hipSuccess) {
      e = nullptr;
      return bfail(RBE_ERR_DEVICE, "hipEventCreate failed");
    }
  b->timing_cap = max_steps;
  return RBE_OK;
}

rbe_status rbe_batch_timing_read(rbe_batch b, double* h_ms, int32_t* h_steps, double* h_np) {
  if (!b || !h_ms || !h_steps || !h_np) return bfail(RBE_ERR_ARG, "NULL argument");
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return bfail(RBE_ERR_DEVICE, "hipStreamSynchronize: %s", hipGetErrorString(e));
  for (int k = 0; k < rbe_batch_s::kKinds; ++k) h_ms[k] = 0.0;
  for (int s = 0; s < b->timed; ++s) {
    const hipEvent_t* t = &b->ev[(size_t)s * (rbe_batch_s::kKinds + 1)];
    for (int k = 0; k < rbe_batch_s::kKinds; ++k) {
      float ms = 0.f;
      e = hipEventElapsedTime(&ms, t[k], t[k + 1]);
      if (e != hipSuccess) return bfail(RBE_ERR_DEVICE, "hipEventElapsedTime: %s", hipGetErrorString(e));
      h_ms[k] += ms;
    }
  }
  *h_steps = b->timed;
  *h_np = b->timed_np;
  b->timed = 0;
  b->timed_np = 0.0;
  return RBE_OK;
}

void rbe_batch_destroy(rbe_batch b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  for (hipEvent_t e : b->ev)
    if (e) (void)hipEventDestroy(e);
  for (Slot& s : b->slots)
    if (s.active || s.mem) release_slot(s);
  for (Stage& st : b->stage) {
    if (st.host) (void)hipHostFree(st.host);
    if (st.dev) (void)hipFree(st.dev);
    if (st.done) (void)hipEventDestroy(st.done);
  }
  delete b;
}

}  // extern "C"
