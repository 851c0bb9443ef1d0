// C ABI of the Langevin NPT integrator (declarations and contracts in include/rbe.h).
#include "rbe_md_internal.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <new>
#include <vector>

using namespace rbe;

namespace rbe {
rbe_status set_error(rbe_status st, const char* msg);
}

struct rbe_md_ctx_s {
  rbe_md_config cfg;
  hipStream_t stream = nullptr;
  MDArgs a{};
  MDCell* d_cell = nullptr;    // [0] start of step, [1] mid step
  double* d_mass = nullptr;
  double* d_part = nullptr;
  uint32_t* d_cnt = nullptr;
  int32_t* d_flags = nullptr;
};

namespace {

rbe_status mfail(rbe_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return rbe::set_error(st, buf);
}

bool pos_fin(double v) { return std::isfinite(v) && v > 0.0; }

void mfree(rbe_md_ctx_s* c) {
  void* b[] = {c->d_cell, c->d_mass, c->d_part, c->d_cnt, c->d_flags};
  for (void* p : b)
    if (p) (void)hipFree(p);
}

}  // namespace

namespace rbe {

rbe_status md_first_args(rbe_md_ctx c, uint64_t step, double* d_x, double* d_y, double* d_z,
                         double* d_px, double* d_py, double* d_pz, const double* d_fx,
                         const double* d_fy, const double* d_fz, MDArgs* out) {
  if (!c || !d_x || !d_y || !d_z || !d_px || !d_py || !d_pz || !d_fx || !d_fy || !d_fz)
    return mfail(RBE_ERR_ARG, "NULL argument");
  MDArgs a = c->a;
  a.x = d_x; a.y = d_y; a.z = d_z; a.px = d_px; a.py = d_py; a.pz = d_pz;
  a.fx = d_fx; a.fy = d_fy; a.fz = d_fz;
  a.step = step;
  a.cell_in = c->d_cell; a.cell_out = c->d_cell + 1;
  *out = a;
  return RBE_OK;
}

rbe_status md_second_args(rbe_md_ctx c, const double* d_x, const double* d_y, const double* d_z,
                          double* d_px, double* d_py, double* d_pz,
                          const double* d_fx, const double* d_fy, const double* d_fz,
                          const double* d_virial_k, const double* d_virial_r, MDArgs* out) {
  if (!c || !d_x || !d_y || !d_z || !d_px || !d_py || !d_pz || !d_fx || !d_fy || !d_fz)
    return mfail(RBE_ERR_ARG, "NULL argument");
  MDArgs a = c->a;
  a.x = const_cast<double*>(d_x); a.y = const_cast<double*>(d_y); a.z = const_cast<double*>(d_z);
  a.px = d_px; a.py = d_py; a.pz = d_pz;
  a.fx = d_fx; a.fy = d_fy; a.fz = d_fz;
  a.virial_k = d_virial_k; a.virial_r = d_virial_r;
  a.cell_in = c->d_cell + 1; a.cell_out = c->d_cell;
  *out = a;
  return RBE_OK;
}

int64_t md_footprint(int64_t n) {
  auto r = [](int64_t b) { return (b + 255) / 256 * 256; };
  const int64_t blocks = md_blocks(n), groups = md_groups(blocks);
  return r(2 * sizeof(MDCell)) + r(8 * n) + r(128 * (blocks + groups)) + r(4 * (groups + 1)) + r(4);
}

}  // namespace rbe

extern "C" {

rbe_status rbe_md_init(const rbe_md_config* cfg, const double* d_mass, const double* box_host,
                       void* stream, rbe_md_ctx* out) {
  if (!cfg || !d_mass || !box_host || !out) return mfail(RBE_ERR_ARG, "NULL argument to rbe_md_init");
  *out = nullptr;
  if (cfg->n < 1) return mfail(RBE_ERR_ARG, "n must be >= 1");
  if (cfg->box_mode != RBE_BOX_ISO && cfg->box_mode != RBE_BOX_SEMIISO && cfg->box_mode != RBE_BOX_ANISO)
    return mfail(RBE_ERR_ARG, "box_mode must be RBE_BOX_ISO, RBE_BOX_SEMIISO or RBE_BOX_ANISO");
  if (cfg->reserved != 0) return mfail(RBE_ERR_ARG, "reserved field must be 0");
  if (!pos_fin(cfg->dt) || !pos_fin(cfg->kT) || !(std::isfinite(cfg->p_ext)) || !pos_fin(cfg->ftm))
    return mfail(RBE_ERR_ARG, "dt, kT and ftm must be positive, p_ext finite");
  if (!(cfg->gamma_p >= 0.0) || !(cfg->gamma_cell >= 0.0)) return mfail(RBE_ERR_ARG, "frictions must be >= 0");
  if (!pos_fin(cfg->mass_cell) || (cfg->box_mode != RBE_BOX_ISO && !pos_fin(cfg->mass_cell_z)))
    return mfail(RBE_ERR_ARG, "barostat masses must be positive");
  for (int d = 0; d < 3; ++d)
    if (!pos_fin(box_host[d])) return mfail(RBE_ERR_ARG, "box[%d] must be positive", d);
  const double tol = 1e-12 * box_host[0];
  if (cfg->box_mode == RBE_BOX_SEMIISO && std::fabs(box_host[1] - box_host[0]) > tol)
    return mfail(RBE_ERR_ARG, "semi-isotropic mode needs lx == ly");
  rbe_md_ctx_s* c = new (std::nothrow) rbe_md_ctx_s();
  if (!c) return mfail(RBE_ERR_ALLOC, "host allocation failed");
  c->cfg = *cfg;
  c->stream = (hipStream_t)stream;
  const size_t n = (size_t)cfg->n;
  // sized for n units (no rigid molecules); rigid molecules need fewer
  const size_t blocks = (size_t)md_blocks((int64_t)n), groups = (size_t)md_groups((int64_t)blocks);
  bool ok = hipMalloc(&c->d_cell, 2 * sizeof(MDCell)) == hipSuccess &&
            hipMalloc(&c->d_mass, n * sizeof(double)) == hipSuccess &&
            hipMalloc(&c->d_part, (blocks + groups) * 16 * sizeof(double)) == hipSuccess &&
            hipMalloc(&c->d_cnt, (groups + 1) * sizeof(uint32_t)) == hipSuccess &&
            hipMalloc(&c->d_flags, sizeof(int32_t)) == hipSuccess;
  if (!ok) { mfree(c); delete c; return mfail(RBE_ERR_ALLOC, "device allocation failed"); }
  MDCell cell{};
  cell.mode = cfg->box_mode == RBE_BOX_ISO ? 0 : (cfg->box_mode == RBE_BOX_SEMIISO ? 1 : 2);
  cell.V = box_host[0] * box_host[1] * box_host[2];
  cell.M = cfg->mass_cell;
  cell.A = box_host[0] * box_host[1];
  cell.L = box_host[2];
  cell.MA = cfg->mass_cell;
  cell.ML = cfg->mass_cell_z;
  for (int d = 0; d < 3; ++d) cell.l[d] = box_host[d];
  cell.Ml[0] = cell.Ml[1] = cfg->mass_cell;
  cell.Ml[2] = cfg->mass_cell_z;
  // isotropic coupling keeps the initial aspect ratio (exactly 1:1:1 for a cubic cell)
  const bool cubic = box_host[1] == box_host[0] && box_host[2] == box_host[0];
  const double L0 = std::cbrt(cell.V);
  for (int d = 0; d < 3; ++d) cell.asp[d] = cubic ? 1.0 : box_host[d] / L0;
  MDCell cells[2] = {cell, cell};
  hipError_t e = hipSuccess;
  do {
    if ((e = hipMemcpyAsync(c->d_mass, d_mass, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream)) != hipSuccess) break;
    if ((e = hipMemcpyAsync(c->d_cell, cells, sizeof cells, hipMemcpyHostToDevice, c->stream)) != hipSuccess) break;
    if ((e = hipMemsetAsync(c->d_cnt, 0, (groups + 1) * sizeof(uint32_t), c->stream)) != hipSuccess) break;
    if ((e = hipMemsetAsync(c->d_flags, 0, sizeof(int32_t), c->stream)) != hipSuccess) break;
    e = hipStreamSynchronize(c->stream);
  } while (0);
  if (e != hipSuccess) { mfree(c); delete c; return mfail(RBE_ERR_DEVICE, "init: %s", hipGetErrorString(e)); }
  MDArgs& a = c->a;
  a.mass = c->d_mass; a.n = cfg->n;
  a.dt = cfg->dt; a.kT = cfg->kT; a.P = cfg->p_ext; a.gp = cfg->gamma_p; a.gc = cfg->gamma_cell;
  a.ftm = cfg->ftm; a.seed = cfg->seed; a.sysid = cfg->system_id;
  a.part = c->d_part; a.cnt = c->d_cnt; a.flags = c->d_flags;
  a.rig_first = 0; a.rig_count = 0;
  *out = c;
  return RBE_OK;
}

rbe_status rbe_md_set_rigid(rbe_md_ctx c, int64_t first, int64_t count, double d_oh, double d_hh) {
  if (!c) return mfail(RBE_ERR_ARG, "NULL context");
  if (count == 0) {
    c->a.rig_first = 0;
    c->a.rig_count = 0;
    return RBE_OK;
  }
  if (first < 0 || count < 0 || first + 3 * count > c->a.n)
    return mfail(RBE_ERR_ARG, "rigid block [%lld, %lld + 3 x %lld) is outside the %lld atoms",
                 (long long)first, (long long)first, (long long)count, (long long)c->a.n);
  if (!(d_oh > 0.0 && std::isfinite(d_oh)) || !(d_hh > 0.0 && d_hh < 2.0 * d_oh))
    return mfail(RBE_ERR_ARG, "bond lengths d_oh = %g, d_hh = %g do not form a triangle", d_oh, d_hh);
  std::vector<double> m((size_t)(3 * count));
  hipError_t e = hipMemcpyAsync(m.data(), c->d_mass + first, m.size() * sizeof(double),
                                hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return mfail(RBE_ERR_DEVICE, "read masses: %s", hipGetErrorString(e));
  const double mo = m[0], mh = m[1];
  for (int64_t k = 0; k < count; ++k)
    if (m[3 * k] != mo || m[3 * k + 1] != mh || m[3 * k + 2] != mh)
      return mfail(RBE_ERR_ARG, "rigid molecule %lld: masses differ from the first molecule's (O, H, H)",
                   (long long)k);
  if (!(mo > 0.0 && mh > 0.0)) return mfail(RBE_ERR_ARG, "masses must be positive");
  const double M = mo + 2.0 * mh;
  const double rc = 0.5 * d_hh;
  const double hgt = std::sqrt(d_oh * d_oh - rc * rc);
  c->a.rig_first = first;
  c->a.rig_count = count;
  c->a.rc = rc;
  c->a.ra = 2.0 * mh * hgt / M;
  c->a.rb = hgt - c->a.ra;
  return RBE_OK;
}

rbe_status rbe_md_pressure(rbe_md_ctx c, const double* d_x, const double* d_y, const double* d_z,
                           double* d_px, double* d_py, double* d_pz, const double* d_fx,
                           const double* d_fy, const double* d_fz, const double* d_virial_k,
                           const double* d_virial_r) {
  MDArgs a;
  rbe_status st = rbe::md_second_args(c, d_x, d_y, d_z, d_px, d_py, d_pz, d_fx, d_fy, d_fz,
                                      d_virial_k, d_virial_r, &a);
  if (st != RBE_OK) return st;
  a.cell_in = c->d_cell; a.cell_out = c->d_cell;
  hipError_t e = launch_md_second(a, 1, c->stream);
  if (e != hipSuccess) return mfail(RBE_ERR_DEVICE, "pressure kernel: %s", hipGetErrorString(e));
  return RBE_OK;
}

rbe_status rbe_md_first_half(rbe_md_ctx c, uint64_t step, double* d_x, double* d_y, double* d_z,
                             double* d_px, double* d_py, double* d_pz, const double* d_fx,
                             const double* d_fy, const double* d_fz) {
  MDArgs a;
  rbe_status st = rbe::md_first_args(c, step, d_x, d_y, d_z, d_px, d_py, d_pz, d_fx, d_fy, d_fz, &a);
  if (st != RBE_OK) return st;
  hipError_t e = launch_md_first(a, c->stream);
  if (e != hipSuccess) return mfail(RBE_ERR_DEVICE, "first half kernel: %s", hipGetErrorString(e));
  return RBE_OK;
}

rbe_status rbe_md_second_half(rbe_md_ctx c, const double* d_x, const double* d_y, const double* d_z,
                              double* d_px, double* d_py, double* d_pz,
                              const double* d_fx, const double* d_fy, const double* d_fz,
                              const double* d_virial_k, const double* d_virial_r) {
  MDArgs a;
  rbe_status st = rbe::md_second_args(c, d_x, d_y, d_z, d_px, d_py, d_pz, d_fx, d_fy, d_fz,
                                      d_virial_k, d_virial_r, &a);
  if (st != RBE_OK) return st;
  hipError_t e = launch_md_second(a, 0, c->stream);
  if (e != hipSuccess) return mfail(RBE_ERR_DEVICE, "second half kernel: %s", hipGetErrorString(e));
  return RBE_OK;
}

const double* rbe_md_box_dev(rbe_md_ctx c) { return c ? c->d_cell[1].l : nullptr; }

rbe_status rbe_md_get_state(rbe_md_ctx c, double* h) {
  if (!c || !h) return mfail(RBE_ERR_ARG, "NULL argument");
  MDCell cell;
  if (hipMemcpyAsync(&cell, c->d_cell, sizeof cell, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return mfail(RBE_ERR_DEVICE, "copy cell state");
  const double f = c->cfg.ftm;
  h[0] = cell.l[0]; h[1] = cell.l[1]; h[2] = cell.l[2];
  h[3] = cell.mode == 0 ? cell.V : (cell.mode == 1 ? cell.A * cell.L : cell.l[0] * cell.l[1] * cell.l[2]);
  h[4] = cell.pV; h[5] = cell.pA; h[6] = cell.pL;
  if (cell.mode == 2) { h[4] = cell.pl[0]; h[5] = cell.pl[1]; h[6] = cell.pl[2]; }
  for (int k = 0; k < 6; ++k) { h[7 + k] = cell.P_ins[k] / f; h[13 + k] = cell.K[k] / f; }
  h[19] = (double)cell.err;
  h[20] = (double)cell.step;
  h[21] = cell.A; h[22] = cell.L; h[23] = cell.V;
  for (int k = 0; k < 6; ++k) h[24 + k] = cell.C[k];
  h[30] = (double)c->a.rig_count;
  h[31] = 0.0;
  return RBE_OK;
}

rbe_status rbe_md_check(rbe_md_ctx c) {
  double h[32];
  rbe_status st = rbe_md_get_state(c, h);
  if (st != RBE_OK) return st;
  if (h[19] != 0.0) return mfail(RBE_ERR_STATE, "the cell collapsed or became non-finite");
  int32_t flags = 0;
  if (hipMemcpy(&flags, c->d_flags, sizeof flags, hipMemcpyDeviceToHost) != hipSuccess)
    return mfail(RBE_ERR_DEVICE, "read constraint flags");
  if (flags) {
    const int32_t zero = 0;
    (void)hipMemcpy(c->d_flags, &zero, sizeof zero, hipMemcpyHostToDevice);
    return mfail(RBE_ERR_STATE, "a rigid-molecule position constraint had no solution (step too long)");
  }
  return RBE_OK;
}

void rbe_md_destroy(rbe_md_ctx c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  mfree(c);
  delete c;
}

}  // extern "C"
