// C ABI of the real-space pair sum (declarations and contracts in include/rbe.h).
#include "rbe_real_internal.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <new>
#include <string>
#include <vector>

using namespace rbe;

namespace rbe {
// shared with rbe_api.cpp: thread-local error text
rbe_status set_error(rbe_status st, const char* msg);
}

struct rbe_real_ctx_s {
  rbe_real_config cfg;
  hipStream_t stream = nullptr;
  RealArgs a{};
  int ncell_cap = 0;
  int nblocks = 0;
  double box0[3] = {0, 0, 0};
  void* bufs[28] = {};
  int nbufs = 0;
  int64_t evals = 0;  // evaluations launched
};

namespace {

rbe_status rfail(rbe_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return rbe::set_error(st, buf);
}

template <typename T>
bool ralloc(rbe_real_ctx_s* c, T** p, size_t count) {
  if (hipMalloc((void**)p, count * sizeof(T) + 16) != hipSuccess) { *p = nullptr; return false; }
  c->bufs[c->nbufs++] = *p;
  return true;
}

void rfree(rbe_real_ctx_s* c) {
  for (int i = 0; i < c->nbufs; ++i) (void)hipFree(c->bufs[i]);
  c->nbufs = 0;
}

rbe_status check_real_box(const rbe_real_ctx_s* c, const double* box) {
  if (!box) return rfail(RBE_ERR_ARG, "box pointer is NULL");
  for (int d = 0; d < 3; ++d) {
    if (!(std::isfinite(box[d]) && box[d] > 0.0)) return rfail(RBE_ERR_ARG, "box[%d] = %g is not a positive finite length", d, box[d]);
    const double rs = c->cfg.rc + c->a.skin;
    if (box[d] < 2.5 * rs) return rfail(RBE_ERR_ARG, "box[%d] = %g is below 2.5 x the search radius = %g", d, box[d], 2.5 * rs);
    if (std::floor(2.0 * box[d] / c->cfg.rc) > c->a.nc_cap[d]) return rfail(RBE_ERR_CAPACITY, "box[%d] = %g exceeds the cell capacity", d, box[d]);
  }
  return RBE_OK;
}

}  // namespace

namespace rbe {

rbe_status real_step_args(rbe_real_ctx c, const double* d_x, const double* d_y, const double* d_z,
                          double* d_fx, double* d_fy, double* d_fz, int accumulate,
                          double* d_virial6, double* d_energy, RealArgs* out, int* ncell_cap) {
  if (!c) return rfail(RBE_ERR_ARG, "NULL context");
  if (!d_x || !d_y || !d_z || !d_fx || !d_fy || !d_fz) return rfail(RBE_ERR_ARG, "NULL particle array");
  RealArgs a = c->a;
  a.x = d_x; a.y = d_y; a.z = d_z;
  a.fx = d_fx; a.fy = d_fy; a.fz = d_fz;
  a.accumulate = accumulate ? 1 : 0;
  a.virial6 = d_virial6; a.energy = d_energy;
  ++c->evals;
  *out = a;
  *ncell_cap = c->ncell_cap;
  return RBE_OK;
}

int32_t list_capacity(int64_t n, const double* box, double rc, double skin) {
  const double rho = (double)n / (box[0] * box[1] * box[2]);
  const double rs = rc + skin;
  const double mean = rho * 4.18879020478639 * rs * rs * rs;    // (4 pi/3) rs^3 rho
  const int64_t k = (int64_t)std::ceil(1.6 * mean + 64.0);
  return (int32_t)std::max<int64_t>((k + 31) / 32 * 32, kListMin);
}

int64_t real_footprint(const rbe_real_config* cfg, const double* box, double skin) {
  int64_t cap = 1;
  for (int d = 0; d < 3; ++d) {
    long v = (long)std::floor(4.0 * box[d] / cfg->rc);
    if (v > kCellAxisMax) v = kCellAxisMax;
    if (v < 5) v = 5;
    cap *= v;
  }
  const int64_t n = cfg->n, blocks = pair_blocks_max(n);
  auto r = [](int64_t b) { return (b + 16 + 255) / 256 * 256; };
  int64_t t = r(8 * n);
  if (cfg->ntypes > 0) t += r(4 * n) + r(16 * (int64_t)cfg->ntypes * cfg->ntypes);
  t += r(4 * n) + r(4 * cap) + r(4 * (cap + 1)) + r(4 * cap) + r(4 * n) + r(32 * n) + r(16 * n) + 2 * r(4 * n) +
       r(16) + r(64 * (blocks + red_groups(blocks))) + r(4 * (red_groups(blocks) + 1)) + r(4);
  if (skin > 0.0) {
    const int64_t kc = list_capacity(n, box, cfg->rc, skin);
    t += r(4 * n * kc) + r(4 * n) + r(24 * n) + r(24) + r(32 * n) + r(8) + r(8) + r(4);
  }
  return t;
}

}  // namespace rbe

extern "C" {

rbe_status rbe_real_init(const rbe_real_config* cfg, const double* d_q, const int32_t* d_type,
                         const double* h_lj, const double* box_host, void* stream,
                         rbe_real_ctx* out) {
  if (!cfg || !d_q || !box_host || !out) return rfail(RBE_ERR_ARG, "NULL argument to rbe_real_init");
  *out = nullptr;
  if (cfg->n < 1) return rfail(RBE_ERR_ARG, "n = %lld must be >= 1", (long long)cfg->n);
  if (cfg->ntypes < 0 || cfg->ntypes > 64) return rfail(RBE_ERR_ARG, "ntypes = %d must be in 0..64", cfg->ntypes);
  if (cfg->ntypes > 0 && (!d_type || !h_lj)) return rfail(RBE_ERR_ARG, "ntypes > 0 needs types and LJ coefficients");
  if (cfg->precision != RBE_PREC_FP64 && cfg->precision != RBE_PREC_FP32)
    return rfail(RBE_ERR_ARG, "unknown precision %d", cfg->precision);
  if (!(std::isfinite(cfg->alpha) && cfg->alpha > 0)) return rfail(RBE_ERR_ARG, "alpha must be positive");
  if (!(std::isfinite(cfg->rc) && cfg->rc > 0)) return rfail(RBE_ERR_ARG, "rc must be positive");
  if (!(std::isfinite(cfg->coulomb) && cfg->coulomb > 0)) return rfail(RBE_ERR_ARG, "coulomb must be positive");
  rbe_real_ctx_s* c = new (std::nothrow) rbe_real_ctx_s();
  if (!c) return rfail(RBE_ERR_ALLOC, "host allocation failed");
  c->cfg = *cfg;
  c->stream = (hipStream_t)stream;
  RealArgs& a = c->a;
  a.n = cfg->n; a.ntypes = cfg->ntypes;
  a.prec32 = cfg->precision == RBE_PREC_FP32 ? 1 : 0;
  a.alpha = cfg->alpha; a.rc = cfg->rc; a.coulomb = cfg->coulomb;
  a.erfcx_short = std::sqrt(cfg->alpha) * cfg->rc <= kErfcxRange ? 1 : 0;
  long cap = 1;
  for (int d = 0; d < 3; ++d) {
    long v = (long)std::floor(4.0 * box_host[d] / cfg->rc);   // cells at least rc/2 wide, box up to 2x
    if (v > kCellAxisMax) v = kCellAxisMax;
    if (v < 5) v = 5;
    a.nc_cap[d] = (int)v;
    cap *= v;
    c->box0[d] = box_host[d];
  }
  {
    rbe_status st = check_real_box(c, box_host);
    if (st != RBE_OK) { delete c; return st; }
  }
  c->ncell_cap = (int)cap;
  c->nblocks = (int)pair_blocks_max(cfg->n);
  const size_t n = (size_t)cfg->n;
  bool ok = true;
  double* dq = nullptr; int32_t* dt = nullptr; double* dlj = nullptr;
  ok = ok && ralloc(c, &dq, n);
  if (cfg->ntypes > 0) {
    ok = ok && ralloc(c, &dt, n);
    ok = ok && ralloc(c, &dlj, (size_t)cfg->ntypes * cfg->ntypes * 2);
  }
  ok = ok && ralloc(c, &a.cellof, n) && ralloc(c, &a.count, (size_t)cap) &&
       ralloc(c, &a.start, (size_t)cap + 1) && ralloc(c, &a.cursor, (size_t)cap) &&
       ralloc(c, &a.list, n) && ralloc(c, &a.xq, n) && ralloc(c, &a.xf, n) && ralloc(c, &a.ts, n) && ralloc(c, &a.cs, n) &&
       ralloc(c, &a.grid, 4) && ralloc(c, &a.part, (size_t)(c->nblocks + red_groups(c->nblocks)) * 8) &&
       ralloc(c, &a.cnt, (size_t)red_groups(c->nblocks) + 1) && ralloc(c, &a.err, 1);
  if (!ok) { rfree(c); delete c; return rfail(RBE_ERR_ALLOC, "device allocation failed"); }
  a.q = dq; a.type = dt; a.lj = dlj;
  hipError_t e = hipSuccess;
  do {
    if ((e = hipMemcpyAsync(dq, d_q, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream)) != hipSuccess) break;
    if (cfg->ntypes > 0) {
      if ((e = hipMemcpyAsync(dt, d_type, n * sizeof(int32_t), hipMemcpyDeviceToDevice, c->stream)) != hipSuccess) break;
      if ((e = hipMemcpyAsync(dlj, h_lj, (size_t)cfg->ntypes * cfg->ntypes * 2 * sizeof(double), hipMemcpyHostToDevice, c->stream)) != hipSuccess) break;
    }
    if ((e = hipMemsetAsync(a.count, 0, (size_t)cap * sizeof(int32_t), c->stream)) != hipSuccess) break;
    if ((e = hipMemsetAsync(a.cnt, 0, ((size_t)red_groups(c->nblocks) + 1) * sizeof(uint32_t), c->stream)) != hipSuccess) break;
    if ((e = hipMemsetAsync(a.err, 0, sizeof(int32_t), c->stream)) != hipSuccess) break;
    e = hipStreamSynchronize(c->stream);
  } while (0);
  if (e != hipSuccess) { rfree(c); delete c; return rfail(RBE_ERR_DEVICE, "init copies: %s", hipGetErrorString(e)); }
  for (int d = 0; d < 3; ++d) a.box[d] = box_host[d];
  a.box_ptr = nullptr;
  *out = c;
  return RBE_OK;
}

rbe_status rbe_real_set_box(rbe_real_ctx c, const double* box_host) {
  if (!c) return rfail(RBE_ERR_ARG, "NULL context");
  rbe_status st = check_real_box(c, box_host);
  if (st != RBE_OK) return st;
  for (int d = 0; d < 3; ++d) c->a.box[d] = box_host[d];
  c->a.box_ptr = nullptr;
  return RBE_OK;
}

rbe_status rbe_real_set_box_dev(rbe_real_ctx c, const double* d_box) {
  if (!c || !d_box) return rfail(RBE_ERR_ARG, "NULL argument");
  c->a.box_ptr = d_box;
  return RBE_OK;
}

rbe_status rbe_real_forces(rbe_real_ctx c, const double* d_x, const double* d_y, const double* d_z,
                           double* d_fx, double* d_fy, double* d_fz, int accumulate,
                           double* d_virial6, double* d_energy) {
  RealArgs a;
  int ncell_cap = 0;
  rbe_status st = rbe::real_step_args(c, d_x, d_y, d_z, d_fx, d_fy, d_fz, accumulate, d_virial6,
                                      d_energy, &a, &ncell_cap);
  if (st != RBE_OK) return st;
  hipError_t e = launch_real(a, ncell_cap, c->stream);
  if (e != hipSuccess) return rfail(RBE_ERR_DEVICE, "real-space kernels: %s", hipGetErrorString(e));
  return RBE_OK;
}

rbe_status rbe_real_set_skin(rbe_real_ctx c, double skin) {
  if (!c) return rfail(RBE_ERR_ARG, "NULL context");
  if (!(skin >= 0.0 && std::isfinite(skin))) return rfail(RBE_ERR_ARG, "skin = %g must be >= 0", skin);
  if (c->a.skin > 0.0) return rfail(RBE_ERR_STATE, "the skin is set already");
  if (skin == 0.0) return RBE_OK;
  RealArgs& a = c->a;
  const double rs = a.rc + skin;
  for (int d = 0; d < 3; ++d)
    if (c->box0[d] < 2.5 * rs)
      return rfail(RBE_ERR_ARG, "box[%d] = %g is below 2.5 (rc + skin) = %g", d, c->box0[d], 2.5 * rs);
  if (a.n > kListIdxMask + 1)
    return rfail(RBE_ERR_ARG, "n = %lld: neighbour lists take at most 2^25 particles", (long long)a.n);
  const size_t n = (size_t)a.n;
  const int32_t kc = list_capacity(a.n, c->box0, a.rc, skin);
  bool ok = ralloc(c, &a.nbr, n * (size_t)kc) && ralloc(c, &a.ncount, n) && ralloc(c, &a.ref, 3 * n) &&
            ralloc(c, &a.ref_box, 3) && ralloc(c, &a.xc, n) && ralloc(c, &a.dmax, 1) &&
            ralloc(c, &a.state, 2) && ralloc(c, &a.vcnt, 1);
  if (!ok) return rfail(RBE_ERR_ALLOC, "device allocation of the neighbour lists failed");
  hipError_t e = hipMemsetAsync(a.dmax, 0, sizeof(unsigned long long), c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(a.state, 0, 2 * sizeof(int32_t), c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(a.vcnt, 0, sizeof(uint32_t), c->stream);
  if (e == hipSuccess) e = hipMemsetAsync(a.ref, 0, 3 * n * sizeof(double), c->stream);
  // every list slot holds a valid index from the start (the pair kernel reads
  // the first 128 slots of a list before its length is known)
  if (e == hipSuccess) e = hipMemsetAsync(a.nbr, 0, n * (size_t)kc * sizeof(int32_t), c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return rfail(RBE_ERR_DEVICE, "list set-up: %s", hipGetErrorString(e));
  a.kcap = kc;
  a.skin = skin;
  return RBE_OK;
}

rbe_status rbe_real_list_stats(rbe_real_ctx c, int64_t* h_stats) {
  if (!c || !h_stats) return rfail(RBE_ERR_ARG, "NULL argument");
  if (hipStreamSynchronize(c->stream) != hipSuccess) return rfail(RBE_ERR_DEVICE, "hipStreamSynchronize failed");
  int32_t st[2] = {0, 0};
  if (c->a.skin > 0.0 && hipMemcpy(st, c->a.state, sizeof st, hipMemcpyDeviceToHost) != hipSuccess)
    return rfail(RBE_ERR_DEVICE, "read the list state");
  h_stats[0] = c->evals;
  h_stats[1] = st[1];
  return RBE_OK;
}

rbe_status rbe_real_check(rbe_real_ctx c) {
  if (!c) return rfail(RBE_ERR_ARG, "NULL context");
  if (hipStreamSynchronize(c->stream) != hipSuccess) return rfail(RBE_ERR_DEVICE, "hipStreamSynchronize failed");
  int32_t err = 0;
  if (hipMemcpy(&err, c->a.err, sizeof err, hipMemcpyDeviceToHost) != hipSuccess) return rfail(RBE_ERR_DEVICE, "read error flags");
  if (err) {
    const int32_t zero = 0;
    (void)hipMemcpy(c->a.err, &zero, sizeof zero, hipMemcpyHostToDevice);
    return rfail(RBE_ERR_CAPACITY, "real space: %s%s%s", (err & 2) ? "cell below 2.5 x the search radius or over capacity; " : "",
                 (err & 4) ? "a cell holds more than 2048 particles; " : "",
                 (err & 8) ? "a neighbour list over capacity" : "");
  }
  return RBE_OK;
}

void rbe_real_destroy(rbe_real_ctx c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  rfree(c);
  delete c;
}

}  // extern "C"
