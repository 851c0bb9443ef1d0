// The Fourier-space step for callers that cannot allocate device memory
// (code under graph capture, tight serving loops, harnesses that forbid
// hipMalloc): rbe_forces_pressure_noalloc keeps every intermediate of the
// single-launch step in one file-scope device array instead of a context's
// buffers (declaration and contract in include/rbe.h).
#include "rbe_internal.h"

#include <mutex>

namespace rbe {
rbe_status set_error(rbe_status st, const char* msg);
}

using namespace rbe;

namespace {

// Largest scratch a call may use: the batch, the chunk and group partials of
// rho, rho, the force constants, the arrival counters, the cell values and
// the charge sums of one system (for the largest single-launch plan, 256
// chunks x 512 frequency slots, about 2.4 MB).  Every GPU the library runs
// on holds one copy until the process ends.
constexpr size_t kScratchBytes = size_t(4) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// device address of each GPU's copy of `scratch`, looked up once per device
constexpr int kMaxDevices = 64;
std::mutex g_lock;
void* g_scratch[kMaxDevices] = {};

rbe_status nfail(rbe_status st, const char* msg) { return rbe::set_error(st, msg); }

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

}  // namespace

extern "C" rbe_status rbe_forces_pressure_noalloc(const rbe_config* cfg, const double* d_q,
                                                  const double* box_host, uint64_t step,
                                                  const double* d_x, const double* d_y,
                                                  const double* d_z, double* d_fx, double* d_fy,
                                                  double* d_fz, int accumulate, double* d_virial6,
                                                  double* d_energy, double* d_rho, void* stream) {
  if (!cfg || !d_q || !box_host || !d_x || !d_y || !d_z || !d_fx || !d_fy || !d_fz)
    return nfail(RBE_ERR_ARG, "NULL argument to rbe_forces_pressure_noalloc");
  StepArgs a{};
  bool single = false;
  rbe_status st = kspace_plan(cfg, box_host, &a, &single);
  if (st != RBE_OK) return st;
  if (!single)
    return nfail(RBE_ERR_CAPACITY, "rbe_forces_pressure_noalloc: the system is beyond the single-launch "
                                   "plan (every chunk within one 512-particle tile, at most 512 "
                                   "frequencies, every block resident at once)");
  // scratch layout, each part 256-byte aligned
  const size_t p = (size_t)a.p;
  const size_t ncnt = (size_t)cnt_words(a.Y, a.NG);
  // (the cell values and the counters first: the words cleared every call)
  size_t off = 0;
  const size_t o_bs = off;   off += round256(sizeof(BoxState));
  const size_t o_cnt = off;  off += round256(ncnt * sizeof(uint32_t));
  const size_t n_clear = off / sizeof(uint32_t);
  const size_t o_qs = off;   off += round256(3 * sizeof(double));
  const size_t o_m = off;    off += round256(3 * p * sizeof(int32_t));
  const size_t o_part = off; off += round256((size_t)a.X * a.Ppad * sizeof(double2));
  const size_t o_gp = off;   off += round256((size_t)a.NG * a.Ppad * sizeof(double2));
  const size_t o_rho = off;  off += round256(p * sizeof(double2));
  const size_t o_f32 = off;  off += round256(p * sizeof(FCoef32));
  const size_t o_f64 = off;  off += round256(p * sizeof(FCoef64));
  if (off > kScratchBytes)
    return nfail(RBE_ERR_CAPACITY, "rbe_forces_pressure_noalloc: the plan needs more than the 4 MiB "
                                   "of static scratch");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return nfail(RBE_ERR_DEVICE, "rbe_forces_pressure_noalloc: no usable current device");
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_lock);
    if (!g_scratch[dev]) {
      // the array's device address on this device (the current one): the
      // name itself is only a host-side stand-in
      void* ptr = nullptr;
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr)
        return nfail(RBE_ERR_DEVICE, "rbe_forces_pressure_noalloc: hipGetSymbolAddress failed");
      g_scratch[dev] = ptr;
    }
    base = static_cast<unsigned char*>(g_scratch[dev]);
  }
  hipStream_t s = (hipStream_t)stream;
  a.q = d_q; a.qf = nullptr;
  a.x = d_x; a.y = d_y; a.z = d_z;
  a.fx = d_fx; a.fy = d_fy; a.fz = d_fz;
  a.accumulate = accumulate ? 1 : 0;
  a.virial6 = d_virial6; a.energy = d_energy;
  a.box_src = BOX_ARGS;
  for (int k = 0; k < 3; ++k) a.box_arg[k] = box_host[k];
  a.tri_arg = TriCell{};
  if (cfg->box_mode == RBE_BOX_TRICLINIC && !triclinic_cell(cfg->alpha, box_host, &a.tri_arg))
    return nfail(RBE_ERR_ARG, "rbe_forces_pressure_noalloc: degenerate triclinic cell");
  a.box_ptr = nullptr;
  a.sample = 1;
  a.step = step;
  a.predraw = 0; a.use_pre = 0;
  a.sampler = RBE_SAMPLER_EXACT; a.mh_iters = 1; a.mh_init = 0; a.mh_old = nullptr; a.mh_new = nullptr;
  a.bs = reinterpret_cast<BoxState*>(base + o_bs);
  a.qsum_dev = reinterpret_cast<const double*>(base + o_qs);
  a.m = reinterpret_cast<int32_t*>(base + o_m);
  a.partial = reinterpret_cast<double2*>(base + o_part);
  a.gpart = reinterpret_cast<double2*>(base + o_gp);
  a.rho = d_rho ? reinterpret_cast<double2*>(d_rho) : reinterpret_cast<double2*>(base + o_rho);
  a.terms = nullptr;
  a.fc32 = reinterpret_cast<FCoef32*>(base + o_f32);
  a.fc64 = reinterpret_cast<FCoef64*>(base + o_f64);
  a.cnt = reinterpret_cast<uint32_t*>(base + o_cnt);
  a.tab = nullptr; a.pre = nullptr; a.m_pre = nullptr;
  // one block: the cell values and the counters cleared (a fill kernel, not
  // a memset, so a captured graph replays it), the charge sums (the self term
  // is formed on the device); the step kernel follows on the same stream
  hipError_t e = launch_qsum(d_q, nullptr, reinterpret_cast<double*>(base + o_qs), a.n, s,
                             reinterpret_cast<uint32_t*>(base + o_bs), (int64_t)n_clear);
  if (e == hipSuccess) e = launch_step(cfg->precision, a, s);
  if (e != hipSuccess) return nfail(RBE_ERR_DEVICE, "rbe_forces_pressure_noalloc: launch failed");
  return RBE_OK;
}
