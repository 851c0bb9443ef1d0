// Issue-rate microbenchmarks behind the roofline peaks: the device's own
// rates of FP32 sines (the transcendental unit), FP32 and FP64 fused
// multiply-adds, and sines mixed with multiply-adds (whether the two kinds
// of instruction issue side by side).  Declaration in include/rbe.h
// (rbe_measure_issue_rates).
#include "rbe_internal.h"

#include <vector>

namespace rbe {
rbe_status set_error(rbe_status st, const char* msg);
}

namespace {

constexpr int kChains = 8;         // independent dependency chains per thread
constexpr int kThreads = 256;

// kind 0: FP32 sines; 1: FP32 FMAs; 2: FP64 FMAs; 3: one sine and four FP32
// FMAs per chain step.  Every chain is folded into one store per thread.
template <int Kind>
__global__ void __launch_bounds__(kThreads) k_rate(int iters, float* out32, double* out64) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (Kind == 2) {
    double v[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) v[c] = 1.0 + 1e-3 * (t % 7) + 1e-4 * c;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
      for (int c = 0; c < kChains; ++c) v[c] = fma(v[c], 0.999999, 1e-7);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += v[c];
    out64[t] = s;
    return;
  }
  float v[kChains], w[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) { v[c] = 0.1f + 1e-3f * (t % 7) + 1e-4f * c; w[c] = v[c]; }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      if (Kind == 0) {
        v[c] = __builtin_amdgcn_sinf(v[c]);
      } else if (Kind == 1) {
        v[c] = fmaf(v[c], 0.999999f, 1e-7f);
      } else {
        v[c] = __builtin_amdgcn_sinf(v[c]);
        w[c] = fmaf(w[c], 0.999999f, 1e-7f);
        w[c] = fmaf(w[c], 0.999999f, 1e-7f);
        w[c] = fmaf(w[c], 0.999999f, 1e-7f);
        w[c] = fmaf(w[c], 0.999999f, 1e-7f);
      }
    }
  }
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += v[c] + w[c];
  out32[t] = s;
}

template <int Kind>
hipError_t time_kind(int blocks, int iters, float* o32, double* o64, hipEvent_t e0, hipEvent_t e1,
                     float* ms) {
  hipLaunchKernelGGL(k_rate<Kind>, dim3(blocks), dim3(kThreads), 0, 0, iters, o32, o64);  // warm-up
  hipError_t e = hipEventRecord(e0, 0);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_rate<Kind>, dim3(blocks), dim3(kThreads), 0, 0, iters, o32, o64);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, 0);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
  return e;
}

}  // namespace

extern "C" rbe_status rbe_measure_issue_rates(double* h_out) {
  if (!h_out) return rbe::set_error(RBE_ERR_ARG, "NULL argument");
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return rbe::set_error(RBE_ERR_DEVICE, "rbe_measure_issue_rates: device query failed");
  const int blocks = cus * 16;              // 16 blocks of 4 waves per compute unit
  const int iters = 4096;
  float* o32 = nullptr;
  double* o64 = nullptr;
  const size_t n = (size_t)blocks * kThreads;
  if (hipMalloc(&o32, n * sizeof(float)) != hipSuccess) return rbe::set_error(RBE_ERR_ALLOC, "rates buffer");
  if (hipMalloc(&o64, n * sizeof(double)) != hipSuccess) {
    (void)hipFree(o32);
    return rbe::set_error(RBE_ERR_ALLOC, "rates buffer");
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  float ms[4] = {0, 0, 0, 0};
  if (e == hipSuccess) e = time_kind<0>(blocks, iters, o32, o64, e0, e1, &ms[0]);
  if (e == hipSuccess) e = time_kind<1>(blocks, iters, o32, o64, e0, e1, &ms[1]);
  if (e == hipSuccess) e = time_kind<2>(blocks, iters, o32, o64, e0, e1, &ms[2]);
  if (e == hipSuccess) e = time_kind<3>(blocks, iters, o32, o64, e0, e1, &ms[3]);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(o32);
  (void)hipFree(o64);
  if (e != hipSuccess) return rbe::set_error(RBE_ERR_DEVICE, "rbe_measure_issue_rates: a launch failed");
  const double ops = (double)n * iters * kChains;
  h_out[0] = ops / (ms[0] * 1e-3);          // FP32 sines per second
  h_out[1] = ops / (ms[1] * 1e-3);          // FP32 FMAs per second
  h_out[2] = ops / (ms[2] * 1e-3);          // FP64 FMAs per second
  h_out[3] = ops / (ms[3] * 1e-3);          // sines per second with 4 FMAs beside each
  h_out[4] = (double)cus;
  return RBE_OK;
}
