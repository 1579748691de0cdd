// LDS read-bandwidth probe (include/gato_probe.h): the peak against which the
// solver kernels' LDS traffic is reported. One 512-thread workgroup per CU
// (100 KB of LDS each, so no second workgroup fits) reads 16-byte vectors from
// LDS in an unrolled loop; every lane accumulates what it reads so that no load
// is dead. Two access patterns:
//   0: every lane its own 16 bytes, consecutive lanes consecutive addresses
//      (no bank conflicts: 1 KB of distinct data per wavefront load);
//   1: groups of 16 lanes read the same 16 bytes (the broadcast pattern of the
//      PCG's block-row products: 4 distinct addresses per wavefront load).
// Delivered bytes count 16 per lane per load in both patterns.
#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/gato_probe.h"

namespace {

constexpr int kProbeThreads = 512;
constexpr int kProbeDoubles = 12800;   // 100 KB
constexpr int kProbeUnroll = 16;

__global__ __launch_bounds__(kProbeThreads) void lds_probe_kernel(int pattern, int iters, double *sink,
                                                                   unsigned long long *cycles) {
  __shared__ __align__(16) double buf[kProbeDoubles];
  const int tid = threadIdx.x;
  for (int i = tid; i < kProbeDoubles; i += kProbeThreads) buf[i] = 0.5 * i;
  __syncthreads();
  // Index of the first double of this lane's 16 bytes (even, so 16-byte aligned).
  const int base = pattern == 0 ? 2 * tid : 2 * (tid / 16);
  double a0 = 0.0, a1 = 0.0;
  const unsigned long long t0 = clock64();
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) {
      // Stride 768 doubles between unrolled loads: the highest index read is
      // 2 * 511 + 1 + 768 * 15 < kProbeDoubles.
      const double2 v = *reinterpret_cast<const double2 *>(&buf[base + 768 * u]);
      a0 += v.x;
      a1 += v.y;
    }
    // Keeps the loads inside the loop (the values do not change between passes).
    asm volatile("" : "+v"(a0), "+v"(a1));
  }
  const unsigned long long t1 = clock64();
  sink[(size_t)blockIdx.x * kProbeThreads + tid] = a0 + a1;
  if (tid == 0) cycles[blockIdx.x] = t1 - t0;
}

}  // namespace

extern "C" int gato_probe_lds(int pattern, int iters, double *bytes_per_clk_cu, double *bytes_per_s) {
  if ((pattern != 0 && pattern != 1) || iters < 1 || iters > (1 << 20)) return -1;
  static_assert(2 * (kProbeThreads - 1) + 1 + 768 * (kProbeUnroll - 1) < kProbeDoubles, "probe indices");
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -3;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -3;
  double *sink = nullptr;
  unsigned long long *cyc = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = 0;
  auto done = [&]() {
    if (sink) (void)hipFree(sink);
    if (cyc) (void)hipFree(cyc);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return rc;
  };
  if (hipMalloc((void **)&sink, (size_t)cus * kProbeThreads * sizeof(double)) != hipSuccess ||
      hipMalloc((void **)&cyc, (size_t)cus * sizeof(unsigned long long)) != hipSuccess ||
      hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    rc = -2;
    return done();
  }
  // A warm-up launch, then the timed one.
  for (int r = 0; r < 2; ++r) {
    if (r == 1 && hipEventRecord(e0, nullptr) != hipSuccess) { rc = -3; return done(); }
    hipLaunchKernelGGL(lds_probe_kernel, dim3(cus), dim3(kProbeThreads), 0, nullptr, pattern, iters, sink, cyc);
    if (hipGetLastError() != hipSuccess) { rc = -3; return done(); }
  }
  float ms = 0.f;
  if (hipEventRecord(e1, nullptr) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
      hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
    rc = -3;
    return done();
  }
  std::vector<unsigned long long> c(cus);
  if (hipMemcpy(c.data(), cyc, (size_t)cus * sizeof(unsigned long long), hipMemcpyDeviceToHost) != hipSuccess) {
    rc = -3;
    return done();
  }
  unsigned long long cmax = 0;
  for (unsigned long long v : c) cmax = v > cmax ? v : cmax;
  const double bytes_cu = (double)kProbeThreads * 16.0 * kProbeUnroll * (double)iters;
  if (bytes_per_clk_cu) *bytes_per_clk_cu = cmax ? bytes_cu / (double)cmax : 0.0;
  if (bytes_per_s) *bytes_per_s = ms > 0.f ? bytes_cu * cus / (ms * 1e-3) : 0.0;
  return done();
}
