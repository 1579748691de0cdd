// The mixed-shape SQP kernel (double Schur rows and PCG vectors): one launch for a
// batch of uneven DoF and horizon.
#include "gato_launch.hpp"
#include "gato_sqp.hpp"

namespace gato {

hipError_t launch_sqp_mixed_f64(int grid, const KArgs &a, hipStream_t s) {
  hipLaunchKernelGGL((sqp_mixed_kernel<double>), dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

// With split long solves: a cooperative launch (the parts of a solve are
// resident together).
hipError_t launch_sqp_mixed_f64_split(int grid, const KArgs &a, hipStream_t s) {
  const void *f = reinterpret_cast<const void *>(&sqp_mixed_kernel<double, false, true>);
  const hipError_t e = cooperative_fits(f, grid);
  if (e != hipSuccess) return e;
  KArgs arg = a;
  void *args[] = {&arg};
  return hipLaunchCooperativeKernel(f, dim3(grid),
                                    dim3(kBlock), args, 0, s);
}

// The split mixed-shape kernel itself, for launches built as graph nodes.
const void *sqp_mixed_f64_split_fn() {
  return reinterpret_cast<const void *>(&sqp_mixed_kernel<double, false, true>);
}

}  // namespace gato
