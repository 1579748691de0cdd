// Instantiations of the fused SQP kernel for n = 6 degrees of freedom.
#include "gato_launch.hpp"
#include "gato_sqp.hpp"

namespace gato {

hipError_t launch_sqp_n6(int kpt, bool f64, int grid, const KArgs &a, hipStream_t s) {
  const dim3 g(grid), b(kBlock);
  switch (kpt * 2 + (f64 ? 1 : 0)) {
    case 2: hipLaunchKernelGGL((sqp_kernel<6, 1, float>), g, b, 0, s, a); break;
    case 3: hipLaunchKernelGGL((sqp_kernel<6, 1, double>), g, b, 0, s, a); break;
    case 4: hipLaunchKernelGGL((sqp_kernel<6, 2, float>), g, b, 0, s, a); break;
    case 5: hipLaunchKernelGGL((sqp_kernel<6, 2, double>), g, b, 0, s, a); break;
    case 8: hipLaunchKernelGGL((sqp_kernel<6, 4, float>), g, b, 0, s, a); break;
    case 9: hipLaunchKernelGGL((sqp_kernel<6, 4, double>), g, b, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Split long solves (four knots per lane group, FP64 Schur): a cooperative
// launch, so that the parts of a solve are resident together.
hipError_t launch_sqp_n6_split(int grid, bool f64, const KArgs &a, hipStream_t s) {
  const void *f = f64 ? reinterpret_cast<const void *>(&sqp_kernel<6, 4, double, false, true>)
                      : reinterpret_cast<const void *>(&sqp_kernel<6, 4, float, false, true>);
  const hipError_t e = cooperative_fits(f, grid);
  if (e != hipSuccess) return e;
  KArgs arg = a;
  void *args[] = {&arg};
  return hipLaunchCooperativeKernel(f, dim3(grid),
                                    dim3(kBlock), args, 0, s);
}

}  // namespace gato
