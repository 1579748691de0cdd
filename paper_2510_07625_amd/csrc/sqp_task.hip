// Instantiations of the task-space (tip tracking) variant of the fused SQP
// kernel: 3, 6 and 7 degrees of freedom, one or two knots per lane group.
#include "gato_launch.hpp"
#include "gato_sqp.hpp"

namespace gato {

hipError_t launch_sqp_task(int nd, int kpt, bool f64, int grid, const KArgs &a, hipStream_t s) {
  const dim3 g(grid), b(kBlock);
  switch (nd * 8 + kpt * 2 + (f64 ? 1 : 0)) {
    case 7 * 8 + 2: hipLaunchKernelGGL((sqp_kernel<7, 1, float, true>), g, b, 0, s, a); break;
    case 7 * 8 + 3: hipLaunchKernelGGL((sqp_kernel<7, 1, double, true>), g, b, 0, s, a); break;
    case 7 * 8 + 4: hipLaunchKernelGGL((sqp_kernel<7, 2, float, true>), g, b, 0, s, a); break;
    case 7 * 8 + 5: hipLaunchKernelGGL((sqp_kernel<7, 2, double, true>), g, b, 0, s, a); break;
    case 6 * 8 + 2: hipLaunchKernelGGL((sqp_kernel<6, 1, float, true>), g, b, 0, s, a); break;
    case 6 * 8 + 3: hipLaunchKernelGGL((sqp_kernel<6, 1, double, true>), g, b, 0, s, a); break;
    case 6 * 8 + 4: hipLaunchKernelGGL((sqp_kernel<6, 2, float, true>), g, b, 0, s, a); break;
    case 6 * 8 + 5: hipLaunchKernelGGL((sqp_kernel<6, 2, double, true>), g, b, 0, s, a); break;
    case 3 * 8 + 2: hipLaunchKernelGGL((sqp_kernel<3, 1, float, true>), g, b, 0, s, a); break;
    case 3 * 8 + 3: hipLaunchKernelGGL((sqp_kernel<3, 1, double, true>), g, b, 0, s, a); break;
    case 3 * 8 + 4: hipLaunchKernelGGL((sqp_kernel<3, 2, float, true>), g, b, 0, s, a); break;
    case 3 * 8 + 5: hipLaunchKernelGGL((sqp_kernel<3, 2, double, true>), g, b, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace gato
