// Instantiations of the fused SQP kernel for n = 3 degrees of freedom.
#include "gato_launch.hpp"
#include "gato_sqp.hpp"

namespace gato {

hipError_t launch_sqp_n3(int kpt, bool f64, int grid, const KArgs &a, hipStream_t s) {
  const dim3 g(grid), b(kBlock);
  switch (kpt * 2 + (f64 ? 1 : 0)) {
    case 2: hipLaunchKernelGGL((sqp_kernel<3, 1, float>), g, b, 0, s, a); break;
    case 3: hipLaunchKernelGGL((sqp_kernel<3, 1, double>), g, b, 0, s, a); break;
    case 4: hipLaunchKernelGGL((sqp_kernel<3, 2, float>), g, b, 0, s, a); break;
    case 5: hipLaunchKernelGGL((sqp_kernel<3, 2, double>), g, b, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace gato
