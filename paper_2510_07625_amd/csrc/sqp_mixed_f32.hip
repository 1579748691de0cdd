// The mixed-shape SQP kernel (float Schur rows and PCG vectors): one launch for a
// batch of uneven DoF and horizon.
#include "gato_launch.hpp"
#include "gato_sqp.hpp"

namespace gato {

hipError_t launch_sqp_mixed_f32(int grid, const KArgs &a, hipStream_t s) {
  hipLaunchKernelGGL((sqp_mixed_kernel<float>), dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace gato
