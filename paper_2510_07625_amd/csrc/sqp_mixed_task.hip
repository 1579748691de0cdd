// The mixed-shape SQP kernel of the task-space variant (tip tracking costs),
// both precisions: one launch for an uneven batch with task-space solves.
#include "gato_launch.hpp"
#include "gato_sqp.hpp"

namespace gato {

hipError_t launch_sqp_mixed_task(int grid, bool f64, const KArgs &a, hipStream_t s) {
  if (f64) hipLaunchKernelGGL((sqp_mixed_kernel<double, true>), dim3(grid), dim3(kBlock), 0, s, a);
  else hipLaunchKernelGGL((sqp_mixed_kernel<float, true>), dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace gato
