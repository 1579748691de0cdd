// The mixed-shape SQP kernel of the task-space variant (tip tracking costs),
// both precisions: one launch for an uneven batch with task-space solves; and
// its split form, whose long solves (6-7 DoF, N > 64) run on four workgroups.
#include "gato_launch.hpp"
#include "gato_sqp.hpp"

namespace gato {

hipError_t launch_sqp_mixed_task(int grid, bool f64, const KArgs &a, hipStream_t s) {
  if (f64) hipLaunchKernelGGL((sqp_mixed_kernel<double, true>), dim3(grid), dim3(kBlock), 0, s, a);
  else hipLaunchKernelGGL((sqp_mixed_kernel<float, true>), dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

// With split long solves (FP64 only): a cooperative launch, the four parts of
// a long solve resident together.
hipError_t launch_sqp_mixed_task_split(int grid, const KArgs &a, hipStream_t s) {
  const void *f = sqp_mixed_task_split_fn();
  const hipError_t e = cooperative_fits(f, grid);
  if (e != hipSuccess) return e;
  KArgs arg = a;
  void *args[] = {&arg};
  return hipLaunchCooperativeKernel(f, dim3(grid), dim3(kBlock), args, 0, s);
}

const void *sqp_mixed_task_split_fn() {
  return reinterpret_cast<const void *>(&sqp_mixed_kernel<double, true, true>);
}

}  // namespace gato
