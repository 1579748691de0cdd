// Kernel instantiation table shared by the host library and the translation
// units that instantiate the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "gato_internal.hpp"

namespace gato {

// Launches the fused SQP kernel for n = nd, knots-per-group kpt, precision f64
// on `grid` workgroups. Returns hipErrorInvalidValue for shapes that were not
// compiled.
hipError_t launch_sqp(int nd, int kpt, bool f64, int grid, const KArgs &a, hipStream_t s);

// The same for the task-space variant (tip tracking costs): kpt 1 and 2.
hipError_t launch_sqp_task(int nd, int kpt, bool f64, int grid, const KArgs &a, hipStream_t s);
// The mixed-shape kernel of the task-space variant.
hipError_t launch_sqp_mixed_task(int grid, bool f64, const KArgs &a, hipStream_t s);
// Its split form (FP64; a cooperative launch, as the other split kernels).
hipError_t launch_sqp_mixed_task_split(int grid, const KArgs &a, hipStream_t s);
// Largest knots per lane group of the one-workgroup task-space kernels; longer
// task-space solves run only split.
constexpr int kTaskKptMax = 2;

// The number of workgroups of kernel f (kBlock threads) that fit the current
// device at once.
inline hipError_t cooperative_capacity(const void *f, int *cap) {
  int per_cu = 0, dev = 0, cus = 0;
  *cap = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kBlock, 0);
  if (e != hipSuccess) return e;
  e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  *cap = per_cu * cus;
  return hipSuccess;
}

// hipSuccess when `grid` workgroups of kernel f fit the device at once (the
// condition of a cooperative launch), hipErrorCooperativeLaunchTooLarge when
// they do not (nothing is launched then).
inline hipError_t cooperative_fits(const void *f, int grid) {
  int cap = 0;
  const hipError_t e = cooperative_capacity(f, &cap);
  if (e != hipSuccess) return e;
  return cap >= grid ? hipSuccess : hipErrorCooperativeLaunchTooLarge;
}

// Launches the closed-loop plant step (RK4, one thread per instance).
hipError_t launch_plant(const PlantArgs &a, hipStream_t s);

// Fills n doubles with v.
hipError_t launch_fill(double *p, size_t n, double v, hipStream_t s);
// The fill kernel (double *p, size_t n, double v; 256 threads per workgroup),
// for launches built as graph nodes.
const void *fill_kernel_fn();
// The split mixed-shape kernels (one KArgs argument, kBlock threads).
const void *sqp_mixed_f64_split_fn();
const void *sqp_mixed_f32_split_fn();
const void *sqp_mixed_task_split_fn();

// Exchange-tag epoch of split launches replayed from a graph. Eager launches
// cycle through 1..kGraphEpoch-1, so words a replay leaves behind never carry
// an eager launch's tag; every replay clears the words before its kernel.
constexpr unsigned kGraphEpoch = 65535u;

// Shifts the resident trajectories and multipliers of n slots one knot.
hipError_t launch_shift(const SolveDesc *desc, int M, int n, const int *slots, int N_max, int nx_max, int nu_max,
                        float *X, float *U, double *lam, hipStream_t s);

// Hypothesis selection of P instances with H solves each (slots p H + j):
// distances of the predictions to the measured states, argmin, estimate update
// and re-centred forces in the device descriptors.
hipError_t launch_select(SolveDesc *desc, int P, int H, int nx_max, const float *pred, const float *meas,
                         const double *off, double *est, int *sel, double *dist, hipStream_t s);

// Launches the tip kinematics of every knot: X [M][N_max][nx_max] -> P [M][N_max][3].
hipError_t launch_tips(const SolveDesc *desc, int M, int N_max, int nx_max, const float *X, float *P,
                       hipStream_t s);

// Largest compiled knots-per-group value for n DoF (3 DoF: 64 lane groups
// of 8, so 2 knots per group reach the maximum horizon).
inline int kpt_max(int n) { return 2 * n > 8 ? 4 : 2; }

// Register-resident PCG rows: the smallest knots per lane group for a solve
// of n DoF and N knots (0 if N is too large).
inline int kpt_for(int n, int N) {
  const int G = (2 * n > 8) ? 16 : 8;
  const int slots = kBlock / G;
  for (int k = 1; k <= kpt_max(n); k *= 2)
    if (N <= k * slots) return k;
  return 0;
}

}  // namespace gato
