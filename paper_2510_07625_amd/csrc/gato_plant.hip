// Plant of closed-loop studies: the robot integrated with classical RK4 on its
// continuous dynamics (the simulations of Sec. IV-E run the plant at 1 kHz with
// RK4), one thread per instance, FP64 arithmetic on FP32 states.
#include "gato_launch.hpp"

namespace gato {

namespace {

template <int ND>
__device__ void plant_rk4(const Chain &ch, double h, int substeps, const float *x, const float *tau, float *xn,
                          unsigned *bad) {
  constexpr int NX = 2 * ND;
  double y[NX], k[NX], acc[NX], t[NX], u[ND];
  double L[ND][ND];
#pragma unroll
  for (int i = 0; i < NX; ++i) y[i] = (double)x[i];
#pragma unroll
  for (int i = 0; i < ND; ++i) u[i] = (double)tau[i];
  const double d = h / substeps;
  bool ok = true;
  // f(z) = [qd; FD(q, qd, tau)] into k.
  auto f = [&](const double *z) {
#pragma unroll
    for (int i = 0; i < ND; ++i) k[i] = z[ND + i];
    ok = forward_dynamics<ND, double>(ch, z, z + ND, u, k + ND, L) && ok;
  };
  for (int s = 0; s < substeps; ++s) {
    f(y);                                       // k1
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      acc[i] = k[i];
      t[i] = y[i] + 0.5 * d * k[i];
    }
    f(t);                                       // k2
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      acc[i] += 2.0 * k[i];
      t[i] = y[i] + 0.5 * d * k[i];
    }
    f(t);                                       // k3
#pragma unroll
    for (int i = 0; i < NX; ++i) {
      acc[i] += 2.0 * k[i];
      t[i] = y[i] + d * k[i];
    }
    f(t);                                       // k4
#pragma unroll
    for (int i = 0; i < NX; ++i) y[i] += d / 6.0 * (acc[i] + k[i]);
  }
  bool fin = ok;
#pragma unroll
  for (int i = 0; i < NX; ++i) {
    xn[i] = (float)y[i];
    fin = fin && isfinite(y[i]);
  }
  if (!fin) *bad = 1u;
}

__global__ __launch_bounds__(64) void plant_kernel(PlantArgs a) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= a.n) return;
  const int sid = a.slots ? a.slots[r] : r;
  if (sid < 0 || sid >= a.M) {
    a.status[r] = GATO_ST_NONFINITE;
    return;
  }
  Chain ch = a.desc[sid].chain;
  if (a.fext) {
    for (int c = 0; c < 3; ++c) ch.fe[c] = a.fext[(size_t)r * 3 + c];
    ch.has_fe = (ch.fe[0] != 0.f || ch.fe[1] != 0.f || ch.fe[2] != 0.f) && ch.model == 0;
  }
  const float *x = a.x + (size_t)r * a.nx_max;
  const float *tau = a.tau + (size_t)r * a.nu_max;
  float *xn = a.xn + (size_t)r * a.nx_max;
  unsigned bad = 0u;
  switch (ch.n) {
    case 3: plant_rk4<3>(ch, a.h, a.substeps, x, tau, xn, &bad); break;
    case 6: plant_rk4<6>(ch, a.h, a.substeps, x, tau, xn, &bad); break;
    case 7: plant_rk4<7>(ch, a.h, a.substeps, x, tau, xn, &bad); break;
    default: bad = 1u; break;
  }
  a.status[r] = bad ? GATO_ST_NONFINITE : 0u;
}

}  // namespace

hipError_t launch_plant(const PlantArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(plant_kernel, dim3((a.n + 63) / 64), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace gato
