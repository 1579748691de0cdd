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

// Tip position of every knot of every solve, one thread per (solve, knot);
// zero beyond a solve's horizon and for the double-integrator model.
__global__ __launch_bounds__(256) void tip_kernel(const SolveDesc *desc, int M, int N_max, int nx_max,
                                                  const float *X, float *P) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= M * N_max) return;
  const int sid = t / N_max, k = t % N_max;
  const SolveDesc &D = desc[sid];
  float p[3] = {0.f, 0.f, 0.f};
  if (k < D.N && D.chain.model == 0) {
    const float *q = X + (size_t)t * nx_max;
    switch (D.n) {
      case 3: tip_position<3>(D.chain, q, p); break;
      case 6: tip_position<6>(D.chain, q, p); break;
      case 7: tip_position<7>(D.chain, q, p); break;
      default: break;
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) P[(size_t)t * 3 + c] = p[c];
}

}  // namespace

hipError_t launch_tips(const SolveDesc *desc, int M, int N_max, int nx_max, const float *X, float *P,
                       hipStream_t s) {
  const int n = M * N_max;
  hipLaunchKernelGGL(tip_kernel, dim3((n + 255) / 256), dim3(256), 0, s, desc, M, N_max, nx_max, X, P);
  return hipGetLastError();
}

hipError_t launch_plant(const PlantArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(plant_kernel, dim3((a.n + 63) / 64), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace gato
