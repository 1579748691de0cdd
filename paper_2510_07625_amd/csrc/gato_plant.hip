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

// Fills n doubles with v (a kernel, so that callers may capture it in a graph).
__global__ __launch_bounds__(256) void fill_kernel(double *p, size_t n, double v) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Shifts the resident trajectory and multipliers of slot slots[b] one knot
// towards the start, the last knot repeated; one workgroup per slot, staged
// through LDS so that the in-place update reads only old values.
__global__ __launch_bounds__(256) void shift_kernel(const SolveDesc *desc, int M, int n, const int *slots, int N_max,
                                                    int nx_max, int nu_max, float *X, float *U, double *lam) {
  __shared__ float xs[GATO_MAX_KNOTS * 2 * kMaxDof];
  __shared__ float us[GATO_MAX_KNOTS * kMaxDof];
  __shared__ double ls[GATO_MAX_KNOTS * 2 * kMaxDof];
  if ((int)blockIdx.x >= n) return;
  const int sid = slots[blockIdx.x];
  if (sid < 0 || sid >= M) return;   // uniform across the workgroup
  const int N = desc[sid].N;
  float *Xs = X + (size_t)sid * N_max * nx_max;
  float *Us = U + (size_t)sid * (N_max - 1) * nu_max;
  double *Ls = lam + (size_t)sid * N_max * nx_max;
  const int nxe = N * nx_max, nue = (N - 1) * nu_max;
  for (int t = threadIdx.x; t < nxe; t += blockDim.x) {
    xs[t] = Xs[t];
    ls[t] = Ls[t];
  }
  for (int t = threadIdx.x; t < nue; t += blockDim.x) us[t] = Us[t];
  __syncthreads();
  for (int t = threadIdx.x; t < nxe; t += blockDim.x) {
    const int k = t / nx_max, j = t - k * nx_max;
    const int ks = min(k + 1, N - 1);
    Xs[t] = xs[ks * nx_max + j];
    Ls[t] = ls[ks * nx_max + j];
  }
  for (int t = threadIdx.x; t < nue; t += blockDim.x) {
    const int k = t / nu_max, j = t - k * nu_max;
    Us[t] = us[min(k + 1, N - 2) * nu_max + j];
  }
}

// Hypothesis selection (gato_select_hypotheses): one wavefront per instance p.
// Lane l scores hypotheses j = l, l + 64, ... by the Euclidean distance between
// their one-step predictions and the measured state (FP64 sums in index
// order), a butterfly takes the smallest distance (the smaller j on ties), the
// estimate moves to that hypothesis and the instance's hypotheses are
// re-centred on it in the device descriptors.
__global__ __launch_bounds__(64) void select_kernel(SolveDesc *desc, int P, int H, int nx_max, const float *pred,
                                                    const float *meas, const double *off, double *est, int *sel,
                                                    double *dist) {
  __shared__ double e[3];
  const int p = blockIdx.x;
  if (p >= P) return;   // uniform across the workgroup
  const int lane = threadIdx.x;
  const size_t first = (size_t)p * H;
  const int nx = 2 * desc[first].n;
  const float *ms = meas + (size_t)p * nx_max;
  double best = INFINITY;
  int bj = H;   // none yet
  for (int j = lane; j < H; j += 64) {
    const float *q = pred + (first + j) * nx_max;
    double s = 0.0;
    for (int i = 0; i < nx; ++i) {
      const double d = (double)q[i] - (double)ms[i];
      s += d * d;
    }
    const double dj = sqrt(s);
    if (dist) dist[first + j] = dj;
    if (dj < best) {   // j ascends per lane, so ties keep the smaller j; NaN never wins
      best = dj;
      bj = j;
    }
  }
  for (int w = 32; w >= 1; w >>= 1) {
    const double ob = __shfl_xor(best, w);
    const int oj = __shfl_xor(bj, w);
    if (ob < best || (ob == best && oj < bj)) {
      best = ob;
      bj = oj;
    }
  }
  const int j = bj < H ? bj : 0;   // every distance non-finite: keep the estimate
  if (lane < 3) {
    const double v = est[(size_t)p * 3 + lane] + off[(size_t)j * 3 + lane];
    est[(size_t)p * 3 + lane] = v;
    e[lane] = v;
  }
  if (lane == 0 && sel) sel[p] = j;
  __syncthreads();
  for (int jj = lane; jj < H; jj += 64) {
    Chain &c = desc[first + jj].chain;
    float f[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      f[a] = (float)(e[a] + off[(size_t)jj * 3 + a]);
      c.fe[a] = f[a];
    }
    c.has_fe = (f[0] != 0.f || f[1] != 0.f || f[2] != 0.f) ? 1 : 0;
  }
}

}  // namespace

hipError_t launch_select(SolveDesc *desc, int P, int H, int nx_max, const float *pred, const float *meas,
                         const double *off, double *est, int *sel, double *dist, hipStream_t s) {
  hipLaunchKernelGGL(select_kernel, dim3(P), dim3(64), 0, s, desc, P, H, nx_max, pred, meas, off, est, sel, dist);
  return hipGetLastError();
}

const void *fill_kernel_fn() { return reinterpret_cast<const void *>(&fill_kernel); }

hipError_t launch_fill(double *p, size_t n, double v, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_shift(const SolveDesc *desc, int M, int n, const int *slots, int N_max, int nx_max, int nu_max,
                        float *X, float *U, double *lam, hipStream_t s) {
  hipLaunchKernelGGL(shift_kernel, dim3(n), dim3(256), 0, s, desc, M, n, slots, N_max, nx_max, nu_max, X, U, lam);
  return hipGetLastError();
}

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
