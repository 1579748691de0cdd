// The fused SQP iteration for one trajectory-optimisation solve per workgroup.
//
// One workgroup of kBlock threads owns one solve and runs whole SQP iterations
// (Algorithm 1) without returning to the host:
//   1. LQ:     rigid-body dynamics + derivatives at every knot (Sec. III-A,
//              Eq. (1)); lane (knot, direction) runs one dual-number RNEA.
//   2. Schur:  lane (knot, row) forms its row of theta_k, phi_k and gamma~
//              (Eqs. (5)-(6)) and, inside the knot's lane group, the inverse of
//              the diagonal block by Gauss-Jordan elimination.
//   3. Precon: its row of the stair preconditioner (Eq. (6)), which needs the
//              neighbouring knots' inverses (the paper's single grid-wide
//              synchronisation becomes a workgroup barrier here).
//   4. PCG:    (Sec. II-B, III-B) with the rows of S~ and P held in registers,
//              vectors exchanged through LDS and dot products reduced across
//              the wavefronts of the workgroup.
//   5. Step:   dZ = -G^-1 (g - C^T lambda) (Eq. (4)).
//   6. Line search: lane (alpha, knot) evaluates one trial knot (forward
//              dynamics + stage cost + defect), a fixed-order reduction gives
//              the merit of Eq. (3) per alpha and the argmin of Eq. (7) picks
//              the step.
// The S~ rows, gamma~, PCG vectors and dot products use Real (double by
// default; float for the all-FP32 variant); the dynamics, line search and the
// preconditioner application use float.
#pragma once

#include <hip/hip_runtime.h>

#include "gato_internal.hpp"

namespace gato {

template <int ND>
struct Shape {
  static constexpr int NX = 2 * ND;
  static constexpr int NU = ND;
  static constexpr int G = (2 * ND > 8) ? 16 : 8;  // lanes per knot (power of two >= NX)
  static constexpr int SLOTS = kBlock / G;          // knots handled at once
};

template <int ND, int KPT, class Real>
struct Smem {
  using Sh = Shape<ND>;
  static constexpr int G = Sh::G;
  static constexpr int KN = KPT * Sh::SLOTS;
  float X[KN][G];          // iterate
  float U[KN][8];
  float dX[KN][G];         // step
  float dU[KN][8];
  float e[KN][G];          // defects e_k = f(x_k, u_k) - x_{k+1}
  float qg[KN][G];         // state gradients q_k
  float rg[KN][8];         // control gradients r_k
  float rv[KN][G];         // PCG residual, shared for the preconditioner
  float gv[KN][G];         // gamma~, shared for the reference norm
  Real pv[KN][G];          // PCG direction / multipliers, shared
  Real sv[KN][G];          // Q_k^-1 times pv
  Real piv[Sh::SLOTS][G];  // Gauss-Jordan pivot rows, one per lane group
  Real red[2][2][kBlock / 64];
  double mp[kMaxAlpha + 1][KN];  // per-knot merit terms; row n_alpha: current point
  double merit[kMaxAlpha + 1];
  float alpha[kMaxAlpha];
  float xs[G], xg[G], c0[G];
  int bad[2];  // per-iteration flag, indexed by iteration parity
};

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <class R>
__device__ __forceinline__ R wave_sum(R v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Sum over the workgroup of two values; every thread gets bit-identical
// results (butterfly inside the wavefront, fixed order across wavefronts).
template <class Real>
__device__ __forceinline__ void block_sum2(Real (*red)[2][kBlock / 64], int &buf, Real &a, Real &b) {
  a = wave_sum(a);
  b = wave_sum(b);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[buf][0][wave] = a;
    red[buf][1][wave] = b;
  }
  __syncthreads();
  Real sa = 0, sb = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) {
    sa += red[buf][0][w];
    sb += red[buf][1][w];
  }
  buf ^= 1;
  a = sa;
  b = sb;
}

template <class Real>
__device__ __forceinline__ Real block_sum(Real (*red)[2][kBlock / 64], int &buf, Real a) {
  a = wave_sum(a);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[buf][0][wave] = a;
  __syncthreads();
  Real s = 0;
#pragma unroll
  for (int w = 0; w < kBlock / 64; ++w) s += red[buf][0][w];
  buf ^= 1;
  return s;
}

template <int ND, int KPT, class Real>
__device__ void sqp_solve(const KArgs &a, int sid, char *smem_raw) {
  using Sh = Shape<ND>;
  constexpr int NX = Sh::NX, NU = Sh::NU, G = Sh::G, SLOTS = Sh::SLOTS;
  using SM = Smem<ND, KPT, Real>;
  SM &sm = *reinterpret_cast<SM *>(smem_raw);
  const SolveDesc &D = a.desc[sid];
  const Chain &ch = D.chain;
  const int tid = threadIdx.x;
  const int lane = tid % G;
  const int slot = tid / G;
  const int N = D.N;
  const float h = D.dt;
  const int n_alpha = a.n_alpha;
  char *ws = a.ws + D.ws_off;
  float *gA = reinterpret_cast<float *>(ws + D.offA);    // [N-1][NX][NX]
  float *gB = reinterpret_cast<float *>(ws + D.offB);    // [N-1][NX][NU]
  Real *gD = reinterpret_cast<Real *>(ws + D.offD);      // [N][NX][NX]
  const size_t xoff = (size_t)sid * a.N_max * a.nx_max;
  double *gL = a.lam + xoff;                             // [N][nx_max]
  const size_t uoff = (size_t)sid * (a.N_max - 1) * a.nu_max;

  // ---- Stage the iterate and the solve constants in LDS.
  for (int t = tid; t < N * G; t += kBlock) {
    const int k = t / G, j = t % G;
    sm.X[k][j] = (j < NX && a.mode != kModeKkt) ? a.X[xoff + (size_t)k * a.nx_max + j] : 0.f;
  }
  for (int t = tid; t < (N - 1) * 8; t += kBlock) {
    const int k = t / 8, j = t % 8;
    sm.U[k][j] = (j < NU && a.mode != kModeKkt) ? a.U[uoff + (size_t)k * a.nu_max + j] : 0.f;
  }
  if (tid < G) {
    const bool in = tid < NX && a.mode != kModeKkt;
    sm.xs[tid] = in ? a.xs[(size_t)sid * a.nx_max + tid] : 0.f;
    sm.xg[tid] = (in && tid < ND) ? a.goal[(size_t)sid * a.nu_max + tid] : 0.f;
  }
  if (tid == 0) {
    sm.bad[0] = 0;
    sm.bad[1] = 0;
    float al = 1.f;
    for (int i = 0; i < n_alpha; ++i) {
      sm.alpha[i] = al;
      al = al / a.beta;
    }
  }

  // Multipliers of the rows this thread owns (warm start across iterations).
  Real lam[KPT];
#pragma unroll
  for (int p = 0; p < KPT; ++p) {
    const int k = slot + p * SLOTS;
    lam[p] = (a.warm && a.mode == kModeSqp && k < N && lane < NX) ? (Real)gL[k * a.nx_max + lane] : (Real)0;
  }
  int redbuf = 0;
  __syncthreads();

  for (int it = 0; it < a.iters; ++it) {
    int &bad_flag = sm.bad[it & 1];
    // ================= 1. LQ: dynamics, derivatives, defects, gradients.
    if (a.mode != kModeKkt) {
      for (int k = slot; k < N - 1; k += SLOTS) {
        float q[ND], qd[ND], u[ND], qdd[ND], L[ND][ND];
#pragma unroll
        for (int i = 0; i < ND; ++i) {
          q[i] = sm.X[k][i];
          qd[i] = sm.X[k][ND + i];
          u[i] = sm.U[k][i];
        }
        const bool ok = forward_dynamics<ND>(ch, q, qd, u, qdd, L);
        if (lane < NX) {
          float col[ND];
          fd_jacobian_column<ND>(ch, q, qd, qdd, L, lane, col);
          float *Ak = gA + (size_t)k * NX * NX;
#pragma unroll
          for (int i = 0; i < ND; ++i) {
            Ak[i * NX + lane] = (i == lane ? 1.f : 0.f) + (lane == ND + i ? h : 0.f);
            Ak[(ND + i) * NX + lane] = h * col[i] + (lane == ND + i ? 1.f : 0.f);
          }
          if (lane < ND) {
            float mi[ND];
#pragma unroll
            for (int i = 0; i < ND; ++i) mi[i] = (i == lane) ? 1.f : 0.f;
            chol_solve<ND>(L, mi);
            float *Bk = gB + (size_t)k * NX * NU;
#pragma unroll
            for (int i = 0; i < ND; ++i) {
              Bk[i * NU + lane] = 0.f;
              Bk[(ND + i) * NU + lane] = h * mi[i];
            }
          }
        }
        if (lane == 0) {
          float viol = 0.f, cost = 0.f;
#pragma unroll
          for (int i = 0; i < ND; ++i) {
            const float e0 = (q[i] + h * qd[i]) - sm.X[k + 1][i];
            const float e1 = (qd[i] + h * qdd[i]) - sm.X[k + 1][ND + i];
            sm.e[k][i] = e0;
            sm.e[k][ND + i] = e1;
            viol += fabsf(e0) + fabsf(e1);
          }
#pragma unroll
          for (int i = 0; i < NX; ++i) {
            const float d = sm.X[k][i] - sm.xg[i];
            cost += 0.5f * D.Wq[i] * d * d;
          }
#pragma unroll
          for (int i = 0; i < NU; ++i) cost += 0.5f * D.Wr[i] * u[i] * u[i];
          sm.mp[n_alpha][k] = (double)cost + (double)a.mu * (double)viol;
          if (!ok || !isfinite(viol) || !isfinite(cost)) bad_flag = 1;
        }
      }
      for (int t = tid; t < N * G; t += kBlock) {
        const int k = t / G, j = t % G;
        const float *W = (k < N - 1) ? D.Wq : D.Wn;
        sm.qg[k][j] = j < NX ? W[j] * (sm.X[k][j] - sm.xg[j]) : 0.f;
        if (k < N - 1 && j < 8) sm.rg[k][j] = j < NU ? D.Wr[j] * sm.U[k][j] : 0.f;
      }
      if (tid < G) sm.c0[tid] = tid < NX ? sm.xs[tid] - sm.X[0][tid] : 0.f;
      if (tid == kBlock - 1) {
        float cost = 0.f, viol = 0.f;
        for (int i = 0; i < NX; ++i) {
          const float d = sm.X[N - 1][i] - sm.xg[i];
          cost += 0.5f * D.Wn[i] * d * d;
          viol += fabsf(sm.xs[i] - sm.X[0][i]);
        }
        sm.mp[n_alpha][N - 1] = (double)cost + (double)a.mu * (double)viol;
      }
      if (a.mode == kModeLq) {
        __syncthreads();
        const size_t ao = (size_t)sid * (a.N_max - 1) * a.nx_max * a.nx_max;
        const size_t bo = (size_t)sid * (a.N_max - 1) * a.nx_max * a.nu_max;
        const size_t eo = (size_t)sid * (a.N_max - 1) * a.nx_max;
        for (int t = tid; t < (N - 1) * NX * NX; t += kBlock) {
          const int k = t / (NX * NX), r = (t / NX) % NX, c = t % NX;
          a.outA[ao + ((size_t)k * a.nx_max + r) * a.nx_max + c] = gA[t];
        }
        for (int t = tid; t < (N - 1) * NX * NU; t += kBlock) {
          const int k = t / (NX * NU), r = (t / NU) % NX, c = t % NU;
          a.outB[bo + ((size_t)k * a.nx_max + r) * a.nu_max + c] = gB[t];
        }
        for (int t = tid; t < (N - 1) * NX; t += kBlock) {
          const int k = t / NX, r = t % NX;
          a.oute[eo + (size_t)k * a.nx_max + r] = sm.e[k][r];
        }
        return;
      }
    } else {
      // Stage entry point: QP data supplied by the caller.
      const size_t ao = (size_t)sid * (a.N_max - 1) * a.nx_max * a.nx_max;
      const size_t bo = (size_t)sid * (a.N_max - 1) * a.nx_max * a.nu_max;
      for (int t = tid; t < (N - 1) * NX * NX; t += kBlock) {
        const int k = t / (NX * NX), r = (t / NX) % NX, c = t % NX;
        gA[t] = a.inA[ao + ((size_t)k * a.nx_max + r) * a.nx_max + c];
      }
      for (int t = tid; t < (N - 1) * NX * NU; t += kBlock) {
        const int k = t / (NX * NU), r = (t / NU) % NX, c = t % NU;
        gB[t] = a.inB[bo + ((size_t)k * a.nx_max + r) * a.nu_max + c];
      }
      for (int t = tid; t < N * G; t += kBlock) {
        const int k = t / G, j = t % G;
        sm.qg[k][j] = j < NX ? a.inq[xoff + (size_t)k * a.nx_max + j] : 0.f;
        if (k < N - 1) {
          sm.e[k][j] = j < NX ? a.ine[(size_t)sid * (a.N_max - 1) * a.nx_max + (size_t)k * a.nx_max + j] : 0.f;
          if (j < 8) sm.rg[k][j] = j < NU ? a.inr[uoff + (size_t)k * a.nu_max + j] : 0.f;
        }
      }
      if (tid < G) sm.c0[tid] = tid < NX ? a.inc0[(size_t)sid * a.nx_max + tid] : 0.f;
    }
    __syncthreads();
    // The other parity's flag was last read before the previous iteration's
    // closing barrier; clear it for the next iteration.
    if (tid == 0) sm.bad[(it + 1) & 1] = 0;

    // ================= 2. Schur complement rows and diagonal-block inverses.
    Real th[KPT][NX];     // row of the diagonal block theta_{k-1} (Q_0^-1 for k = 0)
    float Am[KPT][NX];    // row `lane` of A_{k-1}: S~_{k,k-1} = -A_{k-1} Q_{k-1}^-1
    float Ac[KPT][NX];    // column `lane` of A_k: S~_{k,k+1} = -Q_k^-1 A_k^T
    Real gam[KPT];
    Real qown[KPT];       // Q_k^-1 at (lane, lane)
    Real dinv[KPT][NX];   // row of the inverse of the diagonal block
#pragma unroll
    for (int p = 0; p < KPT; ++p) {
      const int k = slot + p * SLOTS;
      const bool valid = k < N && lane < NX;
#pragma unroll
      for (int m = 0; m < NX; ++m) {
        th[p][m] = 0;
        Am[p][m] = 0.f;
        Ac[p][m] = 0.f;
        dinv[p][m] = 0;
      }
      gam[p] = 0;
      qown[p] = 0;
      if (valid) {
        const double *Qik = (k < N - 1) ? D.Qi : D.Qni;
        qown[p] = (Real)Qik[lane];
        if (k == 0) {
#pragma unroll
          for (int m = 0; m < NX; ++m) th[p][m] = (m == lane) ? (Real)D.Qi[lane] : (Real)0;
          gam[p] = (Real)sm.c0[lane] + (Real)D.Qi[lane] * (Real)sm.qg[0][lane];
        } else {
          const int km = k - 1;
          const float *A = gA + (size_t)km * NX * NX;
          const float *B = gB + (size_t)km * NX * NU;
          float Ar[NX], Br[NU];
#pragma unroll
          for (int m = 0; m < NX; ++m) Ar[m] = A[lane * NX + m];
#pragma unroll
          for (int m = 0; m < NU; ++m) Br[m] = B[lane * NU + m];
          Real ArQ[NX], BrR[NU];
#pragma unroll
          for (int m = 0; m < NX; ++m) ArQ[m] = (Real)Ar[m] * (Real)D.Qi[m];
#pragma unroll
          for (int m = 0; m < NU; ++m) BrR[m] = (Real)Br[m] * (Real)D.Ri[m];
#pragma unroll
          for (int c = 0; c < NX; ++c) {
            Real t = (c == lane) ? (Real)Qik[lane] : (Real)0;
#pragma unroll
            for (int m = 0; m < NX; ++m) t += ArQ[m] * (Real)A[c * NX + m];
#pragma unroll
            for (int m = 0; m < NU; ++m) t += BrR[m] * (Real)B[c * NU + m];
            th[p][c] = t;
          }
          Real z = (Real)sm.e[km][lane] + (Real)Qik[lane] * (Real)sm.qg[k][lane];
#pragma unroll
          for (int m = 0; m < NX; ++m) z -= ArQ[m] * (Real)sm.qg[km][m];
#pragma unroll
          for (int m = 0; m < NU; ++m) z -= BrR[m] * (Real)sm.rg[km][m];
          gam[p] = z;
#pragma unroll
          for (int m = 0; m < NX; ++m) Am[p][m] = Ar[m];
        }
        if (k < N - 1) {
          const float *A = gA + (size_t)k * NX * NX;
#pragma unroll
          for (int m = 0; m < NX; ++m) Ac[p][m] = A[m * NX + lane];
        }
      }
      // Inverse of the diagonal block: Gauss-Jordan inside the lane group
      // (the block is SPD, so no pivoting is needed).
      if (k < N) {
        if (k == 0) {
          const Real d0 = lane < NX ? (Real)1 / (Real)D.Qi[lane] : (Real)0;
#pragma unroll
          for (int m = 0; m < NX; ++m) dinv[p][m] = (m == lane) ? d0 : (Real)0;
        } else {
          Real row[NX];
#pragma unroll
          for (int c = 0; c < NX; ++c) row[c] = th[p][c];
#pragma unroll
          for (int pv = 0; pv < NX; ++pv) {
            if (lane == pv) {
#pragma unroll
              for (int c = 0; c < NX; ++c) sm.piv[slot][c] = row[c];
            }
            wave_sync();
            Real prow[NX];
#pragma unroll
            for (int c = 0; c < NX; ++c) prow[c] = sm.piv[slot][c];
            wave_sync();
            const Real pinv = (Real)1 / prow[pv];
            if (lane == pv) {
#pragma unroll
              for (int c = 0; c < NX; ++c) row[c] = (c == pv) ? pinv : row[c] * pinv;
            } else {
              const Real f = row[pv] * pinv;
#pragma unroll
              for (int c = 0; c < NX; ++c) row[c] = (c == pv) ? -f : row[c] - f * prow[c];
            }
          }
#pragma unroll
          for (int c = 0; c < NX; ++c) dinv[p][c] = row[c];
        }
        if (lane < NX) {
          Real *Dk = gD + (size_t)k * NX * NX + lane * NX;
#pragma unroll
          for (int c = 0; c < NX; ++c) Dk[c] = dinv[p][c];
        }
      }
    }
    __syncthreads();

    // ================= 3. Rows of the stair preconditioner P = -Phi^-1.
    float Pd[KPT][NX], Pm[KPT][NX], Pp[KPT][NX];
#pragma unroll
    for (int p = 0; p < KPT; ++p) {
      const int k = slot + p * SLOTS;
      const bool valid = k < N && lane < NX;
#pragma unroll
      for (int m = 0; m < NX; ++m) {
        Pd[p][m] = (float)dinv[p][m];
        Pm[p][m] = 0.f;
        Pp[p][m] = 0.f;
      }
      if (valid && k >= 1) {
        // row of -D_k^-1 phi_{k-1} D_{k-1}^-1, phi_{k-1} = -A_{k-1} Q_{k-1}^-1
        const float *A = gA + (size_t)(k - 1) * NX * NX;
        const Real *Dm = gD + (size_t)(k - 1) * NX * NX;
        Real t[NX];
#pragma unroll
        for (int c = 0; c < NX; ++c) {
          Real s = 0;
#pragma unroll
          for (int m = 0; m < NX; ++m) s += dinv[p][m] * (Real)A[m * NX + c];
          t[c] = s * (Real)D.Qi[c];   // = -(D_k^-1 phi_{k-1})[lane][c]
        }
#pragma unroll
        for (int c2 = 0; c2 < NX; ++c2) {
          Real s = 0;
#pragma unroll
          for (int c = 0; c < NX; ++c) s += t[c] * Dm[c * NX + c2];
          Pm[p][c2] = (float)s;
        }
      }
      if (valid && k <= N - 2) {
        // row of (-D_{k+1}^-1 phi_k D_k^-1)^T = column of the block below.
        const float *A = gA + (size_t)k * NX * NX;
        const Real *Dp = gD + (size_t)(k + 1) * NX * NX;
        Real v[NX];
#pragma unroll
        for (int m = 0; m < NX; ++m) {
          Real s = 0;
#pragma unroll
          for (int c = 0; c < NX; ++c) s += (Real)A[m * NX + c] * ((Real)D.Qi[c] * dinv[p][c]);
          v[m] = s;   // = -(phi_k D_k^-1 e_lane)[m]
        }
#pragma unroll
        for (int m2 = 0; m2 < NX; ++m2) {
          Real s = 0;
#pragma unroll
          for (int m = 0; m < NX; ++m) s += Dp[m2 * NX + m] * v[m];
          Pp[p][m2] = (float)s;
        }
      }
    }

    // ================= 4. PCG on S~ lambda = gamma~.
    auto share_p = [&](const Real *vals) {
#pragma unroll
      for (int p = 0; p < KPT; ++p) {
        const int k = slot + p * SLOTS;
        if (k < N) {
          const bool valid = lane < NX;
          sm.pv[k][lane] = valid ? vals[p] : (Real)0;
          sm.sv[k][lane] = valid ? qown[p] * vals[p] : (Real)0;
        }
      }
    };
    auto apply_S = [&](int p) -> Real {
      const int k = slot + p * SLOTS;
      Real acc = 0;
#pragma unroll
      for (int m = 0; m < NX; ++m) acc += th[p][m] * sm.pv[k][m];
      if (k > 0) {
#pragma unroll
        for (int m = 0; m < NX; ++m) acc -= (Real)Am[p][m] * sm.sv[k - 1][m];
      }
      if (k < N - 1) {
        Real t = 0;
#pragma unroll
        for (int m = 0; m < NX; ++m) t += (Real)Ac[p][m] * sm.pv[k + 1][m];
        acc -= qown[p] * t;
      }
      return acc;
    };
    auto apply_P = [&](int p, float (*buf)[G]) -> float {
      const int k = slot + p * SLOTS;
      float acc = 0.f;
#pragma unroll
      for (int m = 0; m < NX; ++m) acc += Pd[p][m] * buf[k][m];
      if (k > 0) {
#pragma unroll
        for (int m = 0; m < NX; ++m) acc += Pm[p][m] * buf[k - 1][m];
      }
      if (k < N - 1) {
#pragma unroll
        for (int m = 0; m < NX; ++m) acc += Pp[p][m] * buf[k + 1][m];
      }
      return acc;
    };

    Real r[KPT], z[KPT], pd[KPT];
    share_p(lam);
    __syncthreads();
#pragma unroll
    for (int p = 0; p < KPT; ++p) {
      const int k = slot + p * SLOTS;
      const bool valid = k < N && lane < NX;
      r[p] = valid ? gam[p] - apply_S(p) : (Real)0;
      if (k < N) {
        sm.rv[k][lane] = valid ? (float)r[p] : 0.f;
        sm.gv[k][lane] = valid ? (float)gam[p] : 0.f;
      }
    }
    __syncthreads();
    Real eta = 0, eta_ref = 0;
#pragma unroll
    for (int p = 0; p < KPT; ++p) {
      const int k = slot + p * SLOTS;
      const bool valid = k < N && lane < NX;
      z[p] = valid ? (Real)apply_P(p, sm.rv) : (Real)0;
      const Real pg = valid ? (Real)apply_P(p, sm.gv) : (Real)0;
      pd[p] = z[p];
      eta += r[p] * z[p];
      eta_ref += gam[p] * pg;
    }
    block_sum2(sm.red, redbuf, eta, eta_ref);
    const Real stop = (Real)a.pcg_tol * (Real)a.pcg_tol * eta_ref;
    const int max_it = a.pcg_max_iter > 0 ? a.pcg_max_iter : N * NX;
    int its = 0;
    while (eta > stop && its < max_it) {
      share_p(pd);
      __syncthreads();
      Real pw = 0, w[KPT];
#pragma unroll
      for (int p = 0; p < KPT; ++p) {
        const int k = slot + p * SLOTS;
        const bool valid = k < N && lane < NX;
        w[p] = valid ? apply_S(p) : (Real)0;
        pw += pd[p] * w[p];
      }
      pw = block_sum(sm.red, redbuf, pw);
      const Real alpha = eta / pw;
#pragma unroll
      for (int p = 0; p < KPT; ++p) {
        const int k = slot + p * SLOTS;
        lam[p] += alpha * pd[p];
        r[p] -= alpha * w[p];
        if (k < N) sm.rv[k][lane] = (float)r[p];
      }
      __syncthreads();
      Real eta_new = 0;
#pragma unroll
      for (int p = 0; p < KPT; ++p) {
        const int k = slot + p * SLOTS;
        const bool valid = k < N && lane < NX;
        z[p] = valid ? (Real)apply_P(p, sm.rv) : (Real)0;
        eta_new += r[p] * z[p];
      }
      eta_new = block_sum(sm.red, redbuf, eta_new);
      const Real beta = eta_new / eta;
      eta = eta_new;
#pragma unroll
      for (int p = 0; p < KPT; ++p) pd[p] = z[p] + beta * pd[p];
      ++its;
    }
    unsigned status = (eta > stop) ? GATO_ST_PCG_MAXITER : 0u;

    // ================= 5. Step recovery dZ = -G^-1 (g - C^T lambda).
    share_p(lam);
    __syncthreads();
#pragma unroll
    for (int p = 0; p < KPT; ++p) {
      const int k = slot + p * SLOTS;
      if (k < N && lane < NX) {
        Real s = (Real)sm.qg[k][lane] - lam[p];
        if (k < N - 1) {
#pragma unroll
          for (int m = 0; m < NX; ++m) s += (Real)Ac[p][m] * sm.pv[k + 1][m];
        }
        const float dx = (float)(-qown[p] * s);
        sm.dX[k][lane] = dx;
        if (!isfinite(dx)) bad_flag = 1;
        if (lane < NU && k < N - 1) {
          const float *B = gB + (size_t)k * NX * NU;
          Real su = (Real)sm.rg[k][lane];
#pragma unroll
          for (int m = 0; m < NX; ++m) su += (Real)B[m * NU + lane] * sm.pv[k + 1][m];
          const float du = (float)(-(Real)D.Ri[lane] * su);
          sm.dU[k][lane] = du;
          if (!isfinite(du)) bad_flag = 1;
        }
      }
    }
    if (a.mode == kModeKkt) {
      __syncthreads();
#pragma unroll
      for (int p = 0; p < KPT; ++p) {
        const int k = slot + p * SLOTS;
        if (k < N && lane < NX) {
          a.outdX[xoff + (size_t)k * a.nx_max + lane] = sm.dX[k][lane];
          a.outlam[xoff + (size_t)k * a.nx_max + lane] = (double)lam[p];
          if (lane < NU && k < N - 1) a.outdU[uoff + (size_t)k * a.nu_max + lane] = sm.dU[k][lane];
        }
      }
      if (tid == 0 && a.outits) a.outits[sid] = its;
      return;
    }
    __syncthreads();

    // ================= 6. Line search over alpha_i = beta^-i (Eqs. (3), (7)).
    const int ntask = n_alpha * (N - 1);
    for (int t = tid; t < ntask; t += kBlock) {
      const int i = t / (N - 1), k = t - i * (N - 1);
      const float al = sm.alpha[i];
      float q[ND], qd[ND], u[ND], qdd[ND], L[ND][ND], xn[NX];
#pragma unroll
      for (int j = 0; j < ND; ++j) {
        q[j] = sm.X[k][j] + al * sm.dX[k][j];
        qd[j] = sm.X[k][ND + j] + al * sm.dX[k][ND + j];
        u[j] = sm.U[k][j] + al * sm.dU[k][j];
      }
#pragma unroll
      for (int j = 0; j < NX; ++j) xn[j] = sm.X[k + 1][j] + al * sm.dX[k + 1][j];
      forward_dynamics<ND>(ch, q, qd, u, qdd, L);
      float viol = 0.f, cost = 0.f;
#pragma unroll
      for (int j = 0; j < ND; ++j) {
        viol += fabsf((q[j] + h * qd[j]) - xn[j]) + fabsf((qd[j] + h * qdd[j]) - xn[ND + j]);
        const float d0 = q[j] - sm.xg[j], d1 = qd[j] - sm.xg[ND + j];
        cost += 0.5f * D.Wq[j] * d0 * d0 + 0.5f * D.Wq[ND + j] * d1 * d1 + 0.5f * D.Wr[j] * u[j] * u[j];
      }
      sm.mp[i][k] = (double)cost + (double)a.mu * (double)viol;
    }
    for (int i = tid; i < n_alpha; i += kBlock) {
      const float al = sm.alpha[i];
      float cost = 0.f, viol = 0.f;
      for (int j = 0; j < NX; ++j) {
        const float d = (sm.X[N - 1][j] + al * sm.dX[N - 1][j]) - sm.xg[j];
        cost += 0.5f * D.Wn[j] * d * d;
        viol += fabsf(sm.xs[j] - (sm.X[0][j] + al * sm.dX[0][j]));
      }
      sm.mp[i][N - 1] = (double)cost + (double)a.mu * (double)viol;
    }
    __syncthreads();
    if (tid <= n_alpha) {
      double s = 0.0;
      for (int k = 0; k < N; ++k) s += sm.mp[tid][k];
      sm.merit[tid] = s;
    }
    __syncthreads();
    int best = -1;
    for (int i = 0; i < n_alpha; ++i) {
      const double m = sm.merit[i];
      if (isfinite(m) && (best < 0 || m < sm.merit[best])) best = i;
    }
    const bool bad = bad_flag != 0 || best < 0;
    if (bad) status |= GATO_ST_NONFINITE;
    else if (!(sm.merit[best] < sm.merit[n_alpha])) status |= GATO_ST_NO_DESCENT;
    const float al = bad ? 0.f : sm.alpha[best];
    if (!bad) {
      for (int t = tid; t < N * G; t += kBlock) {
        const int k = t / G, j = t % G;
        sm.X[k][j] += al * sm.dX[k][j];
        if (k < N - 1 && j < 8) sm.U[k][j] += al * sm.dU[k][j];
      }
    }
    if (tid == 0 && a.stats) {
      gato_solve_stats st;
      st.merit0 = (float)sm.merit[n_alpha];
      st.merit = bad ? (float)sm.merit[n_alpha] : (float)sm.merit[best];
      st.alpha = al;
      st.pcg_iters = its;
      st.status = status;
      a.stats[(size_t)sid * a.stats_stride + it] = st;
    }
    __syncthreads();
  }

  // ---- Write back the iterate and the warm-start multipliers.
  if (a.mode == kModeSqp) {
    for (int t = tid; t < N * G; t += kBlock) {
      const int k = t / G, j = t % G;
      if (j < NX) a.X[xoff + (size_t)k * a.nx_max + j] = sm.X[k][j];
      if (k < N - 1 && j < NU) a.U[uoff + (size_t)k * a.nu_max + j] = sm.U[k][j];
    }
#pragma unroll
    for (int p = 0; p < KPT; ++p) {
      const int k = slot + p * SLOTS;
      if (k < N && lane < NX) gL[k * a.nx_max + lane] = (double)lam[p];
    }
  }
}

template <int ND, int KPT, class Real>
__global__ __launch_bounds__(kBlock) void sqp_kernel(KArgs a) {
  __shared__ __align__(16) char smem[sizeof(Smem<ND, KPT, Real>)];
  const int sid = a.order ? a.order[blockIdx.x] : a.sid_base + (int)blockIdx.x;
  sqp_solve<ND, KPT, Real>(a, sid, smem);
}

}  // namespace gato
