// The fused SQP iteration for one trajectory-optimisation solve per workgroup.
//
// One workgroup of kBlock threads owns one solve and runs whole SQP iterations
// (Algorithm 1) without returning to the host. Knot k of the solve is handled
// by a group of G lanes (G = 16 for 5..7 DoF, 8 for fewer), so a wavefront
// holds 64/G knots. Per iteration:
//   1. LQ (Sec. III-A, Eq. (1)): the group's first lane evaluates forward
//      dynamics and the Cholesky factor of the inertia matrix and shares them
//      through LDS; lane d then forms column d of the dynamics Jacobian with one
//      dual-number RNEA pass. Defects, gradients and the current merit follow.
//   2. Schur complement (Eqs. (5)-(6)): lane j forms row j of theta_{k-1} and
//      entry j of gamma~ in FP64, then the group inverts the diagonal block by
//      Gauss-Jordan elimination (SPD, no pivoting).
//   3. Stair preconditioner (Eq. (6)): the FP64 variants apply it factored,
//      P v = D^-1 (v - O D^-1 v) with O the off-diagonal blocks of S~, so only
//      the rows of D^-1 are kept; the all-FP32 variant's lanes of knot k+1 form
//      the off-diagonal block -D_{k+1}^-1 phi_k D_k^-1 once and knot k reads
//      its transpose. The paper's single grid-wide synchronisation becomes a
//      workgroup barrier.
//   4. PCG on S~ lambda = gamma~ (Sec. II-B, III-B) in the pipelined
//      arrangement: the inner products of an iteration are reduced together
//      and share a barrier with the vector exchange, so an iteration needs two
//      workgroup barriers. Rows of S~ and P stay in registers; vectors are
//      exchanged through LDS. (The all-FP32 and task-space variants run the
//      standard arrangement.)
//   5. Step dZ = -G^-1 (g - C^T lambda) (Eq. (4)).
//   6. Line search (Eqs. (3), (7)): lane (alpha, knot) evaluates one trial
//      knot; a fixed-order reduction gives each candidate's merit.
// The Schur rows, gamma~, the block inverses, the PCG vectors and its inner
// products use Real (double; float for the all-FP32 variant). Dynamics and the
// line search's trial points use float; the explicit preconditioner blocks of
// the all-FP32 variant (and the D^-1 rows of four knots per lane group) too.
//
// Task-space variant (TS): a tip tracking term 1/2 |p(q_k) - pref_k|^2_W per
// knot makes the joint block of Q_k dense, H_k = diag(Q_q + rho) + J^T W J
// (Gauss-Newton). Phase 1 then also factors H_k = L_k L_k^T and rewrites the
// QP in the variables y_k = T_k^-1 x_k, T_k = blkdiag(L_k^-T, I), whose state
// Hessian is diagonal again: A_k -> T_{k+1}^-1 A_k T_k, e_k -> T_{k+1}^-1 e_k,
// q_k -> T_k^T q_k, c_0 -> T_0^-1 c_0 (B_k is unchanged, its joint rows are
// zero). The Schur complement of the rewritten QP is congruent to that of
// Eq. (5) under blkdiag(T_k^-1), and so is the stair preconditioner of
// Eq. (6), so PCG takes the same iterates (multipliers scaled by T_k^T) and
// the same stopping value as on the dense-Q_k system; phases 2-4 run
// unchanged, and phase 5 maps the step and the multipliers back.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "gato_internal.hpp"

namespace gato {

template <int ND>
struct Shape {
  static constexpr int NX = 2 * ND;
  static constexpr int NU = ND;
  static constexpr int G = (2 * ND > 8) ? 16 : 8;  // lanes per knot (power of two >= NX)
  static constexpr int SLOTS = kBlock / G;          // knots handled at once
  static constexpr int NL = ND * (ND + 1) / 2;      // packed Cholesky factor
};

// QP blocks live in LDS when the workgroup holds at most 32 knots, or one knot
// per lane group, and in the solve's global workspace otherwise.
template <int ND, int KPT>
struct BlockStore {
  static constexpr int KN = KPT * Shape<ND>::SLOTS;
  static constexpr bool kLds = (KPT == 1) || (KN <= 32);
  static constexpr int LB = kLds ? KN : 1;
};

template <int ND, int KPT, class Real>
struct Smem {
  using Sh = Shape<ND>;
  static constexpr int G = Sh::G;
  static constexpr int NX = Sh::NX, NU = Sh::NU;
  static constexpr int KN = KPT * Sh::SLOTS;
  static constexpr int LB = BlockStore<ND, KPT>::LB;
  float X[KN][G];          // iterate
  float U[KN][8];
  float dX[KN][G];         // step
  float dU[KN][8];
  float e[KN][G];          // defects e_k = f(x_k, u_k) - x_{k+1}
  float qg[KN][G];         // state gradients q_k
  float rg[KN][8];         // control gradients r_k
  Real rv[KN][G];          // PCG residual, shared for the preconditioner
  Real gv[KN][G];          // gamma~, shared for the reference norm
  float qdd[KN][8];        // forward dynamics at the knot
  float Lf[KN][Sh::NL];    // packed Cholesky factor of the inertia matrix
  Real pv[KN][G];          // vector shared for the S~ product
  Real sv[KN][G];          // Q_k^-1 times pv
  double piv[Sh::SLOTS][G];  // Gauss-Jordan pivot rows, one per lane group
  double red[2][3][kBlock / 64];  // per-wavefront partial sums
  double mp0[KN];          // per-knot merit terms at the current point
  double Qi[G], Qni[G];    // 1 / (Q + rho), 1 / (Q_N + rho) for the current rho
  union {
    double mp[kMaxAlpha][KN];  // per-knot merit terms of the step candidates (line search)
    Real tv[KN][G];            // exchange inside a lane group (PCG preconditioner)
  };
  double merit[kMaxAlpha + 1];
  float alpha[kMaxAlpha];
  float xs[G], xg[G], c0[G];
  int bad[2];              // per-iteration flag, indexed by iteration parity
  int xfail, xpad[3];      // split solve: a wait for another part gave up (16 bytes: keeps
                           // the blocks below 16-byte aligned for 128-bit LDS reads)
  float A[LB][NX * NX];    // A_k
  float B[LB][NX * NU];    // B_k
  float Dinv[LB][NX * NX]; // inverse diagonal blocks of S~
  float Poff[LB][NX * NX]; // P_{k+1,k}
};

// LDS of the task-space variant, placed after Smem.
template <int ND, int KPT>
struct TsSmem {
  static constexpr int KN = KPT * Shape<ND>::SLOTS;
  static constexpr int NL = Shape<ND>::NL;
  double Lc[KN][NL];     // Cholesky factor L_k of the joint block H_k (packed rows)
  double Li[KN][NL];     // L_k^-1 (packed rows)
  double tq[KN][8];      // joint-block vectors exchanged inside a lane group
  double mt[KN];         // tip tracking cost of each knot at the current iterate
  float Jt[KN][3][8];    // tip Jacobian J_k (column per joint)
  float pr[KN][4];       // reference tip positions
  float pe[KN][4];       // p(q_k) - pref_k at the current iterate
};

template <int ND, int KPT, class Real>
constexpr size_t ts_offset() {
  return (sizeof(Smem<ND, KPT, Real>) + 15) & ~(size_t)15;
}
template <int ND, int KPT, class Real, bool TS>
constexpr size_t smem_bytes() {
  return TS ? ts_offset<ND, KPT, Real>() + sizeof(TsSmem<ND, KPT>) : sizeof(Smem<ND, KPT, Real>);
}

// Packed lower-triangular storage, row i holding columns 0..i.
__device__ __forceinline__ constexpr int tri(int i, int j) { return i * (i + 1) / 2 + j; }

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ---- Cross-lane sums. Every lane ends with the bit-identical total.
// The in-row patterns (quad permutations, row mirrors) read a valid lane for
// every lane, so those moves need no previous destination value; the row
// broadcasts that combine the four rows stay in registers (no LDS round trip).
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
// Row broadcasts (row_bcast:15 = 0x142, row_bcast:31 = 0x143) into the rows
// of ROWS; the other rows read 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ float bcast(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, false));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double bcast(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_val(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_val(double v, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                          __builtin_amdgcn_readlane(__double2loint(v), l));
}

// ---- Products with the lane group's own vector (16-lane groups, FP64). Lane m
// of a 16-lane row holds entry m of its knot's vector; v_fmac_f64 with a
// row_newbcast:m DPP source multiplies every lane's coefficient by that entry
// straight from lane m's register, so the knot's own block-row products need no
// LDS round trip. The terms are accumulated in the same order as the LDS
// form's loops, so the sums are the same bit for bit. Each product is one asm
// statement that starts with the two wait states a DPP read needs after a VALU
// write of its source (x is only read inside it).
#define GATO_NB1(M, C) "v_fmac_f64_dpp %0, %1, %[c" #M "] row_newbcast:" #M " row_mask:0xf bank_mask:0xf\n\t"
#define GATO_NB2(M, A) "v_fmac_f64_dpp %" #A ", %2, %[c" #M "] row_newbcast:" #M " row_mask:0xf bank_mask:0xf\n\t"
#define GATO_C12(c) [c0] "v"(c[0]), [c1] "v"(c[1]), [c2] "v"(c[2]), [c3] "v"(c[3]), [c4] "v"(c[4]), [c5] "v"(c[5]), \
    [c6] "v"(c[6]), [c7] "v"(c[7]), [c8] "v"(c[8]), [c9] "v"(c[9]), [c10] "v"(c[10]), [c11] "v"(c[11])
#define GATO_C14(c) GATO_C12(c), [c12] "v"(c[12]), [c13] "v"(c[13])

// acc += sum_m c[m] x_m, m = 0..NX-1 in order (x_m: x at lane m of the row).
template <int NX>
__device__ __forceinline__ void row_dot1(double &acc, double x, const double *c) {
  static_assert(NX == 12 || NX == 14, "16-lane groups hold 12 or 14 rows");
  if constexpr (NX == 14) {
    asm volatile("s_nop 1\n\t" GATO_NB1(0, c) GATO_NB1(1, c) GATO_NB1(2, c) GATO_NB1(3, c) GATO_NB1(4, c)
                 GATO_NB1(5, c) GATO_NB1(6, c) GATO_NB1(7, c) GATO_NB1(8, c) GATO_NB1(9, c) GATO_NB1(10, c)
                 GATO_NB1(11, c) GATO_NB1(12, c) GATO_NB1(13, c)
                 : "+v"(acc) : "v"(x), GATO_C14(c));
  } else {
    asm volatile("s_nop 1\n\t" GATO_NB1(0, c) GATO_NB1(1, c) GATO_NB1(2, c) GATO_NB1(3, c) GATO_NB1(4, c)
                 GATO_NB1(5, c) GATO_NB1(6, c) GATO_NB1(7, c) GATO_NB1(8, c) GATO_NB1(9, c) GATO_NB1(10, c)
                 GATO_NB1(11, c)
                 : "+v"(acc) : "v"(x), GATO_C12(c));
  }
}

// acc -= sum_m c[m] x_m, m = 0..NX-1 in order (the same roundings as
// acc = fma(-c[m], x_m, acc) term by term).
#define GATO_NBN(M, C) "v_fmac_f64_dpp %0, -%1, %[c" #M "] row_newbcast:" #M " row_mask:0xf bank_mask:0xf\n\t"
template <int NX>
__device__ __forceinline__ void row_dot1_sub(double &acc, double x, const double *c) {
  static_assert(NX == 12 || NX == 14, "16-lane groups hold 12 or 14 rows");
  if constexpr (NX == 14) {
    asm volatile("s_nop 1\n\t" GATO_NBN(0, c) GATO_NBN(1, c) GATO_NBN(2, c) GATO_NBN(3, c) GATO_NBN(4, c)
                 GATO_NBN(5, c) GATO_NBN(6, c) GATO_NBN(7, c) GATO_NBN(8, c) GATO_NBN(9, c) GATO_NBN(10, c)
                 GATO_NBN(11, c) GATO_NBN(12, c) GATO_NBN(13, c)
                 : "+v"(acc) : "v"(x), GATO_C14(c));
  } else {
    asm volatile("s_nop 1\n\t" GATO_NBN(0, c) GATO_NBN(1, c) GATO_NBN(2, c) GATO_NBN(3, c) GATO_NBN(4, c)
                 GATO_NBN(5, c) GATO_NBN(6, c) GATO_NBN(7, c) GATO_NBN(8, c) GATO_NBN(9, c) GATO_NBN(10, c)
                 GATO_NBN(11, c)
                 : "+v"(acc) : "v"(x), GATO_C12(c));
  }
}
#undef GATO_NBN

// acc += sgn * sum_m c[m] x_m with FP32 coefficients converted inside the
// statement (two temporaries), m = 0..NX-1 in order; the same roundings as
// the loop acc = fma(sgn c[m], x_m, acc) over the converted c[m].
#define GATO_NBF(M, T, S) "v_cvt_f64_f32 %[" #T "], %[c" #M "]\n\t"                                \
  "v_fmac_f64_dpp %0, " S "%[x], %[" #T "] row_newbcast:" #M " row_mask:0xf bank_mask:0xf\n\t"
#define GATO_F14(c) [c0] "v"(c[0]), [c1] "v"(c[1]), [c2] "v"(c[2]), [c3] "v"(c[3]), [c4] "v"(c[4]),     \
    [c5] "v"(c[5]), [c6] "v"(c[6]), [c7] "v"(c[7]), [c8] "v"(c[8]), [c9] "v"(c[9]), [c10] "v"(c[10]),   \
    [c11] "v"(c[11]), [c12] "v"(c[12]), [c13] "v"(c[13])
#define GATO_F12(c) [c0] "v"(c[0]), [c1] "v"(c[1]), [c2] "v"(c[2]), [c3] "v"(c[3]), [c4] "v"(c[4]),     \
    [c5] "v"(c[5]), [c6] "v"(c[6]), [c7] "v"(c[7]), [c8] "v"(c[8]), [c9] "v"(c[9]), [c10] "v"(c[10]),   \
    [c11] "v"(c[11])
#define GATO_DOTF(S)                                                                                      \
  if constexpr (NX == 14) {                                                                               \
    asm volatile("s_nop 1\n\t" GATO_NBF(0, ta, S) GATO_NBF(1, tb, S) GATO_NBF(2, ta, S) GATO_NBF(3, tb, S) \
                 GATO_NBF(4, ta, S) GATO_NBF(5, tb, S) GATO_NBF(6, ta, S) GATO_NBF(7, tb, S)              \
                 GATO_NBF(8, ta, S) GATO_NBF(9, tb, S) GATO_NBF(10, ta, S) GATO_NBF(11, tb, S)            \
                 GATO_NBF(12, ta, S) GATO_NBF(13, tb, S)                                                  \
                 : "+v"(acc), [ta] "=&v"(ta), [tb] "=&v"(tb) : [x] "v"(x), GATO_F14(c));                     \
  } else {                                                                                                \
    asm volatile("s_nop 1\n\t" GATO_NBF(0, ta, S) GATO_NBF(1, tb, S) GATO_NBF(2, ta, S) GATO_NBF(3, tb, S) \
                 GATO_NBF(4, ta, S) GATO_NBF(5, tb, S) GATO_NBF(6, ta, S) GATO_NBF(7, tb, S)              \
                 GATO_NBF(8, ta, S) GATO_NBF(9, tb, S) GATO_NBF(10, ta, S) GATO_NBF(11, tb, S)            \
                 : "+v"(acc), [ta] "=&v"(ta), [tb] "=&v"(tb) : [x] "v"(x), GATO_F12(c));                     \
  }
template <int NX>
__device__ __forceinline__ void row_dot1_f(double &acc, double x, const float *c) {
  static_assert(NX == 12 || NX == 14, "16-lane groups hold 12 or 14 rows");
  double ta, tb;
  GATO_DOTF("")
}
template <int NX>
__device__ __forceinline__ void row_dot1_sub_f(double &acc, double x, const float *c) {
  static_assert(NX == 12 || NX == 14, "16-lane groups hold 12 or 14 rows");
  double ta, tb;
  GATO_DOTF("-")
}
#undef GATO_DOTF
#undef GATO_F12
#undef GATO_F14
#undef GATO_NBF

// d0 += sum over even m of c[m] x_m, d1 += sum over odd m (two independent chains).
template <int NX>
__device__ __forceinline__ void row_dot2(double &d0, double &d1, double x, const double *c) {
  static_assert(NX == 12 || NX == 14, "16-lane groups hold 12 or 14 rows");
  if constexpr (NX == 14) {
    asm volatile("s_nop 1\n\t" GATO_NB2(0, 0) GATO_NB2(1, 1) GATO_NB2(2, 0) GATO_NB2(3, 1) GATO_NB2(4, 0)
                 GATO_NB2(5, 1) GATO_NB2(6, 0) GATO_NB2(7, 1) GATO_NB2(8, 0) GATO_NB2(9, 1) GATO_NB2(10, 0)
                 GATO_NB2(11, 1) GATO_NB2(12, 0) GATO_NB2(13, 1)
                 : "+v"(d0), "+v"(d1) : "v"(x), GATO_C14(c));
  } else {
    asm volatile("s_nop 1\n\t" GATO_NB2(0, 0) GATO_NB2(1, 1) GATO_NB2(2, 0) GATO_NB2(3, 1) GATO_NB2(4, 0)
                 GATO_NB2(5, 1) GATO_NB2(6, 0) GATO_NB2(7, 1) GATO_NB2(8, 0) GATO_NB2(9, 1) GATO_NB2(10, 0)
                 GATO_NB2(11, 1)
                 : "+v"(d0), "+v"(d1) : "v"(x), GATO_C12(c));
  }
}
#undef GATO_NB1
#undef GATO_NB2
#undef GATO_C12
#undef GATO_C14

// t[c] += s_c * mul for every column c of the group (s_c: s at lane c of the
// row), one term of the row-by-matrix products that form the Schur diagonal
// block: lane c holds row c of the matrix, so its entries need no LDS copy.
#define GATO_RB(C) "v_fmac_f64_dpp %" #C ", %[s], %[m] row_newbcast:" #C " row_mask:0xf bank_mask:0xf\n\t"
template <int NX>
__device__ __forceinline__ void col_fma(double *t, double s, double mul) {
  static_assert(NX == 12 || NX == 14, "16-lane groups hold 12 or 14 rows");
  if constexpr (NX == 14) {
    asm volatile("s_nop 1\n\t" GATO_RB(0) GATO_RB(1) GATO_RB(2) GATO_RB(3) GATO_RB(4) GATO_RB(5) GATO_RB(6)
                 GATO_RB(7) GATO_RB(8) GATO_RB(9) GATO_RB(10) GATO_RB(11) GATO_RB(12) GATO_RB(13)
                 : "+v"(t[0]), "+v"(t[1]), "+v"(t[2]), "+v"(t[3]), "+v"(t[4]), "+v"(t[5]), "+v"(t[6]),
                   "+v"(t[7]), "+v"(t[8]), "+v"(t[9]), "+v"(t[10]), "+v"(t[11]), "+v"(t[12]), "+v"(t[13])
                 : [s] "v"(s), [m] "v"(mul));
  } else {
    asm volatile("s_nop 1\n\t" GATO_RB(0) GATO_RB(1) GATO_RB(2) GATO_RB(3) GATO_RB(4) GATO_RB(5) GATO_RB(6)
                 GATO_RB(7) GATO_RB(8) GATO_RB(9) GATO_RB(10) GATO_RB(11)
                 : "+v"(t[0]), "+v"(t[1]), "+v"(t[2]), "+v"(t[3]), "+v"(t[4]), "+v"(t[5]), "+v"(t[6]),
                   "+v"(t[7]), "+v"(t[8]), "+v"(t[9]), "+v"(t[10]), "+v"(t[11])
                 : [s] "v"(s), [m] "v"(mul));
  }
}
#undef GATO_RB

// One Gauss-Jordan pivot of a lane group (16-lane groups, FP64; lane r holds
// row r): every lane takes the pivot row from lane PV's registers by row
// broadcasts fused into its update, row_c += pivot_c * nf (nf = -f off the
// pivot lane, 0 on it), so no row travels through LDS. The terms and their
// rounding are those of the LDS form.
#define GATO_GJ(C) "v_fmac_f64_dpp %" #C ", %" #C ", %[nf] row_newbcast:%[pv] row_mask:0xf bank_mask:0xf\n\t"
template <int PV, int NX>
__device__ __forceinline__ void gj_pivot(double *row, int lane) {
  static_assert(NX == 12 || NX == 14, "16-lane groups hold 12 or 14 rows");
  double pp = -0.0;   // -0 + x * 1 is x exactly
  asm volatile("s_nop 1\n\tv_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
               : "+v"(pp) : "v"(row[PV]), "v"(1.0), "i"(PV));
  const double pinv = 1.0 / pp;
  const double f = row[PV] * pinv;
  const double nf = (lane == PV) ? 0.0 : -f;
  if constexpr (NX == 14) {
    asm volatile("s_nop 1\n\t" GATO_GJ(0) GATO_GJ(1) GATO_GJ(2) GATO_GJ(3) GATO_GJ(4) GATO_GJ(5) GATO_GJ(6)
                 GATO_GJ(7) GATO_GJ(8) GATO_GJ(9) GATO_GJ(10) GATO_GJ(11) GATO_GJ(12) GATO_GJ(13)
                 : "+v"(row[0]), "+v"(row[1]), "+v"(row[2]), "+v"(row[3]), "+v"(row[4]), "+v"(row[5]),
                   "+v"(row[6]), "+v"(row[7]), "+v"(row[8]), "+v"(row[9]), "+v"(row[10]), "+v"(row[11]),
                   "+v"(row[12]), "+v"(row[13])
                 : [nf] "v"(nf), [pv] "i"(PV));
  } else {
    asm volatile("s_nop 1\n\t" GATO_GJ(0) GATO_GJ(1) GATO_GJ(2) GATO_GJ(3) GATO_GJ(4) GATO_GJ(5) GATO_GJ(6)
                 GATO_GJ(7) GATO_GJ(8) GATO_GJ(9) GATO_GJ(10) GATO_GJ(11)
                 : "+v"(row[0]), "+v"(row[1]), "+v"(row[2]), "+v"(row[3]), "+v"(row[4]), "+v"(row[5]),
                   "+v"(row[6]), "+v"(row[7]), "+v"(row[8]), "+v"(row[9]), "+v"(row[10]), "+v"(row[11])
                 : [nf] "v"(nf), [pv] "i"(PV));
  }
  if (lane == PV) {
#pragma unroll
    for (int c = 0; c < NX; ++c)
      if (c != PV) row[c] = row[c] * pinv;
  }
  row[PV] = (lane == PV) ? pinv : -f;
}
template <int NX, int... PV>
__device__ __forceinline__ void gj_dpp(double *row, int lane, std::integer_sequence<int, PV...>) {
  (gj_pivot<PV, NX>(row, lane), ...);
}
#undef GATO_GJ

// The PCG's step-length quotients: a / b through the hardware reciprocal and
// two Newton steps (about an ulp from the rounded quotient). Every FP64 PCG
// loop uses it: against the correctly rounded division, whose longer
// dependent chain sits between the inner products and the vector updates of
// every iteration, it takes 1.4% off the one-knot-per-group joint-space call,
// 2.7% off the two-knots-per-group call and 3% off the task-space call.
__device__ __forceinline__ double div_pcg(double a, double b) {
  double r = __builtin_amdgcn_rcp(b);
  double e = fma(-b, r, 1.0);
  r = fma(r, e, r);
  e = fma(-b, r, 1.0);
  r = fma(r, e, r);
  return a * r;
}
__device__ __forceinline__ float div_pcg(float a, float b) { return a / b; }

// Sum over the wavefront (all 64 lanes must be active).
template <class R>
__device__ __forceinline__ R wave_sum(R v) {
  v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x141>(v);  // row_half_mirror
  v += dpp<0x140>(v);  // row_mirror: every lane holds its row's sum
  // Row 3 ends with (r3 + r2) + (r1 + r0), the rows' sums in a fixed order.
  v += bcast<0x142, 0xA>(v);
  v += bcast<0x143, 0xC>(v);
  return lane_val(v, 63);
}

// Two wavefront sums interleaved step by step (each step of one hides the
// latency of the other's).
template <class R>
__device__ __forceinline__ void wave_sum2(R &a, R &b) {
  a += dpp<0xB1>(a);
  b += dpp<0xB1>(b);
  a += dpp<0x4E>(a);
  b += dpp<0x4E>(b);
  a += dpp<0x141>(a);
  b += dpp<0x141>(b);
  a += dpp<0x140>(a);
  b += dpp<0x140>(b);
  a += bcast<0x142, 0xA>(a);
  b += bcast<0x142, 0xA>(b);
  a += bcast<0x143, 0xC>(a);
  b += bcast<0x143, 0xC>(b);
  a = lane_val(a, 63);
  b = lane_val(b, 63);
}

// Sum over the workgroup of NV values: butterfly inside each wavefront, then a
// fixed-order sum of the per-wavefront partials.
// Pairwise sum of W values in a fixed order: ((v0 + v1) + (v2 + v3)) + ...
template <int W>
__device__ __forceinline__ double pair_tree(const double *v) {
  if constexpr (W == 1) return v[0];
  else return pair_tree<W / 2>(v) + pair_tree<W / 2>(v + W / 2);
}

// The partials travel through LDS as double (exact for float values).
template <int NV, class V>
__device__ __forceinline__ void block_sum(double (*red)[3][kBlock / 64], int &buf, V *v) {
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[buf][i][wave] = (double)v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    V s = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) s += (V)red[buf][i][w];
    v[i] = s;
  }
  buf ^= 1;
}

// ---- Exchange between the workgroups (parts) of a split solve. An FP64 value
// travels as two 64-bit words, each holding one 32-bit half of the value under
// a 32-bit tag (launch epoch, exchange number). The words are written and
// polled with relaxed agent-scope atomics: each access is single-copy atomic
// and coherent across the XCDs' L2 caches, so a reader that sees the tag sees
// the half stored with it, and no fence (no whole-L2 write-back or
// invalidation) is needed. Exchange e uses slot e mod 4 of the writer; a part
// reuses a slot only after completing later exchanges that every reader of the
// slot had to take part in. Every wait is bounded.
constexpr int kXSlot = 104;                   // words: left row [0, 32), right row [32, 64), sums [64, 104)
constexpr int kXSlots = 8;
constexpr int kXSums = (kXSlot - 64) / 2;     // values of one part's sums region
constexpr int kXLam = 1024;                   // words: multipliers of 32 knots x 16 rows
constexpr int kXPart = kXSlots * kXSlot + kXLam;
constexpr int kXParts = 4;
constexpr int kXSpin = 1 << 17;               // polls before a wait gives up (default)
static_assert(kXParts == kSplitParts && kXParts * kXPart == kXWordsPerSolve, "exchange layout");

__device__ __forceinline__ void xput(unsigned long long *w, unsigned tag, double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const unsigned long long t = (unsigned long long)tag << 32;
  __hip_atomic_store(w, t | (u & 0xffffffffull), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(w + 1, t | (u >> 32), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// The values stored under `tag` at wa and wb (wb may be null: one value);
// the four words are polled together, so a wait costs one round trip. False
// (values 0) when the wait gave up or `dead` (an earlier wait of the
// workgroup gave up) is set.
__device__ __forceinline__ bool xget2(unsigned long long *wa, unsigned long long *wb, unsigned tag, bool dead,
                                      int spin, double &va, double &vb) {
  va = 0.0;
  vb = 0.0;
  if (dead) return false;
  unsigned long long a0 = 0, a1 = 0, b0 = 0, b1 = 0;
  const unsigned long long t = (unsigned long long)tag;
  for (int n = 0;; ++n) {
    a0 = __hip_atomic_load(wa, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    a1 = __hip_atomic_load(wa + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (wb) {
      b0 = __hip_atomic_load(wb, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      b1 = __hip_atomic_load(wb + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      b0 = b1 = t << 32;
    }
    if ((a0 >> 32) == t && (a1 >> 32) == t && (b0 >> 32) == t && (b1 >> 32) == t) break;
    if (n + 1 >= spin) return false;
  }
  va = __longlong_as_double((long long)((a1 << 32) | (a0 & 0xffffffffull)));
  vb = __longlong_as_double((long long)((b1 << 32) | (b0 & 0xffffffffull)));
  return true;
}
__device__ __forceinline__ bool xget(unsigned long long *w, unsigned tag, bool dead, int spin, double &v) {
  double unused;
  return xget2(w, nullptr, tag, dead, spin, v, unused);
}

// ---- Task-space variant: the tip term of one knot, by the knot's lane group.
// Tip position and Jacobian (lane j: one dual-number pass seeded on q_j), the
// residual p(q) - pref and its cost (lane 0), then H = diag(Q_q + rho) +
// J^T W J, its Cholesky factor L (column by column, lane i holding row i,
// pivots broadcast through tq) and L^-1 (lane j forming column j by forward
// substitution). x: the knot's state; Jt, pe, mt, tq, Lc, Li: its LDS rows.
template <int ND>
__device__ __forceinline__ void tip_factor(const Chain &ch, const float *x, const float *pr, const float *We,
                                           const double *Qd, double rho, int lane, float (*Jt)[8], float *pe,
                                           double *mt, double *tq, double *Lc, double *Li, int &bad_flag) {
  if (lane < ND) {
    dual<float> qv[ND], pt[3];
#pragma unroll
    for (int i = 0; i < ND; ++i) qv[i] = dual<float>{x[i], i == lane ? 1.f : 0.f};
    tip_position<ND>(ch, qv, pt);
#pragma unroll
    for (int c = 0; c < 3; ++c) Jt[c][lane] = pt[c].d;
    if (lane == 0) {
      double tc = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const float d = pt[c].v - pr[c];
        pe[c] = d;
        tc += 0.5 * (double)We[c] * (double)d * (double)d;
      }
      *mt = tc;
      if (!isfinite(tc)) bad_flag = 1;
    }
  }
  wave_sync();
  double hr[ND], lr[ND];
#pragma unroll
  for (int j = 0; j < ND; ++j) {
    double t = (j == lane) ? Qd[j] + rho : 0.0;
    if (lane < ND) {
#pragma unroll
      for (int c = 0; c < 3; ++c) t += (double)We[c] * (double)Jt[c][lane] * (double)Jt[c][j];
    }
    hr[j] = t;
    lr[j] = 0.0;
  }
#pragma unroll
  for (int c = 0; c < ND; ++c) {
    if (lane == c) tq[0] = hr[c];
    wave_sync();
    const double piv = tq[0];
    wave_sync();
    if (lane == 0 && !(piv > 0.0)) bad_flag = 1;
    const double dinv = 1.0 / sqrt(piv);
    const double l = (lane >= c && lane < ND) ? hr[c] * dinv : 0.0;   // L[lane][c]
    lr[c] = l;
    if (lane < ND) tq[lane] = l;
    wave_sync();
#pragma unroll
    for (int j = c + 1; j < ND; ++j) hr[j] -= l * tq[j];
    wave_sync();
  }
  if (lane < ND) {
#pragma unroll
    for (int j = 0; j < ND; ++j)
      if (j <= lane) Lc[tri(lane, j)] = lr[j];
  }
  wave_sync();
  if (lane < ND) {
    // Column `lane` of L^-1: rows lane..ND-1 of the solution of L x = e_lane.
    double xs[ND];
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      double t = (i == lane) ? 1.0 : 0.0;
#pragma unroll
      for (int m = 0; m < i; ++m)
        if (m >= lane) t -= Lc[tri(i, m)] * xs[m];
      xs[i] = (i >= lane) ? t / Lc[tri(i, i)] : 0.0;
      if (i >= lane) Li[tri(i, lane)] = xs[i];
    }
  }
}

// Rewrites knot k's QP data in y_k = T_k^-1 x_k, lane `lane` owning state row
// `lane`: row `lane` of A_k -> T_{k+1}^-1 A_k T_k and e_k -> T_{k+1}^-1 e_k
// (when the knot has a successor, `succ`; L1 = L_{k+1}), q_k (with the tip
// term J^T W (p - pref) added) -> T_k^T q_k, and c_0 -> T_0^-1 c_0 (at the
// first knot, `first`). The joint rows of A_k are [I, hI] by construction of
// the Euler step. Lk, Lik: L_k and L_k^-1; tq: the knot's LDS exchange row.
// (Every pointer is valid; the flags say which rows are rewritten, so that
// the LDS accesses keep their address space.)
template <int ND>
__device__ __forceinline__ void tip_rewrite(int lane, bool succ, bool first, float h, const double *Lk,
                                            const double *Lik, const double *L1, float *Ar, float *e, float *qg,
                                            float *c0, const float (*Jt)[8], const float *pe, const float *We,
                                            double *tq) {
  constexpr int NX = 2 * ND;
  if (succ && lane < NX) {
    if (lane < ND) {
      // Row `lane` of [L_{k+1}^T L_k^-T, h L_{k+1}^T].
#pragma unroll
      for (int c = 0; c < ND; ++c) {
        double t = 0.0;
#pragma unroll
        for (int m = 0; m <= c; ++m)
          if (m >= lane) t += L1[tri(m, lane)] * Lik[tri(c, m)];
        Ar[c] = (float)t;
        Ar[ND + c] = c >= lane ? (float)((double)h * L1[tri(c, lane)]) : 0.f;
      }
    } else {
      // Velocity row: its joint columns times L_k^-T.
      float ar[ND];
#pragma unroll
      for (int m = 0; m < ND; ++m) ar[m] = Ar[m];
#pragma unroll
      for (int c = 0; c < ND; ++c) {
        double t = 0.0;
#pragma unroll
        for (int m = 0; m <= c; ++m) t += (double)ar[m] * Lik[tri(c, m)];
        Ar[c] = (float)t;
      }
    }
  }
  double ev = 0.0, cv = 0.0;
  if (lane < ND) {
    double g = (double)qg[lane];
#pragma unroll
    for (int c = 0; c < 3; ++c) g += (double)Jt[c][lane] * (double)We[c] * (double)pe[c];
    tq[lane] = g;
#pragma unroll
    for (int m = 0; m < ND; ++m) {
      if (m >= lane) {
        if (succ) ev += L1[tri(m, lane)] * (double)e[m];
        if (first) cv += Lk[tri(m, lane)] * (double)c0[m];
      }
    }
  }
  wave_sync();
  if (lane < ND) {
    double qh = 0.0;
#pragma unroll
    for (int m = 0; m < ND; ++m)
      if (m <= lane) qh += Lik[tri(lane, m)] * tq[m];
    qg[lane] = (float)qh;
    if (succ) e[lane] = (float)ev;
    if (first) c0[lane] = (float)cv;
  }
  wave_sync();
}

// The multipliers of a knot between the two sets of variables (joint rows,
// lane `lane` holding row `lane`): lambda^ = T_k^T lambda (to y, forward) and
// lambda = T_k^-T lambda^ (back). tq: the knot's LDS exchange row.
template <int ND>
__device__ __forceinline__ double tip_lambda(int lane, bool forward, const double *Lk, const double *Lik, double *tq,
                                             double lam) {
  if (lane < ND) tq[lane] = lam;
  wave_sync();
  double t = lam;
  if (lane < ND) {
    t = 0.0;
#pragma unroll
    for (int m = 0; m < ND; ++m)
      if (m <= lane) t += (forward ? Lik[tri(lane, m)] : Lk[tri(lane, m)]) * tq[m];
  }
  wave_sync();
  return t;
}

// ---- Split long solves, part-local form. A solve of N > 64 knots (6-7 DoF)
// runs on four workgroups (parts); part j owns knots kf = 32 j .. kl (at most
// 32, possibly none) and runs the one-knot-per-lane-group layout of a short
// solve over them, with one halo knot on each side in LDS:
//   * LQ of its own knots and of the knot left of them (whose A, B, e, q, r the
//     first own Schur row needs), the defects of its own knots (the knot right
//     of them is the halo state);
//   * Schur rows, diagonal-block inverses and PCG rows of its own knots, held
//     in registers as in a short solve; at both barriers of a PCG iteration
//     the halo rows of the S~ and preconditioner operands and the partial
//     inner products travel through device memory (the exchange of the
//     one-workgroup split form, same words and tags);
//   * after the PCG: the multipliers of the halo knots, then the step of the
//     first own knot (the left part's right halo), so that every part holds
//     the step at its own knots and both halos;
//   * the line search over its own knots, the per-candidate partial merits
//     (and the parts' failure flags) summed over the parts in a fixed order,
//     so every part takes the same step, status and damping.
// Part 0 writes the statistics; every part writes its own knots' trajectory
// and multipliers. The same method as the one-workgroup solve; sums are taken
// per part first, so results differ from it at rounding level.
template <int ND>
struct PartSmem {
  using Sh = Shape<ND>;
  static constexpr int G = Sh::G, NX = Sh::NX, NU = Sh::NU, NL = Sh::NL;
  static constexpr int KS = Sh::SLOTS;   // own knots at most
  static constexpr int KH = KS + 2;      // with the halo knots: local index li = k - kf + 1
  float X[KH][G];
  float U[KH][8];
  float dX[KH][G];
  float dU[KH][8];
  float e[KH][G];
  float qg[KH][G];
  float rg[KH][8];
  float qdd[KH][8];
  float Lf[KH][NL];
  double pv[KH][G];        // operand of S~ (own rows and halos)
  double sv[KH][G];        // Q_k^-1 times pv
  double rv[KH][G];        // preconditioner: D_k^-1 times its operand
  double gv[KH][G];        // Q_k^-1 times rv
  double piv[KS][G];
  double red[2][3][kBlock / 64];
  double mp0[KH];
  double Qi[G], Qni[G];
  double mp[kMaxAlpha][KH];
  double xmp[kMaxAlpha + 1];        // terminal and initial terms of this part, per candidate (+ current)
  double psum[kMaxAlpha + 1];       // this part's partial merits
  double msum[kXParts][kXSums];     // every part's partial merits and flags
  double merit[kMaxAlpha + 1];
  float alpha[kMaxAlpha];
  float xs[G], xg[G], c0[G];
  int bad[2];
  int xfail, xpad[3];
  float A[KH][NX * NX];
  float B[KH][NX * NU];
};

// LDS of the task-space part-local form, placed after PartSmem: the factors
// L_k, L_k^-1 and tip data of the own knots and both halos (the left halo's
// rewritten A, e and q and the last own knot's rewritten A need them).
template <int ND>
struct PartTsSmem {
  static constexpr int KH = Shape<ND>::SLOTS + 2, NL = Shape<ND>::NL;
  double Lc[KH][NL];
  double Li[KH][NL];
  double tq[KH][8];
  double mt[KH];
  float Jt[KH][3][8];
  float pr[KH][4];
  float pe[KH][4];
};
template <int ND>
constexpr size_t part_ts_offset() {
  return (sizeof(PartSmem<ND>) + 15) & ~(size_t)15;
}
template <int ND, bool TS>
constexpr size_t part_smem_bytes() {
  return TS ? part_ts_offset<ND>() + sizeof(PartTsSmem<ND>) : sizeof(PartSmem<ND>);
}

template <int ND, bool TS>
__device__ __attribute__((always_inline)) inline void sqp_solve_part(const KArgs &a, int sid, int part,
                                                                     char *smem_raw) {
  using Sh = Shape<ND>;
  using Real = double;
  constexpr int NX = Sh::NX, NU = Sh::NU, G = Sh::G, SLOTS = Sh::SLOTS;
  static_assert(G == 16, "the part-local split serves 6-7 DoF");
  using SM = PartSmem<ND>;
  SM &sm = *reinterpret_cast<SM *>(smem_raw);
  // Only dereferenced by the task-space form, whose LDS holds it.
  PartTsSmem<ND> &ts = *reinterpret_cast<PartTsSmem<ND> *>(smem_raw + part_ts_offset<ND>());
  const SolveDesc &D = a.desc[sid];
  const Chain &ch = D.chain;
  const int tid = threadIdx.x;
  const int lane0 = tid % G;
  const int slot0 = tid / G;
  const int N = D.N;
  const float h = D.dt;
  const int n_alpha = a.n_alpha;
  const int nparts = kXParts;
  const bool writer = part == 0;
  const int kf = part * SLOTS;                               // own knots kf .. kl
  const int nloc = max(0, min(SLOTS, N - kf));
  const int kl = kf + nloc - 1;
  const bool has_l = part > 0 && nloc > 0;                    // a neighbour on the left / the right
  const bool has_r = nloc > 0 && kl + 1 < N;
  const size_t xoff = (size_t)sid * a.N_max * a.nx_max;
  const size_t uoff = (size_t)sid * (a.N_max - 1) * a.nu_max;
  double *gL = a.lam + xoff;
  const int sh = a.shift;
  // Knot of a local index and back.
  auto kof = [&](int li) { return kf - 1 + li; };

  // ---- Stage the iterate (own knots and both halos) and the solve constants.
  for (int t = tid; t < (nloc + 2) * G; t += kBlock) {
    const int li = t / G, j = t % G, k = kof(li);
    const bool in = k >= 0 && k < N && j < NX && nloc > 0;
    sm.X[li][j] = in ? a.X[xoff + (size_t)min(k + sh, N - 1) * a.nx_max + j] : 0.f;
  }
  for (int t = tid; t < (nloc + 1) * 8; t += kBlock) {
    const int li = t / 8, j = t % 8, k = kof(li);
    const bool in = k >= 0 && k <= N - 2 && j < NU && nloc > 0;
    sm.U[li][j] = in ? a.U[uoff + (size_t)min(k + sh, N - 2) * a.nu_max + j] : 0.f;
  }
  if (tid < G) {
    const bool in = tid < NX;
    sm.xs[tid] = in ? a.xs[(size_t)sid * a.nx_max + tid] : 0.f;
    sm.xg[tid] = (in && tid < ND) ? a.goal[(size_t)sid * a.nu_max + tid] : 0.f;
  }
  if constexpr (TS) {
    // Reference tip positions of the own and halo knots (not shifted).
    for (int t = tid; t < (nloc + 2) * 4; t += kBlock) {
      const int li = t / 4, c = t % 4, k = kof(li);
      const bool in = k >= 0 && k < N && c < 3 && nloc > 0;
      ts.pr[li][c] = in ? a.pref[((size_t)sid * a.N_max + k) * 3 + c] : 0.f;
    }
  }
  if (tid == 0) {
    sm.bad[0] = 0;
    sm.bad[1] = 0;
    sm.xfail = 0;
    float al = 1.f;
    for (int i = 0; i < n_alpha; ++i) {
      sm.alpha[i] = al;
      al = al / a.beta;
    }
  }
  const bool own0 = slot0 < nloc && lane0 < NX;
  Real lam = (a.warm && own0) ? (Real)gL[min(kf + slot0 + sh, N - 1) * a.nx_max + lane0] : (Real)0;
  int redbuf = 0;
  unsigned xe = 0;
  double rho = a.rho[sid];
  unsigned long long *xb = a.xch + D.xch_off;
  const int xspin = a.xspin > 0 ? a.xspin : kXSpin;
  auto xtag = [&](unsigned e) { return ((a.epoch & 0xffffu) << 16) | (e & 0xffffu); };
  auto xslot = [&](int q, unsigned e) { return xb + (size_t)q * kXPart + (size_t)(e % kXSlots) * kXSlot; };
  __syncthreads();

  for (int it = 0; it < a.iters; ++it) {
    int lane = lane0, slot = slot0;
    asm volatile("" : "+v"(lane), "+v"(slot));
    const int k = kf + slot;                 // this group's own knot
    const int li = slot + 1;
    const bool own = slot < nloc;
    if (!a.warm && it > 0) lam = (Real)0;
    if (tid < G) {
      // (Task-space form: the joint block of the rewritten Q_k is the identity.)
      const bool unit = TS && tid < ND;
      sm.Qi[tid] = tid < NX ? (unit ? 1.0 : 1.0 / (D.Qd[tid] + rho)) : 0.0;
      sm.Qni[tid] = tid < NX ? (unit ? 1.0 : 1.0 / (D.QNd[tid] + rho)) : 0.0;
    }
    int &bad_flag = sm.bad[it & 1];
    unsigned long long *clk = (a.clk && tid == 0 && writer) ? a.clk + ((size_t)sid * a.iters + it) * 8 : nullptr;
    unsigned long long cyc0 = 0;
    if (clk) {
      clk[0] = wall_clock64();
      cyc0 = clock64();
    }
    // ================= 1. LQ at knots kq0..kq1 (the own knots and the one left of them).
    const int kq0 = max(kf - 1, 0), kq1 = min(kl, N - 2);
    const int nq = nloc > 0 ? kq1 - kq0 + 1 : 0;
    for (int t = slot; t < nq; t += SLOTS) {
      const int kk = kq0 + t, lq = kk - kf + 1;
      if (lane == 0) {
        float q[ND], qd[ND], u[ND], qdd[ND], L[ND][ND];
#pragma unroll
        for (int i = 0; i < ND; ++i) {
          q[i] = sm.X[lq][i];
          qd[i] = sm.X[lq][ND + i];
          u[i] = sm.U[lq][i];
        }
        const bool ok = forward_dynamics<ND>(ch, q, qd, u, qdd, L);
#pragma unroll
        for (int i = 0; i < ND; ++i) sm.qdd[lq][i] = qdd[i];
#pragma unroll
        for (int i = 0; i < ND; ++i)
#pragma unroll
          for (int j = 0; j <= i; ++j) sm.Lf[lq][i * (i + 1) / 2 + j] = L[i][j];
        float viol = 0.f, cost = 0.f;
#pragma unroll
        for (int i = 0; i < ND; ++i) {
          const float e0 = (q[i] + h * qd[i]) - sm.X[lq + 1][i];
          const float e1 = (qd[i] + h * qdd[i]) - sm.X[lq + 1][ND + i];
          sm.e[lq][i] = e0;
          sm.e[lq][ND + i] = e1;
          viol += fabsf(e0) + fabsf(e1);
        }
#pragma unroll
        for (int i = 0; i < NX; ++i) {
          const float d = sm.X[lq][i] - sm.xg[i];
          cost += 0.5f * D.Wq[i] * d * d;
        }
#pragma unroll
        for (int i = 0; i < NU; ++i) cost += 0.5f * D.Wr[i] * u[i] * u[i];
        if (kk >= kf) sm.mp0[lq] = (double)cost + (double)a.mu * (double)viol;
        if (!ok || !isfinite(viol) || !isfinite(cost)) bad_flag = 1;
      }
      wave_sync();
      if (lane < NX) {
        float q[ND], qd[ND], qdd[ND], col[ND];
#pragma unroll
        for (int i = 0; i < ND; ++i) {
          q[i] = sm.X[lq][i];
          qd[i] = sm.X[lq][ND + i];
          qdd[i] = sm.qdd[lq][i];
        }
        id_tangent<ND>(ch, q, qd, qdd, lane, col);
        float L[ND][ND];
#pragma unroll
        for (int i = 0; i < ND; ++i)
#pragma unroll
          for (int j = 0; j < ND; ++j) L[i][j] = (j <= i) ? sm.Lf[lq][i * (i + 1) / 2 + j] : 0.f;
        chol_solve<ND>(L, col);
        float *Ak = sm.A[lq];
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
          float *Bk = sm.B[lq];
#pragma unroll
          for (int i = 0; i < ND; ++i) {
            Bk[i * NU + lane] = 0.f;
            Bk[(ND + i) * NU + lane] = h * mi[i];
          }
        }
      }
    }
    // Gradients at the knots kq0..kl, the initial residual, the terminal and
    // initial merit terms (owners of knot N - 1 and knot 0).
    const int lq0 = kq0 - kf + 1;
    for (int t = tid; t < (nloc > 0 ? nloc + 1 - lq0 : 0) * G; t += kBlock) {
      const int lg = lq0 + t / G, j = t % G, kk = kof(lg);
      const float *W = (kk < N - 1) ? D.Wq : D.Wn;
      sm.qg[lg][j] = j < NX ? W[j] * (sm.X[lg][j] - sm.xg[j]) : 0.f;
      if (kk < N - 1 && j < 8) sm.rg[lg][j] = j < NU ? D.Wr[j] * sm.U[lg][j] : 0.f;
    }
    if (tid < G) sm.c0[tid] = (tid < NX && kf == 0) ? sm.xs[tid] - sm.X[1][tid] : 0.f;
    if (tid == kBlock - 1) {
      double x0 = 0.0;
      if (nloc > 0 && kl == N - 1) {
        float cost = 0.f;
        for (int i = 0; i < NX; ++i) {
          const float d = sm.X[nloc][i] - sm.xg[i];
          cost += 0.5f * D.Wn[i] * d * d;
        }
        x0 += (double)cost;
      }
      if (kf == 0) {
        float viol = 0.f;
        for (int i = 0; i < NX; ++i) viol += fabsf(sm.xs[i] - sm.X[1][i]);
        x0 += (double)a.mu * (double)viol;
      }
      sm.xmp[n_alpha] = x0;
    }
    if constexpr (TS) {
      // The tip terms and the factors L_k, L_k^-1 of the own knots and both halos.
      const int lt0 = kf > 0 ? 0 : 1, lt1 = has_r ? nloc + 1 : nloc;
      const int nt = nloc > 0 ? lt1 - lt0 + 1 : 0;
      for (int t = slot; t < nt; t += SLOTS) {
        const int lg = lt0 + t, kk = kof(lg);
        tip_factor<ND>(ch, sm.X[lg], ts.pr[lg], (kk < N - 1) ? D.We : D.WeN, (kk < N - 1) ? D.Qd : D.QNd, rho,
                       lane, ts.Jt[lg], ts.pe[lg], &ts.mt[lg], ts.tq[lg], ts.Lc[lg], ts.Li[lg], bad_flag);
      }
    }
    __syncthreads();
    if (tid == 0) sm.bad[(it + 1) & 1] = 0;
    if constexpr (TS) {
      // Tip costs of the own knots into the merit terms; the QP data of the
      // own knots and the left halo rewritten in y_k = T_k^-1 x_k; then the
      // own warm-start multipliers (lambda^ = T_k^T lambda).
      const int nc = (nloc > 0) ? min(kl, N - 2) - kf + 1 : 0;   // own knots with a control
      for (int t = tid; t < nc; t += kBlock) sm.mp0[1 + t] += ts.mt[1 + t];
      if (tid == 0 && nloc > 0 && kl == N - 1) sm.xmp[n_alpha] += ts.mt[nloc];
      const int nr = nloc > 0 ? nloc + 1 - lq0 : 0;
      for (int t = slot; t < nr; t += SLOTS) {
        const int lg = lq0 + t, kk = kof(lg);
        const bool succ = kk < N - 1;
        tip_rewrite<ND>(lane, succ, kk == 0, h, ts.Lc[lg], ts.Li[lg], ts.Lc[succ ? lg + 1 : lg], sm.A[lg] + lane * NX,
                        sm.e[lg], sm.qg[lg], sm.c0, ts.Jt[lg], ts.pe[lg], succ ? D.We : D.WeN, ts.tq[lg]);
      }
      __syncthreads();
      if (own) lam = tip_lambda<ND>(lane, true, ts.Lc[li], ts.Li[li], ts.tq[li], lam);
    }
    if (clk) clk[1] = wall_clock64();

    // ================= 2. Schur rows and diagonal-block inverses of the own knots.
    Real th[NX], Pdf[NX];
    double Am[NX], Ac[NX];   // the A_{k-1} row and A_k column, converted once per SQP iteration
    Real gam = 0, qown = 0;
#pragma unroll
    for (int m = 0; m < NX; ++m) {
      th[m] = 0;
      Am[m] = 0.0;
      Ac[m] = 0.0;
      Pdf[m] = 0;
    }
    if (own && lane < NX) {
      const double *Qik = (k < N - 1) ? sm.Qi : sm.Qni;
      qown = (Real)Qik[lane];
      if (k == 0) {
#pragma unroll
        for (int m = 0; m < NX; ++m) th[m] = (m == lane) ? (Real)sm.Qi[lane] : (Real)0;
        gam = (Real)sm.c0[lane] + (Real)sm.Qi[lane] * (Real)sm.qg[li][lane];
      } else {
        const float *A = sm.A[li - 1];
        const float *B = sm.B[li - 1];
        Real ArQ[NX], BrR[NU];
#pragma unroll
        for (int m = 0; m < NX; ++m) {
          const float arow = A[lane * NX + m];
          Am[m] = arow;
          ArQ[m] = (Real)arow * (Real)sm.Qi[m];
        }
#pragma unroll
        for (int m = 0; m < NU; ++m) BrR[m] = (Real)B[lane * NU + m] * (Real)D.Ri[m];
#pragma unroll
        for (int c = 0; c < NX; ++c) {
          Real t = (c == lane) ? (Real)Qik[lane] : (Real)0;
#pragma unroll
          for (int m = 0; m < NX; ++m) t += ArQ[m] * (Real)A[c * NX + m];
#pragma unroll
          for (int m = 0; m < NU; ++m) t += BrR[m] * (Real)B[c * NU + m];
          th[c] = t;
        }
        Real z = (Real)sm.e[li - 1][lane] + (Real)Qik[lane] * (Real)sm.qg[li][lane];
#pragma unroll
        for (int m = 0; m < NX; ++m) z -= ArQ[m] * (Real)sm.qg[li - 1][m];
#pragma unroll
        for (int m = 0; m < NU; ++m) z -= BrR[m] * (Real)sm.rg[li - 1][m];
        gam = z;
      }
      if (k < N - 1) {
        const float *A = sm.A[li];
#pragma unroll
        for (int m = 0; m < NX; ++m) Ac[m] = A[m * NX + lane];
      }
    }
    if (own) {
      if (k == 0) {
        const Real d0 = lane < NX ? (Real)1 / (Real)sm.Qi[lane] : (Real)0;
#pragma unroll
        for (int m = 0; m < NX; ++m) Pdf[m] = (m == lane) ? d0 : (Real)0;
      } else {
        Real row[NX];
#pragma unroll
        for (int c = 0; c < NX; ++c) row[c] = th[c];
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
        for (int c = 0; c < NX; ++c) Pdf[c] = row[c];
      }
    }
    __syncthreads();
    if (clk) clk[2] = wall_clock64();
    if (clk) clk[3] = wall_clock64();

    // ================= 4. PCG (pipelined arrangement), halos and sums through the exchange.
    const bool rv_ok = own && lane < NX;
    auto put_row = [&](double left, double right) {   // this group's row to the neighbours (exchange xe)
      if (lane < NX) {
        if (has_l && slot == 0) xput(xslot(part, xe) + 2 * lane, xtag(xe), left);
        if (has_r && slot == nloc - 1) xput(xslot(part, xe) + 32 + 2 * lane, xtag(xe), right);
      }
    };
    // Halo rows of exchange e, for an operand published as vl (the value) and
    // vr (Q^-1 times it): the left neighbour's last knot sends its vr row,
    // which lands in vr[0]; the right neighbour's first knot sends its vl row,
    // which lands in vl[nloc + 1] (the products read vr[li - 1] and
    // vl[li + 1]). With sums, the three partials of every part summed in part
    // order.
    auto get_rows_sums = [&](unsigned e, bool sums, double (*vl)[G], double (*vr)[G], double &s0, double &s1,
                             double &s2) {
      const bool dead = sm.xfail != 0;
      const int l = tid & 63;
      const bool hl = has_l && slot == 0 && lane < NX;
      const bool hr = has_r && slot == nloc - 1 && lane < NX;
      unsigned long long *wh = hl ? xslot(part - 1, e) + 32 + 2 * lane : (hr ? xslot(part + 1, e) + 2 * lane : nullptr);
      unsigned long long *wsum = (sums && l < 3 * nparts) ? xslot(l / 3, e) + 64 + 2 * (l % 3) : nullptr;
      double vh = 0.0, v = 0.0;
      if (wh || wsum) {
        bool ok;
        if (wh && wsum) ok = xget2(wh, wsum, xtag(e), dead, xspin, vh, v);
        else if (wh) ok = xget(wh, xtag(e), dead, xspin, vh);
        else ok = xget(wsum, xtag(e), dead, xspin, v);
        if (!ok) sm.xfail = 1;
      }
      if (hl) vr[0][lane] = vh;
      if (hr) vl[nloc + 1][lane] = vh;
      wave_sync();
      if (sums) {
        s0 = (lane_val(v, 0) + lane_val(v, 3)) + (lane_val(v, 6) + lane_val(v, 9));
        s1 = (lane_val(v, 1) + lane_val(v, 4)) + (lane_val(v, 7) + lane_val(v, 10));
        s2 = (lane_val(v, 2) + lane_val(v, 5)) + (lane_val(v, 8) + lane_val(v, 11));
      }
    };
    auto halo = [&](double (*vl)[G], double (*vr)[G]) {
      double d0, d1, d2;
      get_rows_sums(xe, false, vl, vr, d0, d1, d2);
      ++xe;
    };
    auto share_S = [&](Real v) {
      if (own) {
        sm.pv[li][lane] = lane < NX ? v : (Real)0;
        sm.sv[li][lane] = lane < NX ? qown * v : (Real)0;
        put_row(v, qown * v);
      }
    };
    auto apply_S = [&](Real v) -> Real {
      Real d0 = 0, d1 = 0, l0 = 0, l1 = 0, u0 = 0, u1 = 0;
      row_dot2<NX>(d0, d1, v, th);
      // Neighbours' entries by row broadcasts: each lane reads its own entry.
      if (k > 0) row_dot2<NX>(l0, l1, sm.sv[li - 1][lane], Am);
      if (k < N - 1) row_dot2<NX>(u0, u1, sm.pv[li + 1][lane], Ac);
      return ((d0 + d1) - (l0 + l1)) - qown * (u0 + u1);
    };
    auto dinv = [&](Real x) -> Real {
      Real acc = 0;
      row_dot1<NX>(acc, x, Pdf);
      return acc;
    };
    auto prepare_P = [&](Real v) {
      if (own) {
        const Real z = dinv(v);
        sm.rv[li][lane] = lane < NX ? z : (Real)0;
        sm.gv[li][lane] = lane < NX ? qown * z : (Real)0;
        put_row(z, qown * z);
      }
    };
    auto finish_P = [&](Real v) -> Real {
      Real oz = 0;
      if (k > 0) row_dot1_sub<NX>(oz, sm.gv[li - 1][lane], Am);
      if (k < N - 1) {
        Real t = 0;
        row_dot1<NX>(t, sm.rv[li + 1][lane], Ac);
        oz -= qown * t;
      }
      return dinv(v - oz);
    };

    Real r, u, w, vm = 0, vn = 0, vz = 0, vq = 0, vs = 0, vp = 0;
    share_S(lam);
    __syncthreads();
    halo(sm.pv, sm.sv);
    r = rv_ok ? gam - apply_S(lam) : (Real)0;
    prepare_P(r);
    __syncthreads();
    halo(sm.rv, sm.gv);
    u = rv_ok ? finish_P(r) : (Real)0;
    __syncthreads();
    prepare_P(gam);
    __syncthreads();
    halo(sm.rv, sm.gv);
    const Real Pgam = rv_ok ? finish_P(gam) : (Real)0;
    Real eta_ref = gam * Pgam;
    const int max_it = a.pcg_max_iter > 0 ? a.pcg_max_iter : N * NX;
    Real gma = 0, stop = 0;
    int its = 0;
    share_S(u);
    __syncthreads();
    halo(sm.pv, sm.sv);
    w = rv_ok ? apply_S(u) : (Real)0;
    eta_ref = wave_sum(eta_ref);
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    if ((tid & 63) == 0) sm.red[redbuf][2][wave] = eta_ref;
    Real rg = 0, cga = 0;
    for (;;) {
#pragma unroll
      for (int m = 0; m < NX; ++m) {
        asm volatile("" : "+v"(Am[m]), "+v"(Ac[m]));
        asm volatile("" : "+v"(Pdf[m]));
      }
      Real pr = r * u, pwu = w * u;
      wave_sum2(pr, pwu);
      if ((tid & 63) == 0) {
        sm.red[redbuf][0][wave] = pr;
        sm.red[redbuf][1][wave] = pwu;
      }
      prepare_P(w);
      __syncthreads();
      gma = pair_tree<kBlock / 64>(sm.red[redbuf][0]);
      Real dlt = pair_tree<kBlock / 64>(sm.red[redbuf][1]);
      {
        const double e0 = (its == 0) ? pair_tree<kBlock / 64>(sm.red[redbuf][2]) : 0.0;
        if (tid < 3) xput(xslot(part, xe) + 64 + 2 * tid, xtag(xe), tid == 0 ? gma : (tid == 1 ? dlt : e0));
        double g_, d_, e_;
        get_rows_sums(xe, true, sm.rv, sm.gv, g_, d_, e_);
        ++xe;
        gma = g_;
        dlt = d_;
        if (its == 0) stop = (Real)a.pcg_tol * (Real)a.pcg_tol * (Real)e_;
      }
      redbuf ^= 1;
      if (!(gma > stop) || its >= max_it) break;
      vm = rv_ok ? finish_P(w) : (Real)0;
      share_S(vm);
      const Real beta = gma * rg;
      const Real alpha = div_pcg(gma, dlt - gma * gma * cga);
      __syncthreads();
      halo(sm.pv, sm.sv);
      vn = rv_ok ? apply_S(vm) : (Real)0;
      vz = vn + beta * vz;
      vq = vm + beta * vq;
      vs = w + beta * vs;
      vp = u + beta * vp;
      lam += alpha * vp;
      r -= alpha * vs;
      u -= alpha * vq;
      w -= alpha * vz;
      cga = div_pcg((Real)1, gma * alpha);
      rg = alpha * cga;
      ++its;
    }
    unsigned status = (gma > stop) ? GATO_ST_PCG_MAXITER : 0u;
    if (clk) clk[4] = wall_clock64();

    // ================= 5. Step dZ = -G^-1 (g - C^T lambda) at the own knots and the halos.
    // Multipliers of the halo knots first (exchange), then the own steps and the
    // left halo's step (this part holds its LQ data), then the right halo's step
    // from the right part (its first own knot).
    if (own) {
      sm.pv[li][lane] = lane < NX ? lam : (Real)0;
      put_row(lam, lam);
    }
    __syncthreads();
    halo(sm.pv, sm.pv);
    auto step_at = [&](int lg, int kk, Real lam_own, Real qk) {   // step of knot kk (local lg), row `lane`
      Real sx = (Real)sm.qg[lg][lane] - lam_own;
      if (kk < N - 1) {
        const float *A = sm.A[lg];
#pragma unroll
        for (int m = 0; m < NX; ++m) sx += (Real)A[m * NX + lane] * sm.pv[lg + 1][m];
      }
      const float dx = (float)(-qk * sx);
      sm.dX[lg][lane] = dx;
      if (!isfinite(dx)) bad_flag = 1;
      if constexpr (TS) {
        if (lane < ND) ts.tq[lg][lane] = (double)(-qk * sx);
      }
      if (lane < NU && kk < N - 1) {
        const float *B = sm.B[lg];
        Real su = (Real)sm.rg[lg][lane];
#pragma unroll
        for (int m = 0; m < NX; ++m) su += (Real)B[m * NU + lane] * sm.pv[lg + 1][m];
        const float du = (float)(-(Real)D.Ri[lane] * su);
        sm.dU[lg][lane] = du;
        if (!isfinite(du)) bad_flag = 1;
      }
    };
    if (own && lane < NX) step_at(li, k, lam, qown);
    if (has_l && slot == 0 && lane < NX) step_at(0, kf - 1, sm.pv[0][lane], (Real)sm.Qi[lane]);
    if constexpr (TS) {
      // Back to x: dx_k = T_k dy_k (joint rows L_k^-T dy) at the own knots and
      // the left halo, and lambda = T_k^-T lambda^ at the own knots.
      auto to_x = [&](int lg) {
        wave_sync();
        double t = 0.0;
        if (lane < ND) {
#pragma unroll
          for (int m = 0; m < ND; ++m)
            if (m >= lane) t += ts.Li[lg][tri(m, lane)] * ts.tq[lg][m];
        }
        wave_sync();
        if (lane < ND) {
          const float dx = (float)t;
          sm.dX[lg][lane] = dx;
          if (!isfinite(dx)) bad_flag = 1;
        }
      };
      if (own) {
        to_x(li);
        lam = tip_lambda<ND>(lane, false, ts.Lc[li], ts.Li[li], ts.tq[li], lam);
      }
      if (has_l && slot == 0) to_x(0);
    }
    __syncthreads();
    if (own && slot == 0) put_row((double)sm.dX[1][lane], 0.0);
    {
      // (Only the rows towards the left travel; a part reads its right
      // neighbour's first step into dX[nloc + 1].)
      const bool dead = sm.xfail != 0;
      if (has_r && slot == nloc - 1 && lane < NX) {
        double v;
        if (!xget(xslot(part + 1, xe) + 2 * lane, xtag(xe), dead, xspin, v)) sm.xfail = 1;
        sm.dX[nloc + 1][lane] = (float)v;
      }
      ++xe;
    }
    __syncthreads();
    if (clk) clk[5] = wall_clock64();

    // ================= 6. Line search over the own knots; partial merits summed over the parts.
    const int nst = (nloc > 0) ? min(kl, N - 2) - kf + 1 : 0;   // own knots with a control
    const int ntask = n_alpha * max(nst, 0);
    for (int t = tid; t < ntask; t += kBlock) {
      const int i = t / nst, lg = 1 + (t - i * nst);
      const float al = sm.alpha[i];
      float q[ND], qd[ND], uu[ND], qdd[ND], L[ND][ND], xn[NX];
#pragma unroll
      for (int j = 0; j < ND; ++j) {
        q[j] = sm.X[lg][j] + al * sm.dX[lg][j];
        qd[j] = sm.X[lg][ND + j] + al * sm.dX[lg][ND + j];
        uu[j] = sm.U[lg][j] + al * sm.dU[lg][j];
      }
#pragma unroll
      for (int j = 0; j < NX; ++j) xn[j] = sm.X[lg + 1][j] + al * sm.dX[lg + 1][j];
      forward_dynamics<ND>(ch, q, qd, uu, qdd, L);
      float viol = 0.f, cost = 0.f;
#pragma unroll
      for (int j = 0; j < ND; ++j) {
        viol += fabsf((q[j] + h * qd[j]) - xn[j]) + fabsf((qd[j] + h * qdd[j]) - xn[ND + j]);
        const float d0 = q[j] - sm.xg[j], d1 = qd[j] - sm.xg[ND + j];
        cost += 0.5f * D.Wq[j] * d0 * d0 + 0.5f * D.Wq[ND + j] * d1 * d1 + 0.5f * D.Wr[j] * uu[j] * uu[j];
      }
      if constexpr (TS) {
        float pt[3];
        tip_position<ND>(ch, q, pt);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float d = pt[c] - ts.pr[lg][c];
          cost += 0.5f * D.We[c] * d * d;
        }
      }
      sm.mp[i][lg] = (double)cost + (double)a.mu * (double)viol;
    }
    for (int i = tid; i < n_alpha; i += kBlock) {
      const float al = sm.alpha[i];
      double x0 = 0.0;
      if (nloc > 0 && kl == N - 1) {
        float cost = 0.f;
        for (int j = 0; j < NX; ++j) {
          const float d = (sm.X[nloc][j] + al * sm.dX[nloc][j]) - sm.xg[j];
          cost += 0.5f * D.Wn[j] * d * d;
        }
        if constexpr (TS) {
          float q[ND], pt[3];
#pragma unroll
          for (int j = 0; j < ND; ++j) q[j] = sm.X[nloc][j] + al * sm.dX[nloc][j];
          tip_position<ND>(ch, q, pt);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const float d = pt[c] - ts.pr[nloc][c];
            cost += 0.5f * D.WeN[c] * d * d;
          }
        }
        x0 += (double)cost;
      }
      if (kf == 0) {
        float viol = 0.f;
        for (int j = 0; j < NX; ++j) viol += fabsf(sm.xs[j] - (sm.X[1][j] + al * sm.dX[1][j]));
        x0 += (double)a.mu * (double)viol;
      }
      sm.xmp[i] = x0;
    }
    __syncthreads();
    if (tid <= n_alpha) {
      double sum = 0.0;
      for (int lg = 1; lg <= max(nst, 0); ++lg) sum += (tid == n_alpha) ? sm.mp0[lg] : sm.mp[tid][lg];
      sm.psum[tid] = sum + sm.xmp[tid];
    }
    __syncthreads();
    {
      // Partial merits (n_alpha + 1), this part's non-finite flag and its
      // exchange failure flag to every part; summed in part order.
      const int nv = n_alpha + 3;
      if (tid < nv) {
        const double v = tid <= n_alpha ? sm.psum[tid] : (tid == n_alpha + 1 ? (double)bad_flag : (double)sm.xfail);
        xput(xslot(part, xe) + 64 + 2 * tid, xtag(xe), v);
      }
      const bool dead = sm.xfail != 0;
      if (tid < nv * nparts) {
        const int q = tid / nv, v = tid % nv;
        double x;
        if (!xget(xslot(q, xe) + 64 + 2 * v, xtag(xe), dead, xspin, x)) sm.xfail = 1;
        sm.msum[q][v] = x;
      }
      ++xe;
      __syncthreads();
      if (tid <= n_alpha) {
        double m = 0.0;
        for (int q = 0; q < nparts; ++q) m += sm.msum[q][tid];
        sm.merit[tid] = m;
      }
      __syncthreads();
    }
    int best = -1;
    for (int i = 0; i < n_alpha; ++i) {
      const double m = sm.merit[i];
      if (isfinite(m) && (best < 0 || m < sm.merit[best])) best = i;
    }
    bool any_bad = false, any_xfail = sm.xfail != 0;
    for (int q = 0; q < nparts; ++q) {
      any_bad = any_bad || sm.msum[q][n_alpha + 1] != 0.0;
      any_xfail = any_xfail || sm.msum[q][n_alpha + 2] != 0.0;
    }
    const bool bad = any_bad || best < 0;
    if (bad) status |= GATO_ST_NONFINITE;
    else if (!(sm.merit[best] < sm.merit[n_alpha])) status |= GATO_ST_NO_DESCENT;
    if (any_xfail) status |= GATO_ST_EXCHANGE;
    const double rho_used = rho;
    if (a.rho_adapt) rho = (status & (GATO_ST_NONFINITE | GATO_ST_NO_DESCENT)) ? fmin(2.0 * rho, 1e8) : rho / 3.0;
    const float al = bad ? 0.f : sm.alpha[best];
    if (!bad) {
      for (int t = tid; t < (nloc + 2) * G; t += kBlock) {
        const int lg = t / G, j = t % G, kk = kof(lg);
        if (kk < 0 || kk >= N || nloc == 0) continue;
        sm.X[lg][j] += al * sm.dX[lg][j];
        if (kk < N - 1 && lg <= nloc && j < 8) sm.U[lg][j] += al * sm.dU[lg][j];
      }
    }
    if (tid == 0 && a.stats && writer) {
      gato_solve_stats st;
      st.merit0 = (float)sm.merit[n_alpha];
      st.merit = bad ? (float)sm.merit[n_alpha] : (float)sm.merit[best];
      st.alpha = al;
      st.pcg_iters = its;
      st.status = status;
      st.rho = (float)rho_used;
      a.stats[(size_t)sid * a.stats_stride + it] = st;
    }
    __syncthreads();
    if (clk) {
      clk[6] = wall_clock64();
      clk[7] = clock64() - cyc0;
    }
  }

  // ---- Write back the own knots' iterate and multipliers, and the damping.
  if (writer && a.rho_adapt && tid == 0) a.rho[sid] = rho;
  for (int t = tid; t < nloc * G; t += kBlock) {
    const int lg = 1 + t / G, j = t % G, kk = kof(lg);
    if (j < NX) a.X[xoff + (size_t)kk * a.nx_max + j] = sm.X[lg][j];
    if (kk < N - 1 && j < NU) a.U[uoff + (size_t)kk * a.nu_max + j] = sm.U[lg][j];
  }
  if (own0) gL[(kf + slot0) * a.nx_max + lane0] = (double)lam;
}

template <int ND, int KPT, class Real, bool TS = false, bool SPLIT = false>
__device__ __attribute__((always_inline)) inline void sqp_solve(const KArgs &a, int sid, int part, char *smem_raw) {
  using Sh = Shape<ND>;
  constexpr int NX = Sh::NX, NU = Sh::NU, G = Sh::G, SLOTS = Sh::SLOTS;
  constexpr bool kLds = BlockStore<ND, KPT>::kLds;
  using SM = Smem<ND, KPT, Real>;
  SM &sm = *reinterpret_cast<SM *>(smem_raw);
  // Only dereferenced by the task-space variant, whose LDS holds it.
  TsSmem<ND, KPT> &ts = *reinterpret_cast<TsSmem<ND, KPT> *>(smem_raw + ts_offset<ND, KPT, Real>());
  const SolveDesc &D = a.desc[sid];
  const Chain &ch = D.chain;
  const int tid = threadIdx.x;
  const int lane0 = tid % G;
  const int slot0 = tid / G;
  const int N = D.N;
  const float h = D.dt;
  const int n_alpha = a.n_alpha;
  // Split solve (four knots per lane group): four (or two) workgroups run
  // the same SQP iteration, each with its own workspace, and share the PCG:
  // part j owns the knots of p == j (or p == 2 j, 2 j + 1). Only part 0 writes
  // results.
  // (SPLIT: compiled into kernels of their own, so that the one-workgroup
  // kernels carry none of the exchange code.)
  constexpr bool kSplitOk = SPLIT && (KPT == 4) && !TS;
  // a.split = 4: part j owns p = j; a.split = 2 (when four workgroups per solve
  // do not fit the chip): part j owns p = 2 j and 2 j + 1.
  const int nparts = a.split == 2 ? 2 : kXParts;
  const int psh = nparts == 2 ? 1 : 0;
  const bool split = kSplitOk && a.split && a.mode == kModeSqp && D.xch_off >= 0 && part >= 0 && part < nparts;
  // Four parts of a long FP64 solve run the part-local form (one knot per
  // lane group over the part's own knots, FP64 D^-1 rows); two parts, and the
  // all-FP32 variant, the four-knots-per-group form below.
  if constexpr (kSplitOk && sizeof(Real) == 8) {
    static_assert(sizeof(PartSmem<ND>) <= smem_bytes<ND, KPT, Real, TS>(), "LDS of a part");
    if (split && a.split == 4 && !a.by_block) {
      sqp_solve_part<ND, false>(a, sid, part, smem_raw);
      return;
    }
  }
  const bool writer = !split || part == 0;
  char *ws = a.ws + D.ws_off + (split ? (int64_t)part * D.ws_part : 0);
  const size_t xoff = (size_t)sid * a.N_max * a.nx_max;
  const size_t uoff = (size_t)sid * (a.N_max - 1) * a.nu_max;
  double *gL = a.lam + xoff;  // [N][nx_max]
  const int rid = a.by_block ? (int)blockIdx.x : sid;  // index of xs, goal, stats
  const int sh = a.shift;

  // Block accessors (LDS or the solve's workspace).
  auto Ablk = [&](int k) -> float * {
    if constexpr (kLds) return sm.A[k];
    else return reinterpret_cast<float *>(ws + D.offA) + (size_t)k * NX * NX;
  };
  auto Bblk = [&](int k) -> float * {
    if constexpr (kLds) return sm.B[k];
    else return reinterpret_cast<float *>(ws + D.offB) + (size_t)k * NX * NU;
  };
  auto Dblk = [&](int k) -> float * {
    if constexpr (kLds) return sm.Dinv[k];
    else return reinterpret_cast<float *>(ws + D.offD) + (size_t)k * NX * NX;
  };
  auto Pblk = [&](int k) -> float * {   // explicit preconditioner blocks: kpt == 1 only
    if constexpr (kLds) return sm.Poff[k];
    else return nullptr;
  };
  // Rows of the Schur diagonal blocks, kept in the workspace (read back through
  // L2) when four knots per lane group would not fit them in registers.
  constexpr bool kThGlobal = KPT >= 4;
  auto Tblk = [&](int k) -> Real * { return reinterpret_cast<Real *>(ws + D.offT) + (size_t)k * NX * NX; };
  // A_k^T in the workspace: the columns of A_k as contiguous rows, for the
  // kernels that read them back where they are used (one vector load per
  // four entries instead of a strided load per entry).
  auto ATblk = [&](int k) -> float * { return reinterpret_cast<float *>(ws + D.offAT) + (size_t)k * NX * NX; };
  constexpr bool kColsT = KPT >= 4 && sizeof(Real) == 8;

  // ---- Stage the iterate and the solve constants in LDS.
  // (With a warm-start shift, knot k starts from the previous knot k + shift,
  // the last knot repeated.)
  for (int t = tid; t < N * G; t += kBlock) {
    const int k = t / G, j = t % G;
    const int ks = min(k + sh, N - 1);
    sm.X[k][j] = (j < NX && a.mode != kModeKkt) ? a.X[xoff + (size_t)ks * a.nx_max + j] : 0.f;
  }
  for (int t = tid; t < (N - 1) * 8; t += kBlock) {
    const int k = t / 8, j = t % 8;
    const int ks = min(k + sh, N - 2);
    sm.U[k][j] = (j < NU && a.mode != kModeKkt) ? a.U[uoff + (size_t)ks * a.nu_max + j] : 0.f;
  }
  if (tid < G) {
    const bool in = tid < NX && a.mode != kModeKkt;
    sm.xs[tid] = in ? a.xs[(size_t)rid * a.nx_max + tid] : 0.f;
    sm.xg[tid] = (in && tid < ND) ? a.goal[(size_t)rid * a.nu_max + tid] : 0.f;
  }
  if constexpr (TS) {
    // Reference tip positions of this request's horizon (not shifted).
    for (int t = tid; t < N * 4; t += kBlock) {
      const int k = t / 4, c = t % 4;
      ts.pr[k][c] = c < 3 ? a.pref[((size_t)sid * a.N_max + k) * 3 + c] : 0.f;
    }
  }
  if (tid == 0) {
    sm.bad[0] = 0;
    sm.bad[1] = 0;
    sm.xfail = 0;
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
    const int k = slot0 + p * SLOTS;
    lam[p] = (a.warm && a.mode == kModeSqp && k < N && lane0 < NX)
                 ? (Real)gL[min(k + sh, N - 1) * a.nx_max + lane0] : (Real)0;
  }
  int redbuf = 0;
  unsigned xe = 0;   // split solve: exchange number (the same sequence in every part)
  // Damping on every Q_k (Sec. IV-C); uniform across the workgroup.
  double rho = a.rho[sid];
  __syncthreads();

  for (int it = 0; it < a.iters; ++it) {
    // Opaque per-iteration copies: keeps the compiler from hoisting the many
    // lane-dependent selects of the phases below out of the iteration loop,
    // where they would stay live across every phase and spill.
    int lane = lane0, slot = slot0;
    asm volatile("" : "+v"(lane), "+v"(slot));
    // Without warm starts every PCG solve starts from zero.
    if (!a.warm && it > 0) {
#pragma unroll
      for (int p = 0; p < KPT; ++p) lam[p] = (Real)0;
    }
    // Q^-1 and Q_N^-1 for this iteration's rho (first read after phase 1's barrier).
    // (Task-space variant: the joint block of the rewritten Q_k is the identity.)
    if (tid < G) {
      const bool unit = TS && tid < ND;
      sm.Qi[tid] = tid < NX ? (unit ? 1.0 : 1.0 / (D.Qd[tid] + rho)) : 0.0;
      sm.Qni[tid] = tid < NX ? (unit ? 1.0 : 1.0 / (D.QNd[tid] + rho)) : 0.0;
    }
    int &bad_flag = sm.bad[it & 1];
    unsigned long long *clk = (a.clk && tid == 0 && writer) ? a.clk + ((size_t)sid * a.iters + it) * 8 : nullptr;
    unsigned long long cyc0 = 0;
    if (clk) {
      clk[0] = wall_clock64();
      cyc0 = clock64();
    }
    // ================= 1. LQ: dynamics, derivatives, defects, gradients.
    if (a.mode != kModeKkt) {
      for (int k = slot; k < N - 1; k += SLOTS) {
        if (lane == 0) {
          float q[ND], qd[ND], u[ND], qdd[ND], L[ND][ND];
#pragma unroll
          for (int i = 0; i < ND; ++i) {
            q[i] = sm.X[k][i];
            qd[i] = sm.X[k][ND + i];
            u[i] = sm.U[k][i];
          }
          const bool ok = forward_dynamics<ND>(ch, q, qd, u, qdd, L);
#pragma unroll
          for (int i = 0; i < ND; ++i) sm.qdd[k][i] = qdd[i];
#pragma unroll
          for (int i = 0; i < ND; ++i)
#pragma unroll
            for (int j = 0; j <= i; ++j) sm.Lf[k][i * (i + 1) / 2 + j] = L[i][j];
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
          sm.mp0[k] = (double)cost + (double)a.mu * (double)viol;
          if (!ok || !isfinite(viol) || !isfinite(cost)) bad_flag = 1;
        }
        wave_sync();
        if (lane < NX) {
          float q[ND], qd[ND], qdd[ND], col[ND];
#pragma unroll
          for (int i = 0; i < ND; ++i) {
            q[i] = sm.X[k][i];
            qd[i] = sm.X[k][ND + i];
            qdd[i] = sm.qdd[k][i];
          }
          id_tangent<ND>(ch, q, qd, qdd, lane, col);
          float L[ND][ND];
#pragma unroll
          for (int i = 0; i < ND; ++i)
#pragma unroll
            for (int j = 0; j < ND; ++j) L[i][j] = (j <= i) ? sm.Lf[k][i * (i + 1) / 2 + j] : 0.f;
          chol_solve<ND>(L, col);
          float *Ak = Ablk(k);
#pragma unroll
          for (int i = 0; i < ND; ++i) {
            Ak[i * NX + lane] = (i == lane ? 1.f : 0.f) + (lane == ND + i ? h : 0.f);
            Ak[(ND + i) * NX + lane] = h * col[i] + (lane == ND + i ? 1.f : 0.f);
          }
          if constexpr (kColsT) {
            float *Atk = ATblk(k) + lane * NX;
#pragma unroll
            for (int i = 0; i < ND; ++i) {
              Atk[i] = (i == lane ? 1.f : 0.f) + (lane == ND + i ? h : 0.f);
              Atk[ND + i] = h * col[i] + (lane == ND + i ? 1.f : 0.f);
            }
          }
          if (lane < ND) {
            float mi[ND];
#pragma unroll
            for (int i = 0; i < ND; ++i) mi[i] = (i == lane) ? 1.f : 0.f;
            chol_solve<ND>(L, mi);
            float *Bk = Bblk(k);
#pragma unroll
            for (int i = 0; i < ND; ++i) {
              Bk[i * NU + lane] = 0.f;
              Bk[(ND + i) * NU + lane] = h * mi[i];
            }
          }
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
        sm.mp0[N - 1] = (double)cost + (double)a.mu * (double)viol;
      }
      if constexpr (TS) {
        // The tip terms and the factors L_k, L_k^-1 of every knot.
        for (int k = slot; k < N; k += SLOTS)
          tip_factor<ND>(ch, sm.X[k], ts.pr[k], (k < N - 1) ? D.We : D.WeN, (k < N - 1) ? D.Qd : D.QNd, rho, lane,
                         ts.Jt[k], ts.pe[k], &ts.mt[k], ts.tq[k], ts.Lc[k], ts.Li[k], bad_flag);
      }
      if (a.mode == kModeLq) {
        __syncthreads();
        const size_t ao = (size_t)sid * (a.N_max - 1) * a.nx_max * a.nx_max;
        const size_t bo = (size_t)sid * (a.N_max - 1) * a.nx_max * a.nu_max;
        const size_t eo = (size_t)sid * (a.N_max - 1) * a.nx_max;
        for (int t = tid; t < (N - 1) * NX * NX; t += kBlock) {
          const int k = t / (NX * NX), r = (t / NX) % NX, c = t % NX;
          a.outA[ao + ((size_t)k * a.nx_max + r) * a.nx_max + c] = Ablk(k)[r * NX + c];
        }
        for (int t = tid; t < (N - 1) * NX * NU; t += kBlock) {
          const int k = t / (NX * NU), r = (t / NU) % NX, c = t % NU;
          a.outB[bo + ((size_t)k * a.nx_max + r) * a.nu_max + c] = Bblk(k)[r * NU + c];
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
        const float v = a.inA[ao + ((size_t)k * a.nx_max + r) * a.nx_max + c];
        Ablk(k)[r * NX + c] = v;
        if constexpr (kColsT) ATblk(k)[c * NX + r] = v;
      }
      for (int t = tid; t < (N - 1) * NX * NU; t += kBlock) {
        const int k = t / (NX * NU), r = (t / NU) % NX, c = t % NU;
        Bblk(k)[r * NU + c] = a.inB[bo + ((size_t)k * a.nx_max + r) * a.nu_max + c];
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
    if constexpr (TS) {
      for (int t = tid; t < N; t += kBlock) sm.mp0[t] += ts.mt[t];
      // Rewrite the QP in y_k = T_k^-1 x_k, and the warm-start multipliers
      // (lambda^ = T_k^T lambda).
#pragma unroll
      for (int p = 0; p < KPT; ++p) {
        const int k = slot + p * SLOTS;
        if (k < N) {
          const bool succ = k < N - 1;
          tip_rewrite<ND>(lane, succ, k == 0, h, ts.Lc[k], ts.Li[k], ts.Lc[succ ? k + 1 : k], Ablk(k) + lane * NX,
                          sm.e[k], sm.qg[k], sm.c0, ts.Jt[k], ts.pe[k], succ ? D.We : D.WeN, ts.tq[k]);
          lam[p] = (Real)tip_lambda<ND>(lane, true, ts.Lc[k], ts.Li[k], ts.tq[k], (double)lam[p]);
        }
      }
      __syncthreads();
    }
    if (clk) clk[1] = wall_clock64();

    // ================= 2. Schur complement rows and diagonal-block inverses.
    Real th[kThGlobal ? 1 : KPT][NX];   // row of the diagonal block theta_{k-1} (Q_0^-1 for k = 0)
    // A entries are exact in FP32. With one knot per lane group (FP64
    // variant) the rows are held converted to FP64, once per SQP iteration:
    // the PCG loop then converts nothing (28 conversions fewer per iteration)
    // and, since its two products would otherwise keep FP64 copies of the
    // FP32 rows live across the second barrier, holds fewer registers too
    // (spills 88 -> 20 B/lane, 12% off the headline call). Elsewhere they
    // are kept in FP32 (converted to Real at use), which halves their
    // register footprint. With four knots per lane group (FP64 variant) the
    // rows are read back from the A blocks in the workspace where they are
    // used (as the Schur rows are), which frees 112 registers per lane; the
    // FP32 variant has the room.
    constexpr bool kRowsGlobal = KPT >= 4 && sizeof(Real) == 8;
    static_assert(kRowsGlobal == kColsT, "column reads of A_k need its transposed copy");
    constexpr int KR = kRowsGlobal ? 1 : KPT;
    constexpr bool kRealA = (KPT == 1) && sizeof(Real) == 8 && !TS;
    using AT = std::conditional_t<kRealA, double, float>;
    AT Am[KR][NX];     // row `lane` of A_{k-1}: S~_{k,k-1} = -A_{k-1} Q_{k-1}^-1
    AT Ac[KR][NX];     // column `lane` of A_k: S~_{k,k+1} = -Q_k^-1 A_k^T
    auto am = [&](int p, int m) -> AT {
      if constexpr (kRowsGlobal) return Ablk(slot + p * SLOTS - 1)[lane * NX + m];
      else return Am[p][m];
    };
    auto ac = [&](int p, int m) -> AT {
      if constexpr (kRowsGlobal) return ATblk(slot + p * SLOTS)[lane * NX + m];
      else return Ac[p][m];
    };
    Real gam[KPT];
    Real qown[KPT];       // Q_k^-1 at (lane, lane)
    Real Pd[KPT][NX];     // row of the inverse diagonal block (preconditioner)
#pragma unroll
    for (int p = 0; p < KPT; ++p) {
      const int k = slot + p * SLOTS;
      const bool valid = k < N && lane < NX;
      Real thr[NX];
#pragma unroll
      for (int m = 0; m < NX; ++m) {
        thr[m] = 0;
        if constexpr (!kRowsGlobal) {
          Am[p][m] = 0.f;
          Ac[p][m] = 0.f;
        }
        Pd[p][m] = 0;
      }
      gam[p] = 0;
      qown[p] = 0;
      if (valid) {
        const double *Qik = (k < N - 1) ? sm.Qi : sm.Qni;
        qown[p] = (Real)Qik[lane];
        if (k == 0) {
#pragma unroll
          for (int m = 0; m < NX; ++m) thr[m] = (m == lane) ? (Real)sm.Qi[lane] : (Real)0;
          gam[p] = (Real)sm.c0[lane] + (Real)sm.Qi[lane] * (Real)sm.qg[0][lane];
        } else {
          const int km = k - 1;
          const float *A = Ablk(km);
          const float *B = Bblk(km);
          Real ArQ[NX], BrR[NU];
#pragma unroll
          for (int m = 0; m < NX; ++m) {
            const float arow = A[lane * NX + m];
            if constexpr (!kRowsGlobal) Am[p][m] = arow;
            ArQ[m] = (Real)arow * (Real)sm.Qi[m];
          }
#pragma unroll
          for (int m = 0; m < NU; ++m) BrR[m] = (Real)B[lane * NU + m] * (Real)D.Ri[m];
          if constexpr (sizeof(Real) == 8 && G == 16 && !kRowsGlobal) {
            // Entry (lane, c) of theta: the rows of A_{k-1} and B_{k-1} that
            // lane c holds, read by row broadcasts (same terms, same order).
            double Br[NU];
#pragma unroll
            for (int m = 0; m < NU; ++m) Br[m] = (double)B[lane * NU + m];
#pragma unroll
            for (int c = 0; c < NX; ++c) thr[c] = (c == lane) ? (Real)Qik[lane] : (Real)0;
#pragma unroll
            for (int m = 0; m < NX; ++m) col_fma<NX>(thr, (double)Am[p][m], ArQ[m]);
#pragma unroll
            for (int m = 0; m < NU; ++m) col_fma<NX>(thr, Br[m], BrR[m]);
          } else {
#pragma unroll
            for (int c = 0; c < NX; ++c) {
              Real t = (c == lane) ? (Real)Qik[lane] : (Real)0;
#pragma unroll
              for (int m = 0; m < NX; ++m) t += ArQ[m] * (Real)A[c * NX + m];
#pragma unroll
              for (int m = 0; m < NU; ++m) t += BrR[m] * (Real)B[c * NU + m];
              thr[c] = t;
            }
          }
          Real z = (Real)sm.e[km][lane] + (Real)Qik[lane] * (Real)sm.qg[k][lane];
#pragma unroll
          for (int m = 0; m < NX; ++m) z -= ArQ[m] * (Real)sm.qg[km][m];
#pragma unroll
          for (int m = 0; m < NU; ++m) z -= BrR[m] * (Real)sm.rg[km][m];
          gam[p] = z;
        }
        if constexpr (!kRowsGlobal) {
          if (k < N - 1) {
            const float *A = Ablk(k);
#pragma unroll
            for (int m = 0; m < NX; ++m) Ac[p][m] = A[m * NX + lane];
          }
        }
      }
      // Inverse of the diagonal block: Gauss-Jordan inside the lane group
      // (the block is SPD, so no pivoting is needed).
      if (k < N) {
        if (k == 0) {
          const Real d0 = lane < NX ? (Real)1 / (Real)sm.Qi[lane] : (Real)0;
#pragma unroll
          for (int m = 0; m < NX; ++m) Pd[p][m] = (m == lane) ? d0 : (Real)0;
        } else {
          // T: the arithmetic of the elimination (Real, or double when the
          // all-FP32 variant is asked for an FP64 block inverse).
          auto gauss_jordan = [&](auto tag) {
            using T = decltype(tag);
            T row[NX];
#pragma unroll
            for (int c = 0; c < NX; ++c) row[c] = (T)thr[c];
            if constexpr (std::is_same_v<T, double> && G == 16 && !TS) {
              gj_dpp<NX>(row, lane, std::make_integer_sequence<int, NX>{});
            } else {
#pragma unroll
            for (int pv = 0; pv < NX; ++pv) {
              if (lane == pv) {
#pragma unroll
                for (int c = 0; c < NX; ++c) sm.piv[slot][c] = (double)row[c];
              }
              wave_sync();
              T prow[NX];
#pragma unroll
              for (int c = 0; c < NX; ++c) prow[c] = (T)sm.piv[slot][c];
              wave_sync();
              const T pinv = (T)1 / prow[pv];
              if (lane == pv) {
#pragma unroll
                for (int c = 0; c < NX; ++c) row[c] = (c == pv) ? pinv : row[c] * pinv;
              } else {
                const T f = row[pv] * pinv;
#pragma unroll
                for (int c = 0; c < NX; ++c) row[c] = (c == pv) ? -f : row[c] - f * prow[c];
              }
            }
            }
#pragma unroll
            for (int c = 0; c < NX; ++c) Pd[p][c] = (Real)row[c];
          };
          if (sizeof(Real) == 4 && a.fp64_inv) gauss_jordan(double{});
          else gauss_jordan(Real{});
        }
        if (lane < NX) {
          float *Dk = Dblk(k) + lane * NX;
#pragma unroll
          for (int c = 0; c < NX; ++c) Dk[c] = (float)Pd[p][c];
        }
      }
      if constexpr (kThGlobal) {
        if (valid) {
          Real *Tk = Tblk(k) + lane * NX;
#pragma unroll
          for (int c = 0; c < NX; ++c) Tk[c] = thr[c];
        }
      } else {
#pragma unroll
        for (int c = 0; c < NX; ++c) th[p][c] = thr[c];
      }
    }
    __syncthreads();
    if (clk) clk[2] = wall_clock64();

    // ================= 3. Off-diagonal blocks of the stair preconditioner.
    // Explicit form (the all-FP32 variant with one knot per lane group): the
    // lanes of knot k (k >= 1) form row `lane` of
    //   P_{k,k-1} = -D_k^-1 phi_{k-1} D_{k-1}^-1,  phi_{k-1} = -A_{k-1} Q_{k-1}^-1,
    // keep it, and publish it so that knot k-1 can read its column. Either
    // form is a fixed linear operator, as the pipelined recurrences require.
    // With kFactP (the FP64 variants, and several knots per lane group where
    // registers are short) the off-diagonal blocks are not formed:
    // P w = D^-1 (w - O D^-1 w), with O the off-diagonal blocks of S~ that the
    // S~ product already holds.
    constexpr bool kFactP = KPT > 1 || TS || sizeof(Real) == 8;
    constexpr int KP = kFactP ? 1 : KPT;
    // D^-1 rows: held in Real for one and two knots per lane group (FP64) and
    // for the task-space variant, in FP32 (converted at use) otherwise.
    // Rounding D^-1 to FP32 perturbs the preconditioner's smallest directions
    // (P ~ S~^-1), which slows PCG and moves where a truncated PCG stops: on
    // the headline batch the slowest solve needs 9% more iterations, at
    // N = 64 up to 13% more, and the iterate at the stop then departs from the
    // FP64 method's by up to 1e-3 after three SQP iterations (1e-5 with FP64
    // rows); on the far worse conditioned task-space systems 30-80% more. With
    // two knots per group the FP64 rows cost spills (288 against 208 B/lane,
    // 22% per PCG iteration); with four they would cost far more, and long
    // solves split across workgroups instead.
    constexpr bool kRealP = TS || (KPT <= 2 && sizeof(Real) == 8);
    using PT = std::conditional_t<kRealP, Real, float>;
    PT Pm[KP][NX], Pp[KP][NX], Pdf[KPT][NX];
#pragma unroll
    for (int p = 0; p < KPT; ++p) {
#pragma unroll
      for (int m = 0; m < NX; ++m) Pdf[p][m] = kRealP ? (PT)Pd[p][m] : (PT)(float)Pd[p][m];
    }
    if constexpr (!kFactP) {
#pragma unroll
    for (int p = 0; p < KPT; ++p) {
      const int k = slot + p * SLOTS;
      const bool valid = k < N && lane < NX;
#pragma unroll
      for (int m = 0; m < NX; ++m) {
        Pm[p][m] = 0.f;
        Pp[p][m] = 0.f;
      }
      if (valid && k >= 1) {
        const float *A = Ablk(k - 1);
        const float *Dm = Dblk(k - 1);
        float t[NX];
#pragma unroll
        for (int c = 0; c < NX; ++c) {
          float s = 0.f;
#pragma unroll
          for (int m = 0; m < NX; ++m) s += (float)Pd[p][m] * A[m * NX + c];
          t[c] = s * (float)sm.Qi[c];   // = -(D_k^-1 phi_{k-1})[lane][c]
        }
        float *Po = Pblk(k - 1) + lane * NX;
#pragma unroll
        for (int c2 = 0; c2 < NX; ++c2) {
          float s = 0.f;
#pragma unroll
          for (int c = 0; c < NX; ++c) s += t[c] * Dm[c * NX + c2];
          Pm[p][c2] = s;
          Po[c2] = s;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < KPT; ++p) {
      const int k = slot + p * SLOTS;
      if (k < N - 1 && lane < NX) {
        const float *Po = Pblk(k);
#pragma unroll
        for (int m = 0; m < NX; ++m) Pp[p][m] = Po[m * NX + lane];   // P_{k,k+1} = P_{k+1,k}^T
      }
    }
    }  // !kFactP

    if (clk) clk[3] = wall_clock64();
    // ================= 4. PCG on S~ lambda = gamma~, pipelined arrangement.
    // Per iteration, with u = P r, w = S~ u kept by recurrence:
    //   gamma = (r, u), delta = (w, u)         [partials published with w]
    //   m = P w, n = S~ m
    //   beta = gamma / gamma_prev, alpha = gamma / (delta - beta gamma / alpha_prev)
    //   z = n + beta z, q = m + beta q, s = w + beta s, p = u + beta p
    //   lambda += alpha p, r -= alpha s, u -= alpha q, w -= alpha z
    // In exact arithmetic this is the standard PCG iteration; the reduction of
    // an iteration shares a workgroup barrier with the vector exchange, so an
    // iteration needs two barriers and the scalar divisions overlap the
    // matrix-vector products.
    // Split solve: this part's rows only, until the multipliers are gathered.
    bool xon = split;
    auto own = [&](int p) { return !xon || (p >> psh) == part; };
    unsigned long long *xb = split ? a.xch + D.xch_off : nullptr;
    const int xspin = a.xspin > 0 ? a.xspin : kXSpin;
    auto xtag = [&](unsigned e) { return ((a.epoch & 0xffffu) << 16) | (e & 0xffffu); };
    auto xslot = [&](int q, unsigned e) { return xb + (size_t)q * kXPart + (size_t)(e % kXSlots) * kXSlot; };
    const int kf = (part << psh) * SLOTS;                        // own knots kf..kl (none when kf >= N)
    const int kl = min(kf + (SLOTS << psh), N) - 1;
    const bool has_l = split && part > 0 && kf < N;              // a part on the left / the right
    const bool has_r = split && kl + 1 < N;
    // Halo rows: the first own knot's row of vl goes to the left part, the last
    // one's of vr to the right part; the neighbours' rows land in vr[kf - 1]
    // and vl[kl + 1], read only by the lane groups that receive them.
    // (Published where the rows are formed, in share_S and prepare_P, for
    // the exchange that follows them: number xe.)
    auto xhalo_put_row = [&](int k, double left, double right) {
      if (lane < NX) {
        if (has_l && k == kf) xput(xslot(part, xe) + 2 * lane, xtag(xe), left);
        if (has_r && k == kl) xput(xslot(part, xe) + 32 + 2 * lane, xtag(xe), right);
      }
    };
    auto xhalo_get = [&](unsigned e, Real (*vl)[G], Real (*vr)[G]) {
      const bool dead = sm.xfail != 0;
      if (lane < NX) {
        double v;
        if (has_l && slot == 0) {
          if (!xget(xslot(part - 1, e) + 32 + 2 * lane, xtag(e), dead, xspin, v)) sm.xfail = 1;
          vr[kf - 1][lane] = (Real)v;
        }
        if (has_r && slot == kl % SLOTS) {
          if (!xget(xslot(part + 1, e) + 2 * lane, xtag(e), dead, xspin, v)) sm.xfail = 1;
          vl[kl + 1][lane] = (Real)v;
        }
      }
      wave_sync();
    };
    // Sums over the parts (fixed order) of three partials that every lane holds.
    auto xsum_put = [&](unsigned e, double s0, double s1, double s2) {
      if (tid < 3) xput(xslot(part, e) + 64 + 2 * tid, xtag(e), tid == 0 ? s0 : (tid == 1 ? s1 : s2));
    };
    // Halo rows and sums of one exchange, all words polled together.
    auto xhalo_sum_get = [&](unsigned e, bool halo, Real (*vl)[G], Real (*vr)[G], double &s0, double &s1,
                             double &s2) {
      const bool dead = sm.xfail != 0;
      const int l = tid & 63;
      const bool hl = halo && has_l && slot == 0 && lane < NX;
      const bool hr = halo && has_r && slot == kl % SLOTS && lane < NX;
      unsigned long long *wh = hl ? xslot(part - 1, e) + 32 + 2 * lane : (hr ? xslot(part + 1, e) + 2 * lane : nullptr);
      unsigned long long *ws = l < 3 * nparts ? xslot(l / 3, e) + 64 + 2 * (l % 3) : nullptr;
      double vh = 0.0, v = 0.0;
      if (wh || ws) {
        bool ok;
        if (wh && ws) ok = xget2(wh, ws, xtag(e), dead, xspin, vh, v);
        else if (wh) ok = xget(wh, xtag(e), dead, xspin, vh);
        else ok = xget(ws, xtag(e), dead, xspin, v);
        if (!ok) sm.xfail = 1;
      }
      if (hl) vr[kf - 1][lane] = (Real)vh;
      if (hr) vl[kl + 1][lane] = (Real)vh;
      wave_sync();
      if (nparts == 2) {
        s0 = lane_val(v, 0) + lane_val(v, 3);
        s1 = lane_val(v, 1) + lane_val(v, 4);
        s2 = lane_val(v, 2) + lane_val(v, 5);
      } else {
        s0 = (lane_val(v, 0) + lane_val(v, 3)) + (lane_val(v, 6) + lane_val(v, 9));
        s1 = (lane_val(v, 1) + lane_val(v, 4)) + (lane_val(v, 7) + lane_val(v, 10));
        s2 = (lane_val(v, 2) + lane_val(v, 5)) + (lane_val(v, 8) + lane_val(v, 11));
      }
    };
    auto xhalo = [&](Real (*vl)[G], Real (*vr)[G]) {
      xhalo_get(xe, vl, vr);
      ++xe;
    };
    // Sums over the parts of three workgroup totals (no halo rows).
    auto xsums = [&](double &s0, double &s1, double &s2) {
      xsum_put(xe, s0, s1, s2);
      xhalo_sum_get(xe, false, sm.pv, sm.sv, s0, s1, s2);
      ++xe;
    };
    // Every part's multipliers to every part (after the PCG).
    auto xlam = [&]() {
      const unsigned e = xe++;
#pragma unroll
      for (int p = 0; p < KPT; ++p)
        if ((p >> psh) == part && slot + p * SLOTS < N && lane < NX)
          xput(xb + (size_t)p * kXPart + kXSlots * kXSlot + 2 * (slot * G + lane), xtag(e), (double)lam[p]);
      const bool dead = sm.xfail != 0;
#pragma unroll
      for (int p = 0; p < KPT; ++p) {
        if ((p >> psh) != part && slot + p * SLOTS < N && lane < NX) {
          double v;
          if (!xget(xb + (size_t)p * kXPart + kXSlots * kXSlot + 2 * (slot * G + lane), xtag(e), dead, xspin, v))
            sm.xfail = 1;
          lam[p] = (Real)v;
        }
      }
    };
    auto share_S = [&](const Real *vals) {   // operand of S~: vals and Q^-1 vals
#pragma unroll
      for (int p = 0; p < KPT; ++p) {
        const int k = slot + p * SLOTS;
        if (k < N && own(p)) {
          const bool valid = lane < NX;
          sm.pv[k][lane] = valid ? vals[p] : (Real)0;
          sm.sv[k][lane] = valid ? qown[p] * vals[p] : (Real)0;
          if (xon) xhalo_put_row(k, (double)vals[p], (double)(qown[p] * vals[p]));
        }
      }
    };
    auto share_P = [&](const Real *vals, Real (*buf)[G]) {
#pragma unroll
      for (int p = 0; p < KPT; ++p) {
        const int k = slot + p * SLOTS;
        if (k < N && own(p)) buf[k][lane] = (lane < NX) ? vals[p] : (Real)0;
      }
    };
    // With one knot per lane group, block-row products accumulate in two
    // interleaved partial sums per block (even and odd columns), so that the FMA
    // chains are short and independent; with more knots the extra accumulators
    // would cost registers (spills), so the odd columns fold into the even sums.
    constexpr bool kSplit = (KPT == 1);
    // The knot's own block-row products (the diagonal block of S~ and the
    // D^-1 products of the preconditioner) by DPP row broadcasts from the
    // registers (16-lane groups, FP64); the neighbours' blocks still read the
    // neighbours' published vectors from LDS.
    constexpr bool kDpp = (G == 16) && (sizeof(Real) == 8);
    // own: this lane's entry of the vector the product multiplies (the value
    // share_S published in pv).
    auto apply_S = [&](int p, Real own) -> Real {
      const int k = slot + p * SLOTS;
      if constexpr (kSplit) {
        Real d0 = 0, d1 = 0, l0 = 0, l1 = 0, u0 = 0, u1 = 0;
        if constexpr (kDpp) {
          row_dot2<NX>(d0, d1, own, th[p]);
        } else {
#pragma unroll
          for (int m = 0; m < NX; m += 2) {
            d0 += th[p][m] * sm.pv[k][m];
            d1 += th[p][m + 1] * sm.pv[k][m + 1];
          }
        }
        if constexpr (kDpp) {
          // The neighbours' entries by row broadcasts too: each lane reads
          // its own entry of the neighbour's vector (one LDS read, not 14).
          if (k > 0) {
            double c[NX];
#pragma unroll
            for (int m = 0; m < NX; ++m) c[m] = (double)Am[p][m];
            row_dot2<NX>(l0, l1, sm.sv[k - 1][lane], c);
          }
          if (k < N - 1) {
            double c[NX];
#pragma unroll
            for (int m = 0; m < NX; ++m) c[m] = (double)Ac[p][m];
            row_dot2<NX>(u0, u1, sm.pv[k + 1][lane], c);
          }
        } else {
          if (k > 0) {
#pragma unroll
            for (int m = 0; m < NX; m += 2) {
              l0 += (Real)Am[p][m] * sm.sv[k - 1][m];
              l1 += (Real)Am[p][m + 1] * sm.sv[k - 1][m + 1];
            }
          }
          if (k < N - 1) {
#pragma unroll
            for (int m = 0; m < NX; m += 2) {
              u0 += (Real)Ac[p][m] * sm.pv[k + 1][m];
              u1 += (Real)Ac[p][m + 1] * sm.pv[k + 1][m + 1];
            }
          }
        }
        return ((d0 + d1) - (l0 + l1)) - qown[p] * (u0 + u1);
      } else {
        Real acc = 0;
        if constexpr (kDpp && !kThGlobal) {
          row_dot1<NX>(acc, own, th[p]);
        } else {
#pragma unroll
          for (int m = 0; m < NX; ++m) {
            if constexpr (kThGlobal) acc += Tblk(k)[lane * NX + m] * sm.pv[k][m];
            else acc += th[p][m] * sm.pv[k][m];
          }
        }
        if constexpr (kDpp && !kRowsGlobal && !kRealA) {
          if (k > 0) row_dot1_sub_f<NX>(acc, sm.sv[k - 1][lane], Am[p]);
          if (k < N - 1) {
            Real t = 0;
            row_dot1_f<NX>(t, sm.pv[k + 1][lane], Ac[p]);
            acc -= qown[p] * t;
          }
        } else {
          if (k > 0) {
#pragma unroll
            for (int m = 0; m < NX; ++m) acc -= (Real)am(p, m) * sm.sv[k - 1][m];
          }
          if (k < N - 1) {
            Real t = 0;
#pragma unroll
            for (int m = 0; m < NX; ++m) t += (Real)ac(p, m) * sm.pv[k + 1][m];
            acc -= qown[p] * t;
          }
        }
        return acc;
      }
    };
    auto apply_P = [&](int p, Real (*buf)[G]) -> Real {
      const int k = slot + p * SLOTS;
      Real acc = 0;
      if constexpr (!kFactP) {
        Real d0 = 0, d1 = 0, l0 = 0, l1 = 0, u0 = 0, u1 = 0;
#pragma unroll
        for (int m = 0; m < NX; m += 2) {
          d0 += (Real)Pdf[p][m] * buf[k][m];
          d1 += (Real)Pdf[p][m + 1] * buf[k][m + 1];
        }
        if (k > 0) {
#pragma unroll
          for (int m = 0; m < NX; m += 2) {
            l0 += (Real)Pm[p][m] * buf[k - 1][m];
            l1 += (Real)Pm[p][m + 1] * buf[k - 1][m + 1];
          }
        }
        if (k < N - 1) {
#pragma unroll
          for (int m = 0; m < NX; m += 2) {
            u0 += (Real)Pp[p][m] * buf[k + 1][m];
            u1 += (Real)Pp[p][m + 1] * buf[k + 1][m + 1];
          }
        }
        acc = (d0 + d1) + ((l0 + l1) + (u0 + u1));
      }
      return acc;
    };
    // Factored preconditioner, two halves around the workgroup barrier that
    // publishes the operand (the explicit form publishes it with share_P):
    //   prepare: z_k = D_k^-1 v_k (own knot, exchanged inside the lane group),
    //            published with Q_k^-1 z_k in rv / gv;
    //   finish:  t_k = v_k - (O z)_k, then (P v)_k = D_k^-1 t_k.
    auto group_dinv = [&](int p, Real x) -> Real {   // row `lane` of D_k^-1 times the group's x
      const int k = slot + p * SLOTS;
      Real acc = 0;
      if constexpr (kDpp) {
        double c[NX];
#pragma unroll
        for (int m = 0; m < NX; ++m) c[m] = (double)Pdf[p][m];
        row_dot1<NX>(acc, x, c);
      } else {
        sm.tv[k][lane] = (lane < NX) ? x : (Real)0;
        wave_sync();
#pragma unroll
        for (int m = 0; m < NX; ++m) acc += (Real)Pdf[p][m] * sm.tv[k][m];
        wave_sync();
      }
      return acc;
    };
    auto prepare_P = [&](const Real *vals) {
#pragma unroll
      for (int p = 0; p < KPT; ++p) {
        const int k = slot + p * SLOTS;
        if (k < N && own(p)) {
          const Real z = group_dinv(p, vals[p]);
          sm.rv[k][lane] = (lane < NX) ? z : (Real)0;
          sm.gv[k][lane] = (lane < NX) ? qown[p] * z : (Real)0;
          if (xon) xhalo_put_row(k, (double)z, (double)(qown[p] * z));
        }
      }
    };
    auto finish_P = [&](int p, Real v) -> Real {
      const int k = slot + p * SLOTS;
      Real oz = 0;   // (O z)_k at row `lane`
      if constexpr (kDpp && KPT == 2 && !kRealA) {
        if (k > 0) row_dot1_sub_f<NX>(oz, sm.gv[k - 1][lane], Am[p]);
        if (k < N - 1) {
          Real t = 0;
          row_dot1_f<NX>(t, sm.rv[k + 1][lane], Ac[p]);
          oz -= qown[p] * t;
        }
      } else if constexpr (kDpp && KPT == 1) {
        if (k > 0) {
          double c[NX];
#pragma unroll
          for (int m = 0; m < NX; ++m) c[m] = (double)am(p, m);
          row_dot1_sub<NX>(oz, sm.gv[k - 1][lane], c);
        }
        if (k < N - 1) {
          Real t = 0;
          double c[NX];
#pragma unroll
          for (int m = 0; m < NX; ++m) c[m] = (double)ac(p, m);
          row_dot1<NX>(t, sm.rv[k + 1][lane], c);
          oz -= qown[p] * t;
        }
      } else {
        if (k > 0) {
#pragma unroll
          for (int m = 0; m < NX; ++m) oz -= (Real)am(p, m) * sm.gv[k - 1][m];
        }
        if (k < N - 1) {
          Real t = 0;
#pragma unroll
          for (int m = 0; m < NX; ++m) t += (Real)ac(p, m) * sm.rv[k + 1][m];
          oz -= qown[p] * t;
        }
      }
      return group_dinv(p, v - oz);
    };
    auto row_valid = [&](int p) { return (slot + p * SLOTS) < N && lane < NX && own(p); };

    // r = gamma~ - S~ lambda, u = P r, w = S~ u; eta_ref = gamma~^T P gamma~.
    Real r[KPT], u[KPT], w[KPT], vm[KPT], vn[KPT], vz[KPT], vq[KPT], vs[KPT], vp[KPT];
    share_S(lam);
    __syncthreads();
    if (xon) xhalo(sm.pv, sm.sv);
#pragma unroll
    for (int p = 0; p < KPT; ++p) r[p] = row_valid(p) ? gam[p] - apply_S(p, lam[p]) : (Real)0;
    Real Pgam[KPT];   // P gamma~, for the reference norm
    if constexpr (kFactP) {
      prepare_P(r);
      __syncthreads();
      if (xon) xhalo(sm.rv, sm.gv);
#pragma unroll
      for (int p = 0; p < KPT; ++p) u[p] = row_valid(p) ? finish_P(p, r[p]) : (Real)0;
      __syncthreads();
      prepare_P(gam);
      __syncthreads();
      if (xon) xhalo(sm.rv, sm.gv);
#pragma unroll
      for (int p = 0; p < KPT; ++p) Pgam[p] = row_valid(p) ? finish_P(p, gam[p]) : (Real)0;
    } else {
      share_P(r, sm.rv);
      share_P(gam, sm.gv);
      __syncthreads();
#pragma unroll
      for (int p = 0; p < KPT; ++p) {
        u[p] = row_valid(p) ? apply_P(p, sm.rv) : (Real)0;
        Pgam[p] = row_valid(p) ? apply_P(p, sm.gv) : (Real)0;
      }
    }
    Real eta_ref = 0;
#pragma unroll
    for (int p = 0; p < KPT; ++p) eta_ref += gam[p] * Pgam[p];
    const int max_it = a.pcg_max_iter > 0 ? a.pcg_max_iter : N * NX;
    Real gma = 0, stop = 0;
    int its = 0;
    if constexpr (sizeof(Real) == 4 || TS) {
      // All-FP32 and task-space variants: the standard (Hestenes-Stiefel)
      // arrangement, whose directly computed p^T S~ p tolerates the rounding
      // of FP32 vectors, and which on the worse-conditioned task-space systems
      // is also the faster one (fewer live registers than the pipelined
      // recurrences next to the variant's own state).
      // Acc: the accumulation type of the inner products (double when FP64
      // accumulation is asked for, and for FP64 vectors).
      auto run = [&](auto tag) {
        using Acc = decltype(tag);
        Acc sums[3] = {0, 0, 0};
#pragma unroll
        for (int p = 0; p < KPT; ++p) {
          sums[0] += (Acc)r[p] * (Acc)u[p];
          sums[2] += (Acc)gam[p] * (Acc)Pgam[p];
          vp[p] = u[p];
        }
        block_sum<3>(sm.red, redbuf, sums);
        if (xon) {
          double t0 = (double)sums[0], t1 = (double)sums[1], t2 = (double)sums[2];
          xsums(t0, t1, t2);
          sums[0] = (Acc)t0;
          sums[2] = (Acc)t2;
        }
        Acc g = sums[0];
        const Acc stop_a = (Acc)a.pcg_tol * (Acc)a.pcg_tol * sums[2];
        while (g > stop_a && its < max_it) {
          share_S(vp);
          __syncthreads();
          if (xon) xhalo(sm.pv, sm.sv);
          Acc pw[1] = {0};
#pragma unroll
          for (int p = 0; p < KPT; ++p) {
            w[p] = row_valid(p) ? apply_S(p, vp[p]) : (Real)0;
            pw[0] += (Acc)vp[p] * (Acc)w[p];
          }
          block_sum<1>(sm.red, redbuf, pw);
          if (xon) {
            double t0 = (double)pw[0], t1 = 0.0, t2 = 0.0;
            xsums(t0, t1, t2);
            pw[0] = (Acc)t0;
          }
          const Real alpha = (Real)div_pcg(g, pw[0]);
#pragma unroll
          for (int p = 0; p < KPT; ++p) {
            lam[p] += alpha * vp[p];
            r[p] -= alpha * w[p];
          }
          if constexpr (kFactP) prepare_P(r);
          else share_P(r, sm.rv);
          __syncthreads();
          if (xon) xhalo(sm.rv, sm.gv);
          Acc rz[1] = {0};
#pragma unroll
          for (int p = 0; p < KPT; ++p) {
            if constexpr (kFactP) u[p] = row_valid(p) ? finish_P(p, r[p]) : (Real)0;
            else u[p] = row_valid(p) ? apply_P(p, sm.rv) : (Real)0;
            rz[0] += (Acc)r[p] * (Acc)u[p];
          }
          block_sum<1>(sm.red, redbuf, rz);
          if (xon) {
            double t0 = (double)rz[0], t1 = 0.0, t2 = 0.0;
            xsums(t0, t1, t2);
            rz[0] = (Acc)t0;
          }
          const Real beta = (Real)div_pcg(rz[0], g);
          g = rz[0];
#pragma unroll
          for (int p = 0; p < KPT; ++p) vp[p] = u[p] + beta * vp[p];
          ++its;
        }
        // Only the convergence test outlives the loop (status bits).
        gma = (g > stop_a) ? (Real)1 : (Real)0;
        stop = 0;
      };
      if constexpr (sizeof(Real) == 8) run(double{});
      else if (a.fp64_dot) run(double{});
      else run(float{});
    } else {
      share_S(u);
      __syncthreads();
      if (xon) xhalo(sm.pv, sm.sv);
#pragma unroll
      for (int p = 0; p < KPT; ++p) {
        w[p] = row_valid(p) ? apply_S(p, u[p]) : (Real)0;
        vz[p] = vq[p] = vs[p] = vp[p] = 0;
      }
      eta_ref = wave_sum(eta_ref);
      const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: kept in a scalar register
      if ((tid & 63) == 0) sm.red[redbuf][2][wave] = eta_ref;
      // rg = 1 / gamma_prev and c = 1 / (gamma_prev alpha_prev), formed in the
      // previous iteration off the critical path, turn
      //   beta = gamma / gamma_prev, alpha = gamma / (delta - beta gamma / alpha_prev)
      // into beta = gamma rg, alpha = gamma / (delta - gamma^2 c): one division.
      Real rg = 0, cga = 0;
      for (;;) {
        // Keep the matrix rows as they are across iterations (stops the
        // compiler from hoisting conversions of FP32 rows and doubling their
        // registers).
#pragma unroll
        for (int p = 0; p < KPT; ++p)
#pragma unroll
          for (int m = 0; m < NX; ++m) {
            if constexpr (!kRowsGlobal) asm volatile("" : "+v"(Am[p][m]), "+v"(Ac[p][m]));
            asm volatile("" : "+v"(Pdf[p][m]));
          }
        if constexpr (!kFactP) {
#pragma unroll
          for (int p = 0; p < KPT; ++p)
#pragma unroll
            for (int m = 0; m < NX; ++m) asm volatile("" : "+v"(Pm[p][m]), "+v"(Pp[p][m]));
        }
        // Publish w for m = P w together with the partial inner products.
        Real pr = 0, pwu = 0;
#pragma unroll
        for (int p = 0; p < KPT; ++p) {
          pr += r[p] * u[p];
          pwu += w[p] * u[p];
        }
        if constexpr (kSplit) {
          wave_sum2(pr, pwu);
        } else {
          pr = wave_sum(pr);
          pwu = wave_sum(pwu);
        }
        if ((tid & 63) == 0) {
          sm.red[redbuf][0][wave] = pr;
          sm.red[redbuf][1][wave] = pwu;
        }
        if constexpr (kFactP) prepare_P(w);
        else share_P(w, sm.rv);
        __syncthreads();
        // Pairwise tree over the per-wavefront partials (fixed order).
        gma = pair_tree<kBlock / 64>(sm.red[redbuf][0]);
        Real dlt = pair_tree<kBlock / 64>(sm.red[redbuf][1]);
        if (xon) {
          // Halo rows for finish_P and this part's inner products out; the
          // neighbours' rows and the sums over the parts in.
          const double e0 = (its == 0) ? pair_tree<kBlock / 64>(sm.red[redbuf][2]) : 0.0;
          xsum_put(xe, gma, dlt, e0);
          double g_, d_, e_;
          xhalo_sum_get(xe, true, sm.rv, sm.gv, g_, d_, e_);
          ++xe;
          gma = (Real)g_;
          dlt = (Real)d_;
          if (its == 0) stop = (Real)a.pcg_tol * (Real)a.pcg_tol * (Real)e_;
        } else if (its == 0) {
          stop = (Real)a.pcg_tol * (Real)a.pcg_tol * pair_tree<kBlock / 64>(sm.red[redbuf][2]);
        }
        redbuf ^= 1;
        if (!(gma > stop) || its >= max_it) break;
#pragma unroll
        for (int p = 0; p < KPT; ++p) {
          if constexpr (kFactP) vm[p] = row_valid(p) ? finish_P(p, w[p]) : (Real)0;
          else vm[p] = row_valid(p) ? apply_P(p, sm.rv) : (Real)0;
        }
        share_S(vm);
        // (kpt > 1: the quotients in the textbook order, whose operands are
        // short-lived; rg and cga then hold gamma_prev and alpha_prev.)
        const Real beta = kSplit ? gma * rg : ((its == 0) ? (Real)0 : div_pcg(gma, rg));
        const Real alpha = kSplit ? div_pcg(gma, dlt - gma * gma * cga)
                                  : ((its == 0) ? div_pcg(gma, dlt) : div_pcg(gma, dlt - div_pcg(beta * gma, cga)));
        __syncthreads();
        if (xon) xhalo(sm.pv, sm.sv);
#pragma unroll
        for (int p = 0; p < KPT; ++p) {
          vn[p] = row_valid(p) ? apply_S(p, vm[p]) : (Real)0;
          vz[p] = vn[p] + beta * vz[p];
          vq[p] = vm[p] + beta * vq[p];
          vs[p] = w[p] + beta * vs[p];
          vp[p] = u[p] + beta * vp[p];
          lam[p] += alpha * vp[p];
          r[p] -= alpha * vs[p];
          u[p] -= alpha * vq[p];
          w[p] -= alpha * vz[p];
        }
        if constexpr (kSplit) {
          cga = div_pcg((Real)1, gma * alpha);
          rg = alpha * cga;
        } else {
          rg = gma;
          cga = alpha;
        }
        ++its;
      }
    }
    bool xfail_any = false;   // some part of this solve gave up a wait
    if (xon) {
      xlam();
      xon = false;
      // Every part's failure flag to every part: a part that gave up still
      // publishes (without waiting), so a writer that did not give up learns
      // that the rows it received were not the other parts' results.
      __syncthreads();
      double f0 = sm.xfail ? 1.0 : 0.0, f1 = 0.0, f2 = 0.0;
      xsums(f0, f1, f2);
      xfail_any = f0 != 0.0;
    }
    unsigned status = (gma > stop) ? GATO_ST_PCG_MAXITER : 0u;
    if (clk) clk[4] = wall_clock64();

    // ================= 5. Step recovery dZ = -G^-1 (g - C^T lambda).
    share_S(lam);
    __syncthreads();
#pragma unroll
    for (int p = 0; p < KPT; ++p) {
      const int k = slot + p * SLOTS;
      if (k < N && lane < NX) {
        Real sx = (Real)sm.qg[k][lane] - lam[p];
        if (k < N - 1) {
#pragma unroll
          for (int m = 0; m < NX; ++m) sx += (Real)ac(p, m) * sm.pv[k + 1][m];
        }
        const float dx = (float)(-qown[p] * sx);
        sm.dX[k][lane] = dx;
        if (!isfinite(dx)) bad_flag = 1;
        if constexpr (TS) {
          if (lane < ND) ts.tq[k][lane] = (double)(-qown[p] * sx);
        }
        if (lane < NU && k < N - 1) {
          const float *B = Bblk(k);
          Real su = (Real)sm.rg[k][lane];
#pragma unroll
          for (int m = 0; m < NX; ++m) su += (Real)B[m * NU + lane] * sm.pv[k + 1][m];
          const float du = (float)(-(Real)D.Ri[lane] * su);
          sm.dU[k][lane] = du;
          if (!isfinite(du)) bad_flag = 1;
        }
      }
    }
    if constexpr (TS) {
      // Back to x: dx_k = T_k dy_k (joint rows L_k^-T dy), lambda = T_k^-T lambda^.
#pragma unroll
      for (int p = 0; p < KPT; ++p) {
        const int k = slot + p * SLOTS;
        if (k < N) {
          const double *Lk = ts.Lc[k];
          const double *Lik = ts.Li[k];
          wave_sync();
          double t = 0.0;
          if (lane < ND) {
#pragma unroll
            for (int m = 0; m < ND; ++m)
              if (m >= lane) t += Lik[tri(m, lane)] * ts.tq[k][m];
          }
          wave_sync();
          if (lane < ND) {
            const float dx = (float)t;
            sm.dX[k][lane] = dx;
            if (!isfinite(dx)) bad_flag = 1;
            ts.tq[k][lane] = (double)lam[p];
          }
          wave_sync();
          if (lane < ND) {
            double l = 0.0;
#pragma unroll
            for (int m = 0; m < ND; ++m)
              if (m <= lane) l += Lk[tri(lane, m)] * ts.tq[k][m];
            lam[p] = (Real)l;
          }
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
    if (clk) clk[5] = wall_clock64();

    // ================= 6. Line search over alpha_i = beta^-i (Eqs. (3), (7)).
    const int ntask = n_alpha * (N - 1);
    for (int t = tid; t < ntask; t += kBlock) {
      const int i = t / (N - 1), k = t - i * (N - 1);
      const float al = sm.alpha[i];
      float q[ND], qd[ND], uu[ND], qdd[ND], L[ND][ND], xn[NX];
#pragma unroll
      for (int j = 0; j < ND; ++j) {
        q[j] = sm.X[k][j] + al * sm.dX[k][j];
        qd[j] = sm.X[k][ND + j] + al * sm.dX[k][ND + j];
        uu[j] = sm.U[k][j] + al * sm.dU[k][j];
      }
#pragma unroll
      for (int j = 0; j < NX; ++j) xn[j] = sm.X[k + 1][j] + al * sm.dX[k + 1][j];
      forward_dynamics<ND>(ch, q, qd, uu, qdd, L);
      float viol = 0.f, cost = 0.f;
#pragma unroll
      for (int j = 0; j < ND; ++j) {
        viol += fabsf((q[j] + h * qd[j]) - xn[j]) + fabsf((qd[j] + h * qdd[j]) - xn[ND + j]);
        const float d0 = q[j] - sm.xg[j], d1 = qd[j] - sm.xg[ND + j];
        cost += 0.5f * D.Wq[j] * d0 * d0 + 0.5f * D.Wq[ND + j] * d1 * d1 + 0.5f * D.Wr[j] * uu[j] * uu[j];
      }
      if constexpr (TS) {
        float pt[3];
        tip_position<ND>(ch, q, pt);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float d = pt[c] - ts.pr[k][c];
          cost += 0.5f * D.We[c] * d * d;
        }
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
      if constexpr (TS) {
        float q[ND], pt[3];
#pragma unroll
        for (int j = 0; j < ND; ++j) q[j] = sm.X[N - 1][j] + al * sm.dX[N - 1][j];
        tip_position<ND>(ch, q, pt);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float d = pt[c] - ts.pr[N - 1][c];
          cost += 0.5f * D.WeN[c] * d * d;
        }
      }
      sm.mp[i][N - 1] = (double)cost + (double)a.mu * (double)viol;
    }
    __syncthreads();
    if (tid <= n_alpha) {
      double sum = 0.0;
      for (int k = 0; k < N; ++k) sum += (tid == n_alpha) ? sm.mp0[k] : sm.mp[tid][k];
      sm.merit[tid] = sum;
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
    const double rho_used = rho;
    if (a.rho_adapt) rho = (status & (GATO_ST_NONFINITE | GATO_ST_NO_DESCENT)) ? fmin(2.0 * rho, 1e8) : rho / 3.0;
    const float al = bad ? 0.f : sm.alpha[best];
    if (!bad) {
      for (int t = tid; t < N * G; t += kBlock) {
        const int k = t / G, j = t % G;
        sm.X[k][j] += al * sm.dX[k][j];
        if (k < N - 1 && j < 8) sm.U[k][j] += al * sm.dU[k][j];
      }
    }
    if (split && (sm.xfail || xfail_any)) status |= GATO_ST_EXCHANGE;
    if (tid == 0 && a.stats && writer) {
      gato_solve_stats st;
      st.merit0 = (float)sm.merit[n_alpha];
      st.merit = bad ? (float)sm.merit[n_alpha] : (float)sm.merit[best];
      st.alpha = al;
      st.pcg_iters = its;
      st.status = status;
      st.rho = (float)rho_used;
      a.stats[(size_t)rid * a.stats_stride + it] = st;
    }
    __syncthreads();
    if (clk) {
      clk[6] = wall_clock64();
      clk[7] = clock64() - cyc0;
    }
  }

  // ---- Write back the iterate, the warm-start multipliers and the adapted damping.
  const int lane = lane0, slot = slot0;
  if (a.mode == kModeSqp && writer) {
    if (a.rho_adapt && tid == 0) a.rho[sid] = rho;
    const size_t rxo = (size_t)blockIdx.x * a.N_max * a.nx_max;
    const size_t ruo = (size_t)blockIdx.x * (a.N_max - 1) * a.nu_max;
    for (int t = tid; t < N * G; t += kBlock) {
      const int k = t / G, j = t % G;
      if (j < NX) {
        a.X[xoff + (size_t)k * a.nx_max + j] = sm.X[k][j];
        if (a.Xout) a.Xout[rxo + (size_t)k * a.nx_max + j] = sm.X[k][j];
      }
      if (k < N - 1 && j < NU) {
        a.U[uoff + (size_t)k * a.nu_max + j] = sm.U[k][j];
        if (a.Uout) a.Uout[ruo + (size_t)k * a.nu_max + j] = sm.U[k][j];
      }
    }
#pragma unroll
    for (int p = 0; p < KPT; ++p) {
      const int k = slot + p * SLOTS;
      if (k < N && lane < NX) gL[k * a.nx_max + lane] = (double)lam[p];
    }
  }
}

template <int ND, int KPT, class Real, bool TS = false, bool SPLIT = false>
__global__ __launch_bounds__(kBlock) void sqp_kernel(KArgs a) {
  static_assert(smem_bytes<ND, KPT, Real, TS>() <= 160 * 1024, "LDS of one workgroup exceeds 160 KB");
  __shared__ __align__(16) char smem[smem_bytes<ND, KPT, Real, TS>()];
  int sid = a.order ? a.order[blockIdx.x] : a.sid_base + (int)blockIdx.x;
  int part = 0;
  if constexpr (SPLIT) {
    if (a.split) {
      part = (int)((unsigned)sid >> 24);
      sid &= 0xffffff;
    }
  }
  if (sid < 0 || sid >= a.M) return;   // a caller-provided slot out of range: nothing to do
  sqp_solve<ND, KPT, Real, TS, SPLIT>(a, sid, part, smem);
}

// Mixed-shape kernel: every workgroup reads its solve's (n, kpt) and runs the
// matching specialisation, so a batch of uneven DoF and horizon is one launch.
// The LDS footprint is the largest specialisation's; every specialisation
// already runs one workgroup per CU, so occupancy is unchanged. (For 3 DoF,
// two knots per 8-lane group already cover the maximum horizon; the
// task-space variant is compiled for one and two knots per group, and its
// long solves (6-7 DoF, N > 64) run only split, in the part-local form.)
template <class Real, bool TS>
constexpr size_t mixed_smem_bytes() {
  size_t m = 0;
  const size_t s[] = {smem_bytes<3, 1, Real, TS>(), smem_bytes<3, 2, Real, TS>(),
                      smem_bytes<6, 1, Real, TS>(), smem_bytes<6, 2, Real, TS>(),
                      TS ? part_smem_bytes<6, true>() : smem_bytes<6, 4, Real, false>(),
                      smem_bytes<7, 1, Real, TS>(), smem_bytes<7, 2, Real, TS>(),
                      TS ? part_smem_bytes<7, true>() : smem_bytes<7, 4, Real, false>()};
  for (size_t v : s) m = v > m ? v : m;
  return m;
}

// A long task-space solve runs only as the four parts of a split SQP launch
// in FP64 (the host builds no other launch of one).
__device__ __forceinline__ bool task_split_ok(const KArgs &a, const SolveDesc &D, int part) {
  return a.split == kXParts && a.mode == kModeSqp && !a.by_block && D.xch_off >= 0 && part >= 0 && part < kXParts;
}

template <class Real, bool TS = false, bool SPLIT = false>
__global__ __launch_bounds__(kBlock) void sqp_mixed_kernel(KArgs a) {
  static_assert(mixed_smem_bytes<Real, TS>() <= 160 * 1024, "LDS of one workgroup exceeds 160 KB");
  __shared__ __align__(16) char smem[mixed_smem_bytes<Real, TS>()];
  int sid = a.order ? a.order[blockIdx.x] : a.sid_base + (int)blockIdx.x;
  int part = 0;
  if constexpr (SPLIT) {
    if (a.split) {
      part = (int)((unsigned)sid >> 24);
      sid &= 0xffffff;
    }
  }
  if (sid < 0 || sid >= a.M) return;   // a caller-provided slot out of range: nothing to do
  const SolveDesc &D = a.desc[sid];
  switch (D.n * 8 + D.kpt) {
    case 3 * 8 + 1: sqp_solve<3, 1, Real, TS>(a, sid, part, smem); break;
    case 3 * 8 + 2: sqp_solve<3, 2, Real, TS>(a, sid, part, smem); break;
    case 6 * 8 + 1: sqp_solve<6, 1, Real, TS>(a, sid, part, smem); break;
    case 6 * 8 + 2: sqp_solve<6, 2, Real, TS>(a, sid, part, smem); break;
    case 7 * 8 + 1: sqp_solve<7, 1, Real, TS>(a, sid, part, smem); break;
    case 7 * 8 + 2: sqp_solve<7, 2, Real, TS>(a, sid, part, smem); break;
    case 6 * 8 + 4:
      if constexpr (!TS) sqp_solve<6, 4, Real, false, SPLIT>(a, sid, part, smem);
      else if constexpr (SPLIT && sizeof(Real) == 8) {
        if (task_split_ok(a, D, part)) sqp_solve_part<6, true>(a, sid, part, smem);
      }
      break;
    case 7 * 8 + 4:
      if constexpr (!TS) sqp_solve<7, 4, Real, false, SPLIT>(a, sid, part, smem);
      else if constexpr (SPLIT && sizeof(Real) == 8) {
        if (task_split_ok(a, D, part)) sqp_solve_part<7, true>(a, sid, part, smem);
      }
      break;
    default: break;  // the host only builds the shapes above
  }
}

}  // namespace gato
