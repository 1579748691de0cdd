// FP64 CPU oracle for one SQP iteration loop of batched trajectory optimisation
// as described in "GATO: GPU-Accelerated and Batched Trajectory Optimization for
// Scalable Edge Model Predictive Control" (Du, Adabag, Bravo-Palacios, Plancher,
// arXiv 2510.07625).
//
// TEST INFRASTRUCTURE ONLY. This is the plain, slow, obviously-correct statement
// of what the GPU library computes. Only the tests, the smoke check and the CPU
// baseline leg of the benchmark load it. It shares no code, header, table or
// helper with the GPU library, and the GPU library never links or calls it.
//
// Where the paper fixes a result by a plain definition, that definition is
// written out here:
//   * the QP of one SQP step is Eq. (1); its solution is the KKT system Eq. (2),
//     solved by a dense LU with partial pivoting of the whole KKT matrix;
//   * the line search is Eq. (7) over the L1 merit of Eq. (3).
// Two further modes restate the paper's own solution path so that the GPU's
// intermediate results can be checked stage by stage:
//   * Schur complement + symmetric stair preconditioner + PCG, Eqs. (4)-(6)
//     (Sec. II-B), with the sign reading of c described below;
//   * the textbook finite-horizon Riccati recursion for the same QP (used as an
//     exact fast solver for long horizons and as an independent pin).
//
// Readings of the paper (each also listed in the design notes):
//   R1  N counts knot points: states x_0..x_{N-1}, controls u_0..u_{N-2}.
//   R2  Eq. (4)-(6) are consistent with each other only for the constraint
//       right-hand side -c; solving Eq. (1) as stated gives
//       S~ = C G^-1 C^T, gamma~ = c + C G^-1 g, dZ = -G^-1 (g - C^T lambda).
//   R3  PCG runs on S~ = -S with P = -Phi^-1 (both SPD).
//   R4  The (3,3) entry theta_2 of S in Eq. (6) is read as theta_1.
//   R5  P = D^-1 - D^-1 O D^-1 with D, O the block diagonal / off-diagonal of S~,
//       which is Eq. (6)'s Phi^-1 up to the sign of R3.
//   R6  PCG stops when r^T P r <= eps^2 * gamma~^T P gamma~, or after N*nx steps.
//   R7  The line search always steps to the best of alpha_i = beta^-i,
//       i = 0..A-1; ties go to the larger step.
//   R8  Trial merits use the nonlinear defects at the trial point, one knot at a
//       time (multiple shooting), as the per-knot merit blocks of Algorithm 1.
//   R9  Task-space tracking (the experiments of Sec. IV track the end effector):
//       knot k adds 1/2 (p(q_k) - pref_k)^T W (p(q_k) - pref_k) with p the tip
//       position. The QP takes its exact gradient J^T W (p - pref) and its
//       Gauss-Newton Hessian J^T W J, so each Q_k is a dense SPD block and
//       Eq. (5) is used with the dense Q_k^-1 exactly as written.
//
// Robot model (the paper's robots are not available): a serial chain of n
// revolute joints whose axes alternate z, y, z, y, ... starting with joint 0.
// Link i has its frame at joint i; the next joint sits at length_i along the
// link's +z; the centre of mass is at length_i/2 on +z with diagonal inertia
// (Ixx, Iyy, Izz) about it. Gravity acts along -z of the base. The dynamics are
// written as the classical Newton-Euler recursion in base coordinates.
// A second model, a chain of unit masses coupled by springs
// (q'' = u - k T q, T = tridiag(-1, 2, -1)), gives a linear system for the
// Riccati pin.

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <vector>

extern "C" {

typedef struct {
  int model;           /* 0 revolute chain, 1 spring-coupled double integrators */
  int n;               /* degrees of freedom */
  const double *link;  /* [n][5] length, mass, Ixx, Iyy, Izz */
  double gravity;      /* along -z of the base */
  double spring_k;     /* model 1 only */
  double fext[3];      /* external force on the tip of the last link (base frame), model 0 */
} orc_robot;

typedef struct {
  int N;               /* knot points */
  double dt;           /* time step h */
  const double *Qd;    /* [2n] diagonal of Q (stages 0..N-2) */
  const double *Rd;    /* [n]  diagonal of R */
  const double *QNd;   /* [2n] diagonal of Q_N (last knot) */
  /* Task-space (end-effector) tracking, model 0; NULL Wee: none. Each knot
   * adds 1/2 (p(q_k) - pref_k)^T diag(W) (p(q_k) - pref_k), p the tip position
   * in the base frame, W = Wee for k < N-1 and WeeN for the last knot. */
  const double *Wee;   /* [3] */
  const double *WeeN;  /* [3] */
  const double *pref;  /* [N][3] reference tip positions */
} orc_problem;

typedef struct {
  int sqp_iters;
  int kkt_mode;        /* 0 dense LU, 1 Schur + PCG, 2 Riccati */
  double pcg_tol;
  int pcg_max_iter;    /* <= 0: N * nx */
  int warm_lambda;     /* PCG starts from the previous SQP iteration's lambda */
  double mu;           /* merit weight on ||c||_1 */
  double beta;         /* step ratio, alpha_i = beta^-i */
  int n_alpha;         /* number of candidate steps */
  double rho;          /* damping added to the diagonal of every Q_k (initial value) */
  int rho_adapt;       /* 1: rho /= 3 after an iteration with descent, rho *= 2 without (capped at 1e8) */
} orc_params;

#define ORC_MAX_ALPHA 32

typedef struct {
  double merit0;       /* merit at the current iterate */
  double merit;        /* merit at the accepted step */
  double alpha;        /* accepted step */
  double J;            /* cost at the accepted point */
  double c1;           /* ||c||_1 at the accepted point */
  double kkt_res;      /* inf-norm residual of the linear KKT system */
  int pcg_iters;
  int status;          /* 1 PCG max-iter, 2 non-finite, 4 no descent */
  int argmin;
  int pad;
  double rho;          /* damping used in this iteration */
  double merits[ORC_MAX_ALPHA];
  double pcg_stop;     /* r^T P r / (tol^2 gamma^T P gamma) after the last PCG iteration (<= 1: rule met) */
  double pcg_stop_prev;/* the same one iteration earlier (> 1 when the rule first holds at the last one) */
} orc_iter_log;

}  // extern "C"

enum { ST_PCG_MAXITER = 1, ST_NONFINITE = 2, ST_NO_DESCENT = 4 };

namespace {

// ---------------------------------------------------------------------------
// Forward-mode dual numbers (one tangent direction) for exact derivatives.
// ---------------------------------------------------------------------------
struct Dual {
  double v, d;
  Dual(double v_ = 0.0, double d_ = 0.0) : v(v_), d(d_) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual sin(Dual a) { return Dual(std::sin(a.v), a.d * std::cos(a.v)); }
inline Dual cos(Dual a) { return Dual(std::cos(a.v), -a.d * std::sin(a.v)); }
using std::cos;
using std::sin;

template <class T> struct V3 { T x, y, z; };
template <class T> V3<T> v3(T x, T y, T z) { return V3<T>{x, y, z}; }
template <class T> V3<T> operator+(V3<T> a, V3<T> b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T> V3<T> operator-(V3<T> a, V3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T> V3<T> operator*(T s, V3<T> a) { return {s * a.x, s * a.y, s * a.z}; }
template <class T> T dot(V3<T> a, V3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T> V3<T> cross(V3<T> a, V3<T> b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

template <class T> struct M3 { T m[3][3]; };
template <class T> M3<T> eye3() {
  M3<T> r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r.m[i][j] = T(i == j ? 1.0 : 0.0);
  return r;
}
template <class T> V3<T> operator*(const M3<T> &a, V3<T> v) {
  return {a.m[0][0] * v.x + a.m[0][1] * v.y + a.m[0][2] * v.z,
          a.m[1][0] * v.x + a.m[1][1] * v.y + a.m[1][2] * v.z,
          a.m[2][0] * v.x + a.m[2][1] * v.y + a.m[2][2] * v.z};
}
template <class T> M3<T> operator*(const M3<T> &a, const M3<T> &b) {
  M3<T> r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      T s = T(0.0);
      for (int k = 0; k < 3; ++k) s = s + a.m[i][k] * b.m[k][j];
      r.m[i][j] = s;
    }
  return r;
}
template <class T> M3<T> transpose(const M3<T> &a) {
  M3<T> r;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) r.m[i][j] = a.m[j][i];
  return r;
}
// Rotation by angle q about the joint axis: z for even joints, y for odd.
template <class T> M3<T> joint_rotation(int joint, T q) {
  T c = cos(q), s = sin(q);
  M3<T> r = eye3<T>();
  if (joint % 2 == 0) {
    r.m[0][0] = c; r.m[0][1] = -s;
    r.m[1][0] = s; r.m[1][1] = c;
  } else {
    r.m[0][0] = c; r.m[0][2] = s;
    r.m[2][0] = -s; r.m[2][2] = c;
  }
  return r;
}
template <class T> V3<T> joint_axis_local(int joint) {
  return joint % 2 == 0 ? v3<T>(T(0.0), T(0.0), T(1.0)) : v3<T>(T(0.0), T(1.0), T(0.0));
}

// Inverse dynamics tau = M(q) qdd + C(q, qd) qd + g(q), by the Newton-Euler
// recursion written in base coordinates (forward pass for link velocities and
// accelerations, backward pass for joint forces and moments).
template <class T>
void inverse_dynamics(const orc_robot &rb, const T *q, const T *qd, const T *qdd, bool with_gravity,
                      T *tau) {
  const int n = rb.n;
  if (rb.model == 1) {
    // Spring-coupled unit masses: tau = qdd + k T q.
    for (int i = 0; i < n; ++i) {
      T s = T(2.0) * q[i];
      if (i > 0) s = s - q[i - 1];
      if (i < n - 1) s = s - q[i + 1];
      tau[i] = qdd[i] + T(rb.spring_k) * s;
    }
    return;
  }
  std::vector<M3<T>> R(n);
  std::vector<V3<T>> p(n + 1), z(n), c(n), w(n), wd(n), a(n), F(n), Nm(n);
  const T zero(0.0);
  // Kinematics in base coordinates.
  for (int i = 0; i < n; ++i) {
    const double len_parent = i > 0 ? rb.link[5 * (i - 1) + 0] : 0.0;
    if (i == 0) {
      p[0] = v3<T>(zero, zero, zero);
      R[0] = joint_rotation<T>(0, q[0]);
    } else {
      p[i] = p[i - 1] + R[i - 1] * v3<T>(zero, zero, T(len_parent));
      R[i] = R[i - 1] * joint_rotation<T>(i, q[i]);
    }
    z[i] = R[i] * joint_axis_local<T>(i);
    c[i] = p[i] + R[i] * v3<T>(zero, zero, T(0.5 * rb.link[5 * i + 0]));
  }
  p[n] = p[n - 1] + R[n - 1] * v3<T>(zero, zero, T(rb.link[5 * (n - 1) + 0]));

  // Forward pass. Gravity enters as an upward acceleration of the fixed base.
  const V3<T> a_base = v3<T>(zero, zero, T(with_gravity ? rb.gravity : 0.0));
  for (int i = 0; i < n; ++i) {
    const V3<T> w_prev = i > 0 ? w[i - 1] : v3<T>(zero, zero, zero);
    const V3<T> wd_prev = i > 0 ? wd[i - 1] : v3<T>(zero, zero, zero);
    w[i] = w_prev + qd[i] * z[i];
    wd[i] = wd_prev + qdd[i] * z[i] + cross(w_prev, qd[i] * z[i]);
    if (i == 0) {
      a[0] = a_base;
    } else {
      const V3<T> d = p[i] - p[i - 1];
      a[i] = a[i - 1] + cross(wd[i - 1], d) + cross(w[i - 1], cross(w[i - 1], d));
    }
    const V3<T> rc = c[i] - p[i];
    const V3<T> ac = a[i] + cross(wd[i], rc) + cross(w[i], cross(w[i], rc));
    const double m = rb.link[5 * i + 1];
    F[i] = T(m) * ac;
    M3<T> Ib;
    for (int r = 0; r < 3; ++r)
      for (int s = 0; s < 3; ++s) Ib.m[r][s] = T(r == s ? rb.link[5 * i + 2 + r] : 0.0);
    const M3<T> Iw = R[i] * Ib * transpose(R[i]);
    Nm[i] = Iw * wd[i] + cross(w[i], Iw * w[i]);
  }
  // Backward pass: force and moment (about the joint) that link i-1 exerts on link i.
  // An external force f on the tip p[n] of the last link enters as the force
  // -f that a (virtual) next link exerts at p[n]; the joints then supply
  // tau = M qdd + b - J(q)^T f.
  V3<T> f_next = v3<T>(T(-rb.fext[0]), T(-rb.fext[1]), T(-rb.fext[2])), n_next = v3<T>(zero, zero, zero);
  for (int i = n - 1; i >= 0; --i) {
    const V3<T> f = F[i] + f_next;
    const V3<T> mom = Nm[i] + n_next + cross(c[i] - p[i], F[i]) + cross(p[i + 1] - p[i], f_next);
    tau[i] = dot(z[i], mom);
    f_next = f;
    n_next = mom;
  }
}

// Position of the tip (the end of the last link) in base coordinates: the
// frames are chained from the base exactly as in the kinematics above.
template <class T>
V3<T> tip_position(const orc_robot &rb, const T *q) {
  const int n = rb.n;
  const T zero(0.0);
  V3<T> p = v3<T>(zero, zero, zero);
  M3<T> Rm = eye3<T>();
  for (int i = 0; i < n; ++i) {
    if (i > 0) p = p + Rm * v3<T>(zero, zero, T(rb.link[5 * (i - 1) + 0]));
    Rm = Rm * joint_rotation<T>(i, q[i]);
  }
  return p + Rm * v3<T>(zero, zero, T(rb.link[5 * (n - 1) + 0]));
}

// Tip position p[3] and its Jacobian J[3][n] = dp/dq (one dual-number pass per
// joint).
void tip_jacobian(const orc_robot &rb, const double *q, double *p, double *J) {
  const int n = rb.n;
  const V3<double> pv = tip_position<double>(rb, q);
  p[0] = pv.x; p[1] = pv.y; p[2] = pv.z;
  std::vector<Dual> qd(n);
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i < n; ++i) qd[i] = Dual(q[i], i == j ? 1.0 : 0.0);
    const V3<Dual> t = tip_position<Dual>(rb, qd.data());
    J[0 * n + j] = t.x.d;
    J[1 * n + j] = t.y.d;
    J[2 * n + j] = t.z.d;
  }
}

bool has_task(const orc_problem &pr) { return pr.Wee != nullptr && pr.WeeN != nullptr && pr.pref != nullptr; }

// ---------------------------------------------------------------------------
// Small dense linear algebra (row-major, FP64).
// ---------------------------------------------------------------------------

// Cholesky factorisation A = L L^T in place (lower triangle); false if not SPD.
bool cholesky(double *A, int n) {
  for (int j = 0; j < n; ++j) {
    double s = A[j * n + j];
    for (int k = 0; k < j; ++k) s -= A[j * n + k] * A[j * n + k];
    if (!(s > 0.0)) return false;
    const double d = std::sqrt(s);
    A[j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double t = A[i * n + j];
      for (int k = 0; k < j; ++k) t -= A[i * n + k] * A[j * n + k];
      A[i * n + j] = t / d;
    }
  }
  return true;
}

void cholesky_solve(const double *L, int n, double *b) {
  for (int i = 0; i < n; ++i) {
    double s = b[i];
    for (int k = 0; k < i; ++k) s -= L[i * n + k] * b[k];
    b[i] = s / L[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = b[i];
    for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * b[k];
    b[i] = s / L[i * n + i];
  }
}

// LU with partial pivoting, solving A X = B for nrhs right-hand sides stored
// row-major [n][nrhs]. A and B are overwritten. Returns false if singular.
bool lu_solve(double *A, int n, double *B, int nrhs) {
  for (int k = 0; k < n; ++k) {
    int piv = k;
    double best = std::fabs(A[(size_t)k * n + k]);
    for (int i = k + 1; i < n; ++i) {
      const double v = std::fabs(A[(size_t)i * n + k]);
      if (v > best) { best = v; piv = i; }
    }
    if (!(best > 0.0)) return false;
    if (piv != k) {
      for (int j = 0; j < n; ++j) std::swap(A[(size_t)k * n + j], A[(size_t)piv * n + j]);
      for (int j = 0; j < nrhs; ++j) std::swap(B[(size_t)k * nrhs + j], B[(size_t)piv * nrhs + j]);
    }
    const double inv = 1.0 / A[(size_t)k * n + k];
    const double *rowk = A + (size_t)k * n;
    for (int i = k + 1; i < n; ++i) {
      double *rowi = A + (size_t)i * n;
      const double l = rowi[k] * inv;
      if (l == 0.0) continue;
      rowi[k] = l;
      for (int j = k + 1; j < n; ++j) rowi[j] -= l * rowk[j];
      for (int j = 0; j < nrhs; ++j) B[(size_t)i * nrhs + j] -= l * B[(size_t)k * nrhs + j];
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    const double d = A[(size_t)k * n + k];
    for (int j = 0; j < nrhs; ++j) {
      double s = B[(size_t)k * nrhs + j];
      for (int i = k + 1; i < n; ++i) s -= A[(size_t)k * n + i] * B[(size_t)i * nrhs + j];
      B[(size_t)k * nrhs + j] = s / d;
    }
  }
  return true;
}

// Inverse of a small dense matrix by LU with partial pivoting.
bool invert(const double *A, int n, double *Ainv) {
  std::vector<double> a(A, A + (size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Ainv[i * n + j] = (i == j) ? 1.0 : 0.0;
  return lu_solve(a.data(), n, Ainv, n);
}

// C = A (r x k) * B (k x c)
void matmul(const double *A, const double *B, double *C, int r, int k, int c) {
  for (int i = 0; i < r; ++i)
    for (int j = 0; j < c; ++j) {
      double s = 0.0;
      for (int t = 0; t < k; ++t) s += A[i * k + t] * B[t * c + j];
      C[i * c + j] = s;
    }
}

// ---------------------------------------------------------------------------
// Rigid-body quantities built from inverse dynamics.
// ---------------------------------------------------------------------------

// Joint-space inertia: inverse dynamics is affine in qdd, so column j is the
// extra torque that a unit acceleration of joint j needs at rest.
void mass_matrix(const orc_robot &rb, const double *q, double *M) {
  const int n = rb.n;
  std::vector<double> zero(n, 0.0), e(n, 0.0), col(n), base(n);
  inverse_dynamics<double>(rb, q, zero.data(), zero.data(), false, base.data());
  for (int j = 0; j < n; ++j) {
    std::fill(e.begin(), e.end(), 0.0);
    e[j] = 1.0;
    inverse_dynamics<double>(rb, q, zero.data(), e.data(), false, col.data());
    for (int i = 0; i < n; ++i) M[i * n + j] = col[i] - base[i];
  }
}

// qdd = M(q)^-1 (tau - b(q, qd)), b = Coriolis + gravity. Optionally returns
// the Cholesky factor of M.
bool forward_dynamics(const orc_robot &rb, const double *q, const double *qd, const double *tau,
                      double *qdd, double *Lout) {
  const int n = rb.n;
  std::vector<double> M((size_t)n * n), zero(n, 0.0), b(n);
  mass_matrix(rb, q, M.data());
  inverse_dynamics<double>(rb, q, qd, zero.data(), true, b.data());
  if (!cholesky(M.data(), n)) return false;
  for (int i = 0; i < n; ++i) qdd[i] = tau[i] - b[i];
  cholesky_solve(M.data(), n, qdd);
  if (Lout) std::memcpy(Lout, M.data(), sizeof(double) * n * n);
  return true;
}

// Exact derivatives of forward dynamics. Differentiating ID(q, qd, FD(q, qd, tau)) = tau
// gives dqdd/dq = -M^-1 dID/dq and dqdd/dqd = -M^-1 dID/dqd (qdd held fixed),
// dqdd/dtau = M^-1. dID/d(q, qd) comes from forward-mode dual numbers.
bool fd_derivatives(const orc_robot &rb, const double *q, const double *qd, const double *tau,
                    double *qdd, double *dq, double *dqd, double *Minv) {
  const int n = rb.n;
  std::vector<double> L((size_t)n * n);
  if (!forward_dynamics(rb, q, qd, tau, qdd, L.data())) return false;
  std::vector<Dual> Q(n), QD(n), QDD(n), TAU(n);
  std::vector<double> col(n);
  for (int dir = 0; dir < 2 * n; ++dir) {
    for (int i = 0; i < n; ++i) {
      Q[i] = Dual(q[i], (dir == i) ? 1.0 : 0.0);
      QD[i] = Dual(qd[i], (dir == n + i) ? 1.0 : 0.0);
      QDD[i] = Dual(qdd[i], 0.0);
    }
    inverse_dynamics<Dual>(rb, Q.data(), QD.data(), QDD.data(), true, TAU.data());
    for (int i = 0; i < n; ++i) col[i] = -TAU[i].d;
    cholesky_solve(L.data(), n, col.data());
    double *dst = dir < n ? dq : dqd;
    const int j = dir < n ? dir : dir - n;
    for (int i = 0; i < n; ++i) dst[i * n + j] = col[i];
  }
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i < n; ++i) col[i] = (i == j) ? 1.0 : 0.0;
    cholesky_solve(L.data(), n, col.data());
    for (int i = 0; i < n; ++i) Minv[i * n + j] = col[i];
  }
  return true;
}

// Explicit Euler step x' = [q + h qd; qd + h qdd(q, qd, u)].
bool step(const orc_robot &rb, double h, const double *x, const double *u, double *xn) {
  const int n = rb.n;
  std::vector<double> qdd(n);
  if (!forward_dynamics(rb, x, x + n, u, qdd.data(), nullptr)) return false;
  for (int i = 0; i < n; ++i) {
    xn[i] = x[i] + h * x[n + i];
    xn[n + i] = x[n + i] + h * qdd[i];
  }
  return true;
}

// Plant of the closed-loop simulations (Sec. IV-E integrates the robot at
// 1 kHz with RK4): the continuous dynamics x' = f(x) = [qd; FD(q, qd, tau)],
// tau held constant over the interval, advanced by `substeps` classical
// fourth-order Runge-Kutta steps of length h / substeps:
//   k1 = f(x), k2 = f(x + d/2 k1), k3 = f(x + d/2 k2), k4 = f(x + d k3),
//   x <- x + d/6 (k1 + 2 k2 + 2 k3 + k4).
bool plant_rk4(const orc_robot &rb, double h, int substeps, const double *x, const double *tau, double *xn) {
  const int n = rb.n, nx = 2 * n;
  const double d = h / substeps;
  std::vector<double> y(x, x + nx), k1(nx), k2(nx), k3(nx), k4(nx), t(nx);
  auto f = [&](const double *z, double *out) {
    for (int i = 0; i < n; ++i) out[i] = z[n + i];
    return forward_dynamics(rb, z, z + n, tau, out + n, nullptr);
  };
  for (int s = 0; s < substeps; ++s) {
    if (!f(y.data(), k1.data())) return false;
    for (int i = 0; i < nx; ++i) t[i] = y[i] + 0.5 * d * k1[i];
    if (!f(t.data(), k2.data())) return false;
    for (int i = 0; i < nx; ++i) t[i] = y[i] + 0.5 * d * k2[i];
    if (!f(t.data(), k3.data())) return false;
    for (int i = 0; i < nx; ++i) t[i] = y[i] + d * k3[i];
    if (!f(t.data(), k4.data())) return false;
    for (int i = 0; i < nx; ++i) y[i] += d / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
  }
  std::memcpy(xn, y.data(), sizeof(double) * nx);
  return true;
}

// Jacobians of the Euler step: A = [[I, hI], [h dqdd/dq, I + h dqdd/dqd]],
// B = [[0], [h M^-1]].
bool step_jacobians(const orc_robot &rb, double h, const double *x, const double *u, double *xn,
                    double *A, double *B) {
  const int n = rb.n, nx = 2 * n;
  std::vector<double> qdd(n), dq((size_t)n * n), dqd((size_t)n * n), Minv((size_t)n * n);
  if (!fd_derivatives(rb, x, x + n, u, qdd.data(), dq.data(), dqd.data(), Minv.data())) return false;
  for (int i = 0; i < n; ++i) {
    xn[i] = x[i] + h * x[n + i];
    xn[n + i] = x[n + i] + h * qdd[i];
  }
  std::memset(A, 0, sizeof(double) * nx * nx);
  std::memset(B, 0, sizeof(double) * nx * n);
  for (int i = 0; i < n; ++i) {
    A[i * nx + i] = 1.0;
    A[i * nx + n + i] = h;
    for (int j = 0; j < n; ++j) {
      A[(n + i) * nx + j] = h * dq[i * n + j];
      A[(n + i) * nx + n + j] = h * dqd[i * n + j] + (i == j ? 1.0 : 0.0);
      B[(n + i) * n + j] = h * Minv[i * n + j];
    }
  }
  return true;
}

// ---------------------------------------------------------------------------
// The QP of one SQP step, Eq. (1).
// ---------------------------------------------------------------------------
struct Lq {
  int n, nx, nu, N;
  std::vector<double> A, B, e;   // [N-1][nx][nx], [N-1][nx][nu], [N-1][nx]
  std::vector<double> q, r;      // [N][nx], [N-1][nu]
  std::vector<double> Qf;        // [N][nx][nx] state Hessian blocks Q_k (incl. rho)
  std::vector<double> Rh;        // [nu] diagonal of R
  std::vector<double> c0;        // [nx] x_s - x_0
  bool ok;
};

double goal_state(const double *qgoal, int n, int i) { return i < n ? qgoal[i] : 0.0; }

Lq build_lq(const orc_robot &rb, const orc_problem &pr, double rho, const double *xs,
            const double *qgoal, const double *X, const double *U) {
  Lq lq;
  const int n = rb.n, nx = 2 * n, nu = n, N = pr.N;
  lq.n = n; lq.nx = nx; lq.nu = nu; lq.N = N; lq.ok = true;
  lq.A.assign((size_t)(N - 1) * nx * nx, 0.0);
  lq.B.assign((size_t)(N - 1) * nx * nu, 0.0);
  lq.e.assign((size_t)(N - 1) * nx, 0.0);
  lq.q.assign((size_t)N * nx, 0.0);
  lq.r.assign((size_t)(N > 1 ? N - 1 : 0) * nu, 0.0);
  lq.Qf.assign((size_t)N * nx * nx, 0.0);
  lq.Rh.assign(nu, 0.0);
  lq.c0.assign(nx, 0.0);
  std::vector<double> fx(nx);
  for (int k = 0; k < N - 1; ++k) {
    if (!step_jacobians(rb, pr.dt, X + (size_t)k * nx, U + (size_t)k * nu, fx.data(),
                        &lq.A[(size_t)k * nx * nx], &lq.B[(size_t)k * nx * nu]))
      lq.ok = false;
    for (int i = 0; i < nx; ++i) lq.e[(size_t)k * nx + i] = fx[i] - X[(size_t)(k + 1) * nx + i];
  }
  for (int k = 0; k < N; ++k) {
    const double *W = (k < N - 1) ? pr.Qd : pr.QNd;
    double *Qk = &lq.Qf[(size_t)k * nx * nx];
    for (int i = 0; i < nx; ++i) {
      lq.q[(size_t)k * nx + i] = W[i] * (X[(size_t)k * nx + i] - goal_state(qgoal, n, i));
      Qk[i * nx + i] = W[i] + rho;
    }
    if (has_task(pr)) {
      // Gauss-Newton terms of the tip tracking cost: gradient J^T W (p - pref),
      // Hessian J^T W J (the residual's second derivative is dropped).
      const double *We = (k < N - 1) ? pr.Wee : pr.WeeN;
      std::vector<double> p(3), J((size_t)3 * n);
      tip_jacobian(rb, X + (size_t)k * nx, p.data(), J.data());
      for (int c = 0; c < 3; ++c) {
        const double res = p[c] - pr.pref[(size_t)k * 3 + c];
        for (int i = 0; i < n; ++i) lq.q[(size_t)k * nx + i] += J[c * n + i] * We[c] * res;
        for (int i = 0; i < n; ++i)
          for (int j = 0; j < n; ++j) Qk[i * nx + j] += J[c * n + i] * We[c] * J[c * n + j];
      }
    }
  }
  for (int k = 0; k < N - 1; ++k)
    for (int i = 0; i < nu; ++i) lq.r[(size_t)k * nu + i] = pr.Rd[i] * U[(size_t)k * nu + i];
  for (int i = 0; i < nu; ++i) lq.Rh[i] = pr.Rd[i];
  for (int i = 0; i < nx; ++i) lq.c0[i] = xs[i] - X[i];
  return lq;
}

// Offsets of x_k and u_k inside dZ = [x_0 u_0 x_1 u_1 ... u_{N-2} x_{N-1}].
inline size_t off_x(const Lq &lq, int k) { return (size_t)k * (lq.nx + lq.nu); }
inline size_t off_u(const Lq &lq, int k) { return (size_t)k * (lq.nx + lq.nu) + lq.nx; }
inline size_t nz_of(const Lq &lq) { return (size_t)lq.N * lq.nx + (size_t)(lq.N - 1) * lq.nu; }

// Dense G, g, C, c of Eq. (2).
void assemble_kkt_parts(const Lq &lq, std::vector<double> &G, std::vector<double> &g,
                        std::vector<double> &C, std::vector<double> &c) {
  const int nx = lq.nx, nu = lq.nu, N = lq.N;
  const size_t nz = nz_of(lq), nc = (size_t)N * nx;
  G.assign(nz * nz, 0.0);
  g.assign(nz, 0.0);
  C.assign(nc * nz, 0.0);
  c.assign(nc, 0.0);
  for (int k = 0; k < N; ++k) {
    for (int i = 0; i < nx; ++i) {
      const size_t o = off_x(lq, k) + i;
      for (int j = 0; j < nx; ++j) G[o * nz + off_x(lq, k) + j] = lq.Qf[((size_t)k * nx + i) * nx + j];
      g[o] = lq.q[(size_t)k * nx + i];
    }
    if (k < N - 1)
      for (int i = 0; i < nu; ++i) {
        const size_t o = off_u(lq, k) + i;
        G[o * nz + o] = lq.Rh[i];
        g[o] = lq.r[(size_t)k * nu + i];
      }
  }
  // Row block 0: dx_0 = x_s - x_0.
  for (int i = 0; i < nx; ++i) {
    C[(size_t)i * nz + off_x(lq, 0) + i] = 1.0;
    c[i] = lq.c0[i];
  }
  // Row block k+1: dx_{k+1} - A_k dx_k - B_k du_k = e_k.
  for (int k = 0; k < N - 1; ++k) {
    for (int i = 0; i < nx; ++i) {
      const size_t row = (size_t)(k + 1) * nx + i;
      C[row * nz + off_x(lq, k + 1) + i] = 1.0;
      for (int j = 0; j < nx; ++j) C[row * nz + off_x(lq, k) + j] = -lq.A[((size_t)k * nx + i) * nx + j];
      for (int j = 0; j < nu; ++j) C[row * nz + off_u(lq, k) + j] = -lq.B[((size_t)k * nx + i) * nu + j];
      c[row] = lq.e[(size_t)k * nx + i];
    }
  }
}

// Solve [[G, C^T], [C, 0]] [dZ; nu] = [-g; c] by dense LU; lambda = -nu.
bool solve_kkt_dense(const Lq &lq, double *dZ, double *lam) {
  std::vector<double> G, g, C, c;
  assemble_kkt_parts(lq, G, g, C, c);
  const size_t nz = nz_of(lq), nc = (size_t)lq.N * lq.nx, nk = nz + nc;
  std::vector<double> K(nk * nk, 0.0), rhs(nk, 0.0);
  for (size_t i = 0; i < nz; ++i)
    for (size_t j = 0; j < nz; ++j) K[i * nk + j] = G[i * nz + j];
  for (size_t i = 0; i < nc; ++i)
    for (size_t j = 0; j < nz; ++j) {
      K[(nz + i) * nk + j] = C[i * nz + j];
      K[j * nk + nz + i] = C[i * nz + j];
    }
  for (size_t i = 0; i < nz; ++i) rhs[i] = -g[i];
  for (size_t i = 0; i < nc; ++i) rhs[nz + i] = c[i];
  if (!lu_solve(K.data(), (int)nk, rhs.data(), 1)) return false;
  for (size_t i = 0; i < nz; ++i) dZ[i] = rhs[i];
  for (size_t i = 0; i < nc; ++i) lam[i] = -rhs[nz + i];
  return true;
}

// [C^T lambda] in dZ layout, from the block structure of C.
void ct_times(const Lq &lq, const double *lam, double *out) {
  const int nx = lq.nx, nu = lq.nu, N = lq.N;
  for (int k = 0; k < N; ++k) {
    for (int i = 0; i < nx; ++i) {
      double s = lam[(size_t)k * nx + i];
      if (k < N - 1)
        for (int j = 0; j < nx; ++j)
          s -= lq.A[((size_t)k * nx + j) * nx + i] * lam[(size_t)(k + 1) * nx + j];
      out[off_x(lq, k) + i] = s;
    }
    if (k < N - 1)
      for (int i = 0; i < nu; ++i) {
        double s = 0.0;
        for (int j = 0; j < nx; ++j) s -= lq.B[((size_t)k * nx + j) * nu + i] * lam[(size_t)(k + 1) * nx + j];
        out[off_u(lq, k) + i] = s;
      }
  }
}

// Eq. (4), last formula: dZ = -G^-1 (g - C^T lambda).
void recover_step(const Lq &lq, const double *lam, double *dZ) {
  const int nx = lq.nx, nu = lq.nu, N = lq.N;
  std::vector<double> ctl(nz_of(lq)), Qc((size_t)nx * nx), v(nx);
  ct_times(lq, lam, ctl.data());
  for (int k = 0; k < N; ++k) {
    // dx_k = -Q_k^-1 (q_k - [C^T lambda]_k), Q_k SPD.
    for (int i = 0; i < nx; ++i) v[i] = -(lq.q[(size_t)k * nx + i] - ctl[off_x(lq, k) + i]);
    std::copy(&lq.Qf[(size_t)k * nx * nx], &lq.Qf[(size_t)(k + 1) * nx * nx], Qc.begin());
    if (!cholesky(Qc.data(), nx)) {
      for (int i = 0; i < nx; ++i) v[i] = std::nan("");
    } else {
      cholesky_solve(Qc.data(), nx, v.data());
    }
    for (int i = 0; i < nx; ++i) dZ[off_x(lq, k) + i] = v[i];
    if (k < N - 1)
      for (int i = 0; i < nu; ++i) {
        const size_t o = off_u(lq, k) + i;
        dZ[o] = -(lq.r[(size_t)k * nu + i] - ctl[o]) / lq.Rh[i];
      }
  }
}

// inf-norm residual of [[G, C^T], [C, 0]] [dZ; -lambda] - [-g; c].
double kkt_residual(const Lq &lq, const double *dZ, const double *lam) {
  std::vector<double> G, g, C, c;
  assemble_kkt_parts(lq, G, g, C, c);
  const size_t nz = nz_of(lq), nc = (size_t)lq.N * lq.nx;
  double res = 0.0;
  for (size_t i = 0; i < nz; ++i) {
    double s = g[i];
    for (size_t j = 0; j < nz; ++j) s += G[i * nz + j] * dZ[j];
    for (size_t j = 0; j < nc; ++j) s -= C[j * nz + i] * lam[j];
    res = std::fmax(res, std::fabs(s));
  }
  for (size_t i = 0; i < nc; ++i) {
    double s = -c[i];
    for (size_t j = 0; j < nz; ++j) s += C[i * nz + j] * dZ[j];
    res = std::fmax(res, std::fabs(s));
  }
  return res;
}

// ---------------------------------------------------------------------------
// Schur complement, preconditioner and PCG: Eqs. (4)-(6), Sec. II-B.
// ---------------------------------------------------------------------------
struct Schur {
  int nx, N;
  std::vector<double> S;      // dense [N nx][N nx], S~ = C G^-1 C^T
  std::vector<double> gamma;  // [N nx], gamma~ = c + C G^-1 g
  std::vector<double> P;      // dense [N nx][N nx], P = -Phi^-1
  bool ok;
};

// theta_k, phi_k, zeta_k of Eq. (5), with the inverse Q_k^-1 of each (possibly
// dense) state Hessian block and diagonal R, placed into the block tridiagonal
// S~ and gamma~ of Eq. (6) (signs per reading R2/R3), then the stair
// preconditioner of Eq. (6) block by block.
Schur build_schur(const Lq &lq) {
  Schur s;
  const int nx = lq.nx, nu = lq.nu, N = lq.N;
  const size_t dim = (size_t)N * nx;
  s.nx = nx; s.N = N; s.ok = true;
  s.S.assign(dim * dim, 0.0);
  s.P.assign(dim * dim, 0.0);
  s.gamma.assign(dim, 0.0);
  auto Sat = [&](int bi, int bj, int i, int j) -> double & {
    return s.S[((size_t)bi * nx + i) * dim + (size_t)bj * nx + j];
  };
  auto Pat = [&](int bi, int bj, int i, int j) -> double & {
    return s.P[((size_t)bi * nx + i) * dim + (size_t)bj * nx + j];
  };
  // Q_k^-1 for every knot.
  std::vector<double> Qi((size_t)N * nx * nx, 0.0);
  for (int k = 0; k < N; ++k)
    if (!invert(&lq.Qf[(size_t)k * nx * nx], nx, &Qi[(size_t)k * nx * nx])) s.ok = false;
  // Block (0,0) = Q_0^-1 and gamma~_0 = c_0 + Q_0^-1 q_0.
  for (int i = 0; i < nx; ++i) {
    double t = lq.c0[i];
    for (int j = 0; j < nx; ++j) {
      Sat(0, 0, i, j) = Qi[i * nx + j];
      t += Qi[i * nx + j] * lq.q[j];
    }
    s.gamma[i] = t;
  }
  std::vector<double> theta((size_t)N * nx * nx, 0.0), phi((size_t)(N - 1) * nx * nx, 0.0);
  std::vector<double> AQ((size_t)nx * nx);
  for (int k = 0; k < N - 1; ++k) {
    const double *A = &lq.A[(size_t)k * nx * nx];
    const double *B = &lq.B[(size_t)k * nx * nu];
    const double *Qik = &Qi[(size_t)k * nx * nx];
    const double *Qik1 = &Qi[(size_t)(k + 1) * nx * nx];
    double *th = &theta[(size_t)(k + 1) * nx * nx];
    double *ph = &phi[(size_t)k * nx * nx];
    matmul(A, Qik, AQ.data(), nx, nx, nx);          // A_k Q_k^-1
    for (int i = 0; i < nx; ++i)
      for (int j = 0; j < nx; ++j) {
        double t = Qik1[i * nx + j];
        for (int m = 0; m < nx; ++m) t += AQ[i * nx + m] * A[j * nx + m];
        for (int m = 0; m < nu; ++m) t += B[i * nu + m] * B[j * nu + m] / lq.Rh[m];
        th[i * nx + j] = t;                         // theta_k
        ph[i * nx + j] = -AQ[i * nx + j];           // phi_k = -A_k Q_k^-1
      }
    for (int i = 0; i < nx; ++i) {
      double z = 0.0;                               // zeta_k
      for (int m = 0; m < nx; ++m) z -= AQ[i * nx + m] * lq.q[(size_t)k * nx + m];
      for (int m = 0; m < nu; ++m) z -= B[i * nu + m] * lq.r[(size_t)k * nu + m] / lq.Rh[m];
      for (int m = 0; m < nx; ++m) z += Qik1[i * nx + m] * lq.q[(size_t)(k + 1) * nx + m];
      s.gamma[(size_t)(k + 1) * nx + i] = lq.e[(size_t)k * nx + i] + z;
    }
    for (int i = 0; i < nx; ++i)
      for (int j = 0; j < nx; ++j) {
        Sat(k + 1, k + 1, i, j) = th[i * nx + j];
        Sat(k + 1, k, i, j) = ph[i * nx + j];       // below the diagonal: phi_k
        Sat(k, k + 1, j, i) = ph[i * nx + j];       // above: phi_k^T
      }
  }
  // Stair preconditioner: diagonal blocks D_k^-1 (D_0^-1 = Q_0, D_{k+1}^-1 =
  // theta_k^-1), off-diagonal blocks -D_{k+1}^-1 phi_k D_k^-1.
  std::vector<double> Dinv((size_t)N * nx * nx, 0.0);
  for (int i = 0; i < nx * nx; ++i) Dinv[i] = lq.Qf[i];   // (Q_0^-1)^-1
  for (int k = 1; k < N; ++k)
    if (!invert(&theta[(size_t)k * nx * nx], nx, &Dinv[(size_t)k * nx * nx])) s.ok = false;
  std::vector<double> t1((size_t)nx * nx), t2((size_t)nx * nx);
  for (int k = 0; k < N; ++k)
    for (int i = 0; i < nx; ++i)
      for (int j = 0; j < nx; ++j) Pat(k, k, i, j) = Dinv[((size_t)k * nx + i) * nx + j];
  for (int k = 0; k < N - 1; ++k) {
    matmul(&Dinv[(size_t)(k + 1) * nx * nx], &phi[(size_t)k * nx * nx], t1.data(), nx, nx, nx);
    matmul(t1.data(), &Dinv[(size_t)k * nx * nx], t2.data(), nx, nx, nx);
    for (int i = 0; i < nx; ++i)
      for (int j = 0; j < nx; ++j) {
        Pat(k + 1, k, i, j) = -t2[i * nx + j];
        Pat(k, k + 1, j, i) = -t2[i * nx + j];
      }
  }
  return s;
}

// y = A x for a dim x dim matrix (dim = N nx) that is block tridiagonal with
// nx x nx blocks, as S~ and P of Eq. (6) are by construction: row i sums over
// the block columns bi-1..bi+1 of its block row bi in ascending column order,
// so the terms left out are exactly the structural zeros and the sums equal
// those of the full dense product. (N = 1: a plain dense product.)
void tridiag_matvec(const std::vector<double> &A, const double *x, double *y, int nx, int N) {
  const size_t dim = (size_t)N * nx;
  for (size_t i = 0; i < dim; ++i) {
    const int bi = (int)(i / nx);
    const size_t j0 = (size_t)std::max(bi - 1, 0) * nx, j1 = (size_t)std::min(bi + 2, N) * nx;
    double s = 0.0;
    for (size_t j = j0; j < j1; ++j) s += A[i * dim + j] * x[j];
    y[i] = s;
  }
}

// Preconditioned conjugate gradient on S~ lambda = gamma~ (Sec. II-B) with the
// stopping rule of reading R6. lam holds the initial guess on entry. With
// fixed_iters >= 0 the iteration count is prescribed instead (a replay of a
// count decided elsewhere); ratio / ratio_prev (or NULL) receive the stopping
// value r^T P r over tol^2 gamma^T P gamma after the last iteration and after
// the one before it (infinity before the first).
int pcg(const Schur &s, double *lam, double tol, int max_iter, bool *hit_max, int fixed_iters = -1,
        double *ratio = nullptr, double *ratio_prev = nullptr) {
  const size_t dim = (size_t)s.N * s.nx;
  std::vector<double> r(dim), z(dim), p(dim), w(dim), pg(dim);
  auto S_times = [&](const double *x, double *y) { tridiag_matvec(s.S, x, y, s.nx, s.N); };
  auto P_times = [&](const double *x, double *y) { tridiag_matvec(s.P, x, y, s.nx, s.N); };
  P_times(s.gamma.data(), pg.data());
  double eta_ref = 0.0;
  for (size_t i = 0; i < dim; ++i) eta_ref += s.gamma[i] * pg[i];
  S_times(lam, w.data());
  for (size_t i = 0; i < dim; ++i) r[i] = s.gamma[i] - w[i];
  P_times(r.data(), z.data());
  double eta = 0.0;
  for (size_t i = 0; i < dim; ++i) { p[i] = z[i]; eta += r[i] * z[i]; }
  const double stop = tol * tol * eta_ref;
  int it = 0;
  *hit_max = false;
  double eta_prev = std::numeric_limits<double>::infinity();
  while (fixed_iters >= 0 ? (it < fixed_iters && eta > 0.0) : eta > stop) {
    if (fixed_iters < 0 && it >= max_iter) { *hit_max = true; break; }
    eta_prev = eta;
    S_times(p.data(), w.data());
    double pw = 0.0;
    for (size_t i = 0; i < dim; ++i) pw += p[i] * w[i];
    const double a = eta / pw;
    for (size_t i = 0; i < dim; ++i) { lam[i] += a * p[i]; r[i] -= a * w[i]; }
    P_times(r.data(), z.data());
    double eta_new = 0.0;
    for (size_t i = 0; i < dim; ++i) eta_new += r[i] * z[i];
    const double b = eta_new / eta;
    for (size_t i = 0; i < dim; ++i) p[i] = z[i] + b * p[i];
    eta = eta_new;
    ++it;
  }
  if (ratio) *ratio = eta / stop;
  if (ratio_prev) *ratio_prev = eta_prev / stop;
  return it;
}

// ---------------------------------------------------------------------------
// Finite-horizon Riccati recursion for the same QP (textbook dynamic programming).
// ---------------------------------------------------------------------------
bool solve_riccati(const Lq &lq, double *dZ, double *lam) {
  const int nx = lq.nx, nu = lq.nu, N = lq.N;
  std::vector<double> P((size_t)N * nx * nx, 0.0), p((size_t)N * nx, 0.0);
  std::vector<double> K((size_t)(N > 1 ? N - 1 : 0) * nu * nx, 0.0), d((size_t)(N > 1 ? N - 1 : 0) * nu, 0.0);
  double *PN = &P[(size_t)(N - 1) * nx * nx];
  for (int i = 0; i < nx; ++i) {
    for (int j = 0; j < nx; ++j) PN[i * nx + j] = lq.Qf[((size_t)(N - 1) * nx + i) * nx + j];
    p[(size_t)(N - 1) * nx + i] = lq.q[(size_t)(N - 1) * nx + i];
  }
  std::vector<double> PA((size_t)nx * nx), PB((size_t)nx * nu), H((size_t)nu * nu), Gux((size_t)nu * nx),
      hv(nu), v(nx), rhs((size_t)nu * (nx + 1));
  for (int k = N - 2; k >= 0; --k) {
    const double *A = &lq.A[(size_t)k * nx * nx];
    const double *B = &lq.B[(size_t)k * nx * nu];
    const double *P1 = &P[(size_t)(k + 1) * nx * nx];
    const double *p1 = &p[(size_t)(k + 1) * nx];
    const double *e = &lq.e[(size_t)k * nx];
    matmul(P1, A, PA.data(), nx, nx, nx);
    matmul(P1, B, PB.data(), nx, nx, nu);
    for (int i = 0; i < nx; ++i) {               // v = P_{k+1} e_k + p_{k+1}
      double t = p1[i];
      for (int j = 0; j < nx; ++j) t += P1[i * nx + j] * e[j];
      v[i] = t;
    }
    for (int i = 0; i < nu; ++i) {
      for (int j = 0; j < nu; ++j) {             // H = R + B^T P B
        double t = (i == j) ? lq.Rh[i] : 0.0;
        for (int m = 0; m < nx; ++m) t += B[m * nu + i] * PB[m * nu + j];
        H[i * nu + j] = t;
      }
      for (int j = 0; j < nx; ++j) {             // G_ux = B^T P A
        double t = 0.0;
        for (int m = 0; m < nx; ++m) t += B[m * nu + i] * PA[m * nx + j];
        Gux[i * nx + j] = t;
      }
      double t = lq.r[(size_t)k * nu + i];       // g_u = r + B^T v
      for (int m = 0; m < nx; ++m) t += B[m * nu + i] * v[m];
      hv[i] = t;
    }
    // [K | d] = H^-1 [G_ux | g_u]
    for (int i = 0; i < nu; ++i) {
      for (int j = 0; j < nx; ++j) rhs[(size_t)i * (nx + 1) + j] = Gux[i * nx + j];
      rhs[(size_t)i * (nx + 1) + nx] = hv[i];
    }
    std::vector<double> Hc(H);
    if (!lu_solve(Hc.data(), nu, rhs.data(), nx + 1)) return false;
    double *Kk = &K[(size_t)k * nu * nx];
    double *dk = &d[(size_t)k * nu];
    for (int i = 0; i < nu; ++i) {
      for (int j = 0; j < nx; ++j) Kk[i * nx + j] = rhs[(size_t)i * (nx + 1) + j];
      dk[i] = rhs[(size_t)i * (nx + 1) + nx];
    }
    // Joseph form, with Acl = A - B K:
    //   P_k = Q + K^T R K + Acl^T P_{k+1} Acl,
    //   p_k = q + K^T (R d - r) + Acl^T (P_{k+1} (e - B d) + p_{k+1}).
    // It equals the plain update Q + A^T P A - G_ux^T K for the optimal K but
    // stays symmetric positive definite in rounding; the plain form loses
    // symmetry and diverges over long horizons when A is open-loop unstable.
    double *Pk = &P[(size_t)k * nx * nx];
    double *pk = &p[(size_t)k * nx];
    std::vector<double> Acl((size_t)nx * nx), PAcl((size_t)nx * nx), w(nx);
    for (int i = 0; i < nx; ++i)
      for (int j = 0; j < nx; ++j) {
        double t = A[i * nx + j];
        for (int m = 0; m < nu; ++m) t -= B[i * nu + m] * Kk[m * nx + j];
        Acl[i * nx + j] = t;
      }
    matmul(P1, Acl.data(), PAcl.data(), nx, nx, nx);
    for (int i = 0; i < nx; ++i) {               // w = P_{k+1} (e - B d) + p_{k+1}
      double t = p1[i];
      for (int j = 0; j < nx; ++j) {
        double ebd = e[j];
        for (int m = 0; m < nu; ++m) ebd -= B[j * nu + m] * dk[m];
        t += P1[i * nx + j] * ebd;
      }
      w[i] = t;
    }
    for (int i = 0; i < nx; ++i) {
      for (int j = 0; j < nx; ++j) {
        double t = lq.Qf[((size_t)k * nx + i) * nx + j];
        for (int m = 0; m < nu; ++m) t += Kk[m * nx + i] * lq.Rh[m] * Kk[m * nx + j];
        for (int m = 0; m < nx; ++m) t += Acl[m * nx + i] * PAcl[m * nx + j];
        Pk[i * nx + j] = t;
      }
      double t = lq.q[(size_t)k * nx + i];
      for (int m = 0; m < nu; ++m) t += Kk[m * nx + i] * (lq.Rh[m] * dk[m] - lq.r[(size_t)k * nu + m]);
      for (int m = 0; m < nx; ++m) t += Acl[m * nx + i] * w[m];
      pk[i] = t;
    }
    for (int i = 0; i < nx; ++i)
      for (int j = i + 1; j < nx; ++j) {
        const double avg = 0.5 * (Pk[i * nx + j] + Pk[j * nx + i]);
        Pk[i * nx + j] = avg;
        Pk[j * nx + i] = avg;
      }
  }
  // Forward roll from dx_0 = x_s - x_0; lambda_k = P_k dx_k + p_k.
  std::vector<double> dx(lq.c0);
  for (int k = 0; k < N; ++k) {
    for (int i = 0; i < nx; ++i) {
      dZ[off_x(lq, k) + i] = dx[i];
      double t = p[(size_t)k * nx + i];
      for (int j = 0; j < nx; ++j) t += P[((size_t)k * nx + i) * nx + j] * dx[j];
      lam[(size_t)k * nx + i] = t;
    }
    if (k == N - 1) break;
    const double *A = &lq.A[(size_t)k * nx * nx];
    const double *B = &lq.B[(size_t)k * nx * nu];
    std::vector<double> du(nu), dn(nx);
    for (int i = 0; i < nu; ++i) {
      double t = -d[(size_t)k * nu + i];
      for (int j = 0; j < nx; ++j) t -= K[((size_t)k * nu + i) * nx + j] * dx[j];
      du[i] = t;
      dZ[off_u(lq, k) + i] = t;
    }
    for (int i = 0; i < nx; ++i) {
      double t = lq.e[(size_t)k * nx + i];
      for (int j = 0; j < nx; ++j) t += A[i * nx + j] * dx[j];
      for (int j = 0; j < nu; ++j) t += B[i * nu + j] * du[j];
      dn[i] = t;
    }
    dx = dn;
  }
  return true;
}

// ---------------------------------------------------------------------------
// Merit function, Eq. (3): J + mu ||c||_1 with the nonlinear constraints.
// ---------------------------------------------------------------------------
bool cost_and_defect(const orc_robot &rb, const orc_problem &pr, const double *xs, const double *qgoal,
                     const double *X, const double *U, double *J, double *c1) {
  const int n = rb.n, nx = 2 * n, nu = n, N = pr.N;
  double cost = 0.0, viol = 0.0;
  for (int k = 0; k < N; ++k) {
    const double *W = (k < N - 1) ? pr.Qd : pr.QNd;
    for (int i = 0; i < nx; ++i) {
      const double d = X[(size_t)k * nx + i] - goal_state(qgoal, n, i);
      cost += 0.5 * W[i] * d * d;
    }
    if (has_task(pr)) {
      const double *We = (k < N - 1) ? pr.Wee : pr.WeeN;
      const V3<double> p = tip_position<double>(rb, X + (size_t)k * nx);
      const double d[3] = {p.x - pr.pref[(size_t)k * 3 + 0], p.y - pr.pref[(size_t)k * 3 + 1],
                           p.z - pr.pref[(size_t)k * 3 + 2]};
      for (int c = 0; c < 3; ++c) cost += 0.5 * We[c] * d[c] * d[c];
    }
    if (k < N - 1)
      for (int i = 0; i < nu; ++i) cost += 0.5 * pr.Rd[i] * U[(size_t)k * nu + i] * U[(size_t)k * nu + i];
  }
  for (int i = 0; i < nx; ++i) viol += std::fabs(xs[i] - X[i]);
  std::vector<double> fx(nx);
  bool ok = true;
  for (int k = 0; k < N - 1; ++k) {
    if (!step(rb, pr.dt, X + (size_t)k * nx, U + (size_t)k * nu, fx.data())) ok = false;
    for (int i = 0; i < nx; ++i) viol += std::fabs(fx[i] - X[(size_t)(k + 1) * nx + i]);
  }
  *J = cost;
  *c1 = viol;
  return ok;
}

bool all_finite(const double *v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

}  // namespace

// ===========================================================================
// C entry points (ctypes).
// ===========================================================================
extern "C" {

int orc_inverse_dynamics(const orc_robot *rb, const double *q, const double *qd, const double *qdd,
                         int with_gravity, double *tau) {
  inverse_dynamics<double>(*rb, q, qd, qdd, with_gravity != 0, tau);
  return 0;
}

int orc_mass_matrix(const orc_robot *rb, const double *q, double *M) {
  mass_matrix(*rb, q, M);
  return 0;
}

int orc_forward_dynamics(const orc_robot *rb, const double *q, const double *qd, const double *tau,
                         double *qdd) {
  return forward_dynamics(*rb, q, qd, tau, qdd, nullptr) ? 0 : -1;
}

int orc_fd_derivatives(const orc_robot *rb, const double *q, const double *qd, const double *tau,
                       double *qdd, double *dq, double *dqd, double *Minv) {
  return fd_derivatives(*rb, q, qd, tau, qdd, dq, dqd, Minv) ? 0 : -1;
}

int orc_step(const orc_robot *rb, double h, const double *x, const double *u, double *xn) {
  return step(*rb, h, x, u, xn) ? 0 : -1;
}

int orc_plant_rk4(const orc_robot *rb, double h, int substeps, const double *x, const double *tau, double *xn) {
  if (substeps < 1) return -2;
  return plant_rk4(*rb, h, substeps, x, tau, xn) ? 0 : -1;
}

int orc_step_jacobians(const orc_robot *rb, double h, const double *x, const double *u, double *xn,
                       double *A, double *B) {
  return step_jacobians(*rb, h, x, u, xn, A, B) ? 0 : -1;
}

// LQ data of Eq. (1) at (X, U): A[N-1][nx][nx], B[N-1][nx][nu], e[N-1][nx],
// q[N][nx], r[N-1][nu], c0[nx].
int orc_lq(const orc_robot *rb, const orc_problem *pr, double rho, const double *xs, const double *qgoal,
           const double *X, const double *U, double *A, double *B, double *e, double *q, double *r,
           double *c0) {
  Lq lq = build_lq(*rb, *pr, rho, xs, qgoal, X, U);
  std::memcpy(A, lq.A.data(), sizeof(double) * lq.A.size());
  std::memcpy(B, lq.B.data(), sizeof(double) * lq.B.size());
  std::memcpy(e, lq.e.data(), sizeof(double) * lq.e.size());
  std::memcpy(q, lq.q.data(), sizeof(double) * lq.q.size());
  std::memcpy(r, lq.r.data(), sizeof(double) * lq.r.size());
  std::memcpy(c0, lq.c0.data(), sizeof(double) * lq.c0.size());
  return lq.ok ? 0 : -1;
}

// Tip position p[3] (base frame) and Jacobian J[3][n] at joint angles q.
int orc_tip(const orc_robot *rb, const double *q, double *p, double *J) {
  if (!rb || !q || !p || !J || rb->model != 0) return -1;
  tip_jacobian(*rb, q, p, J);
  return 0;
}

// State Hessian blocks Q_k [N][nx][nx] of the QP at (X, U) (diagonal Q plus rho,
// plus the Gauss-Newton tip tracking term when the problem has one).
int orc_lq_hessian(const orc_robot *rb, const orc_problem *pr, double rho, const double *xs, const double *qgoal,
                   const double *X, const double *U, double *Qf) {
  Lq lq = build_lq(*rb, *pr, rho, xs, qgoal, X, U);
  std::copy(lq.Qf.begin(), lq.Qf.end(), Qf);
  return lq.ok ? 0 : -1;
}

// Dense G[nz][nz], g[nz], C[nc][nz], c[nc] of Eq. (2) at (X, U).
int orc_kkt_parts(const orc_robot *rb, const orc_problem *pr, double rho, const double *xs,
                  const double *qgoal, const double *X, const double *U, double *G, double *g, double *C,
                  double *c) {
  Lq lq = build_lq(*rb, *pr, rho, xs, qgoal, X, U);
  std::vector<double> vG, vg, vC, vc;
  assemble_kkt_parts(lq, vG, vg, vC, vc);
  std::memcpy(G, vG.data(), sizeof(double) * vG.size());
  std::memcpy(g, vg.data(), sizeof(double) * vg.size());
  std::memcpy(C, vC.data(), sizeof(double) * vC.size());
  std::memcpy(c, vc.data(), sizeof(double) * vc.size());
  return lq.ok ? 0 : -1;
}

// Dense S~[dim][dim], gamma~[dim], P[dim][dim] (dim = N nx) of Eqs. (5)-(6).
int orc_schur(const orc_robot *rb, const orc_problem *pr, double rho, const double *xs, const double *qgoal,
              const double *X, const double *U, double *S, double *gamma, double *P) {
  Lq lq = build_lq(*rb, *pr, rho, xs, qgoal, X, U);
  Schur s = build_schur(lq);
  std::memcpy(S, s.S.data(), sizeof(double) * s.S.size());
  std::memcpy(gamma, s.gamma.data(), sizeof(double) * s.gamma.size());
  std::memcpy(P, s.P.data(), sizeof(double) * s.P.size());
  return (lq.ok && s.ok) ? 0 : -1;
}

// PCG on caller-given dense S~, P, gamma~ (dim x dim); lam is the initial guess
// on entry and the solution on exit. Returns the iteration count (< 0 on error)
// and sets *hit_max when the cap was reached.
int orc_pcg_dense(int dim, const double *S, const double *P, const double *gamma, double *lam, double tol,
                  int max_iter, int *hit_max) {
  Schur s;
  s.nx = dim; s.N = 1; s.ok = true;
  s.S.assign(S, S + (size_t)dim * dim);
  s.P.assign(P, P + (size_t)dim * dim);
  s.gamma.assign(gamma, gamma + dim);
  bool hm = false;
  const int it = pcg(s, lam, tol, max_iter, &hm);
  if (hit_max) *hit_max = hm ? 1 : 0;
  return it;
}

// One linear solve of the SQP step at (X, U): dZ [nz] and lambda [N nx].
// mode 0 dense LU, 1 Schur + PCG (lam in/out as initial guess), 2 Riccati.
int orc_qp_step(const orc_robot *rb, const orc_problem *pr, double rho, const double *xs, const double *qgoal,
                const double *X, const double *U, int mode, double pcg_tol, int pcg_max_iter, double *dZ,
                double *lam, int *pcg_iters, double *kkt_res) {
  Lq lq = build_lq(*rb, *pr, rho, xs, qgoal, X, U);
  if (!lq.ok) return -1;
  bool ok = true;
  int its = 0;
  if (mode == 0) {
    ok = solve_kkt_dense(lq, dZ, lam);
  } else if (mode == 1) {
    Schur s = build_schur(lq);
    ok = s.ok;
    bool hm = false;
    const int cap = pcg_max_iter > 0 ? pcg_max_iter : lq.N * lq.nx;
    its = pcg(s, lam, pcg_tol, cap, &hm);
    recover_step(lq, lam, dZ);
  } else {
    ok = solve_riccati(lq, dZ, lam);
  }
  if (pcg_iters) *pcg_iters = its;
  if (kkt_res) *kkt_res = kkt_residual(lq, dZ, lam);
  return ok ? 0 : -1;
}

// inf-norm residual of Eq. (2) at (X, U) for a caller-given dZ [nz] and
// lambda [N nx] (the residual every SQP iteration records); -1 if the QP data
// could not be formed.
double orc_kkt_residual(const orc_robot *rb, const orc_problem *pr, double rho, const double *xs,
                        const double *qgoal, const double *X, const double *U, const double *dZ,
                        const double *lam) {
  Lq lq = build_lq(*rb, *pr, rho, xs, qgoal, X, U);
  if (!lq.ok) return -1.0;
  return kkt_residual(lq, dZ, lam);
}

// The KKT solve of one SQP step on caller-given QP data (Eq. (2)):
// A[N-1][nx][nx], B[N-1][nx][nu], e[N-1][nx], q[N][nx], r[N-1][nu], c0[nx],
// Hessian diagonals Qh[N][nx] and Rh[nu]. mode 0 dense LU, 2 Riccati.
// Writes dZ [nz] and lambda [N nx].
int orc_kkt_from_lq(int nx, int nu, int N, const double *A, const double *B, const double *e, const double *q,
                    const double *r, const double *c0, const double *Qh, const double *Rh, int mode, double *dZ,
                    double *lam, double *kkt_res) {
  Lq lq;
  lq.n = nu; lq.nx = nx; lq.nu = nu; lq.N = N; lq.ok = true;
  lq.A.assign(A, A + (size_t)(N - 1) * nx * nx);
  lq.B.assign(B, B + (size_t)(N - 1) * nx * nu);
  lq.e.assign(e, e + (size_t)(N - 1) * nx);
  lq.q.assign(q, q + (size_t)N * nx);
  lq.r.assign(r, r + (size_t)(N - 1) * nu);
  lq.Qf.assign((size_t)N * nx * nx, 0.0);
  for (int k = 0; k < N; ++k)
    for (int i = 0; i < nx; ++i) lq.Qf[((size_t)k * nx + i) * nx + i] = Qh[(size_t)k * nx + i];
  lq.Rh.assign(Rh, Rh + nu);
  lq.c0.assign(c0, c0 + nx);
  const bool ok = (mode == 2) ? solve_riccati(lq, dZ, lam) : solve_kkt_dense(lq, dZ, lam);
  if (kkt_res) *kkt_res = kkt_residual(lq, dZ, lam);
  return ok ? 0 : -1;
}

// Merit of Eq. (3) at (X, U): returns J + mu ||c||_1 and writes J, ||c||_1.
double orc_merit(const orc_robot *rb, const orc_problem *pr, const double *xs, const double *qgoal,
                 const double *X, const double *U, double mu, double *J, double *c1) {
  double j = 0.0, c = 0.0;
  cost_and_defect(*rb, *pr, xs, qgoal, X, U, &j, &c);
  if (J) *J = j;
  if (c1) *c1 = c;
  return j + mu * c;
}

// The SQP loop of Sec. II-A / Algorithm 1 for one solve. X [N][nx] and U [N-1][nu]
// hold the initial guess on entry and the result on exit; lam [N nx] carries the
// PCG warm start in and the last multipliers out. log has sqp_iters entries (or is
// NULL). alpha_replay (or NULL) prescribes the accepted step of each iteration;
// a replayed step still records every candidate merit. descent_replay (or NULL)
// prescribes, per iteration, whether the line search counts as a descent for the
// rho adaptation (1 descent, 0 none), so that a replay follows the same rho
// sequence when two merits tie at FP32 resolution on the other side.
// pcg_replay (or NULL; Schur + PCG mode only) prescribes the PCG iteration
// count of each SQP iteration: the count is an integer that floating point
// decides, so a replay takes the other side's decision and the log's
// pcg_stop / pcg_stop_prev show whether the stopping rule holds there.
int orc_sqp(const orc_robot *rb, const orc_problem *pr, const orc_params *prm, const double *xs,
            const double *qgoal, double *X, double *U, double *lam, orc_iter_log *log,
            const double *alpha_replay, const int *descent_replay, const int *pcg_replay) {
  const int n = rb->n, nx = 2 * n, nu = n, N = pr->N;
  const size_t nX = (size_t)N * nx, nU = (size_t)(N - 1) * nu;
  if (prm->n_alpha < 1 || prm->n_alpha > ORC_MAX_ALPHA) return -2;
  std::vector<double> dZ((size_t)N * nx + nU), lamv((size_t)N * nx, 0.0), Xt(nX), Ut(nU);
  if (lam && prm->warm_lambda) std::memcpy(lamv.data(), lam, sizeof(double) * nX);
  int rc = 0;
  double rho = prm->rho;
  for (int it = 0; it < prm->sqp_iters; ++it) {
    orc_iter_log L;
    std::memset(&L, 0, sizeof(L));
    L.rho = rho;
    Lq lq = build_lq(*rb, *pr, rho, xs, qgoal, X, U);
    bool ok = lq.ok;
    if (prm->kkt_mode == 0) {
      ok = ok && solve_kkt_dense(lq, dZ.data(), lamv.data());
    } else if (prm->kkt_mode == 1) {
      Schur s = build_schur(lq);
      ok = ok && s.ok;
      if (!prm->warm_lambda) std::fill(lamv.begin(), lamv.end(), 0.0);
      bool hm = false;
      const int cap = prm->pcg_max_iter > 0 ? prm->pcg_max_iter : N * nx;
      L.pcg_iters = pcg(s, lamv.data(), prm->pcg_tol, cap, &hm, pcg_replay ? pcg_replay[it] : -1, &L.pcg_stop,
                        &L.pcg_stop_prev);
      if (hm) L.status |= ST_PCG_MAXITER;
      recover_step(lq, lamv.data(), dZ.data());
    } else {
      ok = ok && solve_riccati(lq, dZ.data(), lamv.data());
    }
    L.kkt_res = kkt_residual(lq, dZ.data(), lamv.data());
    if (!ok || !all_finite(dZ.data(), dZ.size())) {
      L.status |= ST_NONFINITE;
      if (log) log[it] = L;
      rc = 1;
      if (prm->rho_adapt) rho = std::min(2.0 * rho, 1e8);
      continue;
    }
    double J0, c0;
    cost_and_defect(*rb, *pr, xs, qgoal, X, U, &J0, &c0);
    L.merit0 = J0 + prm->mu * c0;
    int best = 0;
    double alpha = 1.0;
    for (int i = 0; i < prm->n_alpha; ++i) {
      const double a = std::pow(prm->beta, -(double)i);
      for (int k = 0; k < N; ++k)
        for (int j = 0; j < nx; ++j)
          Xt[(size_t)k * nx + j] = X[(size_t)k * nx + j] + a * dZ[off_x(lq, k) + j];
      for (int k = 0; k < N - 1; ++k)
        for (int j = 0; j < nu; ++j)
          Ut[(size_t)k * nu + j] = U[(size_t)k * nu + j] + a * dZ[off_u(lq, k) + j];
      double Jt, ct;
      cost_and_defect(*rb, *pr, xs, qgoal, Xt.data(), Ut.data(), &Jt, &ct);
      const double m = Jt + prm->mu * ct;
      L.merits[i] = m;
      if (i == 0 || m < L.merits[best]) { best = i; }
    }
    alpha = std::pow(prm->beta, -(double)best);
    L.argmin = best;
    if (alpha_replay) alpha = alpha_replay[it];
    if (!(L.merits[best] < L.merit0)) L.status |= ST_NO_DESCENT;
    for (int k = 0; k < N; ++k)
      for (int j = 0; j < nx; ++j) X[(size_t)k * nx + j] += alpha * dZ[off_x(lq, k) + j];
    for (int k = 0; k < N - 1; ++k)
      for (int j = 0; j < nu; ++j) U[(size_t)k * nu + j] += alpha * dZ[off_u(lq, k) + j];
    double J1, c1;
    cost_and_defect(*rb, *pr, xs, qgoal, X, U, &J1, &c1);
    L.alpha = alpha;
    L.J = J1;
    L.c1 = c1;
    L.merit = J1 + prm->mu * c1;
    if (L.status) rc = 1;
    if (log) log[it] = L;
    if (prm->rho_adapt) {
      const bool descent = descent_replay ? descent_replay[it] != 0 : !(L.status & ST_NO_DESCENT);
      rho = descent ? rho / 3.0 : std::min(2.0 * rho, 1e8);
    }
  }
  if (lam) std::memcpy(lam, lamv.data(), sizeof(double) * nX);
  return rc;
}

}  // extern "C"
