// Rigid-body dynamics of a revolute serial chain for one knot point, written in
// link-local spatial-vector form (6D motion/force vectors, Featherstone style).
//
// The paper computes "gradients and Hessians of the costs and dynamics
// functions across all problems and timesteps" with GRiD (Sec. III-A); that
// library is not used here. These routines give, per lane:
//   * inverse dynamics (recursive Newton-Euler), templated on the scalar so the
//     same code runs on plain floats and on forward-mode dual numbers,
//   * the joint-space inertia matrix (composite rigid bodies),
//   * forward dynamics qdd = M^-1 (tau - b) via an in-register Cholesky.
// Derivatives of forward dynamics follow from d/dx[ID(q, qd, FD(q, qd, u))] = 0:
// dqdd/dx = -M^-1 dID/dx at fixed qdd, with dID/dx from one dual-number RNEA
// pass per state direction.
//
// Chain convention: joint i rotates about z (even i) or y (odd i) of its own
// frame; frame i sits at length_{i-1} along +z of frame i-1 (frame 0 at the
// base origin); the centre of mass of link i is at length_i / 2 on +z with
// diagonal inertia (Ixx, Iyy, Izz) about it; gravity acts along -z of the base.
//
// Everything here is __host__ __device__ so that a CPU build can be checked
// without a GPU; the kernels include it for the device.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>

namespace gato {

constexpr int kMaxDof = 7;

// Per-solve chain parameters, pre-processed once per solve.
struct Chain {
  int n;          // degrees of freedom
  int model;      // 0 revolute chain, 1 spring-coupled unit masses
  float g;        // gravity magnitude
  float ks;       // spring stiffness (model 1)
  float Lp[kMaxDof];      // offset of joint i along +z of link i-1 (0 for i = 0)
  float m[kMaxDof];       // mass
  float cz[kMaxDof];      // centre-of-mass offset along +z
  float Io[kMaxDof][3];   // rotational inertia about the joint (diagonal)
  float Lt;               // offset of the tip along +z of the last link
  float fe[3];            // external force on the tip (base frame)
  int has_fe;             // fe is not zero
};

// ---------------------------------------------------------------------------
// Forward-mode dual number over a base scalar S: value + one tangent.
// ---------------------------------------------------------------------------
template <class S>
struct dual {
  S v, d;
};
template <class S> __host__ __device__ inline dual<S> operator+(dual<S> a, dual<S> b) { return {a.v + b.v, a.d + b.d}; }
template <class S> __host__ __device__ inline dual<S> operator-(dual<S> a, dual<S> b) { return {a.v - b.v, a.d - b.d}; }
template <class S> __host__ __device__ inline dual<S> operator-(dual<S> a) { return {-a.v, -a.d}; }
template <class S> __host__ __device__ inline dual<S> operator*(dual<S> a, dual<S> b) {
  return {a.v * b.v, a.d * b.v + a.v * b.d};
}
template <class S> __host__ __device__ inline dual<S> operator*(float s, dual<S> a) { return {s * a.v, s * a.d}; }
using df = dual<float>;

template <class T> struct base_of { using type = T; };
template <class S> struct base_of<dual<S>> { using type = S; };

template <class T> struct cst_impl {
  __host__ __device__ static T make(float x) { return T(x); }
};
template <class S> struct cst_impl<dual<S>> {
  __host__ __device__ static dual<S> make(float x) { return {S(x), S(0.f)}; }
};
template <class T> __host__ __device__ inline T cst(float x) { return cst_impl<T>::make(x); }

__host__ __device__ inline void sin_cos(float x, float *s, float *c) {
  *s = sinf(x);
  *c = cosf(x);
}
__host__ __device__ inline void sin_cos(double x, double *s, double *c) {
  *s = sin(x);
  *c = cos(x);
}
template <class S>
__host__ __device__ inline void sin_cos(dual<S> x, dual<S> *s, dual<S> *c) {
  S sv, cv;
  sin_cos(x.v, &sv, &cv);
  *s = {sv, x.d * cv};
  *c = {cv, -(x.d * sv)};
}

// ---------------------------------------------------------------------------
// Frame maps. Y selects the joint axis (false: z, true: y). R is the rotation of
// the child frame expressed in the parent frame; E = R^T maps parent
// coordinates into child coordinates.
// ---------------------------------------------------------------------------
template <bool Y, class T>
__host__ __device__ inline void rot_E(T c, T s, T &x, T &y, T &z) {  // a <- E a
  if (Y) {
    T nx = c * x - s * z, nz = s * x + c * z;
    x = nx; z = nz;
  } else {
    T nx = c * x + s * y, ny = c * y - s * x;
    x = nx; y = ny;
  }
}
template <bool Y, class T>
__host__ __device__ inline void rot_R(T c, T s, T &x, T &y, T &z) {  // a <- R a
  if (Y) {
    T nx = c * x + s * z, nz = c * z - s * x;
    x = nx; z = nz;
  } else {
    T nx = c * x - s * y, ny = s * x + c * y;
    x = nx; y = ny;
  }
}

// Motion vector (w, v) at the parent origin -> child frame; the child origin
// sits at r = (0, 0, L) in the parent: v_child = E (v - r x w).
template <bool Y, class T>
__host__ __device__ inline void motion_to_child(T c, T s, float L, T *w, T *v) {
  v[0] = v[0] + L * w[1];
  v[1] = v[1] - L * w[0];
  rot_E<Y>(c, s, w[0], w[1], w[2]);
  rot_E<Y>(c, s, v[0], v[1], v[2]);
}

// Force vector (n, f) at the child origin -> parent frame at the parent origin:
// f_p = R f, n_p = R n + r x f_p.
template <bool Y, class T>
__host__ __device__ inline void force_to_parent(T c, T s, float L, T *n, T *f) {
  rot_R<Y>(c, s, n[0], n[1], n[2]);
  rot_R<Y>(c, s, f[0], f[1], f[2]);
  n[0] = n[0] - L * f[1];
  n[1] = n[1] + L * f[0];
}

// ---------------------------------------------------------------------------
// Inverse dynamics (recursive Newton-Euler). Gravity is an upward acceleration
// of the base. ch.model == 1 gives tau = qdd + ks T q (T = tridiag(-1, 2, -1)).
// ---------------------------------------------------------------------------
// cq, sq: cos and sin of the joint angles (precomputed so that the
// trigonometric routines run before the recursion, with few values live).
template <int ND, class T>
__host__ __device__ inline void rnea(const Chain &ch, const T *q, const T *cq, const T *sq, const T *qd,
                                     const T *qdd, bool gravity, T *tau) {
  if (ch.model == 1) {
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      T s = 2.0f * q[i];
      if (i > 0) s = s - q[i - 1];
      if (i < ND - 1) s = s - q[i + 1];
      tau[i] = qdd[i] + ch.ks * s;
    }
    return;
  }
  T fn[ND][3], ff[ND][3];
  T w[3] = {cst<T>(0.f), cst<T>(0.f), cst<T>(0.f)};
  T v[3] = {cst<T>(0.f), cst<T>(0.f), cst<T>(0.f)};
  T aw[3] = {cst<T>(0.f), cst<T>(0.f), cst<T>(0.f)};
  T av[3] = {cst<T>(0.f), cst<T>(0.f), cst<T>(gravity ? ch.g : 0.f)};
#pragma unroll
  for (int i = 0; i < ND; ++i) {
    const float L = ch.Lp[i];
    if (i & 1) {
      motion_to_child<true>(cq[i], sq[i], L, w, v);
      motion_to_child<true>(cq[i], sq[i], L, aw, av);
      // v += S qd; a += S qdd + v x (S qd) with S = (e_y, 0)
      w[1] = w[1] + qd[i];
      aw[1] = aw[1] + qdd[i];
      aw[0] = aw[0] - w[2] * qd[i];
      aw[2] = aw[2] + w[0] * qd[i];
      av[0] = av[0] - v[2] * qd[i];
      av[2] = av[2] + v[0] * qd[i];
    } else {
      motion_to_child<false>(cq[i], sq[i], L, w, v);
      motion_to_child<false>(cq[i], sq[i], L, aw, av);
      // S = (e_z, 0)
      w[2] = w[2] + qd[i];
      aw[2] = aw[2] + qdd[i];
      aw[0] = aw[0] + w[1] * qd[i];
      aw[1] = aw[1] - w[0] * qd[i];
      av[0] = av[0] + v[1] * qd[i];
      av[1] = av[1] - v[0] * qd[i];
    }
    // Spatial inertia about the joint with the centre of mass at c = (0, 0, cz):
    // I (w, v) = (Io w + m c x v, m v - m c x w).
    const float m = ch.m[i], mc = ch.m[i] * ch.cz[i];
    const float Ix = ch.Io[i][0], Iy = ch.Io[i][1], Iz = ch.Io[i][2];
    T hvn[3] = {Ix * w[0] - mc * v[1], Iy * w[1] + mc * v[0], Iz * w[2]};
    T hvf[3] = {m * v[0] + mc * w[1], m * v[1] - mc * w[0], m * v[2]};
    T han[3] = {Ix * aw[0] - mc * av[1], Iy * aw[1] + mc * av[0], Iz * aw[2]};
    T haf[3] = {m * av[0] + mc * aw[1], m * av[1] - mc * aw[0], m * av[2]};
    // f = I a + v x* (I v), with v x* (hn, hf) = (w x hn + v x hf, w x hf)
    fn[i][0] = han[0] + (w[1] * hvn[2] - w[2] * hvn[1]) + (v[1] * hvf[2] - v[2] * hvf[1]);
    fn[i][1] = han[1] + (w[2] * hvn[0] - w[0] * hvn[2]) + (v[2] * hvf[0] - v[0] * hvf[2]);
    fn[i][2] = han[2] + (w[0] * hvn[1] - w[1] * hvn[0]) + (v[0] * hvf[1] - v[1] * hvf[0]);
    ff[i][0] = haf[0] + (w[1] * hvf[2] - w[2] * hvf[1]);
    ff[i][1] = haf[1] + (w[2] * hvf[0] - w[0] * hvf[2]);
    ff[i][2] = haf[2] + (w[0] * hvf[1] - w[1] * hvf[0]);
  }
#pragma unroll
  for (int i = ND - 1; i >= 0; --i) {
    tau[i] = (i & 1) ? fn[i][1] : fn[i][2];
    if (i > 0) {
      T n[3] = {fn[i][0], fn[i][1], fn[i][2]};
      T f[3] = {ff[i][0], ff[i][1], ff[i][2]};
      if (i & 1) force_to_parent<true>(cq[i], sq[i], ch.Lp[i], n, f);
      else force_to_parent<false>(cq[i], sq[i], ch.Lp[i], n, f);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        fn[i - 1][a] = fn[i - 1][a] + n[a];
        ff[i - 1][a] = ff[i - 1][a] + f[a];
      }
    }
  }
  if (ch.has_fe) {
    // External force f on the tip. The recursion is linear in the link
    // wrenches, so its share is a separate backward pass (after the link
    // wrenches above are dead): rotate f from the base into the last link's
    // frame, take the wrench the joints must supply against it at the last
    // joint, (-(r x f), -f) with r = (0, 0, Lt), and carry it to the base.
    T f[3] = {cst<T>(ch.fe[0]), cst<T>(ch.fe[1]), cst<T>(ch.fe[2])};
#pragma unroll
    for (int i = 0; i < ND; ++i) {
      if (i & 1) rot_E<true>(cq[i], sq[i], f[0], f[1], f[2]);
      else rot_E<false>(cq[i], sq[i], f[0], f[1], f[2]);
    }
    T wn[3] = {ch.Lt * f[1], -(ch.Lt * f[0]), cst<T>(0.f)};
    T wf[3] = {-f[0], -f[1], -f[2]};
#pragma unroll
    for (int i = ND - 1; i >= 0; --i) {
      tau[i] = tau[i] + ((i & 1) ? wn[1] : wn[2]);
      if (i > 0) {
        if (i & 1) force_to_parent<true>(cq[i], sq[i], ch.Lp[i], wn, wf);
        else force_to_parent<false>(cq[i], sq[i], ch.Lp[i], wn, wf);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Position of the tip (Lt along +z of the last link) in the base frame: the
// offset is carried from the last frame back to the base, one joint rotation
// and one link offset at a time. With T a dual number seeded on q_j it also
// gives column j of the tip Jacobian.
// ---------------------------------------------------------------------------
template <int ND, class T>
__host__ __device__ inline void tip_position(const Chain &ch, const T *q, T *p) {
  p[0] = cst<T>(0.f);
  p[1] = cst<T>(0.f);
  p[2] = cst<T>(ch.Lt);
#pragma unroll
  for (int i = ND - 1; i >= 0; --i) {
    T s, c;
    sin_cos(q[i], &s, &c);
    if (i & 1) rot_R<true>(c, s, p[0], p[1], p[2]);
    else rot_R<false>(c, s, p[0], p[1], p[2]);
    if (i > 0) p[2] = p[2] + cst<T>(ch.Lp[i]);
  }
}

// ---------------------------------------------------------------------------
// Joint-space inertia by composite rigid bodies. Each composite is kept as mass
// m, first moment h = m c and rotational inertia I (about the joint, symmetric,
// stored xx yy zz xy xz yz) in its own frame. Only the lower triangle is used
// by the Cholesky below, but the full matrix is written.
// ---------------------------------------------------------------------------
template <bool Y, class S>
__host__ __device__ inline void rotate_inertia(S c, S s, S *I) {
  // I <- R I R^T for R the rotation about the joint axis. Only the entries
  // that the rotation mixes are touched.
  if (Y) {
    // R = [[c, 0, s], [0, 1, 0], [-s, 0, c]]
    const S xx = I[0], yy = I[1], zz = I[2], xy = I[3], xz = I[4], yz = I[5];
    const S cc = c * c, ss = s * s, cs = c * s;
    I[0] = cc * xx + ss * zz + 2.f * (cs * xz);
    I[2] = ss * xx + cc * zz - 2.f * (cs * xz);
    I[4] = cs * (zz - xx) + (cc - ss) * xz;
    I[3] = c * xy + s * yz;
    I[5] = c * yz - s * xy;
    (void)yy;
  } else {
    // R = [[c, -s, 0], [s, c, 0], [0, 0, 1]]
    const S xx = I[0], yy = I[1], xy = I[3], xz = I[4], yz = I[5];
    const S cc = c * c, ss = s * s, cs = c * s;
    I[0] = cc * xx + ss * yy - 2.f * (cs * xy);
    I[1] = ss * xx + cc * yy + 2.f * (cs * xy);
    I[3] = cs * (xx - yy) + (cc - ss) * xy;
    I[4] = c * xz - s * yz;
    I[5] = s * xz + c * yz;
  }
}

template <int ND, class S>
__host__ __device__ inline void crba(const Chain &ch, const S *cq, const S *sq, S (*M)[ND]) {
  if (ch.model == 1) {
#pragma unroll
    for (int i = 0; i < ND; ++i)
#pragma unroll
      for (int j = 0; j < ND; ++j) M[i][j] = S((i == j) ? 1.f : 0.f);
    return;
  }
  S cm[ND], ch3[ND][3], cI[ND][6];
#pragma unroll
  for (int i = 0; i < ND; ++i) {
    cm[i] = S(ch.m[i]);
    ch3[i][0] = S(0.f); ch3[i][1] = S(0.f); ch3[i][2] = S(ch.m[i] * ch.cz[i]);
    cI[i][0] = S(ch.Io[i][0]); cI[i][1] = S(ch.Io[i][1]); cI[i][2] = S(ch.Io[i][2]);
    cI[i][3] = S(0.f); cI[i][4] = S(0.f); cI[i][5] = S(0.f);
  }
  // Accumulate composites towards the base.
#pragma unroll
  for (int i = ND - 1; i >= 1; --i) {
    S h[3] = {ch3[i][0], ch3[i][1], ch3[i][2]};
    S I[6] = {cI[i][0], cI[i][1], cI[i][2], cI[i][3], cI[i][4], cI[i][5]};
    if (i & 1) { rot_R<true>(cq[i], sq[i], h[0], h[1], h[2]); rotate_inertia<true>(cq[i], sq[i], I); }
    else { rot_R<false>(cq[i], sq[i], h[0], h[1], h[2]); rotate_inertia<false>(cq[i], sq[i], I); }
    // Shift from the child joint to the parent joint, r = (0, 0, L):
    // I += -m [r]^2 - [h][r] - [r][h], h += m r.
    const float L = ch.Lp[i];
    const S m = cm[i];
    const S t = (2.f * L) * h[2] + (L * L) * m;
    I[0] = I[0] + t;
    I[1] = I[1] + t;
    I[4] = I[4] - L * h[0];
    I[5] = I[5] - L * h[1];
    h[2] = h[2] + L * m;
    cm[i - 1] = cm[i - 1] + m;
#pragma unroll
    for (int a = 0; a < 3; ++a) ch3[i - 1][a] = ch3[i - 1][a] + h[a];
#pragma unroll
    for (int a = 0; a < 6; ++a) cI[i - 1][a] = cI[i - 1][a] + I[a];
  }
  // Column i: force of unit motion about joint i, carried towards the base.
#pragma unroll
  for (int i = 0; i < ND; ++i) {
    S n[3], f[3];
    if (i & 1) {  // e = e_y: n = I e_y, f = e_y x h
      n[0] = cI[i][3]; n[1] = cI[i][1]; n[2] = cI[i][5];
      f[0] = ch3[i][2]; f[1] = S(0.f); f[2] = -ch3[i][0];
      M[i][i] = n[1];
    } else {      // e = e_z
      n[0] = cI[i][4]; n[1] = cI[i][5]; n[2] = cI[i][2];
      f[0] = -ch3[i][1]; f[1] = ch3[i][0]; f[2] = S(0.f);
      M[i][i] = n[2];
    }
#pragma unroll
    for (int j = i; j >= 1; --j) {
      if (j & 1) force_to_parent<true>(cq[j], sq[j], ch.Lp[j], n, f);
      else force_to_parent<false>(cq[j], sq[j], ch.Lp[j], n, f);
      const S mij = ((j - 1) & 1) ? n[1] : n[2];
      M[i][j - 1] = mij;
      M[j - 1][i] = mij;
    }
  }
}

// In-place Cholesky of an SPD ND x ND matrix (lower triangle); returns false if
// a pivot is not positive.
__host__ __device__ inline bool positive(float x) { return x > 0.f; }
__host__ __device__ inline float sqrt_pos(float x) { return sqrtf(fmaxf(x, 1e-30f)); }
__host__ __device__ inline bool positive(double x) { return x > 0.0; }
__host__ __device__ inline double sqrt_pos(double x) { return sqrt(fmax(x, 1e-300)); }

template <int ND, class S>
__host__ __device__ inline bool cholesky(S (*A)[ND]) {
  bool ok = true;
#pragma unroll
  for (int j = 0; j < ND; ++j) {
    S s = A[j][j];
#pragma unroll
    for (int k = 0; k < j; ++k) s = s - A[j][k] * A[j][k];
    ok = ok && positive(s);
    const S d = sqrt_pos(s);
    const S inv = 1.f / d;
    A[j][j] = d;
#pragma unroll
    for (int i = j + 1; i < ND; ++i) {
      S t = A[i][j];
#pragma unroll
      for (int k = 0; k < j; ++k) t = t - A[i][k] * A[j][k];
      A[i][j] = t * inv;
    }
  }
  return ok;
}

template <int ND, class S>
__host__ __device__ inline void chol_solve(const S (*L)[ND], S *b) {
#pragma unroll
  for (int i = 0; i < ND; ++i) {
    S s = b[i];
#pragma unroll
    for (int k = 0; k < i; ++k) s = s - L[i][k] * b[k];
    b[i] = s / L[i][i];
  }
#pragma unroll
  for (int i = ND - 1; i >= 0; --i) {
    S s = b[i];
#pragma unroll
    for (int k = i + 1; k < ND; ++k) s = s - L[k][i] * b[k];
    b[i] = s / L[i][i];
  }
}

// Forward dynamics qdd = M(q)^-1 (tau - b(q, qd)). Leaves the Cholesky factor
// of M in L for later solves. Returns false if M is not positive definite.
template <int ND, class S>
__host__ __device__ inline bool forward_dynamics(const Chain &ch, const S *q, const S *qd, const S *tau, S *qdd,
                                                 S (*L)[ND]) {
  S cq[ND], sq[ND];
#pragma unroll
  for (int i = 0; i < ND; ++i) sin_cos(q[i], &sq[i], &cq[i]);
  crba<ND, S>(ch, cq, sq, L);
  S zero[ND], b[ND];
#pragma unroll
  for (int i = 0; i < ND; ++i) zero[i] = S(0.f);
  rnea<ND, S>(ch, q, cq, sq, qd, zero, true, b);
  const bool ok = cholesky<ND, S>(L);
#pragma unroll
  for (int i = 0; i < ND; ++i) qdd[i] = tau[i] - b[i];
  chol_solve<ND, S>(L, qdd);
  return ok;
}

// -dID/dx_dir at fixed qdd, by one dual-number RNEA pass: direction dir < ND
// is q_dir, dir >= ND is qd_(dir-ND).
template <int ND, class S>
__host__ __device__ inline void id_tangent(const Chain &ch, const S *q, const S *qd, const S *qdd, int dir,
                                           S *col) {
  S cv[ND], sv[ND];
#pragma unroll
  for (int i = 0; i < ND; ++i) sin_cos(q[i], &sv[i], &cv[i]);
  // Only joint `dir` carries an angle tangent: d sin = cos, d cos = -sin.
  dual<S> Q[ND], CQ[ND], SQ[ND], QD[ND], QDD[ND], TAU[ND];
#pragma unroll
  for (int i = 0; i < ND; ++i) {
    const bool on = (dir == i);
    Q[i] = {q[i], S(on ? 1.f : 0.f)};
    CQ[i] = {cv[i], on ? -sv[i] : S(0.f)};
    SQ[i] = {sv[i], on ? cv[i] : S(0.f)};
    QD[i] = {qd[i], S((dir == ND + i) ? 1.f : 0.f)};
    QDD[i] = {qdd[i], S(0.f)};
  }
  rnea<ND, dual<S>>(ch, Q, CQ, SQ, QD, QDD, true, TAU);
#pragma unroll
  for (int i = 0; i < ND; ++i) col[i] = -TAU[i].d;
}

// One column of the Jacobian of forward dynamics, dqdd/dx_dir = -M^-1 dID/dx_dir,
// using the Cholesky factor L and qdd from forward_dynamics.
template <int ND, class S>
__host__ __device__ inline void fd_jacobian_column(const Chain &ch, const S *q, const S *qd, const S *qdd,
                                                   const S (*L)[ND], int dir, S *col) {
  id_tangent<ND, S>(ch, q, qd, qdd, dir, col);
  chol_solve<ND, S>(L, col);
}

}  // namespace gato
