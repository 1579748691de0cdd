// Arithmetic counts of the per-knot rigid-body routines, obtained by running
// the same templates the kernels use on a counting scalar (host only). Used to
// report algorithmic FLOP rates: every +, -, *, / and sqrt counts one, sin and
// cos count one each, a fused multiply-add counts two.
#include <hip/hip_runtime.h>

#include "../../include/gato.h"

namespace {
thread_local long long g_flops = 0;

struct cf {
  float v;
  cf(float x = 0.f) : v(x) {}
};
inline cf operator+(cf a, cf b) { ++g_flops; return cf(a.v + b.v); }
inline cf operator-(cf a, cf b) { ++g_flops; return cf(a.v - b.v); }
inline cf operator*(cf a, cf b) { ++g_flops; return cf(a.v * b.v); }
inline cf operator/(cf a, cf b) { ++g_flops; return cf(a.v / b.v); }
inline cf operator-(cf a) { return cf(-a.v); }
inline cf operator*(float a, cf b) { ++g_flops; return cf(a * b.v); }
inline cf operator/(float a, cf b) { ++g_flops; return cf(a / b.v); }
}  // namespace

namespace gato {
inline void sin_cos(cf x, cf *s, cf *c);
inline bool positive(cf x);
inline cf sqrt_pos(cf x);
}  // namespace gato

#include "gato_rbd.hpp"

namespace gato {
inline void sin_cos(cf x, cf *s, cf *c) {
  g_flops += 2;
  *s = cf(sinf(x.v));
  *c = cf(cosf(x.v));
}
inline bool positive(cf x) { return x.v > 0.f; }
inline cf sqrt_pos(cf x) {
  ++g_flops;
  return cf(sqrtf(fmaxf(x.v, 1e-30f)));
}
}  // namespace gato

namespace {

template <int ND>
void count(const gato::Chain &ch, double *out) {
  cf q[ND], qd[ND], u[ND], qdd[ND], L[ND][ND], col[ND];
  for (int i = 0; i < ND; ++i) {
    q[i] = cf(0.1f * (i + 1));
    qd[i] = cf(0.05f * i);
    u[i] = cf(0.3f);
  }
  g_flops = 0;
  gato::forward_dynamics<ND, cf>(ch, q, qd, u, qdd, L);
  out[0] = (double)g_flops;
  g_flops = 0;
  gato::fd_jacobian_column<ND, cf>(ch, q, qd, qdd, L, 0, col);
  out[1] = (double)g_flops;
  g_flops = 0;
  gato::chol_solve<ND, cf>(L, col);
  out[2] = (double)g_flops;
}

}  // namespace

extern "C" int gato_rbd_flops(int n_dof, double *out) {
  if (!out) return GATO_EINVAL;
  gato::Chain ch{};
  ch.n = n_dof;
  ch.model = GATO_MODEL_SERIAL_CHAIN;
  ch.g = 9.81f;
  for (int i = 0; i < gato::kMaxDof; ++i) {
    ch.Lp[i] = i ? 0.3f : 0.f;
    ch.m[i] = 2.f;
    ch.cz[i] = 0.15f;
    ch.Io[i][0] = ch.Io[i][1] = ch.Io[i][2] = 0.05f;
  }
  switch (n_dof) {
    case 1: count<1>(ch, out); break;
    case 2: count<2>(ch, out); break;
    case 3: count<3>(ch, out); break;
    case 4: count<4>(ch, out); break;
    case 5: count<5>(ch, out); break;
    case 6: count<6>(ch, out); break;
    case 7: count<7>(ch, out); break;
    default: return GATO_EINVAL;
  }
  return GATO_OK;
}
