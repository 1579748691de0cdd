// Host side of the C ABI declared in include/gato.h: argument validation,
// per-solve descriptors, workspace layout and kernel dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <deque>
#include <mutex>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/gato.h"
#include "gato_internal.hpp"
#include "gato_launch.hpp"

namespace gato {
hipError_t launch_sqp_n3(int kpt, bool f64, int grid, const KArgs &a, hipStream_t s);
hipError_t launch_sqp_n6(int kpt, bool f64, int grid, const KArgs &a, hipStream_t s);
hipError_t launch_sqp_n7(int kpt, bool f64, int grid, const KArgs &a, hipStream_t s);
hipError_t launch_sqp_mixed_f32(int grid, const KArgs &a, hipStream_t s);
hipError_t launch_sqp_mixed_f64(int grid, const KArgs &a, hipStream_t s);
hipError_t launch_sqp_n6_split(int grid, bool f64, const KArgs &a, hipStream_t s);
hipError_t launch_sqp_n7_split(int grid, bool f64, const KArgs &a, hipStream_t s);
hipError_t launch_sqp_mixed_f64_split(int grid, const KArgs &a, hipStream_t s);
hipError_t launch_sqp_mixed_f32_split(int grid, const KArgs &a, hipStream_t s);

hipError_t launch_sqp(int nd, int kpt, bool f64, int grid, const KArgs &a, hipStream_t s) {
  if (a.pref) return launch_sqp_task(nd, kpt, f64, grid, a, s);   // a batch with task-space solves
  switch (nd) {
    case 3: return launch_sqp_n3(kpt, f64, grid, a, s);
    case 6: return launch_sqp_n6(kpt, f64, grid, a, s);
    case 7: return launch_sqp_n7(kpt, f64, grid, a, s);
    default: return hipErrorInvalidValue;
  }
}
}  // namespace gato

using gato::SolveDesc;

namespace {

thread_local std::string g_err = "no error";

int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

int hip_fail(hipError_t e, const char *what) {
  return fail(e == hipErrorOutOfMemory ? GATO_ENOMEM : GATO_EDEVICE,
              std::string(what) + ": " + hipGetErrorString(e));
}

bool dof_supported(int n) { return n == 3 || n == 6 || n == 7; }

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t offA, offB, offD, offT, offAT, total;
};

Layout layout_for(int n, int N) {
  const size_t nx = 2 * (size_t)n, nu = (size_t)n;
  Layout l;
  l.offA = 0;
  l.offB = align256(l.offA + (size_t)(N - 1) * nx * nx * sizeof(float));
  l.offD = align256(l.offB + (size_t)(N - 1) * nx * nu * sizeof(float));
  l.offT = align256(l.offD + (size_t)N * nx * nx * sizeof(float));
  l.offAT = align256(l.offT + (size_t)N * nx * nx * sizeof(double));
  l.total = align256(l.offAT + (size_t)(N - 1) * nx * nx * sizeof(float));
  return l;
}

bool pos_finite(double x) { return std::isfinite(x) && x > 0.0; }

// Knots-per-group choices allowed for a solve of n DoF and N knots.
bool kpt_allowed(int n, int N, int kpt) {
  const int lo = gato::kpt_for(n, N);
  return lo > 0 && (kpt == 1 || kpt == 2 || kpt == 4) && kpt >= lo && kpt <= gato::kpt_max(n);
}

}  // namespace

struct gato_batch;
static int rebuild_dispatch(gato_batch *b);

namespace {

}  // namespace

struct gato_batch {
  int M = 0, n_max = 0, N_max = 0;
  gato_params p{};
  hipStream_t stream = nullptr;
  std::vector<SolveDesc> desc;
  SolveDesc *d_desc = nullptr;
  char *d_ws = nullptr;
  size_t ws_bytes = 0;
  double *d_lam = nullptr;   // [M][N_max][nx_max]
  size_t lam_bytes = 0;
  float *d_Xres = nullptr;   // device-resident trajectories for serving, [M][N_max][nx_max]
  float *d_Ures = nullptr;   // [M][N_max-1][nu_max]
  size_t xres_bytes = 0, ures_bytes = 0;
  gato_solve_stats *d_stats = nullptr;
  size_t stats_cap = 0;
  unsigned *d_plant_status = nullptr;  // [M], used when the caller passes none
  double *d_rho = nullptr;             // [M] per-solve damping
  bool task = false;                   // some solve has a tip tracking term (task-space kernels)
  bool task_long = false;              // ... and some solve is long (6-7 DoF, N > 64): it runs only split
  bool fe_on_device = false;           // tip forces were last set on the device (gato_select_hypotheses)
  float *d_pref = nullptr;             // [M][N_max][3] reference tip positions
  // Launch groups: solves of one (n, kpt) shape, longest horizon first.
  struct Group {
    int n, kpt, count;
    int *d_order;
    int *d_order_split[2];   // the same with four / two blocks per split solve (or null)
    int grid_split[2];
  };
  std::vector<Group> groups;
  int *d_order_all = nullptr;  // every solve, decreasing work (mixed-shape launch)
  // Split long solves (6-7 DoF, N > 64): four workgroups per solve
  // sharing the PCG through the exchange words, when the launch fits the chip.
  unsigned long long *d_xch = nullptr;
  size_t xwords = 0;             // exchange words of all split solves
  int n_split = 0;               // solves that can split
  int split_parts = gato::kSplitParts;   // gato_set_split: 4 (split where possible) or 1
  int split_polls = 0;                   // polls before a wait gives up (0: the kernel's default)
  unsigned epoch = 0;            // tag epoch of the last split launch (1..65535)
  int *d_order_split_all[2] = {nullptr, nullptr};   // four / two blocks per split solve
  int grid_split_all[2] = {0, 0};
  // Batches with long task-space solves: consecutive ranges (offset, length)
  // of the four-part order, each made of whole solves and resident on the
  // device at once; one cooperative launch per range.
  std::vector<std::pair<int, int>> task_chunks;
  int dispatch = GATO_DISPATCH_AUTO;
  std::vector<float> tuned_ms;  // per solve: the tuned time of its bucket (0 if never tuned)
  // Captured step (gato_step_graph).
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t graph = nullptr;
  std::vector<uintptr_t> graph_key;
  unsigned mapping_gen = 0;
};

// Brings the host copy of the descriptors' tip forces up to date after they
// were changed on the device, before the host copy is uploaded again.
static int pull_device_forces(gato_batch *b) {
  if (!b->fe_on_device) return GATO_OK;
  std::vector<SolveDesc> d(b->M);
  hipError_t e = b->stream ? hipStreamSynchronize(b->stream) : hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(d.data(), b->d_desc, b->M * sizeof(SolveDesc), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy(desc forces)");
  for (int i = 0; i < b->M; ++i) {
    for (int a = 0; a < 3; ++a) b->desc[i].chain.fe[a] = d[i].chain.fe[a];
    b->desc[i].chain.has_fe = d[i].chain.has_fe;
  }
  b->fe_on_device = false;
  return GATO_OK;
}

// Uploads the descriptors and rebuilds the launch groups and the decreasing-work
// order from b->desc (after create and after every mapping change).
static int rebuild_dispatch(gato_batch *b) {
  const int M = b->M;
  const auto &desc = b->desc;
  const int frc = pull_device_forces(b);
  if (frc != GATO_OK) return frc;
  hipError_t e = hipMemcpy(b->d_desc, desc.data(), M * sizeof(SolveDesc), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy(desc)");
  for (auto &g : b->groups) {
    if (g.d_order) (void)hipFree(g.d_order);
    for (int *o : g.d_order_split)
      if (o) (void)hipFree(o);
  }
  b->groups.clear();
  for (int q = 0; q < 2; ++q) {
    if (b->d_order_split_all[q]) (void)hipFree(b->d_order_split_all[q]);
    b->d_order_split_all[q] = nullptr;
    b->grid_split_all[q] = 0;
  }
  // A split solve takes `parts` consecutive blocks: the part in bits 24..31.
  auto expand = [&](const std::vector<int> &v, int parts) {
    std::vector<int> o;
    for (int i : v) {
      if (desc[i].xch_off >= 0 && desc[i].kpt == 4)
        for (int j = 0; j < parts; ++j) o.push_back(i | (j << 24));
      else
        o.push_back(i);
    }
    return o;
  };
  auto upload = [&](const std::vector<int> &v, int **dst) -> hipError_t {
    hipError_t e2 = hipMalloc((void **)dst, v.size() * sizeof(int));
    if (e2 != hipSuccess) return e2;
    return hipMemcpy(*dst, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice);
  };
  auto longer = [&](int x, int y) {
    const long wx = (long)desc[x].N * desc[x].n, wy = (long)desc[y].N * desc[y].n;
    return wx != wy ? wx > wy : desc[x].N > desc[y].N;
  };
  std::vector<int> all(M);
  for (int i = 0; i < M; ++i) all[i] = i;
  std::stable_sort(all.begin(), all.end(), longer);
  e = hipMemcpy(b->d_order_all, all.data(), M * sizeof(int), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy(order)");
  b->task_chunks.clear();
  if (b->n_split > 0) {
    for (int q = 0; q < 2; ++q) {
      const std::vector<int> xall = expand(all, q == 0 ? 4 : 2);
      e = upload(xall, &b->d_order_split_all[q]);
      if (e != hipSuccess) return hip_fail(e, "split order");
      b->grid_split_all[q] = (int)xall.size();
      if (q == 0 && b->task_long) {
        // The largest prefixes of whole solves that fit the device at once.
        int cap = 0;
        e = gato::cooperative_capacity(gato::sqp_mixed_task_split_fn(), &cap);
        if (e != hipSuccess) return hip_fail(e, "occupancy query");
        if (cap < gato::kSplitParts) return fail(GATO_EUNSUPPORTED, "the four parts of a long solve do not fit the device");
        int start = 0, len = 0;
        for (size_t t = 0; t < xall.size();) {
          const bool parts = ((unsigned)xall[t] >> 24) == 0 && desc[xall[t] & 0xffffff].xch_off >= 0 &&
                             desc[xall[t] & 0xffffff].kpt == 4;
          const int w = parts ? gato::kSplitParts : 1;   // a solve's consecutive entries
          if (len + w > cap) {
            b->task_chunks.push_back({start, len});
            start += len;
            len = 0;
          }
          len += w;
          t += w;
        }
        if (len > 0) b->task_chunks.push_back({start, len});
      }
    }
  }
  std::vector<std::vector<int>> members(64);
  for (int i : all) members[desc[i].n * 8 + desc[i].kpt].push_back(i);
  for (int key = 0; key < 64; ++key) {
    auto &v = members[key];
    if (v.empty()) continue;
    gato_batch::Group g{key / 8, key % 8, (int)v.size(), nullptr, {nullptr, nullptr}, {0, 0}};
    e = hipMalloc((void **)&g.d_order, v.size() * sizeof(int));
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(order)");
    for (int q = 0; q < 2 && b->n_split > 0; ++q) {
      const std::vector<int> xv = expand(v, q == 0 ? 4 : 2);
      if (xv.size() > v.size()) {
        e = upload(xv, &g.d_order_split[q]);
        if (e != hipSuccess) {
          (void)hipFree(g.d_order);
          for (int *o : g.d_order_split)
            if (o) (void)hipFree(o);
          return hip_fail(e, "split order");
        }
        g.grid_split[q] = (int)xv.size();
      }
    }
    b->groups.push_back(g);
    e = hipMemcpy(g.d_order, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy(order)");
  }
  ++b->mapping_gen;
  return GATO_OK;
}

extern "C" {

void gato_default_params(gato_params *p) {
  if (!p) return;
  p->sqp_iters = 10;
  p->pcg_tol = 1e-5;
  p->pcg_max_iter = 0;
  p->mu = 10.0;
  p->beta = 2.0;
  p->n_alpha = 8;
  p->rho = 0.0;
  p->rho_adapt = 0;
  p->schur_fp64 = 1;
  p->warm_lambda = 1;
  p->fp64_block_inv = 0;
  p->fp64_dot = 0;
}

const char *gato_last_error(void) { return g_err.c_str(); }

static int check_params(const gato_params *p) {
  if (p->sqp_iters < 0) return fail(GATO_EINVAL, "sqp_iters must be >= 0");
  if (!pos_finite(p->pcg_tol)) return fail(GATO_EINVAL, "pcg_tol must be positive and finite");
  if (p->pcg_max_iter < 0) return fail(GATO_EINVAL, "pcg_max_iter must be >= 0");
  if (!(std::isfinite(p->mu) && p->mu >= 0.0)) return fail(GATO_EINVAL, "mu must be >= 0");
  if (!(std::isfinite(p->beta) && p->beta > 1.0)) return fail(GATO_EINVAL, "beta must be > 1");
  if (p->n_alpha < 1 || p->n_alpha > GATO_MAX_ALPHA) return fail(GATO_EINVAL, "n_alpha must be in 1..16");
  if (!(std::isfinite(p->rho) && p->rho >= 0.0)) return fail(GATO_EINVAL, "rho must be >= 0");
  if (p->schur_fp64 != 0 && p->schur_fp64 != 1) return fail(GATO_EINVAL, "schur_fp64 must be 0 or 1");
  if (p->warm_lambda != 0 && p->warm_lambda != 1) return fail(GATO_EINVAL, "warm_lambda must be 0 or 1");
  if (p->fp64_block_inv != 0 && p->fp64_block_inv != 1) return fail(GATO_EINVAL, "fp64_block_inv must be 0 or 1");
  if (p->fp64_dot != 0 && p->fp64_dot != 1) return fail(GATO_EINVAL, "fp64_dot must be 0 or 1");
  if (p->rho_adapt != 0 && p->rho_adapt != 1) return fail(GATO_EINVAL, "rho_adapt must be 0 or 1");
  return GATO_OK;
}

size_t gato_workspace_bytes(int n_dof, int N, const gato_params *p) {
  if (!dof_supported(n_dof) || N < 2 || N > GATO_MAX_KNOTS) return 0;
  if (p && p->n_alpha > GATO_MAX_ALPHA) return 0;
  return layout_for(n_dof, N).total + (size_t)N * 2 * n_dof * sizeof(double) + sizeof(SolveDesc) +
         64 * sizeof(gato_solve_stats);
}

int gato_batch_create(int M, const gato_robot *robots, const gato_problem *probs, const gato_params *p,
                      void *hip_stream, gato_batch **out) {
  if (!out) return fail(GATO_EINVAL, "out is NULL");
  *out = nullptr;
  if (M < 1) return fail(GATO_EINVAL, "M must be >= 1");
  if (!robots || !probs) return fail(GATO_EINVAL, "robots and probs must not be NULL");
  gato_params prm;
  gato_default_params(&prm);
  if (p) prm = *p;
  int rc = check_params(&prm);
  if (rc != GATO_OK) return rc;

  std::vector<SolveDesc> desc(M);
  int n_max = 0, N_max = 0;
  for (int i = 0; i < M; ++i) {
    const gato_robot &r = robots[i];
    const gato_problem &q = probs[i];
    const std::string who = "solve " + std::to_string(i) + ": ";
    if (r.model != GATO_MODEL_SERIAL_CHAIN && r.model != GATO_MODEL_DOUBLE_INTEGRATOR)
      return fail(GATO_EINVAL, who + "unknown robot model");
    if (r.n_dof < 1 || r.n_dof > GATO_MAX_DOF) return fail(GATO_EINVAL, who + "n_dof must be in 1..7");
    if (!dof_supported(r.n_dof))
      return fail(GATO_EUNSUPPORTED, who + "n_dof " + std::to_string(r.n_dof) + " has no compiled kernel (3, 6, 7)");
    if (q.N < 2 || q.N > GATO_MAX_KNOTS) return fail(GATO_EINVAL, who + "N must be in 2..128");
    if (!pos_finite(q.dt)) return fail(GATO_EINVAL, who + "dt must be positive");
    if (!q.Q_diag || !q.R_diag || !q.QN_diag) return fail(GATO_EINVAL, who + "cost weights must not be NULL");
    const int n = r.n_dof, nx = 2 * n;
    for (int j = 0; j < nx; ++j)
      if (!pos_finite(q.Q_diag[j]) || !pos_finite(q.QN_diag[j]))
        return fail(GATO_EINVAL, who + "Q and Q_N must be positive");
    for (int j = 0; j < n; ++j)
      if (!pos_finite(q.R_diag[j])) return fail(GATO_EINVAL, who + "R must be positive");
    SolveDesc &d = desc[i];
    std::memset(&d, 0, sizeof(d));
    d.chain.n = n;
    d.chain.model = r.model;
    d.chain.g = (float)r.gravity;
    d.chain.ks = (float)r.spring_k;
    if (r.model == GATO_MODEL_SERIAL_CHAIN) {
      if (!r.link) return fail(GATO_EINVAL, who + "link parameters must not be NULL");
      if (!std::isfinite(r.gravity)) return fail(GATO_EINVAL, who + "gravity must be finite");
      for (int j = 0; j < n; ++j) {
        const double *l = r.link + 5 * j;
        if (!(std::isfinite(l[0]) && l[0] >= 0.0) || !pos_finite(l[1]) || !pos_finite(l[2]) ||
            !pos_finite(l[3]) || !pos_finite(l[4]))
          return fail(GATO_EINVAL, who + "link length must be >= 0 and mass/inertias > 0");
        const double cz = 0.5 * l[0];
        d.chain.Lp[j] = j > 0 ? (float)r.link[5 * (j - 1)] : 0.f;
        d.chain.m[j] = (float)l[1];
        d.chain.cz[j] = (float)cz;
        d.chain.Io[j][0] = (float)(l[2] + l[1] * cz * cz);
        d.chain.Io[j][1] = (float)(l[3] + l[1] * cz * cz);
        d.chain.Io[j][2] = (float)l[4];
      }
      d.chain.Lt = (float)r.link[5 * (n - 1)];
    } else if (!std::isfinite(r.spring_k)) {
      return fail(GATO_EINVAL, who + "spring_k must be finite");
    }
    d.n = n;
    d.N = q.N;
    d.kpt = gato::kpt_for(n, q.N);
    if (d.kpt == 0) return fail(GATO_EUNSUPPORTED, who + "no compiled mapping covers N = " + std::to_string(q.N));
    d.dt = (float)q.dt;
    for (int j = 0; j < nx; ++j) {
      d.Wq[j] = (float)q.Q_diag[j];
      d.Wn[j] = (float)q.QN_diag[j];
      d.Qd[j] = q.Q_diag[j];
      d.QNd[j] = q.QN_diag[j];
    }
    for (int j = 0; j < n; ++j) {
      d.Wr[j] = (float)q.R_diag[j];
      d.Ri[j] = 1.0 / q.R_diag[j];
    }
    if ((q.Wee_diag == nullptr) != (q.WeeN_diag == nullptr))
      return fail(GATO_EINVAL, who + "Wee_diag and WeeN_diag must both be set or both be NULL");
    if (q.Wee_diag) {
      if (r.model != GATO_MODEL_SERIAL_CHAIN) return fail(GATO_EINVAL, who + "tip tracking needs a serial chain");
      for (int c = 0; c < 3; ++c) {
        if (!(std::isfinite(q.Wee_diag[c]) && q.Wee_diag[c] >= 0.0) ||
            !(std::isfinite(q.WeeN_diag[c]) && q.WeeN_diag[c] >= 0.0))
          return fail(GATO_EINVAL, who + "tip weights must be finite and >= 0");
        d.We[c] = (float)q.Wee_diag[c];
        d.WeN[c] = (float)q.WeeN_diag[c];
      }
      d.task = 1;
    }
    n_max = std::max(n_max, n);
    N_max = std::max(N_max, q.N);
  }

  bool task = false, task_long = false;
  for (const auto &d : desc) task = task || d.task;
  for (int i = 0; i < M; ++i) {
    if (!task || desc[i].kpt <= gato::kTaskKptMax) continue;
    // Long solves of a batch with tip tracking run only as four parts of a
    // split launch (the part-local form is FP64).
    if (!prm.schur_fp64)
      return fail(GATO_EUNSUPPORTED, "solve " + std::to_string(i) +
                                         ": batches with tip tracking take N > 64 (6-7 DoF) with schur_fp64 = 1 only");
    task_long = true;
  }
  gato_batch *b = new gato_batch();
  b->M = M;
  b->task = task;
  b->task_long = task_long;
  b->n_max = n_max;
  b->N_max = N_max;
  b->p = prm;
  b->stream = (hipStream_t)hip_stream;
  size_t off = 0;
  int64_t xwords = 0;
  for (int i = 0; i < M; ++i) {
    const Layout l = layout_for(desc[i].n, desc[i].N);
    desc[i].ws_off = (int64_t)off;
    desc[i].offA = (int64_t)l.offA;
    desc[i].offB = (int64_t)l.offB;
    desc[i].offD = (int64_t)l.offD;
    desc[i].offT = (int64_t)l.offT;
    desc[i].offAT = (int64_t)l.offAT;
    // Long solves (four knots per lane group) can split: a workspace per part
    // and an exchange area.
    const bool can_split = desc[i].kpt == 4 && (!task || prm.schur_fp64);
    desc[i].ws_part = can_split ? (int64_t)l.total : 0;
    desc[i].xch_off = can_split ? xwords : -1;
    if (can_split) {
      xwords += gato::kXWordsPerSolve;
      ++b->n_split;
    }
    off += l.total * (can_split ? gato::kSplitParts : 1);
  }
  b->ws_bytes = off;
  b->xwords = (size_t)xwords;
  b->desc = desc;

  hipError_t e;
  b->tuned_ms.assign(M, 0.f);
  e = hipMalloc((void **)&b->d_desc, M * sizeof(SolveDesc));
  if (e != hipSuccess) { gato_batch_destroy(b); return hip_fail(e, "hipMalloc(desc)"); }
  e = hipMalloc((void **)&b->d_order_all, M * sizeof(int));
  if (e != hipSuccess) { gato_batch_destroy(b); return hip_fail(e, "hipMalloc(order)"); }
  if (xwords > 0) {
    e = hipMalloc((void **)&b->d_xch, (size_t)xwords * sizeof(unsigned long long));
    if (e != hipSuccess) { gato_batch_destroy(b); return hip_fail(e, "hipMalloc(exchange)"); }
    e = hipMemset(b->d_xch, 0, (size_t)xwords * sizeof(unsigned long long));
    if (e != hipSuccess) { gato_batch_destroy(b); return hip_fail(e, "hipMemset(exchange)"); }
  }
  rc = rebuild_dispatch(b);
  if (rc != GATO_OK) { gato_batch_destroy(b); return rc; }
  e = hipMalloc((void **)&b->d_ws, b->ws_bytes);
  if (e != hipSuccess) { gato_batch_destroy(b); return hip_fail(e, "hipMalloc(workspace)"); }
  e = hipMemset(b->d_ws, 0, b->ws_bytes);
  if (e != hipSuccess) { gato_batch_destroy(b); return hip_fail(e, "hipMemset(workspace)"); }
  b->lam_bytes = (size_t)M * N_max * 2 * n_max * sizeof(double);
  e = hipMalloc((void **)&b->d_lam, b->lam_bytes);
  if (e != hipSuccess) { gato_batch_destroy(b); return hip_fail(e, "hipMalloc(lambda)"); }
  e = hipMemset(b->d_lam, 0, b->lam_bytes);
  if (e != hipSuccess) { gato_batch_destroy(b); return hip_fail(e, "hipMemset(lambda)"); }
  b->xres_bytes = (size_t)M * N_max * 2 * n_max * sizeof(float);
  b->ures_bytes = (size_t)M * (N_max - 1) * n_max * sizeof(float);
  e = hipMalloc((void **)&b->d_Xres, b->xres_bytes);
  if (e != hipSuccess) { gato_batch_destroy(b); return hip_fail(e, "hipMalloc(resident X)"); }
  e = hipMalloc((void **)&b->d_Ures, b->ures_bytes);
  if (e != hipSuccess) { gato_batch_destroy(b); return hip_fail(e, "hipMalloc(resident U)"); }
  e = hipMalloc((void **)&b->d_plant_status, M * sizeof(unsigned));
  if (e != hipSuccess) { gato_batch_destroy(b); return hip_fail(e, "hipMalloc(plant status)"); }
  e = hipMalloc((void **)&b->d_rho, M * sizeof(double));
  if (e != hipSuccess) { gato_batch_destroy(b); return hip_fail(e, "hipMalloc(rho)"); }
  if (task) {
    const size_t pb = (size_t)M * N_max * 3 * sizeof(float);
    e = hipMalloc((void **)&b->d_pref, pb);
    if (e == hipSuccess) e = hipMemset(b->d_pref, 0, pb);
    if (e != hipSuccess) { gato_batch_destroy(b); return hip_fail(e, "hipMalloc(tip reference)"); }
  }
  {
    const std::vector<double> r0(M, prm.rho);
    e = hipMemcpy(b->d_rho, r0.data(), M * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) { gato_batch_destroy(b); return hip_fail(e, "hipMemcpy(rho)"); }
  }
  e = hipMemset(b->d_Xres, 0, b->xres_bytes);
  if (e == hipSuccess) e = hipMemset(b->d_Ures, 0, b->ures_bytes);
  if (e != hipSuccess) { gato_batch_destroy(b); return hip_fail(e, "hipMemset(resident X, U)"); }
  e = hipDeviceSynchronize();
  if (e != hipSuccess) { gato_batch_destroy(b); return hip_fail(e, "hipDeviceSynchronize"); }
  *out = b;
  return GATO_OK;
}

void gato_batch_destroy(gato_batch *b) {
  if (!b) return;
  // Every stream that may still run work on this batch's memory (the batch
  // stream, serving contexts' streams, the capture stream) is drained first;
  // then the objects that refer to the memory (the instantiated graph and its
  // capture stream) go before the memory itself.
  (void)hipDeviceSynchronize();
  if (b->graph) (void)hipGraphExecDestroy(b->graph);
  b->graph = nullptr;
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  b->cap_stream = nullptr;
  for (auto &g : b->groups) {
    if (g.d_order) (void)hipFree(g.d_order);
    for (int *o : g.d_order_split)
      if (o) (void)hipFree(o);
  }
  if (b->d_order_all) (void)hipFree(b->d_order_all);
  for (int *o : b->d_order_split_all)
    if (o) (void)hipFree(o);
  if (b->d_xch) (void)hipFree(b->d_xch);
  if (b->d_desc) (void)hipFree(b->d_desc);
  if (b->d_ws) (void)hipFree(b->d_ws);
  if (b->d_lam) (void)hipFree(b->d_lam);
  if (b->d_Xres) (void)hipFree(b->d_Xres);
  if (b->d_Ures) (void)hipFree(b->d_Ures);
  if (b->d_stats) (void)hipFree(b->d_stats);
  if (b->d_plant_status) (void)hipFree(b->d_plant_status);
  if (b->d_rho) (void)hipFree(b->d_rho);
  if (b->d_pref) (void)hipFree(b->d_pref);
  delete b;
}

int gato_batch_shape(const gato_batch *b, int *M, int *n_max, int *N_max) {
  if (!b) return fail(GATO_EINVAL, "batch is NULL");
  if (M) *M = b->M;
  if (n_max) *n_max = b->n_max;
  if (N_max) *N_max = b->N_max;
  return GATO_OK;
}

}  // extern "C"

namespace {

gato::KArgs base_args(gato_batch *b) {
  gato::KArgs a;
  std::memset(&a, 0, sizeof(a));
  a.desc = b->d_desc;
  a.M = b->M;
  a.ws = b->d_ws;
  a.lam = b->d_lam;
  a.nx_max = 2 * b->n_max;
  a.nu_max = b->n_max;
  a.N_max = b->N_max;
  a.pcg_tol = b->p.pcg_tol;
  a.pcg_max_iter = b->p.pcg_max_iter;
  a.mu = (float)b->p.mu;
  a.beta = (float)b->p.beta;
  a.n_alpha = b->p.n_alpha;
  a.warm = b->p.warm_lambda;
  a.rho = b->d_rho;
  a.rho_adapt = b->p.rho_adapt;
  a.fp64_inv = b->p.fp64_block_inv;
  a.fp64_dot = b->p.fp64_dot;
  a.pref = b->task ? b->d_pref : nullptr;
  return a;
}

bool use_mixed(const gato_batch *b) {
  return b->dispatch == GATO_DISPATCH_MIXED || (b->dispatch == GATO_DISPATCH_AUTO && b->groups.size() > 1);
}

hipError_t launch_mixed(const gato_batch *b, int grid, const gato::KArgs &a, hipStream_t s) {
  if (b->task) return gato::launch_sqp_mixed_task(grid, b->p.schur_fp64 != 0, a, s);
  return b->p.schur_fp64 ? gato::launch_sqp_mixed_f64(grid, a, s) : gato::launch_sqp_mixed_f32(grid, a, s);
}

// All solves of the batch: one mixed-shape launch over the decreasing-work
// order, or one launch per shape group. Long solves split across four
// workgroups (a cooperative launch), or two when four per solve would not fit
// the chip at once, unless `allow_split` is false (graph capture), the stream is
// under capture or the batch has it switched off; otherwise, and when even two
// do not fit, they run one workgroup each.
int launch_groups(gato_batch *b, gato::KArgs a, hipStream_t s, bool allow_split = true) {
  bool split = allow_split && a.mode == gato::kModeSqp && b->split_parts == gato::kSplitParts && b->n_split > 0;
  if (split) {
    // A stream under capture (the caller's own graph) takes the one-workgroup form.
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) split = false;
  }
  gato::KArgs as = a;
  if (split) {
    b->epoch = b->epoch % (gato::kGraphEpoch - 1u) + 1u;
    as.epoch = b->epoch;
    as.xch = b->d_xch;
    as.xspin = b->split_polls;
  }
  if (b->task_long) {
    // Long task-space solves have no one-workgroup kernel: the whole batch is
    // one split launch of the task-space mixed-shape kernel.
    if (!split)
      return fail(GATO_EUNSUPPORTED, "long solves with tip tracking run only split: not under stream capture "
                                     "(gato_step_graph builds the split launch)");
    // One cooperative launch per range of whole solves that fits the device.
    as.split = gato::kSplitParts;
    for (const auto &c : b->task_chunks) {
      as.order = b->d_order_split_all[0] + c.first;
      const hipError_t e = gato::launch_sqp_mixed_task_split(c.second, as, s);
      if (e != hipSuccess) return hip_fail(e, "kernel launch (split)");
    }
    return GATO_OK;
  }
  if (use_mixed(b)) {
    for (int q = 0; split && q < 2; ++q) {
      if (b->grid_split_all[q] <= b->M) continue;
      as.split = q == 0 ? 4 : 2;
      as.order = b->d_order_split_all[q];
      const hipError_t e = b->p.schur_fp64 ? gato::launch_sqp_mixed_f64_split(b->grid_split_all[q], as, s)
                                           : gato::launch_sqp_mixed_f32_split(b->grid_split_all[q], as, s);
      if (e == hipSuccess) return GATO_OK;
      if (e != hipErrorCooperativeLaunchTooLarge) return hip_fail(e, "kernel launch (split)");
      (void)hipGetLastError();
    }
    a.order = b->d_order_all;
    hipError_t e = launch_mixed(b, b->M, a, s);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return GATO_OK;
  }
  const bool f64 = b->p.schur_fp64 != 0;
  for (const auto &g : b->groups) {
    bool done = false;
    for (int q = 0; split && !done && q < 2 && (g.n == 6 || g.n == 7); ++q) {
      if (!g.d_order_split[q]) continue;
      as.split = q == 0 ? 4 : 2;
      as.order = g.d_order_split[q];
      const hipError_t e = g.n == 7 ? gato::launch_sqp_n7_split(g.grid_split[q], f64, as, s)
                                    : gato::launch_sqp_n6_split(g.grid_split[q], f64, as, s);
      if (e == hipSuccess) done = true;
      else if (e != hipErrorCooperativeLaunchTooLarge) return hip_fail(e, "kernel launch (split)");
      else (void)hipGetLastError();
    }
    if (done) continue;
    a.order = g.d_order;
    hipError_t e = gato::launch_sqp(g.n, g.kpt, f64, g.count, a, s);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
  }
  return GATO_OK;
}
int launch_groups(gato_batch *b, const gato::KArgs &a) { return launch_groups(b, a, b->stream); }

int check_io(gato_batch *b, const void *xs, const void *goal, const void *X, const void *U) {
  if (!b) return fail(GATO_EINVAL, "batch is NULL");
  if (!xs || !goal || !X || !U) return fail(GATO_EINVAL, "device buffers must not be NULL");
  return GATO_OK;
}

}  // namespace

extern "C" {

int gato_step(gato_batch *b, const float *d_xs, const float *d_goal, float *d_X, float *d_U, int n_iters,
              gato_solve_stats *d_stats) {
  int rc = check_io(b, d_xs, d_goal, d_X, d_U);
  if (rc) return rc;
  if (n_iters < 0) return fail(GATO_EINVAL, "n_iters must be >= 0");
  if (n_iters == 0) return GATO_OK;
  gato::KArgs a = base_args(b);
  a.xs = d_xs;
  a.goal = d_goal;
  a.X = d_X;
  a.U = d_U;
  a.iters = n_iters;
  a.stats = d_stats;
  a.stats_stride = n_iters;
  a.mode = gato::kModeSqp;
  return launch_groups(b, a);
}

int gato_step_plain(gato_batch *b, const float *d_xs, const float *d_goal, float *d_X, float *d_U, int n_iters,
                    gato_solve_stats *d_stats) {
  int rc = check_io(b, d_xs, d_goal, d_X, d_U);
  if (rc) return rc;
  if (n_iters < 0) return fail(GATO_EINVAL, "n_iters must be >= 0");
  if (n_iters == 0) return GATO_OK;
  gato::KArgs a = base_args(b);
  a.xs = d_xs;
  a.goal = d_goal;
  a.X = d_X;
  a.U = d_U;
  a.iters = n_iters;
  a.stats = d_stats;
  a.stats_stride = n_iters;
  a.mode = gato::kModeSqp;
  a.order = nullptr;
  const bool f64 = b->p.schur_fp64 != 0;
  for (int i = 0; i < b->M; ++i) {
    a.sid_base = i;
    hipError_t e = gato::launch_sqp(b->desc[i].n, b->desc[i].kpt, f64, 1, a, b->stream);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
  }
  return GATO_OK;
}

int gato_solve(gato_batch *b, const float *d_xs, const float *d_goal, float *d_X, float *d_U,
               gato_solve_stats *h_stats) {
  int rc = check_io(b, d_xs, d_goal, d_X, d_U);
  if (rc) return rc;
  const int iters = b->p.sqp_iters;
  if (iters == 0) return GATO_OK;
  gato_solve_stats *ds = nullptr;
  if (h_stats) {
    const size_t need = (size_t)b->M * iters;
    if (b->stats_cap < need) {
      if (b->d_stats) (void)hipFree(b->d_stats);
      b->d_stats = nullptr;
      b->stats_cap = 0;
      hipError_t e = hipMalloc((void **)&b->d_stats, need * sizeof(gato_solve_stats));
      if (e != hipSuccess) return hip_fail(e, "hipMalloc(stats)");
      b->stats_cap = need;
    }
    ds = b->d_stats;
  }
  rc = gato_step(b, d_xs, d_goal, d_X, d_U, iters, ds);
  if (rc) return rc;
  if (h_stats) {
    const size_t need = (size_t)b->M * iters;
    hipError_t e = hipMemcpyAsync(h_stats, ds, need * sizeof(gato_solve_stats), hipMemcpyDeviceToHost, b->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(stats)");
    e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    for (size_t i = 0; i < need; ++i)
      if (h_stats[i].status) return 1;
  }
  return GATO_OK;
}

int gato_profile_phases(gato_batch *b, const float *d_xs, const float *d_goal, float *d_X, float *d_U,
                        int n_iters, unsigned long long *d_clk) {
  int rc = check_io(b, d_xs, d_goal, d_X, d_U);
  if (rc) return rc;
  if (n_iters < 1 || !d_clk) return fail(GATO_EINVAL, "n_iters must be >= 1 and d_clk non-NULL");
  gato::KArgs a = base_args(b);
  a.xs = d_xs;
  a.goal = d_goal;
  a.X = d_X;
  a.U = d_U;
  a.iters = n_iters;
  a.mode = gato::kModeSqp;
  a.clk = d_clk;
  return launch_groups(b, a);
}

int gato_debug_lq(gato_batch *b, const float *d_xs, const float *d_goal, const float *d_X, const float *d_U,
                  float *d_A, float *d_B, float *d_e) {
  int rc = check_io(b, d_xs, d_goal, d_X, d_U);
  if (rc) return rc;
  if (!d_A || !d_B || !d_e) return fail(GATO_EINVAL, "output buffers must not be NULL");
  if (b->task) return fail(GATO_EUNSUPPORTED, "stage entry points take joint-space batches only");
  gato::KArgs a = base_args(b);
  a.xs = d_xs;
  a.goal = d_goal;
  a.X = const_cast<float *>(d_X);
  a.U = const_cast<float *>(d_U);
  a.iters = 1;
  a.mode = gato::kModeLq;
  a.outA = d_A;
  a.outB = d_B;
  a.oute = d_e;
  return launch_groups(b, a);
}

int gato_debug_kkt(gato_batch *b, const float *d_A, const float *d_B, const float *d_e, const float *d_q,
                   const float *d_r, const float *d_c0, float *d_dX, float *d_dU, double *d_lambda,
                   int *d_pcg_iters) {
  if (!b) return fail(GATO_EINVAL, "batch is NULL");
  if (!d_A || !d_B || !d_e || !d_q || !d_r || !d_c0 || !d_dX || !d_dU || !d_lambda)
    return fail(GATO_EINVAL, "buffers must not be NULL");
  if (b->task) return fail(GATO_EUNSUPPORTED, "stage entry points take joint-space batches only");
  gato::KArgs a = base_args(b);
  a.iters = 1;
  a.mode = gato::kModeKkt;
  a.warm = 0;
  a.inA = d_A;
  a.inB = d_B;
  a.ine = d_e;
  a.inq = d_q;
  a.inr = d_r;
  a.inc0 = d_c0;
  a.outdX = d_dX;
  a.outdU = d_dU;
  a.outlam = d_lambda;
  a.outits = d_pcg_iters;
  return launch_groups(b, a);
}

int gato_set_trajectories(gato_batch *b, const float *d_X, const float *d_U) {
  if (!b || !d_X || !d_U) return fail(GATO_EINVAL, "batch and buffers must not be NULL");
  hipError_t e = hipMemcpyAsync(b->d_Xres, d_X, b->xres_bytes, hipMemcpyDeviceToDevice, b->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(b->d_Ures, d_U, b->ures_bytes, hipMemcpyDeviceToDevice, b->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(trajectories in)");
  return GATO_OK;
}

int gato_get_trajectories(gato_batch *b, float *d_X, float *d_U) {
  if (!b || !d_X || !d_U) return fail(GATO_EINVAL, "batch and buffers must not be NULL");
  hipError_t e = hipMemcpyAsync(d_X, b->d_Xres, b->xres_bytes, hipMemcpyDeviceToDevice, b->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(d_U, b->d_Ures, b->ures_bytes, hipMemcpyDeviceToDevice, b->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(trajectories out)");
  return GATO_OK;
}

int gato_serve_step(gato_batch *b, int n_req, const int *d_slots, const float *d_xs, const float *d_goal,
                    int n_iters, int shift, float *d_Xout, float *d_Uout, gato_solve_stats *d_stats,
                    void *hip_stream) {
  if (!b) return fail(GATO_EINVAL, "batch is NULL");
  if (n_req < 1 || n_req > b->M) return fail(GATO_EINVAL, "n_req must be in 1..M");
  if (!d_slots || !d_xs || !d_goal) return fail(GATO_EINVAL, "slots, xs and goal must not be NULL");
  if (n_iters < 1) return fail(GATO_EINVAL, "n_iters must be >= 1");
  if (shift < 0 || shift > 1) return fail(GATO_EINVAL, "shift must be 0 or 1");
  if (b->task_long) return fail(GATO_EUNSUPPORTED, "serving takes no long solves with tip tracking (they run only split)");
  gato::KArgs a = base_args(b);
  a.xs = d_xs;
  a.goal = d_goal;
  a.X = b->d_Xres;
  a.U = b->d_Ures;
  a.iters = n_iters;
  a.stats = d_stats;
  a.stats_stride = n_iters;
  a.mode = gato::kModeSqp;
  a.order = d_slots;
  a.by_block = 1;
  a.shift = shift;
  a.Xout = d_Xout;
  a.Uout = d_Uout;
  hipStream_t st = hip_stream ? (hipStream_t)hip_stream : b->stream;
  hipError_t e = b->groups.size() == 1
                     ? gato::launch_sqp(b->groups[0].n, b->groups[0].kpt, b->p.schur_fp64 != 0, n_req, a, st)
                     : launch_mixed(b, n_req, a, st);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return GATO_OK;
}

}  // extern "C"

// A launch context of the serving loop: its own stream and completion event,
// pinned host staging that the caller fills and reads in place, and the
// device buffers of one launch.
struct gato_serve_ctx {
  gato_batch *b = nullptr;
  int cap = 0, n_iters = 0, n_last = 0;
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  int *h_slots = nullptr;            // pinned [cap]
  float *h_xs = nullptr, *h_goal = nullptr;      // pinned [cap][nx_max], [cap][nu_max]
  float *h_x1 = nullptr, *h_u0 = nullptr;        // pinned [cap][nx_max], [cap][nu_max]
  gato_solve_stats *h_stats = nullptr;           // pinned [cap][n_iters]
  int *d_slots = nullptr;
  float *d_xs = nullptr, *d_goal = nullptr, *d_X = nullptr, *d_U = nullptr;
  gato_solve_stats *d_stats = nullptr;
};

extern "C" {

void gato_serve_ctx_destroy(gato_serve_ctx *c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  for (void *p : {(void *)c->h_slots, (void *)c->h_xs, (void *)c->h_goal, (void *)c->h_x1, (void *)c->h_u0,
                  (void *)c->h_stats})
    if (p) (void)hipHostFree(p);
  for (void *p : {(void *)c->d_slots, (void *)c->d_xs, (void *)c->d_goal, (void *)c->d_X, (void *)c->d_U,
                  (void *)c->d_stats})
    if (p) (void)hipFree(p);
  if (c->done) (void)hipEventDestroy(c->done);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

int gato_serve_ctx_create(gato_batch *b, int capacity, int n_iters, gato_serve_ctx **out) {
  if (!out) return fail(GATO_EINVAL, "out is NULL");
  *out = nullptr;
  if (!b) return fail(GATO_EINVAL, "batch is NULL");
  if (capacity < 1 || capacity > b->M) return fail(GATO_EINVAL, "capacity must be in 1..M");
  if (n_iters < 1) return fail(GATO_EINVAL, "n_iters must be >= 1");
  gato_serve_ctx *c = new gato_serve_ctx();
  c->b = b;
  c->cap = capacity;
  c->n_iters = n_iters;
  const size_t nx = 2 * (size_t)b->n_max, nu = (size_t)b->n_max, N = (size_t)b->N_max, cap = (size_t)capacity;
  hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&c->done, hipEventDisableTiming);
  if (e == hipSuccess) e = hipHostMalloc((void **)&c->h_slots, cap * sizeof(int), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void **)&c->h_xs, cap * nx * sizeof(float), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void **)&c->h_goal, cap * nu * sizeof(float), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void **)&c->h_x1, cap * nx * sizeof(float), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void **)&c->h_u0, cap * nu * sizeof(float), hipHostMallocDefault);
  if (e == hipSuccess)
    e = hipHostMalloc((void **)&c->h_stats, cap * n_iters * sizeof(gato_solve_stats), hipHostMallocDefault);
  if (e == hipSuccess) e = hipMalloc((void **)&c->d_slots, cap * sizeof(int));
  if (e == hipSuccess) e = hipMalloc((void **)&c->d_xs, cap * nx * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void **)&c->d_goal, cap * nu * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void **)&c->d_X, cap * N * nx * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void **)&c->d_U, cap * (N - 1) * nu * sizeof(float));
  if (e == hipSuccess) e = hipMalloc((void **)&c->d_stats, cap * n_iters * sizeof(gato_solve_stats));
  if (e != hipSuccess) {
    gato_serve_ctx_destroy(c);
    return hip_fail(e, "serve context set-up");
  }
  std::memset(c->h_slots, 0, cap * sizeof(int));
  std::memset(c->h_xs, 0, cap * nx * sizeof(float));
  std::memset(c->h_goal, 0, cap * nu * sizeof(float));
  *out = c;
  return GATO_OK;
}

int gato_serve_ctx_buffers(gato_serve_ctx *c, int **h_slots, float **h_xs, float **h_goal, const float **h_x1,
                           const float **h_u0, const gato_solve_stats **h_stats) {
  if (!c) return fail(GATO_EINVAL, "context is NULL");
  if (h_slots) *h_slots = c->h_slots;
  if (h_xs) *h_xs = c->h_xs;
  if (h_goal) *h_goal = c->h_goal;
  if (h_x1) *h_x1 = c->h_x1;
  if (h_u0) *h_u0 = c->h_u0;
  if (h_stats) *h_stats = c->h_stats;
  return GATO_OK;
}

int gato_serve_ctx_submit(gato_serve_ctx *c, int n_req, int shift) {
  if (!c) return fail(GATO_EINVAL, "context is NULL");
  if (n_req < 1 || n_req > c->cap) return fail(GATO_EINVAL, "n_req must be in 1..capacity");
  gato_batch *b = c->b;
  const size_t nx = 2 * (size_t)b->n_max, nu = (size_t)b->n_max, N = (size_t)b->N_max, R = (size_t)n_req;
  for (int r = 0; r < n_req; ++r)
    if (c->h_slots[r] < 0 || c->h_slots[r] >= b->M) return fail(GATO_EINVAL, "slot outside 0..M-1");
  hipStream_t s = c->stream;
  hipError_t e = hipMemcpyAsync(c->d_slots, c->h_slots, R * sizeof(int), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->d_xs, c->h_xs, R * nx * sizeof(float), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(c->d_goal, c->h_goal, R * nu * sizeof(float), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(serve inputs)");
  const int rc = gato_serve_step(b, n_req, c->d_slots, c->d_xs, c->d_goal, c->n_iters, shift, c->d_X, c->d_U,
                                 c->d_stats, s);
  if (rc != GATO_OK) return rc;
  // The plant's next state x_1 and the control u_0 of every request, and its statistics.
  e = hipMemcpy2DAsync(c->h_x1, nx * sizeof(float), c->d_X + nx, N * nx * sizeof(float), nx * sizeof(float), R,
                       hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpy2DAsync(c->h_u0, nu * sizeof(float), c->d_U, (N - 1) * nu * sizeof(float), nu * sizeof(float), R,
                         hipMemcpyDeviceToHost, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->h_stats, c->d_stats, R * c->n_iters * sizeof(gato_solve_stats), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipEventRecord(c->done, s);
  if (e != hipSuccess) return hip_fail(e, "serve outputs");
  c->n_last = n_req;
  return GATO_OK;
}

int gato_serve_ctx_query(gato_serve_ctx *c) {
  if (!c) return fail(GATO_EINVAL, "context is NULL");
  const hipError_t e = hipEventQuery(c->done);
  if (e == hipSuccess) return 1;
  if (e == hipErrorNotReady) return 0;
  return hip_fail(e, "hipEventQuery");
}

int gato_serve_ctx_trajectories(gato_serve_ctx *c, float *h_X, float *h_U) {
  if (!c || !h_X || !h_U) return fail(GATO_EINVAL, "context and buffers must not be NULL");
  gato_batch *b = c->b;
  const size_t nx = 2 * (size_t)b->n_max, nu = (size_t)b->n_max, N = (size_t)b->N_max, R = (size_t)c->n_last;
  hipError_t e = hipMemcpyAsync(h_X, c->d_X, R * N * nx * sizeof(float), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h_U, c->d_U, R * (N - 1) * nu * sizeof(float), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) return hip_fail(e, "serve trajectories");
  return GATO_OK;
}

int gato_serve_run(gato_batch *b, int n_ctx, int n_iters, int R, const double *h_arrival_s, const int *h_instance,
                   const float *h_goal, float *h_state, int queue_limit, size_t memory_budget, double *h_latency_s,
                   double *h_launch_s, unsigned *h_status, float *h_u0, int *h_launches) {
  if (!b) return fail(GATO_EINVAL, "batch is NULL");
  if (n_ctx < 1 || n_ctx > 16) return fail(GATO_EINVAL, "n_ctx must be in 1..16");
  if (n_iters < 1) return fail(GATO_EINVAL, "n_iters must be >= 1");
  if (R < 0) return fail(GATO_EINVAL, "R must be >= 0");
  if (R > 0 && (!h_arrival_s || !h_instance || !h_goal || !h_latency_s || !h_status))
    return fail(GATO_EINVAL, "request arrays must not be NULL");
  if (!h_state) return fail(GATO_EINVAL, "state must not be NULL");
  for (int r = 0; r < R; ++r) {
    if (h_instance[r] < 0 || h_instance[r] >= b->M) return fail(GATO_EINVAL, "instance outside 0..M-1");
    if (!std::isfinite(h_arrival_s[r]) || (r > 0 && h_arrival_s[r] < h_arrival_s[r - 1]))
      return fail(GATO_EINVAL, "arrival times must be finite and ascending");
  }
  const int M = b->M, nx = 2 * b->n_max, nu = b->n_max;
  const size_t per_req = gato_workspace_bytes(b->n_max, b->N_max, &b->p);
  if (memory_budget > 0 && memory_budget < per_req)
    return fail(GATO_EINVAL, "memory_budget is below one request's workspace (nothing could launch)");
  std::vector<gato_serve_ctx *> ctx(n_ctx, nullptr);
  auto cleanup = [&]() {
    for (auto *c : ctx)
      if (c) gato_serve_ctx_destroy(c);
  };
  for (int i = 0; i < n_ctx; ++i) {
    const int rc = gato_serve_ctx_create(b, M, n_iters, &ctx[i]);
    if (rc != GATO_OK) { cleanup(); return rc; }
  }
  std::vector<std::deque<int>> fifo(M);
  std::deque<int> ready;
  std::vector<char> in_ready(M, 0), busy(M, 0);
  std::vector<std::vector<int>> launched(n_ctx);
  std::vector<double> t_launch(n_ctx, 0.0);
  std::vector<int> free_ctx;
  for (int i = n_ctx - 1; i >= 0; --i) free_ctx.push_back(i);
  size_t inflight_bytes = 0;
  int next = 0, waiting = 0, inflight = 0, launches = 0;
  for (int r = 0; r < R; ++r) {
    h_latency_s[r] = -1.0;
    h_status[r] = 0u;
    if (h_launch_s) h_launch_s[r] = -1.0;
  }
  auto make_ready = [&](int inst) {
    if (!busy[inst] && !in_ready[inst] && !fifo[inst].empty()) {
      ready.push_back(inst);
      in_ready[inst] = 1;
    }
  };
  const auto t0 = std::chrono::steady_clock::now();
  auto now = [&]() { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); };
  while (next < R || waiting > 0 || inflight > 0) {
    const double t = now();
    // 1. Admit arrivals.
    while (next < R && h_arrival_s[next] <= t) {
      if (queue_limit > 0 && waiting >= queue_limit) {
        h_status[next] = GATO_ST_ADMIT_REJECT;
      } else {
        fifo[h_instance[next]].push_back(next);
        ++waiting;
        make_ready(h_instance[next]);
      }
      ++next;
    }
    // 2. Retire finished launches.
    for (int c = 0; c < n_ctx; ++c) {
      if (launched[c].empty()) continue;
      const int q = gato_serve_ctx_query(ctx[c]);
      if (q < 0) { cleanup(); return q; }
      if (q == 0) continue;
      const double td = now();
      for (size_t j = 0; j < launched[c].size(); ++j) {
        const int r = launched[c][j], inst = h_instance[r];
        std::memcpy(h_state + (size_t)inst * nx, ctx[c]->h_x1 + j * nx, nx * sizeof(float));
        if (h_u0) std::memcpy(h_u0 + (size_t)r * nu, ctx[c]->h_u0 + j * nu, nu * sizeof(float));
        unsigned st = 0u;
        for (int it = 0; it < n_iters; ++it) st |= ctx[c]->h_stats[j * n_iters + it].status;
        h_status[r] = st;
        h_latency_s[r] = td - h_arrival_s[r];
        busy[inst] = 0;
        make_ready(inst);
      }
      inflight_bytes -= per_req * launched[c].size();
      launched[c].clear();
      --inflight;
      free_ctx.push_back(c);
    }
    // 3. Launch the oldest request of every ready instance while a context is free.
    if (!free_ctx.empty() && !ready.empty()) {
      size_t room = ready.size();
      if (memory_budget > 0 && per_req > 0)
        room = std::min(room, memory_budget > inflight_bytes ? (memory_budget - inflight_bytes) / per_req : 0);
      if (room > 0) {
        const int c = free_ctx.back();
        free_ctx.pop_back();
        gato_serve_ctx *cx = ctx[c];
        const int n = (int)std::min(room, (size_t)M);
        for (int j = 0; j < n; ++j) {
          const int inst = ready.front();
          ready.pop_front();
          in_ready[inst] = 0;
          const int r = fifo[inst].front();
          fifo[inst].pop_front();
          busy[inst] = 1;
          cx->h_slots[j] = inst;
          std::memcpy(cx->h_xs + (size_t)j * nx, h_state + (size_t)inst * nx, nx * sizeof(float));
          std::memcpy(cx->h_goal + (size_t)j * nu, h_goal + (size_t)r * nu, nu * sizeof(float));
          launched[c].push_back(r);
        }
        waiting -= n;
        const double tl = now();
        for (int r : launched[c])
          if (h_launch_s) h_launch_s[r] = tl;
        const int rc = gato_serve_ctx_submit(cx, n, 1);
        if (rc != GATO_OK) { cleanup(); return rc; }
        inflight_bytes += per_req * n;
        ++inflight;
        ++launches;
        continue;
      }
    }
  }
  cleanup();
  if (h_launches) *h_launches = launches;
  return GATO_OK;
}

int gato_reset_warm_start(gato_batch *b) {
  if (!b) return fail(GATO_EINVAL, "batch is NULL");
  hipError_t e = gato::launch_fill(b->d_lam, b->lam_bytes / sizeof(double), 0.0, b->stream);
  if (e != hipSuccess) return hip_fail(e, "kernel launch (fill)");
  return GATO_OK;
}

int gato_get_multipliers(gato_batch *b, double *d_lam) {
  if (!b || !d_lam) return fail(GATO_EINVAL, "batch and buffer must not be NULL");
  hipError_t e = hipMemcpyAsync(d_lam, b->d_lam, b->lam_bytes, hipMemcpyDeviceToDevice, b->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(multipliers out)");
  return GATO_OK;
}

int gato_set_multipliers(gato_batch *b, const double *d_lam) {
  if (!b || !d_lam) return fail(GATO_EINVAL, "batch and buffer must not be NULL");
  hipError_t e = hipMemcpyAsync(b->d_lam, d_lam, b->lam_bytes, hipMemcpyDeviceToDevice, b->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(multipliers in)");
  return GATO_OK;
}

int gato_shift_warm_start(gato_batch *b, const int *d_slots, int n, void *hip_stream) {
  if (!b || !d_slots) return fail(GATO_EINVAL, "batch and slots must not be NULL");
  if (n < 1 || n > b->M) return fail(GATO_EINVAL, "n must be in 1..M");
  hipError_t e = gato::launch_shift(b->d_desc, b->M, n, d_slots, b->N_max, 2 * b->n_max, b->n_max, b->d_Xres,
                                    b->d_Ures, b->d_lam, hip_stream ? (hipStream_t)hip_stream : b->stream);
  if (e != hipSuccess) return hip_fail(e, "kernel launch (shift)");
  return GATO_OK;
}

int gato_plant_step(gato_batch *b, int n, const int *d_slots, const float *d_x, const float *d_tau,
                    const float *d_fext, double h, int substeps, float *d_xn, unsigned *d_status,
                    void *hip_stream) {
  if (!b) return fail(GATO_EINVAL, "batch is NULL");
  if (n < 1 || n > b->M) return fail(GATO_EINVAL, "n must be in 1..M");
  if (!d_x || !d_tau || !d_xn) return fail(GATO_EINVAL, "x, tau and xn must not be NULL");
  if (!pos_finite(h)) return fail(GATO_EINVAL, "h must be positive");
  if (substeps < 1 || substeps > 100000) return fail(GATO_EINVAL, "substeps must be in 1..100000");
  gato::PlantArgs a;
  a.desc = b->d_desc;
  a.M = b->M;
  a.n = n;
  a.slots = d_slots;
  a.x = d_x;
  a.tau = d_tau;
  a.fext = d_fext;
  a.xn = d_xn;
  a.status = d_status ? d_status : b->d_plant_status;
  a.nx_max = 2 * b->n_max;
  a.nu_max = b->n_max;
  a.h = h;
  a.substeps = substeps;
  hipError_t e = gato::launch_plant(a, hip_stream ? (hipStream_t)hip_stream : b->stream);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return GATO_OK;
}

int gato_tip_positions(gato_batch *b, const float *d_X, float *d_p, void *hip_stream) {
  if (!b || !d_X || !d_p) return fail(GATO_EINVAL, "batch and buffers must not be NULL");
  hipError_t e = gato::launch_tips(b->d_desc, b->M, b->N_max, 2 * b->n_max, d_X, d_p,
                                   hip_stream ? (hipStream_t)hip_stream : b->stream);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return GATO_OK;
}

int gato_set_tip_reference(gato_batch *b, const float *d_pref) {
  if (!b || !d_pref) return fail(GATO_EINVAL, "batch and reference must not be NULL");
  if (!b->task) return fail(GATO_EINVAL, "the batch has no tip tracking term");
  const size_t pb = (size_t)b->M * b->N_max * 3 * sizeof(float);
  hipError_t e = hipMemcpyAsync(b->d_pref, d_pref, pb, hipMemcpyDeviceToDevice, b->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(tip reference)");
  return GATO_OK;
}

int gato_set_external_force(gato_batch *b, const double *h_f) {
  if (!b || !h_f) return fail(GATO_EINVAL, "batch and forces must not be NULL");
  for (int i = 0; i < 3 * b->M; ++i)
    if (!std::isfinite(h_f[i])) return fail(GATO_EINVAL, "forces must be finite");
  for (int i = 0; i < b->M; ++i)
    if (b->desc[i].chain.model != GATO_MODEL_SERIAL_CHAIN &&
        (h_f[3 * i] != 0.0 || h_f[3 * i + 1] != 0.0 || h_f[3 * i + 2] != 0.0))
      return fail(GATO_EINVAL, "external forces apply to serial chains only");
  hipError_t e = b->stream ? hipStreamSynchronize(b->stream) : hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "synchronize");
  for (int i = 0; i < b->M; ++i) {
    gato::Chain &c = b->desc[i].chain;
    for (int a = 0; a < 3; ++a) c.fe[a] = (float)h_f[3 * i + a];
    c.has_fe = (c.fe[0] != 0.f || c.fe[1] != 0.f || c.fe[2] != 0.f) ? 1 : 0;
  }
  e = hipMemcpy(b->d_desc, b->desc.data(), b->M * sizeof(SolveDesc), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy(desc)");
  b->fe_on_device = false;
  return GATO_OK;
}

int gato_select_hypotheses(gato_batch *b, int P, int H, const float *d_pred, const float *d_meas, const double *d_off,
                           double *d_est, int *d_sel, double *d_dist, void *hip_stream) {
  if (!b) return fail(GATO_EINVAL, "batch is NULL");
  if (P < 1 || H < 1 || (long)P * H != b->M) return fail(GATO_EINVAL, "P and H must be >= 1 with P H = M");
  if (!d_pred || !d_meas || !d_off || !d_est) return fail(GATO_EINVAL, "device buffers must not be NULL");
  for (int p = 0; p < P; ++p)
    for (int j = 0; j < H; ++j) {
      const SolveDesc &d = b->desc[(size_t)p * H + j];
      if (d.chain.model != GATO_MODEL_SERIAL_CHAIN)
        return fail(GATO_EINVAL, "external forces apply to serial chains only");
      if (d.n != b->desc[(size_t)p * H].n) return fail(GATO_EINVAL, "the solves of an instance must share the robot");
    }
  hipStream_t s = hip_stream ? (hipStream_t)hip_stream : b->stream;
  const hipError_t e = gato::launch_select(b->d_desc, P, H, 2 * b->n_max, d_pred, d_meas, d_off, d_est, d_sel, d_dist, s);
  if (e != hipSuccess) return hip_fail(e, "kernel launch (hypothesis selection)");
  b->fe_on_device = true;
  return GATO_OK;
}

int gato_set_rho(gato_batch *b, const double *h_rho) {
  if (!b || !h_rho) return fail(GATO_EINVAL, "batch and rho must not be NULL");
  for (int i = 0; i < b->M; ++i)
    if (!(std::isfinite(h_rho[i]) && h_rho[i] >= 0.0)) return fail(GATO_EINVAL, "rho must be finite and >= 0");
  hipError_t e = b->stream ? hipStreamSynchronize(b->stream) : hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(b->d_rho, h_rho, b->M * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy(rho)");
  return GATO_OK;
}

int gato_get_rho(gato_batch *b, double *h_rho) {
  if (!b || !h_rho) return fail(GATO_EINVAL, "batch and rho must not be NULL");
  hipError_t e = b->stream ? hipStreamSynchronize(b->stream) : hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(h_rho, b->d_rho, b->M * sizeof(double), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy(rho)");
  return GATO_OK;
}

int gato_set_split(gato_batch *b, int parts, int max_polls) {
  if (!b) return fail(GATO_EINVAL, "batch is NULL");
  if (parts != 1 && parts != gato::kSplitParts) return fail(GATO_EINVAL, "parts must be 1 or 4");
  if (max_polls < 0) return fail(GATO_EINVAL, "max_polls must be >= 0");
  if (parts == 1 && b->task_long) return fail(GATO_EUNSUPPORTED, "long solves with tip tracking run only split");
  b->split_parts = parts;
  b->split_polls = max_polls;
  return GATO_OK;
}

int gato_set_dispatch(gato_batch *b, int mode) {
  if (!b) return fail(GATO_EINVAL, "batch is NULL");
  if (mode != GATO_DISPATCH_AUTO && mode != GATO_DISPATCH_GROUPED && mode != GATO_DISPATCH_MIXED)
    return fail(GATO_EINVAL, "unknown dispatch mode");
  b->dispatch = mode;
  ++b->mapping_gen;
  return GATO_OK;
}

int gato_buckets(const gato_batch *b, gato_bucket *out, int cap, int *n_out) {
  if (!b || !n_out || (cap > 0 && !out)) return fail(GATO_EINVAL, "batch, n_out or out is NULL");
  std::vector<gato_bucket> v;
  for (int i = 0; i < b->M; ++i) {
    const SolveDesc &d = b->desc[i];
    auto it = std::find_if(v.begin(), v.end(), [&](const gato_bucket &x) { return x.n_dof == d.n && x.N == d.N; });
    if (it == v.end()) v.push_back(gato_bucket{d.n, d.N, 1, d.kpt, b->tuned_ms[i]});
    else ++it->count;
  }
  std::sort(v.begin(), v.end(), [](const gato_bucket &x, const gato_bucket &y) {
    return x.n_dof != y.n_dof ? x.n_dof < y.n_dof : x.N < y.N;
  });
  *n_out = (int)v.size();
  for (int i = 0; i < (int)v.size() && i < cap; ++i) out[i] = v[i];
  return GATO_OK;
}

int gato_set_mapping(gato_batch *b, int n_dof, int N, int kpt) {
  if (!b) return fail(GATO_EINVAL, "batch is NULL");
  if (!kpt_allowed(n_dof, N, kpt)) return fail(GATO_EINVAL, "kpt must be 1, 2 or 4 and cover N");
  if (b->task && kpt > gato::kTaskKptMax && gato::kpt_for(n_dof, N) <= gato::kTaskKptMax)
    return fail(GATO_EUNSUPPORTED, "tip tracking kernels are compiled for kpt 1 and 2 (4: only N > 64, split)");
  bool any = false;
  for (auto &d : b->desc)
    if (d.n == n_dof && d.N == N) {
      d.kpt = kpt;
      any = true;
    }
  if (!any) return fail(GATO_EINVAL, "no solve of this (n_dof, N) in the batch");
  hipError_t e = b->stream ? hipStreamSynchronize(b->stream) : hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "synchronize");
  return rebuild_dispatch(b);
}

int gato_autotune(gato_batch *b, const float *d_xs, const float *d_goal, const float *d_X, const float *d_U,
                  int n_iters, int reps) {
  int rc = check_io(b, d_xs, d_goal, d_X, d_U);
  if (rc) return rc;
  if (n_iters < 1 || reps < 1) return fail(GATO_EINVAL, "n_iters and reps must be >= 1");
  hipStream_t s = b->stream;
  rc = pull_device_forces(b);
  if (rc != GATO_OK) return rc;
  hipError_t e = s ? hipStreamSynchronize(s) : hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "synchronize");
  // Buckets of (n, N) and their members.
  std::vector<std::pair<int, int>> keys;
  std::vector<std::vector<int>> mem;
  for (int i = 0; i < b->M; ++i) {
    const auto key = std::make_pair(b->desc[i].n, b->desc[i].N);
    auto it = std::find(keys.begin(), keys.end(), key);
    if (it == keys.end()) {
      keys.push_back(key);
      mem.push_back({i});
    } else {
      mem[it - keys.begin()].push_back(i);
    }
  }
  float *X = nullptr, *U = nullptr;
  int *order = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  auto cleanup = [&]() {
    if (X) (void)hipFree(X);
    if (U) (void)hipFree(U);
    if (order) (void)hipFree(order);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  e = hipMalloc((void **)&X, b->xres_bytes);
  if (e == hipSuccess) e = hipMalloc((void **)&U, b->ures_bytes);
  if (e == hipSuccess) e = hipMalloc((void **)&order, b->M * sizeof(int));
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) { cleanup(); return hip_fail(e, "autotune set-up"); }
  gato::KArgs a = base_args(b);
  a.xs = d_xs;
  a.goal = d_goal;
  a.X = X;
  a.U = U;
  a.iters = n_iters;
  a.mode = gato::kModeSqp;
  a.order = order;
  for (size_t k = 0; k < keys.size(); ++k) {
    const int n = keys[k].first, N = keys[k].second;
    auto &v = mem[k];
    // Long task-space solves have one mapping (four knots per lane group, split).
    if (b->task && gato::kpt_for(n, N) > gato::kTaskKptMax) continue;
    std::stable_sort(v.begin(), v.end());
    e = hipMemcpy(order, v.data(), v.size() * sizeof(int), hipMemcpyHostToDevice);
    if (e != hipSuccess) { cleanup(); return hip_fail(e, "hipMemcpy(order)"); }
    int best = 0;
    float best_ms = 0.f;
    for (int kpt : {1, 2, 4}) {
      if (!kpt_allowed(n, N, kpt) || (b->task && kpt > gato::kTaskKptMax)) continue;
      for (int i : v) b->desc[i].kpt = kpt;
      e = hipMemcpy(b->d_desc, b->desc.data(), b->M * sizeof(SolveDesc), hipMemcpyHostToDevice);
      if (e != hipSuccess) { cleanup(); return hip_fail(e, "hipMemcpy(desc)"); }
      std::vector<float> ms;
      for (int r = 0; r <= reps; ++r) {
        e = hipMemcpyAsync(X, d_X, b->xres_bytes, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(U, d_U, b->ures_bytes, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = gato::launch_fill(b->d_lam, b->lam_bytes / sizeof(double), 0.0, s);
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        if (e == hipSuccess) e = launch_mixed(b, (int)v.size(), a, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
        if (e != hipSuccess) { cleanup(); return hip_fail(e, "autotune run"); }
        if (r > 0) ms.push_back(t);
      }
      std::sort(ms.begin(), ms.end());
      const float med = ms[ms.size() / 2];
      if (best == 0 || med < best_ms) {
        best = kpt;
        best_ms = med;
      }
    }
    for (int i : v) {
      b->desc[i].kpt = best;
      b->tuned_ms[i] = best_ms;
    }
  }
  cleanup();
  e = gato::launch_fill(b->d_lam, b->lam_bytes / sizeof(double), 0.0, s);
  if (e == hipSuccess) e = s ? hipStreamSynchronize(s) : hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "autotune clean-up");
  return rebuild_dispatch(b);
}

}  // extern "C"

namespace {

// The step of a mixed-shape batch with split long solves as an explicit graph:
// a kernel node that clears the exchange words, then the split kernel as a
// cooperative kernel node (its workgroups resident together), or, for long
// task-space solves, one such node per range of whole solves that fits the
// device, in sequence. *out stays null when the split does not apply (the
// launch does not fit the device, or the runtime refuses the cooperative
// attribute); the caller then captures the one-workgroup form.
int build_split_graph(gato_batch *b, const gato::KArgs &a, hipGraph_t *out) {
  *out = nullptr;
  if (b->split_parts != gato::kSplitParts || b->n_split == 0) return GATO_OK;
  if (b->task ? !b->task_long : !use_mixed(b)) return GATO_OK;
  const void *fn = b->task ? gato::sqp_mixed_task_split_fn()
                           : (b->p.schur_fp64 ? gato::sqp_mixed_f64_split_fn() : gato::sqp_mixed_f32_split_fn());
  for (int q = 0; q < (b->task ? 1 : 2); ++q) {
    const int grid = b->grid_split_all[q];
    if (grid <= b->M) continue;
    std::vector<std::pair<int, int>> ranges;
    if (b->task) {
      ranges = b->task_chunks;
    } else {
      const hipError_t e = gato::cooperative_fits(fn, grid);
      if (e == hipErrorCooperativeLaunchTooLarge) continue;
      if (e != hipSuccess) return hip_fail(e, "occupancy query");
      ranges.push_back({0, grid});
    }
    gato::KArgs as = a;
    as.split = q == 0 ? 4 : 2;
    as.epoch = gato::kGraphEpoch;
    as.xch = b->d_xch;
    as.xspin = b->split_polls;
    hipGraph_t g = nullptr;
    hipError_t e = hipGraphCreate(&g, 0);
    if (e != hipSuccess) return hip_fail(e, "hipGraphCreate");
    double *fp = reinterpret_cast<double *>(b->d_xch);
    size_t fn_words = b->xwords;
    double fv = 0.0;
    void *fargs[] = {&fp, &fn_words, &fv};
    hipKernelNodeParams fparams;
    std::memset(&fparams, 0, sizeof(fparams));
    fparams.func = const_cast<void *>(gato::fill_kernel_fn());
    fparams.gridDim = dim3((unsigned)((fn_words + 255) / 256));
    fparams.blockDim = dim3(256);
    fparams.kernelParams = fargs;
    hipGraphNode_t prev = nullptr;
    e = hipGraphAddKernelNode(&prev, g, nullptr, 0, &fparams);
    bool refused = false;
    for (size_t r = 0; e == hipSuccess && r < ranges.size(); ++r) {
      as.order = b->d_order_split_all[q] + ranges[r].first;
      void *kargs[] = {&as};   // (the node copies its arguments when it is added)
      hipKernelNodeParams kparams;
      std::memset(&kparams, 0, sizeof(kparams));
      kparams.func = const_cast<void *>(fn);
      kparams.gridDim = dim3(ranges[r].second);
      kparams.blockDim = dim3(gato::kBlock);
      kparams.kernelParams = kargs;
      hipGraphNode_t n_sqp = nullptr;
      e = hipGraphAddKernelNode(&n_sqp, g, &prev, 1, &kparams);
      if (e != hipSuccess) break;
      hipLaunchAttributeValue coop;
      std::memset(&coop, 0, sizeof(coop));
      coop.cooperative = 1;
      if (hipGraphKernelNodeSetAttribute(n_sqp, hipKernelNodeAttributeCooperative, &coop) != hipSuccess) {
        (void)hipGetLastError();
        refused = true;
        break;
      }
      prev = n_sqp;
    }
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return hip_fail(e, "hipGraphAddKernelNode");
    }
    if (refused) {
      (void)hipGraphDestroy(g);
      if (b->task_long) return fail(GATO_EUNSUPPORTED, "the runtime refuses a cooperative graph node (long solves "
                                                       "with tip tracking run only split)");
      return GATO_OK;
    }
    *out = g;
    return GATO_OK;
  }
  return GATO_OK;
}

}  // namespace

extern "C" {

int gato_step_graph(gato_batch *b, const float *d_xs, const float *d_goal, float *d_X, float *d_U, int n_iters,
                    gato_solve_stats *d_stats) {
  int rc = check_io(b, d_xs, d_goal, d_X, d_U);
  if (rc) return rc;
  if (n_iters < 0) return fail(GATO_EINVAL, "n_iters must be >= 0");
  if (n_iters == 0) return GATO_OK;
  const std::vector<uintptr_t> key = {(uintptr_t)d_xs, (uintptr_t)d_goal, (uintptr_t)d_X, (uintptr_t)d_U,
                                      (uintptr_t)n_iters, (uintptr_t)d_stats, (uintptr_t)b->mapping_gen};
  hipError_t e;
  if (!b->graph || key != b->graph_key) {
    if (b->graph) {
      e = b->stream ? hipStreamSynchronize(b->stream) : hipDeviceSynchronize();
      if (e != hipSuccess) return hip_fail(e, "synchronize");
      (void)hipGraphExecDestroy(b->graph);
      b->graph = nullptr;
    }
    if (!b->cap_stream) {
      e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
    }
    gato::KArgs a = base_args(b);
    a.xs = d_xs;
    a.goal = d_goal;
    a.X = d_X;
    a.U = d_U;
    a.iters = n_iters;
    a.stats = d_stats;
    a.stats_stride = n_iters;
    a.mode = gato::kModeSqp;
    hipGraph_t g = nullptr;
    rc = build_split_graph(b, a, &g);
    if (rc != GATO_OK) return rc;
    if (!g) {
      e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
      rc = launch_groups(b, a, b->cap_stream, false);
      e = hipStreamEndCapture(b->cap_stream, &g);
      if (rc != GATO_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    }
    e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      b->graph = nullptr;
      return hip_fail(e, "hipGraphInstantiate");
    }
    b->graph_key = key;
  }
  e = hipGraphLaunch(b->graph, b->stream);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  return GATO_OK;
}
}  // extern "C"

// ---- Allocation-free gato_solve (gato_solve_static). The device staging of the
// per-iteration statistics is this file-scope array instead of a buffer the
// batch allocates on demand; each device holds its own copy for the life of
// the process. Host code never passes `scratch` itself to a kernel or a copy
// (in host code the name is a stand-in, not a device address): it uses the
// address hipGetSymbolAddress returns for the current device.
namespace {

constexpr size_t kScratchStats = GATO_STATIC_STATS_MAX;
constexpr size_t kScratchBytes = kScratchStats * sizeof(gato_solve_stats);
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device (looked up once per device).
int scratch_address(void **out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(GATO_EDEVICE, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GATO_OK;
}

}  // namespace

extern "C" {

int gato_solve_static(gato_batch *b, const float *d_xs, const float *d_goal, float *d_X, float *d_U,
                      gato_solve_stats *h_stats) {
  int rc = check_io(b, d_xs, d_goal, d_X, d_U);
  if (rc) return rc;
  const int iters = b->p.sqp_iters;
  if (iters == 0) return GATO_OK;
  const size_t need = (size_t)b->M * iters;
  if (h_stats && need > kScratchStats)
    return fail(GATO_EINVAL, "M * sqp_iters = " + std::to_string(need) + " exceeds the static statistics staging (" +
                                 std::to_string(kScratchStats) + " entries)");
  gato_solve_stats *ds = nullptr;
  if (h_stats) {
    void *p = nullptr;
    rc = scratch_address(&p);
    if (rc != GATO_OK) return rc;
    ds = static_cast<gato_solve_stats *>(p);
    // The staging keeps the previous call's contents: clear the part this call uses.
    static_assert(sizeof(gato_solve_stats) % sizeof(double) == 0, "statistics are whole doubles");
    const hipError_t e = gato::launch_fill(reinterpret_cast<double *>(ds),
                                           need * sizeof(gato_solve_stats) / sizeof(double), 0.0, b->stream);
    if (e != hipSuccess) return hip_fail(e, "kernel launch (clear statistics staging)");
  }
  rc = gato_step(b, d_xs, d_goal, d_X, d_U, iters, ds);
  if (rc) return rc;
  if (h_stats) {
    hipError_t e = hipMemcpyAsync(h_stats, ds, need * sizeof(gato_solve_stats), hipMemcpyDeviceToHost, b->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(stats)");
    e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
    for (size_t i = 0; i < need; ++i)
      if (h_stats[i].status) return 1;
  }
  return GATO_OK;
}

}  // extern "C"
