// Descriptors shared by the host library and the kernels (internal, not ABI).
#pragma once

#include <stdint.h>

#include "../../include/gato.h"
#include "gato_rbd.hpp"

namespace gato {

constexpr int kBlock = 512;        // threads per workgroup (one solve per workgroup)
constexpr int kMaxAlpha = GATO_MAX_ALPHA;

// Per-solve constants, built on the host at create time.
struct SolveDesc {
  Chain chain;
  int n;              // DoF
  int N;              // knot points
  int kpt;            // knots per lane group held in registers by the PCG phase
  int pad0;
  float dt;
  float Wq[16];       // stage state weights (diagonal of Q)
  float Wn[16];       // terminal weights (diagonal of Q_N)
  float Wr[8];        // control weights (diagonal of R)
  double Qd[16];      // diagonal of Q (the kernel forms 1 / (Q + rho) per iteration)
  double QNd[16];     // diagonal of Q_N
  double Ri[8];       // 1 / R
  float We[3], WeN[3];  // tip tracking weights (stages, last knot); task-space solves only
  int task;             // the solve has a tip tracking term
  int pad1;
  int64_t ws_off;     // byte offset of this solve's workspace
  int64_t offA, offB, offD, offT;  // byte offsets inside it: A_k, B_k and the inverse
                                   // diagonal blocks (float); Schur diagonal rows (double)
  int64_t offAT;                   // A_k^T (float), for column reads of A_k
  // Multi-CU split of a long solve (four knots per lane group, FP64 Schur):
  // bytes of one part's workspace (part j at ws_off + j ws_part) and the word
  // offset of the solve's exchange area, or -1 when the solve cannot split.
  int64_t ws_part;
  int64_t xch_off;
};

enum KernelMode { kModeSqp = 0, kModeLq = 1, kModeKkt = 2 };

// Split solves: parts per solve and 64-bit exchange words per solve.
constexpr int kSplitParts = 4;
constexpr int kXWordsPerSolve = kSplitParts * (8 * 104 + 1024);

struct KArgs {
  const SolveDesc *desc;
  char *ws;
  double *lam;               // [M][N_max][nx_max] warm-start multipliers
  const float *xs;
  const float *goal;
  float *X;
  float *U;
  int nx_max, nu_max, N_max;
  int iters;
  gato_solve_stats *stats;   // [M][iters] device, or null
  int stats_stride;
  double pcg_tol;
  int pcg_max_iter;
  float mu;
  float beta;
  int n_alpha;
  int warm;
  double *rho;               // [M] per-solve damping on every Q_k (read at start, written back if adapted)
  int rho_adapt;             // 1: rho /= 3 after an iteration with descent, rho *= 2 otherwise (cap 1e8)
  int fp64_inv;              // all-FP32 variant: FP64 Gauss-Jordan for the diagonal-block inverses
  int fp64_dot;              // all-FP32 variant: FP64 accumulation of the PCG inner products
  int mode;
  int M;                     // solves in the batch: solve indices from `order` outside 0..M-1 are skipped
  int sid_base;              // solve index of blockIdx.x == 0
  const int *order;          // optional block -> solve map (longest first), or null
  const float *pref;         // [M][N_max][3] reference tip positions (task-space kernels)
  // Stage entry points.
  const float *inA, *inB, *ine, *inq, *inr, *inc0;
  float *outA, *outB, *oute;
  float *outdX, *outdU;
  double *outlam;
  int *outits;
  unsigned long long *clk;    // optional [M][iters][8] phase timestamps (profiling)
  // Serving: xs, goal and stats indexed by workgroup (request) instead of
  // solve; the warm start is shifted by `shift` knots when it is loaded; the
  // final trajectories are also gathered per request into Xout / Uout.
  int by_block;
  int shift;
  float *Xout, *Uout;
  // Split launch (split = 4 or 2 parts per long solve, 0: none): `order` entries
  // carry the part in bits 24..31 and the solve in bits 0..23; the parts of a
  // solve exchange through `xch` under tags of this launch's `epoch`
  // (1..65535). All workgroups of such a launch are co-resident (cooperative
  // launch).
  int split;
  unsigned epoch;
  unsigned long long *xch;
  int xspin;                 // polls before a wait gives up (0: the default)
};

// Closed-loop plant step (gato_plant_step).
struct PlantArgs {
  const SolveDesc *desc;
  int M;                     // solves in the batch (slot bound)
  int n;                     // instances in this call
  const int *slots;          // [n] slot of each instance, or null (identity)
  const float *x;            // [n][nx_max]
  const float *tau;          // [n][nu_max]
  const float *fext;         // [n][3] external tip force per instance (base frame), or null: the slot's own
  float *xn;                 // [n][nx_max]
  unsigned *status;          // [n]
  int nx_max, nu_max;
  double h;
  int substeps;
};

}  // namespace gato
