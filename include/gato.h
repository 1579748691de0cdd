/*
 * gato.h - C ABI of the MI355X (gfx950) batched trajectory-optimisation library.
 *
 * The library runs the data-parallel hot path of GATO (Du, Adabag,
 * Bravo-Palacios, Plancher, arXiv 2510.07625): SQP iterations over a batch of M
 * independent trajectory optimisation problems, each iteration forming the QP
 * of Eq. (1) from the rigid-body dynamics at every knot point, reducing its KKT
 * system (Eq. (2)) to the block-tridiagonal Schur complement of Eqs. (4)-(6),
 * solving it with the stair-preconditioned conjugate gradient (Sec. II-B,
 * Sec. III-B), recovering the step (Eq. (4)) and choosing it with the L1-merit
 * line search of Eqs. (3) and (7) (Algorithm 1).
 *
 * Conventions shared by every entry point:
 *   - Sizes: n = DoF (1..GATO_MAX_DOF), nx = 2n (state [q; qd]), nu = n
 *     (joint torques). N counts knot points: states x_0..x_{N-1} and controls
 *     u_0..u_{N-2} (the paper's x_0..x_N has N+1 states; here N is the number
 *     of states).
 *   - Device buffers (d_*) are caller-owned device pointers (e.g. torch
 *     data_ptr()), float32, row-major, padded per solve to the batch maxima:
 *       X     [M][N_max][nx_max]     U   [M][N_max-1][nu_max]
 *       xs    [M][nx_max]            goal[M][nu_max]  (joint-angle goal)
 *     nx_max = 2 n_max, nu_max = n_max. Entries beyond a solve's own n / N are
 *     neither read nor written.
 *   - Ordering: every call is stream-ordered on the HIP stream given at create
 *     time and returns before the GPU finishes, except where stated.
 *   - Errors: functions return an int status (GATO_OK or a negative code) and
 *     never throw; gato_last_error() gives a message for the calling thread.
 *     Per-solve numerical trouble sets status bits and never fails the batch.
 *   - A batch handle is not thread-safe; calls on one handle must not overlap.
 */
#ifndef GATO_H
#define GATO_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define GATO_OK 0
#define GATO_EINVAL (-1)       /* invalid argument; nothing was launched */
#define GATO_ENOMEM (-2)       /* device allocation failed */
#define GATO_EDEVICE (-3)      /* HIP runtime error (launch, copy, sync) */
#define GATO_EUNSUPPORTED (-4) /* shape outside the compiled kernels */

/* Per-solve status bits (gato_solve_stats.status). */
#define GATO_ST_PCG_MAXITER 1u /* PCG hit its iteration cap before the tolerance */
#define GATO_ST_NONFINITE 2u   /* non-finite step or merit; the iterate was kept */
#define GATO_ST_NO_DESCENT 4u  /* no candidate step lowered the merit (stepped anyway) */
#define GATO_ST_ADMIT_REJECT 8u /* serving: the request was refused at admission (queue full) */
#define GATO_ST_EXCHANGE 16u    /* split solve: a wait for another part gave up (result invalid) */

/* Robot models. */
#define GATO_MODEL_SERIAL_CHAIN 0        /* revolute chain, joint axes z, y, z, y, ... */
#define GATO_MODEL_DOUBLE_INTEGRATOR 1   /* unit masses, qdd = u - k T q, T = tridiag(-1, 2, -1) */

#define GATO_MAX_DOF 7
#define GATO_MAX_KNOTS 128
#define GATO_MAX_ALPHA 16

typedef struct gato_batch gato_batch; /* opaque, library-owned */

/*
 * Robot description (host memory, copied at create time).
 * Serial chain: joint i rotates about z (even i) or y (odd i) of its own frame;
 * frame i sits at length_{i-1} along +z of frame i-1; link i has its centre of
 * mass at length_i/2 on +z and diagonal inertia (Ixx, Iyy, Izz) about it;
 * gravity acts along -z of the base. Stands in for the manipulators of Sec. IV.
 */
typedef struct {
  int model;           /* GATO_MODEL_* */
  int n_dof;           /* 1..GATO_MAX_DOF */
  const double *link;  /* [n_dof][5]: length, mass, Ixx, Iyy, Izz (serial chain) */
  double gravity;      /* m/s^2 along -z (serial chain) */
  double spring_k;     /* k (double integrator) */
} gato_robot;

/*
 * One problem of Eq. (1): horizon, Euler time step h and the diagonal tracking
 * weights Q (stages 0..N-2), R and Q_N (knot N-1). The tracked state is
 * [q_goal; 0]. Host memory, copied at create time.
 *
 * Optional task-space term (the end-effector tracking of the paper's
 * experiments, Sec. IV): with Wee_diag and WeeN_diag both non-NULL, knot k
 * also costs 1/2 (p(q_k) - pref_k)^T diag(W) (p(q_k) - pref_k), p the position
 * of the tip of the last link in the base frame, W = Wee_diag for k < N-1 and
 * WeeN_diag at the last knot, pref set with gato_set_tip_reference (zero until
 * then). The QP uses the exact gradient and the Gauss-Newton Hessian J^T W J
 * of this term, so each Q_k gets a dense joint block. Serial chains only; a
 * batch with such a term runs the task-space kernels for all its solves (no
 * stage entry points). Its long solves (6-7 DoF, N > 64) run only on four
 * workgroups each (see gato_set_split), which needs schur_fp64 = 1 (otherwise
 * gato_batch_create returns GATO_EUNSUPPORTED); a step of such a batch is one
 * cooperative launch per range of whole solves that fits the device (one
 * workgroup per short solve, four per long one), and the batch takes no
 * serving steps. Both NULL: no such term
 * (zero-initialise the struct).
 */
typedef struct {
  int N;               /* knot points, 2..GATO_MAX_KNOTS */
  double dt;           /* time step h > 0 */
  const double *Q_diag;  /* [2 n_dof], > 0 */
  const double *R_diag;  /* [n_dof], > 0 */
  const double *QN_diag; /* [2 n_dof], > 0 */
  const double *Wee_diag;  /* [3], >= 0, or NULL */
  const double *WeeN_diag; /* [3], >= 0, or NULL */
} gato_problem;

/*
 * Solver settings. The paper defers its values to its code; the defaults set
 * by gato_default_params are: sqp_iters 10, pcg_tol 1e-5, pcg_max_iter 0
 * (= N nx), mu 10, beta 2, n_alpha 8 (alpha_i = beta^-i, i = 0..7), rho 0,
 * schur_fp64 1, warm_lambda 1, fp64_block_inv 0, fp64_dot 0, rho_adapt 0.
 *
 * Precision: with schur_fp64 = 1 the Schur rows, gamma~, the diagonal-block
 * inverses, the PCG vectors and inner products are FP64 (preconditioner blocks
 * stored in FP32, applied in FP64; dynamics, line search and trajectories in
 * FP32). With schur_fp64 = 0 all of it is FP32, and two toggles move single
 * pieces to FP64: fp64_block_inv (the Gauss-Jordan inversion of the diagonal
 * blocks; the blocks themselves are formed in FP32) and fp64_dot (the
 * accumulation of the PCG inner products). The toggles are ignored when
 * schur_fp64 = 1.
 */
typedef struct {
  int sqp_iters;       /* SQP iterations per gato_solve */
  double pcg_tol;      /* PCG stops when r^T P r <= tol^2 gamma^T P gamma */
  int pcg_max_iter;    /* 0: N * nx */
  double mu;           /* merit weight on ||c||_1, Eq. (3) */
  double beta;         /* > 1, Eq. (7) */
  int n_alpha;         /* candidate steps, 1..GATO_MAX_ALPHA */
  double rho;          /* added to the diagonal of every Q_k (incl. Q_N) in the QP
                          Hessian; the initial per-solve value (see gato_set_rho) */
  int schur_fp64;      /* 1: Schur complement, PCG vectors and dot products in
                          FP64; 0: all FP32 (see the toggles below) */
  int warm_lambda;     /* 1: PCG starts from the solve's previous multipliers (previous SQP
                          iteration, or the previous call's last); 0: from zero */
  int fp64_block_inv;  /* schur_fp64 = 0 only: FP64 diagonal-block inversion */
  int fp64_dot;        /* schur_fp64 = 0 only: FP64 PCG inner-product accumulation */
  int rho_adapt;       /* 1: after each SQP iteration a solve's rho is divided by 3
                          if its line search lowered the merit and doubled (at most
                          1e8) otherwise, as the case study of Sec. IV-C adjusts
                          rho from the line-search status */
} gato_params;

/* Per solve and SQP iteration. */
typedef struct {
  float merit0;        /* merit at the iterate before the step */
  float merit;         /* merit of the accepted candidate */
  float alpha;         /* accepted step */
  int pcg_iters;       /* PCG iterations of this SQP iteration */
  unsigned status;     /* GATO_ST_* bits */
  float rho;           /* damping used in this iteration */
} gato_solve_stats;

/* Fills *p with the defaults listed above. */
void gato_default_params(gato_params *p);

/*
 * Device workspace one solve of this shape needs (bytes). Pure host
 * computation; usable for memory-based admission. Returns 0 for invalid input.
 */
size_t gato_workspace_bytes(int n_dof, int N, const gato_params *p);

/*
 * Creates a batch of M solves (Algorithm 1's M). robots[M] and probs[M] are
 * host arrays; solves may differ in n_dof and N (an uneven batch is launched
 * as one persistent kernel). p may be NULL for the defaults. hip_stream is a
 * hipStream_t (NULL: the null stream). Allocates and zeroes the device
 * workspace (including the per-solve PCG warm-start multipliers) and
 * synchronises. On success *out owns everything until gato_batch_destroy.
 * Errors: GATO_EINVAL (sizes, weights, NULL pointers), GATO_ENOMEM,
 * GATO_EDEVICE.
 */
int gato_batch_create(int M, const gato_robot *robots, const gato_problem *probs, const gato_params *p,
                      void *hip_stream, gato_batch **out);

/*
 * Frees all device memory of the batch. Synchronises the whole device first
 * (work of serving contexts on their own streams may still use the batch),
 * then releases the captured graph, then the memory. Serving contexts of the
 * batch must not be used afterwards. NULL is ignored.
 */
void gato_batch_destroy(gato_batch *b);

/* Number of solves, and the padded maxima n_max, N_max of the batch. */
int gato_batch_shape(const gato_batch *b, int *M, int *n_max, int *N_max);

/*
 * Algorithm 1: runs p->sqp_iters SQP iterations on every solve. d_X / d_U hold
 * the initial trajectories on entry and X*, U* on exit (in place); d_xs and
 * d_goal hold each solve's start state and joint goal. If h_stats is non-NULL
 * it receives [M][sqp_iters] per-iteration statistics and the call
 * synchronises; otherwise the call is asynchronous. Returns GATO_OK, or 1 if
 * some solve set a status bit (only known when h_stats is given).
 */
int gato_solve(gato_batch *b, const float *d_xs, const float *d_goal, float *d_X, float *d_U,
               gato_solve_stats *h_stats);

/*
 * Asynchronous form of gato_solve with a caller-chosen iteration count and
 * device-side statistics: d_stats (device, [M][n_iters] gato_solve_stats, or
 * NULL). No host synchronisation and no host I/O.
 */
int gato_step(gato_batch *b, const float *d_xs, const float *d_goal, float *d_X, float *d_U, int n_iters,
              gato_solve_stats *d_stats);

/*
 * The same iterations as gato_step, one solve per kernel launch (M launches
 * in order on the batch stream): the plain one-solve-per-launch form the
 * batched launch is compared against. Same arguments and results.
 */
int gato_step_plain(gato_batch *b, const float *d_xs, const float *d_goal, float *d_X, float *d_U,
                    int n_iters, gato_solve_stats *d_stats);

/*
 * gato_step with per-phase timing, for profiling: thread 0 of each solve's
 * workgroup writes, per SQP iteration, 8 unsigned 64-bit values to d_clk
 * (device, [M][n_iters][8]): the constant-rate device wall clock at the start
 * of the iteration and after the dynamics, Schur complement, preconditioner,
 * PCG, step-recovery and line-search phases (7 values), then the shader clock
 * cycles of the whole iteration. Results equal gato_step's. Errors as gato_step.
 */
int gato_profile_phases(gato_batch *b, const float *d_xs, const float *d_goal, float *d_X, float *d_U,
                        int n_iters, unsigned long long *d_clk);

/*
 * Stage entry point: the QP data of Eq. (1) at (X, U) for every solve, as the
 * kernel forms it in the first phase of an SQP iteration (dynamics,
 * derivatives and Euler discretisation). Outputs are device buffers:
 *   d_A [M][N_max-1][nx_max][nx_max], d_B [M][N_max-1][nx_max][nu_max],
 *   d_e [M][N_max-1][nx_max]  (e_k = f(x_k, u_k) - x_{k+1}).
 */
int gato_debug_lq(gato_batch *b, const float *d_xs, const float *d_goal, const float *d_X, const float *d_U,
                  float *d_A, float *d_B, float *d_e);

/*
 * Stage entry point: the KKT solve of one SQP step (Eqs. (4)-(6) and the PCG)
 * on caller-given QP data in the layout of gato_debug_lq, plus
 *   d_q [M][N_max][nx_max] (state gradients), d_r [M][N_max-1][nu_max]
 *   (control gradients), d_c0 [M][nx_max] (x_s - x_0).
 * Writes d_dX [M][N_max][nx_max], d_dU [M][N_max-1][nu_max], d_lambda
 * [M][N_max][nx_max] (double) and, if non-NULL, d_pcg_iters [M] (int).
 * The PCG starts from zero multipliers.
 */
int gato_debug_kkt(gato_batch *b, const float *d_A, const float *d_B, const float *d_e, const float *d_q,
                   const float *d_r, const float *d_c0, float *d_dX, float *d_dU, double *d_lambda,
                   int *d_pcg_iters);

/*
 * Serving (MPC re-solves, warm-started from the previous control step as in
 * the experiments of Sec. IV). The batch keeps one device-resident trajectory
 * per solve slot, [M][N_max][nx_max] and [M][N_max-1][nu_max].
 * gato_set_trajectories / gato_get_trajectories copy all slots in or out
 * (device-to-device, stream-ordered on the batch stream).
 */
int gato_set_trajectories(gato_batch *b, const float *d_X, const float *d_U);
int gato_get_trajectories(gato_batch *b, float *d_X, float *d_U);

/*
 * One serving step over n_req requests: request r re-solves slot d_slots[r]
 * (device int array; the slots of one call must be distinct, and a slot must
 * not be in two calls that overlap in time) from start state d_xs[r] and goal
 * d_goal[r] ([n_req][nx_max], [n_req][nu_max], device). With shift = 1 the
 * slot's resident trajectory and PCG multipliers are first shifted one knot
 * (the last knot repeated); shift = 0 re-solves from them as they are. Runs
 * n_iters SQP iterations (1 for a real-time iteration), updates the resident
 * trajectories and, if non-NULL, writes them per request to d_Xout / d_Uout
 * ([n_req][N_max][nx_max], [n_req][N_max-1][nu_max]) and statistics to
 * d_stats ([n_req][n_iters]). Launched on hip_stream (NULL: the batch stream)
 * so that several steps on disjoint slots can overlap. Batches that mix shapes
 * run through the mixed-shape kernel. A slot outside 0..M-1 is skipped (its
 * outputs are left as they were). Errors: GATO_EINVAL, GATO_EUNSUPPORTED (a
 * batch with long solves with tip tracking).
 */
int gato_serve_step(gato_batch *b, int n_req, const int *d_slots, const float *d_xs, const float *d_goal,
                    int n_iters, int shift, float *d_Xout, float *d_Uout, gato_solve_stats *d_stats,
                    void *hip_stream);

/* Resets the PCG warm-start multipliers of every solve to zero (stream-ordered;
 * a kernel, so it may be captured in a graph). */
int gato_reset_warm_start(gato_batch *b);

/*
 * The PCG warm-start multipliers of every slot (FP64, [M][N_max][nx_max],
 * device; the lambda of Eq. (4) per knot): copied out or in, device to device,
 * stream-ordered on the batch stream. Errors: GATO_EINVAL, GATO_EDEVICE.
 */
int gato_get_multipliers(gato_batch *b, double *d_lam);
int gato_set_multipliers(gato_batch *b, const double *d_lam);

/*
 * Shifts the resident trajectory, controls and multipliers of slots
 * d_slots[0..n-1] (device, distinct) one knot towards the start, the last knot
 * repeated: the warm start of the next control step (Sec. IV). A following
 * gato_serve_step with shift = 0 equals one with shift = 1 on the unshifted
 * slot. Slots outside 0..M-1 are skipped. Launched on hip_stream (NULL: the
 * batch stream). Errors: GATO_EINVAL, GATO_EDEVICE.
 */
int gato_shift_warm_start(gato_batch *b, const int *d_slots, int n, void *hip_stream);

/*
 * Serving launch context: the host side of one serving launch in native code,
 * for request loops that must not pay per-launch copies and allocations. A
 * context owns a HIP stream (default priority), a completion event, pinned
 * host staging and the device buffers of one launch of up to `capacity`
 * requests (1..M) running n_iters SQP iterations each.
 *   gato_serve_ctx_buffers: pointers to the pinned staging: inputs h_slots
 *     [capacity], h_xs [capacity][nx_max], h_goal [capacity][nu_max] (the
 *     caller writes requests 0..n_req-1 there), outputs h_x1
 *     [capacity][nx_max] (knot 1 of each new plan, the plant's next state
 *     under the plan), h_u0 [capacity][nu_max] (the first control) and
 *     h_stats [capacity][n_iters]. Any pointer argument may be NULL.
 *   gato_serve_ctx_submit: enqueues on the context's stream the copy of the
 *     first n_req inputs, gato_serve_step (with the given shift) and the copy
 *     of the outputs, then records the event. Returns at once. The outputs
 *     and the inputs' staging must not be touched until the query says done.
 *     Slots are checked on the host (GATO_EINVAL outside 0..M-1).
 *   gato_serve_ctx_query: 1 when the last submit has finished (outputs
 *     valid), 0 while it runs, negative on a device error.
 *   gato_serve_ctx_trajectories: copies the full plans of the last submit,
 *     [n_req][N_max][nx_max] and [n_req][N_max-1][nu_max], to host memory
 *     (synchronous).
 * Contexts of one batch may run at once on disjoint slots; the caller
 * submits a slot again only after the launch that last held it is done.
 * Errors: GATO_EINVAL, GATO_ENOMEM, GATO_EDEVICE.
 */
typedef struct gato_serve_ctx gato_serve_ctx;

int gato_serve_ctx_create(gato_batch *b, int capacity, int n_iters, gato_serve_ctx **out);
void gato_serve_ctx_destroy(gato_serve_ctx *c);
int gato_serve_ctx_buffers(gato_serve_ctx *c, int **h_slots, float **h_xs, float **h_goal, const float **h_x1,
                           const float **h_u0, const gato_solve_stats **h_stats);
int gato_serve_ctx_submit(gato_serve_ctx *c, int n_req, int shift);
int gato_serve_ctx_query(gato_serve_ctx *c);
int gato_serve_ctx_trajectories(gato_serve_ctx *c, float *h_X, float *h_U);

/*
 * Native request loop over R MPC re-solve requests (the serving pattern: new
 * requests join while others run on the device; each re-solve warm-started
 * as in the experiments of Sec. IV), on n_ctx (1..16) launch contexts as above. Request r arrives at
 * h_arrival_s[r] seconds after the call starts (ascending), for instance
 * h_instance[r] (0..M-1) with goal h_goal[r] ([R][nu_max], host). The loop
 * admits requests as they arrive into per-instance FIFOs (GATO_ST_ADMIT_REJECT
 * when queue_limit > 0 requests already wait); whenever one of n_ctx launch
 * contexts is free it launches the oldest waiting request of every instance
 * that has nothing in flight, as many as memory_budget allows
 * (gato_workspace_bytes per request; 0: no limit; a budget below one request
 * is GATO_EINVAL), each re-solved for n_iters
 * SQP iterations from the instance's state h_state[instance] ([M][nx_max],
 * host, updated in place to the plan's x_1 when the result arrives) and its
 * previous plan shifted one knot. Outputs per request: h_latency_s (arrival
 * to host-visible result, -1 if rejected), h_launch_s (launch time, may be
 * NULL), h_status (OR of the iterations' status bits) and h_u0 (the control to
 * apply, [R][nu_max], may be NULL; untouched for rejected requests).
 * *h_launches (may be NULL) gets the number of launches. All host memory is
 * the caller's. Blocking; busy-waits on the calling thread; each context
 * runs on its own stream, so it does not wait on other work of the process.
 * Errors: GATO_EINVAL (bad sizes, NULL arrays, instance out of range,
 * arrival times not ascending or not finite), GATO_ENOMEM, GATO_EDEVICE.
 */
int gato_serve_run(gato_batch *b, int n_ctx, int n_iters, int R, const double *h_arrival_s, const int *h_instance,
                   const float *h_goal, float *h_state, int queue_limit, size_t memory_budget, double *h_latency_s,
                   double *h_launch_s, unsigned *h_status, float *h_u0, int *h_launches);

/*
 * Plant of closed-loop studies (the simulations of Sec. IV-E integrate the
 * robot at 1 kHz with RK4). For r < n, advances the state d_x[r] ([n][nx_max],
 * device) of the robot of slot d_slots[r] (device int array, or NULL for slot
 * r) by h seconds: `substeps` classical fourth-order Runge-Kutta steps on the
 * continuous dynamics x' = [qd; M(q)^-1 (tau - b(q, qd))] with tau = d_tau[r]
 * ([n][nu_max], device) held constant, and an external force on the tip of
 * the last link: d_fext[r] ([n][3], base frame, device) if d_fext is not
 * NULL (the plant's true disturbance), else the slot's own force (see
 * gato_set_external_force). FP64 arithmetic; the result goes to
 * d_xn[r] (may be d_x). d_status[r] (device, may be NULL) is 0, or
 * GATO_ST_NONFINITE for a non-finite result, an indefinite inertia matrix or a
 * slot outside 0..M-1. Launched on hip_stream (NULL: the batch stream).
 * Errors: GATO_EINVAL (n outside 1..M, NULL buffers, h <= 0, substeps outside
 * 1..100000).
 */
int gato_plant_step(gato_batch *b, int n, const int *d_slots, const float *d_x, const float *d_tau,
                    const float *d_fext, double h, int substeps, float *d_xn, unsigned *d_status,
                    void *hip_stream);

/*
 * External force on the tip of the last link of each solve's robot (the
 * disturbance hypotheses of Sec. IV-D: the solves of a batch may differ only
 * in the assumed force). h_f [M][3] (host, base frame, N, finite) replaces
 * every solve's force; the dynamics become M(q) qdd + b(q, qd) = tau + J(q)^T f,
 * with J the positional Jacobian of the tip, and their derivatives follow.
 * Serial chains only (a non-zero force on another model is GATO_EINVAL).
 * Synchronous. Errors: GATO_EINVAL, GATO_EDEVICE.
 */
int gato_set_external_force(gato_batch *b, const double *h_f);

/*
 * Hypothesis selection of the disturbance case study (Sec. IV-D: the solves of
 * a batch differ only in an assumed external force; after a control step the
 * hypothesis whose model best explains the measured motion becomes the
 * estimate and the hypotheses are re-centred on it). The batch holds P
 * instances of H solves each, solve p H + j being hypothesis j of instance p
 * (same robot). For each instance, in one kernel with no host
 * synchronisation:
 *   - hypothesis j scores the Euclidean distance, over the solve's own 2n
 *     state entries and in FP64, between its one-step prediction
 *     d_pred[p H + j] ([P H][nx_max], device; e.g. gato_plant_step of every
 *     slot under its own force) and the measured state d_meas[p]
 *     ([P][nx_max], device);
 *   - the smallest distance wins (ties to the smaller j, so hypothesis 0
 *     wins ties; non-finite distances never win; if none is finite, j = 0);
 *   - the estimate moves to the winner: d_est[p] += d_off[j] (d_est [P][3],
 *     FP64, device, in/out: the current estimates, of which hypothesis j
 *     assumed d_est[p] + d_off[j]; d_off [H][3], FP64, device: the offsets of
 *     the hypotheses from their estimate, d_off[0] = 0 by convention);
 *   - the hypotheses are re-centred: solve p H + j assumes the force
 *     d_est[p] + d_off[j] (rounded to FP32) in every later call, as if set by
 *     gato_set_external_force;
 *   - d_sel[p] = j (device, may be NULL); d_dist[p H + j] = the distances
 *     (device FP64, may be NULL).
 * Stream-ordered on hip_stream (NULL: the batch stream). Errors: GATO_EINVAL
 * (P, H < 1, P H != M, NULL buffers, a solve that is not a serial chain, or
 * the solves of an instance with different DoF), GATO_EDEVICE.
 */
int gato_select_hypotheses(gato_batch *b, int P, int H, const float *d_pred, const float *d_meas, const double *d_off,
                           double *d_est, int *d_sel, double *d_dist, void *hip_stream);

/*
 * Reference tip positions of the task-space term: d_pref [M][N_max][3]
 * (device, base frame, knot k of solve i at (i N_max + k) 3) is copied into
 * the batch on its stream, so the caller may reuse the buffer once the stream
 * passes the copy. Read by every later solve, step and serving launch (not
 * shifted with the warm start). Errors: GATO_EINVAL (NULL arguments, or a
 * batch without task-space solves), GATO_EDEVICE.
 */
int gato_set_tip_reference(gato_batch *b, const float *d_pref);

/*
 * Tip positions (the end of the last link, base frame) of trajectories:
 * d_X [M][N_max][nx_max] device (the boundary layout) -> d_p [M][N_max][3]
 * device; zero beyond a solve's horizon and for the double-integrator model.
 * FP32, the kinematics the task-space term uses. Stream-ordered on hip_stream
 * (NULL: the batch's stream). Errors: GATO_EINVAL, GATO_EDEVICE.
 */
int gato_tip_positions(gato_batch *b, const float *d_X, float *d_p, void *hip_stream);

/*
 * Per-solve damping rho (Sec. IV-C samples rho across the batch): h_rho[M]
 * (host, each finite and >= 0) replaces every solve's current rho; with
 * rho_adapt the kernels update it after every SQP iteration and
 * gato_get_rho reads it back. gato_reset_warm_start leaves rho as it is.
 * Synchronous. Errors: GATO_EINVAL, GATO_EDEVICE.
 */
int gato_set_rho(gato_batch *b, const double *h_rho);
int gato_get_rho(gato_batch *b, double *h_rho);

/*
 * Dispatch of a batch whose solves differ in DoF or horizon (the uneven batch).
 * A solve's kernel shape is (n_dof, kpt), kpt = knots per 16- (8-) lane group
 * held in registers by the PCG (1, 2 or 4, at most 2 for 3 DoF; at least
 * ceil(N / slots), slots = 32 lane groups of 16 for 6-7 DoF, 64 of 8 for 3). The
 * solves run either as one launch per shape (GATO_DISPATCH_GROUPED) or as
 * one launch of the mixed-shape kernel, whose workgroups each pick their
 * solve's specialisation (GATO_DISPATCH_MIXED). AUTO (the default) takes
 * MIXED when the batch has more than one shape. In both, solves are ordered
 * by decreasing work so that the longest start first. Algorithm 1 runs each
 * phase as its own launch over all solves; here a whole SQP step of every
 * solve is one launch.
 */
enum { GATO_DISPATCH_AUTO = 0, GATO_DISPATCH_GROUPED = 1, GATO_DISPATCH_MIXED = 2 };
int gato_set_dispatch(gato_batch *b, int mode);

/*
 * Multi-CU split of long solves. A solve with four knots per lane group (6-7
 * DoF, N > 64) runs on four workgroups (parts = 4, the default), each holding
 * the PCG rows of 32 knots, or on two, each holding those of 64 knots, when
 * four workgroups per solve do not fit the device at once. The parts run the
 * PCG of Sec. III-B (the same Eq. (5) system, preconditioner and stopping
 * rule) together, exchanging halo rows and inner products through device
 * memory at every PCG iteration. With four parts and schur_fp64 = 1 each part
 * forms the LQ data, Schur rows, step and line-search terms of its own 32
 * knots (and of the knots next to them), the merits are summed over the
 * parts, and each part writes its own knots' results; otherwise every part
 * computes the rest of the SQP iteration alike and part 0 writes the results.
 * The split applies to gato_step, gato_solve and gato_profile_phases as a
 * cooperative launch (every workgroup resident at once), and to
 * gato_step_graph of a mixed-shape batch as a cooperative kernel node (after a
 * node that clears the exchange words). Under the caller's own stream
 * capture, in gato_step_graph of a batch launched per shape group, with
 * parts = 1, and when even two workgroups per solve do not fit, every solve
 * of a batch without tip tracking runs on one workgroup; long solves with tip
 * tracking run only on four parts (a batch that does not fit the device at
 * once takes consecutive launches over ranges of whole solves), so under the
 * caller's capture and with parts = 1 they return GATO_EUNSUPPORTED. The
 * inner products are
 * summed per part first, so results differ from the one-workgroup form at
 * rounding level. A part that waits too long for another sets
 * GATO_ST_EXCHANGE: every wait polls at most max_polls times (0: the default,
 * 131072 polls, about 0.1 s), after which the part stops waiting for the rest
 * of the call and its results are invalid. A batch allocates four workspaces
 * and an exchange area (58 KB) per such solve. Errors: GATO_EINVAL (parts not
 * 1 or 4, max_polls < 0), GATO_EUNSUPPORTED (parts = 1 in a batch with long
 * solves with tip tracking).
 */
int gato_set_split(gato_batch *b, int parts, int max_polls);

/* One (n_dof, N) bucket of a batch and the mapping its solves use. */
typedef struct {
  int n_dof;
  int N;
  int count;      /* solves in the bucket */
  int kpt;        /* knots per lane group */
  float tuned_ms; /* time of the winning candidate in the last gato_autotune, 0 if never tuned */
} gato_bucket;

/*
 * Writes up to cap buckets (ordered by n_dof, then N) to out, and their number
 * to *n_out. Errors: GATO_EINVAL.
 */
int gato_buckets(const gato_batch *b, gato_bucket *out, int cap, int *n_out);

/*
 * Sets the knots-per-group mapping of one bucket by hand. kpt must be 1, 2 or
 * 4 (at most 2 for 3 DoF) and at least the minimum for N; in a batch with tip
 * tracking, 4 only where it is the minimum (N > 64). Errors: GATO_EINVAL (no
 * such bucket, or kpt not allowed), GATO_EUNSUPPORTED (kpt 4 with tip tracking
 * at N <= 64).
 */
int gato_set_mapping(gato_batch *b, int n_dof, int N, int kpt);

/*
 * Autotuner: for every (n_dof, N) bucket, times each allowed kpt on the
 * bucket's own solves (mixed-shape kernel, n_iters SQP iterations from d_X,
 * d_U, reps timed runs after one warm-up, HIP events, the median kept) and
 * keeps the fastest (buckets of long solves with tip tracking have one mapping
 * and are not timed). d_X and d_U are read only (the runs use copies); the PCG
 * warm start is cleared afterwards. Synchronous; allocates temporary device
 * memory. Errors: GATO_EINVAL, GATO_ENOMEM, GATO_EDEVICE.
 */
int gato_autotune(gato_batch *b, const float *d_xs, const float *d_goal, const float *d_X, const float *d_U,
                  int n_iters, int reps);

/*
 * gato_step through a HIP graph: the first call with a given argument tuple
 * (and dispatch mapping) captures the step's launch(es) into a graph and
 * instantiates it; later calls with the same tuple replay it with one graph
 * launch on the batch stream. A new tuple or mapping recaptures. A mixed-shape
 * batch with long solves split across workgroups (gato_set_split) is built as
 * two nodes: a kernel that clears the exchange words, then the split kernel as
 * a cooperative node. Same semantics, errors and stream ordering as gato_step.
 */
int gato_step_graph(gato_batch *b, const float *d_xs, const float *d_goal, float *d_X, float *d_U, int n_iters,
                    gato_solve_stats *d_stats);

/*
 * Arithmetic operation counts of the per-knot rigid-body routines the kernels
 * run, for algorithmic FLOP accounting (host only, no GPU needed):
 * out[0] forward dynamics (inertia matrix, bias forces, Cholesky, solve),
 * out[1] one column of the forward-dynamics Jacobian (dual-number inverse
 * dynamics + solve), out[2] one Cholesky solve. A fused multiply-add counts 2,
 * sin and cos count 1 each. Errors: GATO_EINVAL for n_dof outside 1..7.
 */
int gato_rbd_flops(int n_dof, double *out);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): gato_solve with the
 * device staging of the statistics in a static device array of the library
 * instead of a buffer the batch allocates on first use. Same arguments,
 * results and return values as gato_solve; calls no hipMalloc, hipFree or
 * other allocating routine (it launches a fill kernel, the SQP kernels, one
 * device-to-host copy, and synchronises the batch stream when h_stats is
 * given). The staging holds GATO_STATIC_STATS_MAX entries (24 bytes each,
 * 1.5 MiB); every GPU the library runs this on keeps its own copy until the
 * process ends, with the last call's contents. All calls on one GPU share it:
 * calls that overlap in time on one GPU (other threads, other streams) race
 * and must not be made. Errors: as gato_solve, and GATO_EINVAL when h_stats
 * is non-NULL and M * sqp_iters exceeds GATO_STATIC_STATS_MAX (nothing is
 * launched).
 */
#define GATO_STATIC_STATS_MAX 65536
int gato_solve_static(gato_batch *b, const float *d_xs, const float *d_goal, float *d_X, float *d_U,
                      gato_solve_stats *h_stats);

/* Thread-local message describing the last non-OK return (never NULL). */
const char *gato_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GATO_H */
