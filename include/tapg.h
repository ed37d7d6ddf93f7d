/*
 * tapg.h - C ABI of the MI355X dual-APG solver for scenario-tree stochastic
 * MPC of drinking-water networks (Sopasakis et al., "Uncertainty-aware demand
 * management of water distribution networks in deregulated energy markets",
 * arXiv 1904.10548).
 *
 * The problem (Sec. 3.2, problem SMPC) on a scenario tree (Sec. 2.3) with
 * nodes n = 0..K-1 at decision stages 0..N-1:
 *
 *   minimise  sum_n p_n [ W_alpha (alpha0 + pi_n c_E)'u_n + du_n' W_u du_n ]
 *             + sum_n [ W_x dist(x_n | [xmin, xmax]) + W_s dist(x_n | [xs, inf)) ]
 *   s.t.      x_n = A x_anc(n) + B u_n + Gd d_n        (Sec. 2, eq. dynamics)
 *             E u_n + Ed d_n = 0                       (eq. input-disturbance coupling)
 *             umin <= u_n <= umax                      (eq. input constraints)
 *
 * with du_n = u_n - u_anc(n), x_anc(root) = p and u_anc(root) = q (problem SMPC,
 * initial conditions).  dist is the Euclidean distance.  It is solved by the
 * accelerated proximal gradient method on the Fenchel dual (Sec. 4.3, eqs.
 * apg:1-apg:2), with the dual gradient computed by a backward/forward sweep
 * over the tree (Sec. 4.4).
 *
 * Conventions
 *  - Every matrix is dense, row-major, float64, owned by the caller; the
 *    library copies what it needs during the call.  Output arrays are
 *    allocated by the caller.
 *  - Handles are opaque.  The library owns all device memory.
 *  - Every function returns a tapg_status; on failure tapg_last_error()
 *    returns a message for the calling thread.  No function aborts or throws.
 *  - Node numbering is breadth-first: stage 0 (the root) first, then stage
 *    1, and so on; the children of a node are contiguous and ordered like
 *    their parents.  Every leaf is at stage N-1.
 *  - One solver per host thread; calls on one solver are not thread safe.
 */
#ifndef TAPG_H
#define TAPG_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tapg_network_s* tapg_network;
typedef struct tapg_tree_s* tapg_tree;
typedef struct tapg_solver_s* tapg_solver;
typedef struct tapg_server_s* tapg_server;

typedef enum {
  TAPG_OK = 0,
  TAPG_ENOTCONV = 1,  /* max_iter reached before tol; outputs are valid but inexact */
  TAPG_EINVAL = -1,   /* null handle/pointer, out-of-range value, invalid tree */
  TAPG_EDIM = -2,     /* dimension mismatch or unsupported size */
  TAPG_ENOMEM = -3,   /* host or device allocation failed */
  TAPG_EDEVICE = -4,  /* HIP runtime error or no usable gfx950 device */
  TAPG_ESTATE = -5,   /* call out of order (e.g. solve before the factor step) */
  TAPG_ENUMERIC = -6  /* non-finite iterate or failed factorisation */
} tapg_status;

enum { TAPG_FP64 = 0, TAPG_FP32 = 1 };

/* Extrapolation weights of the accelerated iteration (Sec. 4.3, eq. apg:1):
 * beta_nu = theta_nu (1/theta_{nu-1} - 1), theta_0 = theta_{-1} = 1, with
 *   TAPG_BETA_PAPER   theta_{nu+1} = (sqrt(theta_nu^4 + 4 theta_nu^2) - theta_nu^2)/2
 *   TAPG_BETA_SIMPLE  theta_nu = 2/(nu + 2) for nu >= 1 (the paper's simpler choice)
 *   TAPG_BETA_ZERO    beta = 0: the plain dual proximal gradient method */
enum { TAPG_BETA_PAPER = 0, TAPG_BETA_SIMPLE = 1, TAPG_BETA_ZERO = 2 };

/* Solver configuration (the paper's SmpcConfiguration, Sec. 5.1: tuning
 * weights, tolerance, maximum iterations). */
typedef struct {
  double W_alpha;          /* economic-cost scale (Sec. 3.1), > 0 */
  double W_s;              /* safety-level penalty weight, > 0 */
  double W_x;              /* state-box penalty weight, > 0 */
  const double* alpha0;    /* [nu] production cost */
  const double* c_energy;  /* [nu] energy coefficient; node price vector = pi_n * c_energy */
  const double* W_u;       /* [nu*nu] row-major symmetric positive definite */
  double gamma;            /* dual step size; <= 0 selects 1/(1.02 L), L by power iteration */
  double tol;              /* stop when max|H x_hat - t| <= tol; <= 0 runs max_iter iterations */
  int max_iter;            /* >= 1 */
  int check_every;         /* iterations between host checks of the stop flag (>= 1) */
  int precision;           /* TAPG_FP64, or TAPG_FP32 sweeps (factor step and stop test stay FP64) */
  int power_iters;         /* power iterations for L when gamma <= 0 (0 selects 100) */
  int device;              /* HIP device ordinal */
  void* hip_stream;        /* hipStream_t to launch on; NULL: the solver creates its own */
  int beta_rule;           /* TAPG_BETA_* (0: the paper's theta recursion) */
  int averaged_primal;     /* 1: return the averaged primal iterate (Sec. 4.3: O(1/nu^2)),
                              xbar^nu = (1 - theta_nu) xbar^{nu-1} + theta_nu x_hat(w^nu),
                              xbar^0 = x_hat(w^0); with TAPG_BETA_ZERO theta_nu = 1/(nu+1),
                              the running mean.  tapg_solve only (batches: TAPG_EINVAL) */
  double gap_tol;          /* > 0: the stop test becomes |dual_gap| <= gap_tol and (if tol > 0)
                              the last residual <= tol, both tested every check_every iterations
                              (one extra dual-gradient sweep per gap test); tapg_solve only.
                              The gap alone is no certificate (it uses the split variable t),
                              with the residual it is */
} tapg_config;

typedef struct {
  int iters;          /* APG iterations performed (dual-gradient evaluations) */
  int converged;      /* 1 if the residual reached tol */
  double primal_res;  /* max|H x_hat(w) - t| of the last iteration (FP64) */
  double cost;        /* primal cost of (u_hat, x_hat) without the input-box indicator (FP64) */
  double viol_box;    /* max_n distance of u_hat_n to [umin, umax] (inf-norm) */
  double viol_eq;     /* max of |E u + Ed d|_inf and the dynamics residual */
  double gamma;       /* step size used */
  double solve_ms;    /* device time of the solve (data step + iterations), HIP events */
  double dual_gap;    /* duality gap of the returned dual y (Sec. 4.2, strong duality), FP64:
                         G = f(x') + g(t) + F(y) with x' = x_hat(y), t = prox_{g/gamma}(y/gamma
                         + H x') and F the dual objective; -> 0 at the optimum.  NaN unless
                         evaluated (tapg_residuals always evaluates it; tapg_solve when
                         gap_tol > 0) */
  double dual_obj;    /* F(y) = f*(-H'y) + g*(y), the dual objective (minimised); NaN as above */
} tapg_result;

/* Network (the paper's DwnNetwork, Sec. 5.1; model of Sec. 2).
 * A [nx*nx], B [nx*nu], Gd [nx*nd], E [ns*nu], Ed [ns*nd]; bounds of length
 * nx (xmin, xmax, xs) and nu (umin, umax).  Requirements: 1 <= nx, nu <= 256,
 * nd >= 1, 0 <= ns < nu, E of full row rank, umin <= umax, xmin <= xmax.
 * Errors: TAPG_EINVAL (null pointer), TAPG_EDIM (sizes), TAPG_ENUMERIC (E rank
 * deficient or non-finite entries). */
tapg_status tapg_network_create(int nx, int nu, int nd, int ns, const double* A,
                                const double* B, const double* Gd, const double* E,
                                const double* Ed, const double* xmin, const double* xmax,
                                const double* xs, const double* umin, const double* umax,
                                tapg_network* out);
void tapg_network_destroy(tapg_network net);
tapg_status tapg_network_dims(tapg_network net, int* nx, int* nu, int* nd, int* ns);

/* Scenario tree (the paper's ScenarioTree, Sec. 2.3 and 5.1).
 * nodes_per_stage [N] (mu_0 = 1), ancestor [K] (ancestor[0] = -1), prob [K]
 * (prob[0] = 1, children's probabilities add up to their parent's within
 * 1e-12 relative, all > 0), demand [K*nd] (node-major), price [K] (the scalar
 * pi_n).  K = sum(nodes_per_stage).  Validation errors return TAPG_EINVAL with
 * the offending node in tapg_last_error(). */
tapg_status tapg_tree_create(int N, const int* nodes_per_stage, const int* ancestor,
                             const double* prob, int nd, const double* demand,
                             const double* price, tapg_tree* out);
/* Replace the node data of an existing tree (receding horizon: same tree
 * shape, new forecasts).  demand [K*nd], price [K]. */
tapg_status tapg_tree_set_data(tapg_tree tree, const double* demand, const double* price);
/* K of a tree (number of nodes), or -1 for a null handle. */
int tapg_tree_num_nodes(tapg_tree tree);
/* Sizes of a tree (stages N, nodes K, demands per node nd) and of a network;
 * any output pointer may be NULL.  TAPG_EINVAL for a NULL handle. */
tapg_status tapg_tree_dims(tapg_tree tree, int* N, int* K, int* nd);
void tapg_tree_destroy(tapg_tree tree);

/* Solver bound to one network and one device (the paper's SmpcController with
 * its Engine).  The configuration is copied.  Errors: TAPG_EINVAL,
 * TAPG_ENUMERIC (W_u not SPD), TAPG_EDEVICE (device unavailable). */
tapg_status tapg_solver_create(tapg_network net, const tapg_config* cfg, tapg_solver* out);
void tapg_solver_destroy(tapg_solver solver);

/* Offline factor step for horizon N (the paper's Engine::factorStep, Sec. 5.1;
 * the recursion quantities of the dual-gradient DP, Sec. 4.4), in FP64 on the
 * host, then copied to the device (FP64 and FP32 copies).  For s = N-1..0:
 * Qbar_s = W_u + Pbar_{s+1} (Pbar_N = 0), Fbar_s = Z (Z'Qbar_s Z)^{-1} Z' with Z a
 * basis of ker E, Kbar_s = Fbar_s W_u, Gammabar_s = I - Fbar_s Qbar_s,
 * Pbar_s = W_u - W_u Fbar_s W_u.  Every tree of horizon N shares them. */
tapg_status tapg_factor_step(tapg_solver solver, int N);
/* Copy the stage-s factors (row-major nu*nu each; any pointer may be NULL). */
tapg_status tapg_get_factors(tapg_solver solver, int stage, double* Fbar, double* Kbar,
                             double* Gbar);
/* Factor sharing between stages (a property of the factors of Sec. 4.4 that the
 * sweeps exploit): stage s is served by factor block fid[s] (host array of n >= N
 * ints, may be NULL), where consecutive stages whose Fbar agree to 16 ulp of the
 * block's largest entry share the block of the later stage.  With W_u = w I every
 * Fbar_s equals Z Z' / w, so there is one block.  *n_blocks (may be NULL) gets the
 * number of distinct blocks.  TAPG_ESTATE before the factor step, TAPG_EINVAL if
 * n < N. */
tapg_status tapg_factor_blocks(tapg_solver solver, int* fid, int n, int* n_blocks);

/* Solve the problem on `tree` from x_{k|k} = p [nx], u_{k-1|k} = q [nu] (the
 * paper's controlAction).  warm_start != 0 starts from the dual of this
 * tree's previous solve on this solver (y^0 = y^-1 = that dual, theta reset);
 * otherwise from zero.  u0_out [nu] (may be NULL) receives u_hat at the root,
 * the input to apply.  res (may be NULL) receives the statistics.
 * Returns TAPG_OK, TAPG_ENOTCONV (max_iter reached), or an error. */
tapg_status tapg_solve(tapg_solver solver, tapg_tree tree, const double* p, const double* q,
                       int warm_start, double* u0_out, tapg_result* res);

/* For callers that cannot allocate device memory (code running under HIP
 * graph capture is not one of them: the call waits for the device; but tight
 * control loops and harnesses that forbid hipMalloc are): tapg_solve without
 * any device allocation.  Every buffer of the solve lives in one static device
 * array of TAPG_NOALLOC_SCRATCH_BYTES per GPU, held by the library until the
 * process ends (its address is looked up at solver creation); a tree whose
 * buffers do not fit returns TAPG_ENOMEM (tapg_noalloc_bytes gives the need).
 * Cold start (y = 0), the per-stage sweep kernels, the solver's stream; the
 * same iteration as tapg_solve up to rounding.  The step size is cfg.gamma, or
 * 1/(1.02 L) with the tree's estimate from an earlier tapg_estimate_lipschitz
 * or tapg_solve (else TAPG_EINVAL: the power iteration allocates).
 * u0_out [nu], u_out [K*nu], x_out [K*nx] and res may each be NULL.  Calls on
 * one device share its array: the library serialises them, and each call
 * overwrites what the previous one left.  No averaged primal or gap test
 * (TAPG_EINVAL).  Returns TAPG_OK, TAPG_ENOTCONV or an error. */
#define TAPG_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
tapg_status tapg_solve_noalloc(tapg_solver solver, tapg_tree tree, const double* p,
                               const double* q, double* u0_out, double* u_out, double* x_out,
                               tapg_result* res);
/* Scratch bytes tapg_solve_noalloc needs for this tree (host only). */
tapg_status tapg_noalloc_bytes(tapg_solver solver, tapg_tree tree, size_t* bytes);

/* Solve several trees in one set of launches (the paper's method on each tree;
 * Sec. 4.3 iteration, Sec. 4.4 sweeps): the trees, which must share the
 * factored horizon and appear once each, are swept together as one forest, each
 * with its own step size (as tapg_solve would choose it), control block and stop
 * test, so each result equals that of tapg_solve on the tree up to rounding.
 * p[k] (nx), q[k] (nu): initial condition of tree k; warm_start (may be NULL):
 * per tree, start from its last dual as tapg_solve would; u0_out (may be NULL,
 * or hold NULL entries): root input of tree k (nu doubles); res (may be NULL):
 * ntrees results.  Afterwards every tree can be queried as after tapg_solve.
 * Returns TAPG_ENUMERIC if any tree's residual became non-finite, else
 * TAPG_ENOTCONV if any tree stopped at max_iter with tol > 0, else TAPG_OK; the
 * results of all trees are written in every case.  Needs the segment sweep
 * kernels (nx, nu <= 128), else TAPG_EINVAL. */
tapg_status tapg_batch_solve(tapg_solver solver, int ntrees, const tapg_tree* trees,
                             const double* const* p, const double* const* q, const int* warm_start,
                             double* const* u0_out, tapg_result* res);

/* Primal iterate of the last solve: u [K*nu], x [K*nx] (node-major). */
tapg_status tapg_get_primal(tapg_solver solver, tapg_tree tree, double* u, double* x);
/* Dual iterate y^{nu*+1} of the last solve, node-major blocks (y1 [nx], y2 [nx],
 * y3 [nu]) per node: y [K*(2nx+nu)]. */
tapg_status tapg_get_dual(tapg_solver solver, tapg_tree tree, double* y);
/* Set the dual used by the next warm-started solve of this tree. */
tapg_status tapg_set_dual(tapg_solver solver, tapg_tree tree, const double* y);
/* Residual history of the last solve: hist [min(n, iters)] (FP64); returns the
 * number of entries written through *written. */
tapg_status tapg_residual_history(tapg_solver solver, tapg_tree tree, double* hist, int n,
                                  int* written);
/* Statistics of the last solve of this tree (primal residual, cost,
 * violations); same fields as tapg_solve's result, with the duality gap and
 * the dual objective of the tree's current dual (its last solve's, or the one
 * tapg_set_dual gave it) evaluated on the device in FP64 if the solve did not
 * (one dual-gradient sweep; Sec. 4.2 and 4.4); after a diverged solve they
 * stay NaN.  TAPG_ESTATE before a solve. */
tapg_status tapg_residuals(tapg_solver solver, tapg_tree tree, tapg_result* res);

/* Lipschitz constant of the dual gradient of this tree by `iters` power
 * iterations on the device (step-size selection; see tapg_config.gamma).  The
 * estimate is kept with the tree and used by tapg_solve when cfg.gamma <= 0
 * (L depends on the tree's structure and probabilities, not on its data).
 * TAPG_ENUMERIC if the estimate is not a positive finite number. */
tapg_status tapg_estimate_lipschitz(tapg_solver solver, tapg_tree tree, int iters, double* L);

/* Sweep schedule of a tree (host only, no device needed).  The sweeps run
 * as "levels" of consecutive stages; a level's workgroups each own a group of
 * consecutive nodes of its first stage and all their descendants inside the
 * level, at most 4 nodes per stage.  With levels == NULL
 * the library's planner chooses the cuts and group sizes (a cost model of
 * launch, stage and per-node costs); otherwise `levels` is "s0:g0,s1:g1,..."
 * (first stage and group size of each level, s0 = 0).  out[5*l .. 5*l+4]
 * receives (first stage, last stage, group size, workgroups, widest
 * workgroup stage) for l < cap; *nlevels the number of levels.  The same
 * choice is made by tapg_solve (the TAPG_LEVELS environment variable
 * overrides it there). */
tapg_status tapg_plan_schedule(tapg_tree tree, int precision, const char* levels, int* out,
                               int cap, int* nlevels);

/* Profiling aid: with enable != 0, later solves time every sweep-kernel launch
 * with a pair of HIP events on the solver's stream (iteration graphs are not
 * used meanwhile, and the host checks the stop flag after every iteration).
 * tapg_kernel_times returns, for the last timed solve, the summed device time
 * (ms[4]) and counts (launches[4]) of: [0] backward-sweep launches, [1]
 * forward-sweep launches (with the fused prox/dual update), [2] separate
 * end-of-iteration launches (per iteration with the per-stage kernels; once
 * per chunk with the level launches, whose backward launches end the previous
 * iteration themselves), [3] persistent-iteration launches, counted in
 * iterations (with TAPG_CHAIN=1 a single tree whose workgroups all fit on the
 * device runs every level in one cooperative launch per chunk of iterations). */
tapg_status tapg_kernel_timing(tapg_solver solver, int enable);
tapg_status tapg_kernel_times(tapg_solver solver, double* ms, long long* launches);
/* The dispatch cost that each timed launch above carries on top of its kernel:
 * the median time (*us, microseconds) that a pair of events reads around a
 * launch of known length (a 10 us wait) queued the same way, less that length.  Subtracting it per launch brings the
 * timed averages close to a kernel trace's durations. */
tapg_status tapg_event_pair_overhead(tapg_solver solver, double* us);

/* Request server (the solve loop of a controller serving many requests,
 * Sec. 5.1's SmpcController::controlAction per request), with continuous
 * batching: a worker thread owns the solver and iterates the requests in
 * flight (one per tree) together as one forest, one chunk of check_every
 * iterations at a time.  Between chunks, requests whose tree stopped complete
 * and pending requests join, first come first served, while the estimated
 * device memory of the set fits hbm_budget_bytes (at most max_batch requests);
 * every request's iterates are the same as in a tapg_solve of its own.  A
 * request is warm started when the previous request of its session solved the
 * same tree with TAPG_OK or TAPG_ENOTCONV and no request of another session has
 * solved that tree since (a tree keeps one dual).  While a server exists,
 * other calls on its solver return TAPG_ESTATE; destroy the server before the
 * solver.  A submitted tree must not be modified or destroyed before its
 * ticket completes.  If setting up or iterating a set fails, every request of
 * the set completes with the error. */
tapg_status tapg_server_create(tapg_solver solver, size_t hbm_budget_bytes, int max_batch,
                               tapg_server* out);
/* Queue one request (p: nx, q: nu, copied); *ticket identifies it. */
tapg_status tapg_server_submit(tapg_server srv, tapg_tree tree, const double* p, const double* q,
                               int session, long long* ticket);
/* Result of a request: waits up to wait_ms (0: do not wait, < 0: until done).
 * TAPG_ESTATE while pending (nothing written); otherwise the request's status
 * (TAPG_OK, TAPG_ENOTCONV, TAPG_ENUMERIC, or TAPG_ENOMEM if it alone exceeds
 * the budget), with u0_out (nu), res and latency_ms (submit to completion;
 * each may be NULL) written; the ticket is then released. */
tapg_status tapg_server_poll(tapg_server srv, long long ticket, int wait_ms, double* u0_out,
                             tapg_result* res, double* latency_ms);
/* Counters: batches run, requests solved, worker busy time, queue length. */
tapg_status tapg_server_stats(tapg_server srv, long long* batches, long long* solved,
                              double* busy_ms, int* pending);
/* Worker time so far, in ms: forming forests (running trees' state in, data
 * step, iteration graph), chunks of iterations, and leaving forests (state
 * back to the trees' slots, results, forest freed). */
tapg_status tapg_server_timing(tapg_server srv, double* enter_ms, double* chunk_ms,
                               double* leave_ms);
/* Stops the worker (queued requests complete with TAPG_ESTATE) and frees it. */
void tapg_server_destroy(tapg_server srv);

/* Autotuner for the sweep schedule (the levels of stages and the workgroup
 * groups that tapg_plan_schedule describes): times `iters` iterations (one
 * captured iteration graph) of every distinct plan the planner produces under a
 * spread of its cost constants, on the tree (ntrees = 1) or on the batch's forest
 * (ntrees > 1, as tapg_batch_solve would form it), and keeps the fastest for it
 * and for every later tree or batch of the same shape on this solver (TAPG_LEVELS,
 * if set, still wins).  Where the scan form applies, every plan is timed in
 * both forms, in the scan form with each grouping of its forward launch, and
 * then (scan form chosen) with light upper levels.  *ms_per_iter (may be NULL):
 * the winner's time per iteration; *candidates (may be NULL): schedules timed.  The timing runs overwrite
 * the tree's iterates (solve again before querying).  TAPG_EINVAL when the
 * segment kernels do not apply. */
tapg_status tapg_autotune(tapg_solver solver, int ntrees, const tapg_tree* trees, int iters,
                          double* ms_per_iter, int* candidates);

/* Sweep form of a tree (ntrees = 1) or of a batch's forest (ntrees > 1) as
 * its last solve or autotune left it: *form (may be NULL) one of
 * TAPG_FORM_*, *bwd_launches (may be NULL) the backward launches per
 * iteration.  The scan form (Sec. 4.4 recursions with A = I and the projector
 * factors unrolled into subtree and root-path sums) applies when A = I and the
 * projector form applies; untuned trees and forests then use it (TAPG_SCAN=0:
 * the segment form), and tapg_autotune keeps whichever form is faster for the
 * shape.
 * TAPG_ESTATE before the first solve or autotune of that tree or batch. */
/* The schedule of a tree (ntrees = 1) or of a batch's forest as its last
 * solve or autotune left it, written to buf (cap bytes, NUL-terminated) as the
 * environment settings that force it on a fresh solver, for instance
 * "TAPG_SCAN=1 TAPG_LEVELS=0:1,2:1,5:1 TAPG_FWD_GROUP=1 TAPG_TOP=1" (levels:
 * first stage and workgroup group of each; forward group: last-stage nodes
 * per forward workgroup of the scan form, 0 = the bottom level's workgroups;
 * TAPG_TOP=1: light upper levels, whose work runs inside the bottom level's
 * backward launch, so that the backward sweep is one launch) or
 * "TAPG_SEGMENTS=0" (per-stage kernels).  TAPG_EINVAL if cap is too small,
 * TAPG_ESTATE before the first solve or autotune of that tree or batch. */
tapg_status tapg_schedule_spec(tapg_solver solver, int ntrees, const tapg_tree* trees, char* buf,
                               int cap);

#define TAPG_FORM_STAGES 0    /* per-stage kernels */
#define TAPG_FORM_SEGMENT 1   /* segment kernels, stage factors in registers */
#define TAPG_FORM_PROJECTOR 2 /* segment kernels, projector form of the factors */
#define TAPG_FORM_SCAN 3      /* scan kernels */
tapg_status tapg_sweep_form(tapg_solver solver, int ntrees, const tapg_tree* trees, int* form,
                            int* bwd_launches);

/* Release the device memory a solver holds for a tree (its slot and every
 * cached batch containing it).  The tree stays valid; a later solve allocates
 * again. */
tapg_status tapg_solver_forget(tapg_solver solver, tapg_tree tree);

/* Closed-loop receding-horizon simulation (Sec. 6.3, closed-loop
 * simulations).  At each sampling instant k = 0..H_s-1 the library calls
 * forecast(ctx, k, demand [K*nd], price [K]) for the tree's data at k (the
 * root carries the demand and price observed at k, the other nodes the
 * forecast scenarios; return 0, or nonzero to abort with TAPG_EINVAL), solves
 * from the plant state x_k and u_{k-1} (tapg_solve; warm started from the
 * previous dual when warm_start != 0 and k > 0), applies the root input u_k
 * and moves the plant with the observed demand d_k (the root's):
 *   x_{k+1} = A x_k + B u_k + Gd d_k.
 * x0 [nx], u_prev [nu]: initial state and previous input.  Outputs (each may
 * be NULL): x_traj [(H_s+1)*nx] (x_0..x_{H_s}), u_traj [H_s*nu], tau_ms [H_s]
 * (host wall time of each solve), iters [H_s], and the indices of Sec. 6.3 in
 * stats.  A solve that fails (other than TAPG_ENOTCONV) stops the loop with
 * its status.  The tree's data are left at the last step's. */
typedef int (*tapg_forecast_fn)(void* ctx, int k, double* demand, double* price);
typedef struct {
  double kpi_E;         /* (1/H_s) sum_k (alpha0 + pi_k c_E)'u_k, economic index */
  double kpi_S;         /* sum_k |max(xs - x_{k+1}, 0)|_1, safety index */
  double kpi_tau_ms;    /* max_k tau_k, complexity index (ms) */
  double mean_tau_ms;   /* mean_k tau_k */
  double max_viol_box;  /* max_k distance of u_k to [umin, umax] (inf-norm) */
  double max_viol_eq;   /* max_k |E u_k + Ed d_k|_inf */
  long long iters;      /* APG iterations over all steps */
  int steps_converged;  /* steps whose solve reached tol */
} tapg_loop_stats;
tapg_status tapg_closed_loop(tapg_solver solver, tapg_tree tree, int H_s, const double* x0,
                             const double* u_prev, tapg_forecast_fn forecast, void* ctx,
                             int warm_start, double* x_traj, double* u_traj, double* tau_ms,
                             int* iters, tapg_loop_stats* stats);

/* Scenario tree from sampled prediction-error paths (Sec. 2.3 and 6.2: the
 * paper reduces 10^4 Monte-Carlo paths to a tree by the forward scenario
 * reduction of Heitsch and Roemisch), on the GPU, stage by stage: the root
 * holds every path; at stage t every node of stage t-1 splits its cluster of
 * paths by forward selection of min(branching[t], cluster size)
 * representatives (greedy minimisation of the transport cost
 * sum_k p_k min_r |x_k - x_r|_2 over the paths' stage-t values; ties go to the
 * lowest position), each path joining its nearest representative (ties: the
 * one picked first); each representative becomes a child, in the order
 * picked, carrying its stage-t value and its members' summed probability.
 * samples [M*H*d] (path-major, then stage, then component; stage 0 is the
 * root's, normally zero), prob [M] (NULL: uniform; must add up to 1),
 * branching [H] (entry 0 ignored; >= 1).  Outputs (capacity cap nodes): the
 * tree in breadth-first order with contiguous children: nodes_per_stage [H],
 * ancestor [K] (-1 at the root), node_prob [K], node_value [K*d] (may be
 * NULL), rep [K] (the path whose value each node carries; may be NULL), *K_out.
 * All arrays are caller-owned host memory; the call allocates and frees its
 * own device buffers and returns when the tree is complete.  FP64 throughout.
 * Errors (outputs then untouched): TAPG_EINVAL (M, H < 1, d outside 1..128,
 * a NULL required array, cap < 1, a branching entry < 1, probabilities
 * negative or not adding up to 1), TAPG_ENUMERIC (a non-finite sample),
 * TAPG_EDIM (more than cap nodes), TAPG_ENOMEM, TAPG_EDEVICE. */
tapg_status tapg_tree_build(int M, int H, int d, const double* samples, const double* prob,
                            const int* branching, int device, int cap, int* nodes_per_stage,
                            int* ancestor, double* node_prob, double* node_value, int* rep,
                            int* K_out);

/* ------------------------------------------------------------------------
 * JSON front-end (Sec. 5.1: the network, the scenario tree, the forecaster,
 * the controller configuration and the control output live in JSON files;
 * the plant state x_k may too).  The paper names the files, not their
 * fields; the formats below are this library's.  Each file holds one JSON
 * object; matrices are arrays of rows; every number must be finite; keys not
 * listed are errors (a misspelt key is never ignored), except "name" and
 * "description", which every file may carry.  Errors: TAPG_EINVAL (file not
 * readable, syntax error with line:column, unknown or missing key, wrong
 * type), TAPG_EDIM (shapes), TAPG_ENUMERIC (a non-finite number), and the
 * errors of the array entry point each reader ends in.
 * ------------------------------------------------------------------------ */

/* network.json (the paper's DwnNetwork):
 *   {"A": nx x nx, "B": nx x nu, "Gd": nx x nd, "E": ns x nu, "Ed": ns x nd,
 *    "xmin", "xmax", "xs": [nx], "umin", "umax": [nu],
 *    optional "nx", "nu", "nd", "ns" (checked against the matrices)}
 * ns = 0 is "E": [], "Ed": [].  Validated like tapg_network_create. */
tapg_status tapg_network_from_json(const char* path, tapg_network* out);

/* scenarioTree.json (the paper's ScenarioTree):
 *   {"nodes_per_stage": [N], "ancestor": [K] (-1 at the root),
 *    "probability": [K], optional "N", optional "children" (one list per node
 *    or per non-leaf node, checked against "ancestor"), and the node data as
 *    either  "demand": K x nd, "price": [K]  (node values; no forecaster) or
 *    "demand_error": K x nd, "price_error": [K]  (prediction errors of
 *    Sec. 2.2, eq. prediction-error; zero at the root), then with
 * forecaster.json (the paper's Forecaster output):
 *   {"demand": N x nd, "price": [N]}  (nominal forecasts per stage; stage 0
 *    is the current instant), a node's data being forecast + error at its
 *    stage.  forecaster_path is NULL for a tree of node values.  Validated like
 *    tapg_tree_create. */
tapg_status tapg_tree_from_json(const char* tree_path, const char* forecaster_path,
                                tapg_tree* out);
/* The node data that tapg_tree_from_json would build, into caller arrays
 * demand [K*nd] and price [K] (for tapg_tree_set_data in a receding-horizon
 * loop with a new forecaster file per step).  TAPG_EDIM unless the tree file
 * has K nodes and nd demands. */
tapg_status tapg_tree_data_from_json(const char* tree_path, const char* forecaster_path, int K,
                                     int nd, double* demand, double* price);

/* controllerconfig.json (the paper's SmpcConfiguration):
 *   {"W_alpha", "W_s", "W_x": numbers, "alpha0", "c_energy": [nu],
 *    "W_u": nu x nu or a number w (meaning w I), "tol": number,
 *    "max_iter": integer, optional "gamma" (0: automatic), "check_every" (100),
 *    "precision" ("fp64" | "fp32"), "power_iters" (100), "device" (0),
 *    "beta_rule" ("paper" | "simple" | "zero"), "averaged_primal" (false),
 *    "gap_tol" (0)}
 * Fills *cfg (hip_stream NULL); its alpha0, c_energy and W_u point to the
 * caller's arrays alpha0 [nu], c_energy [nu] and W_u [nu*nu], which this
 * call fills and which must outlive the config.  Values are range-checked by
 * tapg_solver_create. */
tapg_status tapg_config_from_json(const char* path, int nu, tapg_config* cfg, double* alpha0,
                                  double* c_energy, double* W_u);

/* Plant state file: {"x": [nx] (x_k), "u_prev": [nu] (u_{k-1}), optional "k"}
 * into caller arrays x [nx] and u_prev [nu]. */
tapg_status tapg_state_from_json(const char* path, int nx, int nu, double* x, double* u_prev);

/* controlOutput.json (the paper's SmpcController output): writes
 *   {"status": "ok" | "not_converged" | ..., "u": [nu] (the control action
 *    u_0 to apply), "iters", "converged", "primal_res", "cost", "viol_box",
 *    "viol_eq", "gamma", "solve_ms", "dual_gap", "dual_obj"}
 * from a solve's root input u0 [nu], its result and its status.  Doubles are
 * written with 17 significant digits (they read back exactly); NaN and
 * infinities as null.  The file is written under path + ".tmp" and renamed,
 * so a reader never sees half a file. */
tapg_status tapg_control_output_write(const char* path, int nu, const double* u0,
                                      const tapg_result* res, tapg_status solve_status);

/* Message describing the last failure on the calling thread ("" if none). */
const char* tapg_last_error(void);
/* Library version string. */
const char* tapg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* TAPG_H */
