/*
 * nrto.h -- C ABI of the MI355X (gfx950) robust-SOCP inner solver.
 *
 * The library solves, for a batch of robust trajectory problems, the tractable
 * linearised problem of one successive-linearisation step (cuNRTO, arXiv
 * 2603.02642, Problem 2):
 *
 *   min_{du, k_v, p}  Q_u(du) + 1/2 k_v' Q_v k_v
 *   s.t.  g0_j + b_j' du + p_j <= 0,  ||A_hat_j k_v + b_hat_j||_2 <= p_j  (j = 1..n_g),
 *         ||F_u du||_2 <= r_trust,
 *
 * by NRTO-DR (inner ADMM with its {k_v, p~} block solved by relaxed
 * Douglas-Rachford splitting, Section III and supplementary II) or by
 * NRTO-FullADMM (Section IV, Algorithm 1, supplementary III).  Problems follow
 * Problem 1: x_{k+1} = f(x_k, u_k) + d_k, x_0 = x0 + d0, disturbances stacked in
 * zeta and bounded by the ball ||zeta|| <= radius (Gamma = S = I, tau = radius^2),
 * affine policy u_k = u_bar_k + K_k zeta_k, constraints required for every zeta.
 *
 * Conventions (all functions):
 *  - Every function returns an nrto_status; no C++ exception or abort crosses
 *    the ABI.  On a non-OK status, nrto_last_error(ctx) (or nrto_last_error(NULL)
 *    for calls without a context) returns a thread-local message.
 *  - Host pointers are read during the call only and never retained; the
 *    context deep-copies problem data.  Device pointers passed to
 *    nrto_project_soc are owned by the caller and must stay valid until the
 *    stream has executed the work.
 *  - A context is bound to one HIP stream (the one given to nrto_setup) and is
 *    not thread-safe.  Calls enqueue work on that stream; calls that return
 *    results to host memory synchronise the stream.  When a context holds
 *    instances of more than one dynamics model, the solve launches of the
 *    second and third model run on two non-blocking streams the context owns,
 *    forked from and joined back into the bound stream with events, so work
 *    queued after a call on the bound stream still sees its results.
 *  - Arrays are row-major float64 unless stated.  Gains K_k (n_u x n_x) are
 *    returned as K[k][u][x]; the paper's k_v stacks vec(K_k) column-major.
 *
 * Constraint order and compact cone layout (shared with the CPU oracle):
 *  state constraints first, by time t = 1..T; within one t, obstacles (arm:
 *  obstacle-major, then link point 0..6), then state upper/lower bounds per
 *  component; then control bounds by step k = 0..T-1, per input upper then
 *  lower.  Cone j stores (t_j, eta_j) with only the structurally non-zero
 *  blocks of eta_j: a state constraint at time t keeps blocks 0..t
 *  (1 + (t+1) n_x entries), a control bound at step k keeps block k
 *  (1 + n_x entries).  The zero blocks stay zero under every update of both
 *  methods, so the compaction is exact.
 */
#ifndef NRTO_H
#define NRTO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nrto_ctx_s *nrto_ctx;

typedef enum {
  NRTO_OK = 0,
  NRTO_MAXITER = 1,        /* iteration limit reached; the iterate is still returned */
  NRTO_INFEASIBLE = 2,     /* consensus residual stagnates (linearisation infeasible) */
  NRTO_FALLBACK_COLD = 3,  /* warm start rejected, cold start used */
  NRTO_ERR_ARG = -1,
  NRTO_ERR_ALLOC = -2,
  NRTO_ERR_HIP = -3,
  NRTO_ERR_STATE = -4
} nrto_status;

typedef enum { NRTO_DR = 0, NRTO_FULLADMM = 1 } nrto_method;
typedef enum { NRTO_FP64 = 0, NRTO_FP32 = 1 } nrto_precision;
typedef enum { NRTO_DYN_UNICYCLE = 0, NRTO_DYN_QUADROTOR = 1, NRTO_DYN_ARM = 2 } nrto_dyn;

/* One robust trajectory problem (Problem 1).  Copied by nrto_setup. */
typedef struct {
  int32_t dyn;               /* nrto_dyn */
  int32_t nx, nu, T;         /* (3,2), (12,4) or (14,7); 1 <= T <= 128 */
  double dt;                 /* forward-Euler step */
  double radius;             /* disturbance ball radius r = sqrt(tau) */
  double mass;               /* quadrotor mass (ignored otherwise) */
  const double *inertia;     /* quadrotor diag(J), 3 values; NULL otherwise */
  const double *links;       /* arm DH link lengths, 7 values; NULL otherwise */
  const double *x0, *xg;     /* nx each: start and goal states */
  const double *Q;           /* nx*nx state tracking weight */
  const double *Ru;          /* nu*nu control weight R_u */
  const double *RK;          /* nu*nu gain weight R_K (cost ||R_K K_k||_F^2) */
  int32_t n_obs;             /* obstacles: rows (centre[d], radius), d = 2 (unicycle) or 3 */
  const double *obs;
  const double *u_lo, *u_hi; /* nu each, +-inf = no bound; NULL = none */
  const double *x_lo, *x_hi; /* nx each, +-inf = no bound; NULL = none */
  const double *u_init;      /* T*nu initial nominal controls */
} nrto_problem;

typedef struct {
  int32_t method;            /* nrto_method */
  int32_t precision;         /* nrto_precision: iteration/projection arithmetic; factor, QP and
                                residual checks are always FP64 */
  int32_t max_admm;          /* ADMM iterations per solve (paper: 40) */
  int32_t max_inner;         /* DR iterations per ADMM step (paper: 100) */
  int32_t check_every;       /* ADMM iterations between KKT residual checks */
  int32_t block_threads;     /* threads per instance workgroup: 64..1024, multiple of 64; 0 = auto */
  double rho;                /* ADMM penalty (paper: 40 NRTO-DR outer ADMM, 10 FullADMM) */
  double alpha;              /* DR relaxation in (0, 2) */
  double sigma_chi, sigma_s; /* DR proximal scalings R_chi = sigma_chi I, R_s = sigma_s I */
  double eps_dr_abs, eps_dr_rel; /* DR stop: ||s~_new - s~|| <= abs + rel max(1, ||s~||) */
  double eps_kkt;            /* stop when the FP64 KKT residual <= eps_kkt (0 = never) */
  double r_trust;            /* trust-region radius ||F_u du|| <= r_trust */
  int32_t cold_init;         /* cold point: 0 = all zeros (the printed initialisation), 1 = every
                                cone at its open-loop value: p = p~ = ||b_hat_j||,
                                s~_j = (||b_hat_j||, b_hat_j), so k_v = 0 is cone-feasible (DR only) */
  int32_t rho_adapt;         /* 1 = residual balancing of rho after each dual update (DR only):
                                rho *= rho_tau if r_p > rho_mu r_d, rho /= rho_tau if
                                r_d > rho_mu r_p, kept in [rho_min, rho_max] */
  double rho_mu, rho_tau, rho_min, rho_max;
  int32_t sigma_adapt;       /* 1 = balance the DR scaling sigma_s during the solve (DR only):
                                after every sigma_every-th DR iteration, with S the affine point,
                                S_hat its projection and K~ the gain state before the iteration,
                                ratio = sqrt((||S_hat - S|| / max(1, ||S||)) /
                                             (||K - K~|| / max(1, ||K||))), skipped while
                                either residual is below 1e-9 of its normaliser;
                                when ratio > sigma_thr or < 1/sigma_thr, sigma_s is multiplied
                                by ratio (kept in [sigma_min, sigma_max]), s~ <- S +
                                (old/new)(s~ - S) and the K blocks are refactored.  The scaling
                                reached is kept per instance for warm solves. */
  int32_t sigma_every;
  double sigma_thr, sigma_min, sigma_max;
  int32_t infeas_window;     /* NRTO-DR: 0 = off; else stop with NRTO_INFEASIBLE when, after an
                                ADMM iteration, the consensus residual r_p = ||p - p~|| has not
                                fallen below 0.99 times its smallest earlier value for this many
                                ADMM iterations while r_p / (1 + ||p~||) > 1e-3 (the linearised
                                problem may be infeasible, e.g. inside a small trust region) */
  int32_t admm_chunk;        /* 0 = a solve is one launch; else a solve is run as launches of at
                                most admm_chunk ADMM iterations each (max_admm in total).  An
                                instance continues from its device state (method state, sigma_s,
                                rho, trust-region multiplier) in the next launch while it has not
                                stopped; stopped instances return at once, so that the slowest
                                solves of a batch are not started late behind the others.  The
                                report sums the counts and times of an instance's launches; the
                                stagnation window (infeas_window) restarts with each launch.
                                Same iterates as one launch up to the order of floating-point
                                sums. */
} nrto_options;

/* Per-instance result of a solve. */
typedef struct {
  int32_t status;            /* NRTO_OK, NRTO_MAXITER or NRTO_INFEASIBLE */
  int32_t admm_iters;
  int32_t inner_iters;       /* total DR iterations (0 for FullADMM) */
  int32_t qp_newton;         /* total Riccati solves in the (du, p) blocks */
  double kkt;                /* FP64 KKT residual of the returned iterate */
  double r_p, r_d;           /* ||p - p~||, rho ||p~ - p~_prev|| of the last ADMM step */
  double mu;                 /* trust-region multiplier */
  double rho;                /* penalty at the end of the solve (differs from the option's
                                value only with rho_adapt) */
  double t_dr_us, t_qp_us, t_kkt_us, t_total_us; /* device wall-clock time of the workgroup in
                                the DR passes with their K-solves, the (du, p) blocks, the KKT
                                checks, and the whole solve */
  double sigma_s;            /* DR scaling at the end of the solve */
  int32_t sigma_updates;     /* changes of sigma_s during the solve */
  int32_t nan_flag;          /* 1 when the residuals became NaN (NaN inputs propagate; the solve
                                stops at the next ADMM iteration with status NRTO_MAXITER) */
} nrto_solve_report;

/* Per-instance result of one successive-linearisation step. */
typedef struct {
  int32_t accepted;          /* step accepted by the merit test */
  int32_t status;            /* solve status */
  double merit_old, merit_new, predicted;
  double r_trust;            /* radius for the next step */
  double kkt;
  int32_t admm_iters, inner_iters; /* of the step's SOCP solve */
} nrto_step_report;

/* Defaults: DR, FP64, 40 ADMM x 100 DR iterations, rho 40, alpha 1,
 * sigma 1, eps_dr 1e-4, eps_kkt 1e-4, r_trust 2 (paper hyperparameter tables);
 * cold_init 0, rho_adapt 0 with rho_mu 10, rho_tau 2, rho_min 1, rho_max 200,
 * sigma_adapt 0 with sigma_every 10, sigma_thr 5, sigma_min 1e-4, sigma_max 1e6. */
void nrto_default_options(nrto_options *opt);

/*
 * Projection of concatenated cones onto second-order cones (supplementary
 * II-C, closed form with its three cases in printed order).
 *  in, out    device arrays of n_entries values (float64 if dtype = 0, float32 if
 *             dtype = 1); in == out is allowed (in-place).
 *  seg_off    device int64 array of n_cones + 1 offsets: cone i is
 *             [seg_off[i], seg_off[i+1]); its first entry is t, the rest eta.  A
 *             length-1 cone is the ray t >= 0; empty cones are allowed.  Must
 *             satisfy seg_off[0] = 0, non-decreasing, seg_off[n_cones] = n_entries.
 *  flags      bit 0: validate seg_off on the device first (synchronises the
 *             stream; NRTO_ERR_ARG if invalid).  Without validation the kernel
 *             still never touches memory outside [0, n_entries).
 *  stream     hipStream_t (NULL = default stream).
 */
nrto_status nrto_project_soc(const void *in, void *out, const int64_t *seg_off,
                             int64_t n_cones, int64_t n_entries, int32_t dtype,
                             int32_t flags, void *stream);

/*
 * nrto_project_soc with offset validation (flags bit 0), for callers that
 * cannot allocate device memory: code that must not call hipMalloc (tight
 * serving loops, harnesses that forbid it).  Arguments, results and errors as
 * nrto_project_soc with flags = 1; the validation flag lives in a fixed 256-byte
 * array the library keeps on every device it runs on until the process ends, so
 * the call allocates nothing.  No input size depends on that array; the limits
 * are those of one launch (at most 2^31 - 1 workgroups of 256 cones or 1024
 * entries), beyond which the call returns NRTO_ERR_ARG.  The current device must
 * be the stream's device.  The array is shared by every call on a device: calls
 * that overlap on one device (other streams or threads) race on the flag.  The
 * call synchronises the stream (it reads the flag back).
 */
nrto_status nrto_project_soc_noalloc(const void *in, void *out, const int64_t *seg_off,
                                     int64_t n_cones, int64_t n_entries, int32_t dtype,
                                     void *stream);

/*
 * Create a context for n_inst problems: device workspace, compact cone layout,
 * wave task schedule.  probs: host array of n_inst problems.  opt: solver
 * options (copied; may be changed later with nrto_set_options).  stream:
 * hipStream_t the context enqueues on.  The nominal controls start at u_init.
 */
nrto_status nrto_setup(const nrto_problem *probs, int32_t n_inst, const nrto_options *opt,
                       void *stream, nrto_ctx *out);
void nrto_destroy(nrto_ctx ctx);
const char *nrto_last_error(nrto_ctx ctx);
nrto_status nrto_set_options(nrto_ctx ctx, const nrto_options *opt);

/* Sizes of instance inst: out[0] n_g, out[1] cone entries, out[2] eta blocks,
 * out[3] n_state (state constraints), out[4] T, out[5] nx, out[6] nu. */
nrto_status nrto_instance_sizes(nrto_ctx ctx, int32_t inst, int64_t out[7]);

/*
 * Constraint-data formation on the device (step a0): nonlinear rollout of the
 * nominal controls, analytic Jacobians, and for every constraint the adjoint
 * recursion lambda_t = grad g_j, b_{j,i} = B_i' lambda_{i+1}, lambda_i = A_i' lambda_{i+1},
 * b_hat_j = r [lambda_0; ...; lambda_t] (supplementary section I).
 */
nrto_status nrto_linearize(nrto_ctx ctx);

/*
 * Replace the linearised data of instance inst by caller-provided host arrays
 * (used to feed both this library and an independent implementation the same
 * SOCP).  Shapes: A T*nx*nx, B T*nx*nu, xhat (T+1)*nx, uhat T*nu, g0 n_g,
 * w n_g*nx (gradient of state constraint j at x_{t_j}; zero rows for control
 * bounds), bhat cone entries (compact layout; the t slot of every cone is 0),
 * bvec blocks*nu (b_{j,k} of every stored block; zero for the last block of a
 * state constraint).
 */
nrto_status nrto_upload_socp(nrto_ctx ctx, int32_t inst, const double *A, const double *B,
                             const double *xhat, const double *uhat, const double *g0,
                             const double *w, const double *bhat, const double *bvec);
/* Copy the device SOCP data of instance inst back (same shapes as upload). */
nrto_status nrto_download_socp(nrto_ctx ctx, int32_t inst, double *A, double *B, double *xhat,
                               double *uhat, double *g0, double *w, double *bhat, double *bvec);

/*
 * Solve the loaded SOCPs of all instances (steps a1-a8: reduced-KKT factor,
 * fused gain-GEMM / projection / relaxation passes, block solves, (du, p)
 * block, dual updates, FP64 KKT residual checks) in one persistent launch.
 * warm = 0 starts every method state from zero; warm = 1 continues from the
 * current state.  rep: host array of n_inst reports (may be NULL).
 */
nrto_status nrto_solve_socp(nrto_ctx ctx, int32_t warm, nrto_solve_report *rep);

/*
 * Device views of a batch's SOCP data and NRTO-DR state for
 * nrto_solve_socp_dev.  Every array is float64 device memory owned by the
 * caller, laid out as the concatenation over instances 0..n_inst-1 (in order)
 * of the per-instance arrays of nrto_upload_socp, nrto_get_solution and
 * nrto_get_state (sizes from nrto_instance_sizes).
 */
typedef struct {
  const double *A, *B, *xhat, *uhat;   /* T*nx*nx, T*nx*nu, (T+1)*nx, T*nu */
  const double *g0, *w;                /* n_g, n_g*nx */
  const double *bhat, *bvec;           /* cone entries, blocks*nu */
} nrto_socp_dev;
typedef struct {
  double *st, *kt, *ptt;               /* DR state: s~ (entries), K~ (T*nu*nx), p~~ (n_g) */
  double *du, *K;                      /* T*nu, T*nu*nx (K[k][u][x]) */
  double *p, *pt, *lam, *pi;           /* n_g each */
} nrto_socp_state_dev;

/*
 * nrto_solve_socp on SOCP data and state held in caller-owned device memory
 * (the context supplies the problem structure, options, stream and its
 * internal scratch).  warm = 0: cold start, the state arrays are outputs;
 * warm = 1: continue from st, kt, ptt, du, K, p, pt, lam (pi is output).  The
 * large arrays (A, B, xhat, uhat, w, bhat, bvec, st, kt, du, K) are read and
 * written in place; the per-cone scalars (g0 in; p, pt, ptt, lam in/out; pi
 * out) are copied device-to-device to and from the context on its stream.  The
 * buffers must stay valid until the stream has executed the call.  NRTO-DR in
 * FP64 only (NRTO_ERR_STATE otherwise); NULL arrays are NRTO_ERR_ARG.  rep:
 * host array of n_inst reports, or NULL (then the call does not synchronise).
 */
nrto_status nrto_solve_socp_dev(nrto_ctx ctx, const nrto_socp_dev *socp, nrto_socp_state_dev *state,
                                int32_t warm, nrto_solve_report *rep);

/*
 * Read the solution of instance inst into host arrays (any may be NULL):
 * du T*nu, K T*nu*nx (K[k][u][x]), p, pt, pi, lam n_g (lam: DR dual lambda,
 * FullADMM scaled dual lambda_p), mu 1.
 */
nrto_status nrto_get_solution(nrto_ctx ctx, int32_t inst, double *du, double *K, double *p,
                              double *pt, double *pi, double *lam, double *mu);
/*
 * Read / write the iteration state of instance inst (compact layout; any
 * pointer may be NULL).  DR: st = s~ (entries), kt = K~ (T*nu*nx), ptt = p~~ (n_g).
 * FullADMM: st = lambda_nu (entries, t slots 0), nu = nu (entries), kt unused.
 */
nrto_status nrto_get_state(nrto_ctx ctx, int32_t inst, double *st, double *nu, double *kt,
                           double *ptt);
nrto_status nrto_set_state(nrto_ctx ctx, int32_t inst, const double *st, const double *nu,
                           const double *kt, const double *ptt, const double *du,
                           const double *K, const double *p, const double *pt,
                           const double *lam);

/*
 * Learned warm start of NRTO-DR (step a10): set the method state of every
 * instance from a prediction row (device float32; row i at pred + i*ld) laid
 * out as du (T*nu), K (T*nu*nx, K[k][u][x]), p~ (n_g), pi (n_g) -- or, with the
 * flag NRTO_WS_NO_GAINS, du, p~, pi only.  The state is rebuilt through the DR
 * fixed-point relations with the cold point's gains (K = K~ = 0; a predicted K
 * is not used): p~_j = max(predicted p~_j, ||eta_j||), p = p~~ = p~,
 * lambda = -pi, s~ = (p~, eta) + y / sigma_s with y_j = pi_j (1, -eta_j/||eta_j||).
 * fallback_test (flags): bit 0 = compare the FP64 KKT residual of the warm point
 * with that of the cold point and keep the cold point where the warm one is
 * worse; NRTO_WS_NO_GAINS (bit 1) = rows without K.  accepted (host, n_inst, may
 * be NULL) receives 1 where the warm point was kept; residuals (host, 2*n_inst,
 * may be NULL) the (warm, cold) residuals.  Follow with nrto_solve_socp(ctx, 1,
 * ...).  Requires method NRTO_DR.
 */
#define NRTO_WS_NO_GAINS 2
nrto_status nrto_warm_start(nrto_ctx ctx, const float *pred, int64_t ld, int32_t fallback_test,
                            int32_t *accepted, double *residuals);

/*
 * One successive-linearisation step for every instance: nrto_linearize, solve,
 * nonlinear rollout of the candidate, merit test, trust-region update and, on
 * acceptance, u_hat += du and the new gains.  rep: n_inst entries or NULL.
 */
nrto_status nrto_scp_step(nrto_ctx ctx, nrto_step_report *rep);
/*
 * The second half of nrto_scp_step on the solution of the last nrto_solve_socp
 * (which must follow an nrto_linearize of the current nominal): nonlinear
 * rollout of the candidate, merit test (penalty weight 10), trust-region update
 * and, on acceptance, u_hat += du and the new gains.  rep: n_inst entries or
 * NULL; its status, kkt and iteration counts are those of the last solve.
 */
nrto_status nrto_scp_accept(nrto_ctx ctx, nrto_step_report *rep);
/*
 * Capture one step -- nrto_linearize (if with_linearize) followed by the solve
 * launches of nrto_solve_socp(ctx, warm, NULL) -- into a HIP graph kept by the context, and
 * replay it with nrto_launch_step (asynchronous on the context's stream; read the
 * results with nrto_get_reports / nrto_get_solution).  For callers that step the
 * same batch many times without host work in between (no allocation, copy or
 * synchronisation happens inside the step).  The context's stream must not be
 * the default stream.  nrto_set_options drops the captured step (its kernels
 * carry the options of the capture).  NRTO-DR, FP64 only.
 */
nrto_status nrto_capture_step(nrto_ctx ctx, int32_t warm, int32_t with_linearize);
nrto_status nrto_launch_step(nrto_ctx ctx);

/* Per-instance reports of the last solve (n_inst entries, host memory), e.g. after
 * nrto_solve_socp with rep = NULL.  Synchronises the context's stream. */
nrto_status nrto_get_reports(nrto_ctx ctx, nrto_solve_report *rep);
/* Current nominal controls of instance inst (T*nu) and gains (T*nu*nx, may be NULL). */
nrto_status nrto_get_nominal(nrto_ctx ctx, int32_t inst, double *uhat, double *K);

/*
 * Learned warm start (a GELU MLP trained on solves of the method itself;
 * the paper names learned warm starts as future work).  BF16 GEMM operands on
 * the matrix cores, FP32 accumulation, FP32 master weights, Adam.
 *  widths     layer widths w_0 .. w_L (host, n_widths = L + 1 >= 2)
 *  max_batch  largest batch passed to infer / train_step / gradients
 *  seed       SplitMix64 seed of the initial weights U(+-sqrt(6/(fan_in+fan_out)))
 *  stream     hipStream_t for every call on this handle
 * X, T, Y are device float32 arrays, row-major (batch x w_0, batch x w_L).
 * Inputs are standardised with (xmean, xstd) and targets with (ymean, ystd)
 * (nrto_ws_set_norm, host arrays; default 0 / 1); nrto_ws_infer returns
 * de-standardised outputs.  Loss: mean squared error on standardised targets.
 */
typedef struct nrto_ws_s *nrto_ws;
nrto_status nrto_ws_create(const int32_t *widths, int32_t n_widths, int32_t max_batch, uint64_t seed,
                           void *stream, nrto_ws *out);
void nrto_ws_destroy(nrto_ws ws);
nrto_status nrto_ws_set_norm(nrto_ws ws, const float *xmean, const float *xstd, const float *ymean,
                             const float *ystd);
nrto_status nrto_ws_infer(nrto_ws ws, const float *X, int32_t batch, float *Y);
/* One Adam step (lr, betas 0.9 / 0.999, eps 1e-8); loss_host may be NULL (no sync). */
nrto_status nrto_ws_train_step(nrto_ws ws, const float *X, const float *T, int32_t batch, float lr,
                               float *loss_host);
/* Gradients without an update, to host memory in the order W_0, b_0, W_1, b_1, ...
 * (W_l is w_{l+1} x w_l row-major). */
nrto_status nrto_ws_gradients(nrto_ws ws, const float *X, const float *T, int32_t batch, float *grads,
                              float *loss_host);
/* Read (get != NULL) and/or write (set != NULL) the FP32 master parameters, same order. */
nrto_status nrto_ws_params(nrto_ws ws, float *get, const float *set);
/* The BF16 matrix-core GEMM the network uses: C (M x N, float32, row-major) =
 * A B with A[m][k] = A[m*sam + k*sak], B[k][n] = B[k*sbk + n*sbn] (bf16 bit
 * patterns, device memory). */
nrto_status nrto_ws_gemm_bf16(const uint16_t *A, int64_t sam, int64_t sak, const uint16_t *B, int64_t sbk,
                              int64_t sbn, int32_t M, int32_t N, int32_t K, float *C, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* NRTO_H */
