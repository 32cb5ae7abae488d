/*
 * libgrim -- MI355X (gfx950) implementation of the per-zone Newton-Raphson
 * method of Chandra, Foucart & Gammie, "grim: A Flexible, Conservative Scheme
 * for Relativistic Fluid Theories" (arXiv:1702.01106).
 *
 * The library advances relativistic ideal MHD (8 primitives) or extended MHD
 * (EMHD, 10 primitives) on a uniform grid in coordinates X^i with a
 * Minkowski or modified Kerr-Schild metric (Sec. 2.1).  One step is the
 * two-stage semi-implicit scheme of Sec. 2.3: each stage computes the
 * explicit fluxes at P^E (PLM reconstruction, LLF, flux-CT; Sec. 2.4, 4.2)
 * and then solves the discrete equations for the primitives of every zone
 * by Newton's method with a finite-difference Jacobian, a dense per-zone LU
 * solve and a quadratic backtracking line search (Sec. 3).
 *
 * Conventions
 *  - Primitive order (Sec. 4): rho, u, utilde^1..3 (normal-observer
 *    four-velocity, equal to u^i in Minkowski), B^1..3, and for EMHD q and
 *    DeltaP.
 *  - Arrays of primitives are FP64, structure of arrays, interior zones only:
 *    P[v][k][j][i] with i fastest, v in [0, nvar), sizes n3 x n2 x n1 (n2 = 1
 *    and n3 = 1 in 1D, n3 = 1 in 2D).
 *  - Pointers: the test hooks take device pointers (memory the caller owns,
 *    e.g. from PyTorch).  grim_set_prims / grim_get_prims take a flag that
 *    says whether the pointer is host or device memory.  The library never
 *    keeps a caller pointer after a call returns.
 *  - Every call returns GRIM_OK (0) or a negative GRIM_E_* code; the message
 *    is available from grim_last_error (per context) or
 *    grim_last_global_error (for failures of grim_create).  No C++ exception
 *    crosses the interface.  Per-zone non-convergence is not an error: it is
 *    reported in the per-zone flags and in grim_stats_t.
 *  - Work is enqueued on the stream given at create time (NULL: the null
 *    stream).  Calls that return data to the host synchronise that stream.
 *  - One context per host thread; calls on one context are not thread-safe.
 */
#ifndef GRIM_H
#define GRIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GRIM_OK 0
#define GRIM_E_INVALID_ARG (-1)
#define GRIM_E_HIP (-2)
#define GRIM_E_OOM (-3)
#define GRIM_E_STATE (-4)

/* models: number of primitives */
#define GRIM_IDEAL_MHD 8
#define GRIM_EMHD 10
/* metrics */
#define GRIM_MINKOWSKI 0
#define GRIM_MKS_KERR 1
/* boundary conditions, per direction */
#define GRIM_BC_PERIODIC 0
#define GRIM_BC_OUTFLOW 1
#define GRIM_BC_POLAR 2
/* precision of the Jacobian difference quotients, storage and LU */
#define GRIM_JAC_F64 0
#define GRIM_JAC_F32 1
/* initial guess of the Newton solve */
#define GRIM_GUESS_PN 0
#define GRIM_GUESS_MLP 1

/* learned-guess network: inputs, hidden width, outputs, parameter count */
#define GRIM_MLP_IN 32
#define GRIM_MLP_HIDDEN 128
#define GRIM_MLP_OUT 16
#define GRIM_MLP_PARAMS 22880
/* Newton system, Riemann solver, reconstruction */
#define GRIM_SYSTEM_REDUCED 0
#define GRIM_SYSTEM_FULL 1
#define GRIM_RIEMANN_LLF 0
#define GRIM_RIEMANN_HLLE 1
#define GRIM_RECON_PLM 0
#define GRIM_RECON_WENO5 1
#define GRIM_RECON_PPM 2
/* per-zone flags */
#define GRIM_FLAG_NOT_CONVERGED 1
#define GRIM_FLAG_LS_EXHAUSTED 2
#define GRIM_FLAG_SINGULAR 4
#define GRIM_FLAG_UNPHYSICAL 8
#define GRIM_FLAG_NONFINITE 16
/* the FP32-Jacobian solve failed in this zone, which was then solved again
 * from P_n with the FP64 Jacobian (the other bits are that solve's) */
#define GRIM_FLAG_F64_RETRY 32

typedef struct grim_ctx grim_ctx_t;

/* Problem and solver description, copied at create (plain value struct). */
typedef struct {
    int ndim;            /* 1, 2 or 3 active directions                      */
    int n1, n2, n3;      /* interior zones per direction (1 if inactive)     */
    int ng;              /* ghost layers per side of active directions: 2, or
                            3 for the five-point reconstructions            */
    int model;           /* GRIM_IDEAL_MHD or GRIM_EMHD                      */
    int metric;          /* GRIM_MINKOWSKI or GRIM_MKS_KERR                  */
    double x_start[3];   /* domain in X^i (Sec. 2.1)                         */
    double x_end[3];
    double spin_a;       /* Kerr spin a                                      */
    double mks_h;        /* mid-plane refinement h of eq. theta_transform    */
    int bc[3];           /* GRIM_BC_* per direction                          */
    double gamma;        /* adiabatic index, P = (gamma - 1) u               */
    double tau_R;        /* EMHD relaxation time (Sec. 4)                    */
    double chi, nu;      /* EMHD thermal and viscous diffusivities           */
    double plm_theta;    /* generalized-minmod parameter (Sec. 2.3, 2.4.1)   */
    double tol;          /* Newton tolerance on the scaled norm              */
    double eps_fd;       /* Jacobian differencing parameter (Sec. 3.1)       */
    double eps_bt;       /* line-search acceptance parameter (Sec. 3.2)      */
    int k_max;           /* maximum Newton iterations                        */
    int ls_max;          /* maximum line-search trials per iteration         */
    int jac_precision;   /* GRIM_JAC_F64 or GRIM_JAC_F32; with F32, zones whose
                            solve fails are solved again with F64 (flag
                            GRIM_FLAG_F64_RETRY, stats.n_f64_retry)          */
    int guess;           /* GRIM_GUESS_PN or GRIM_GUESS_MLP                  */
    int floors;          /* 1: rho >= rho_floor r^-3/2, u >= u_floor r^-5/2   */
    double rho_floor, u_floor;
    int ls_safeguard;    /* line search (Sec. 3.2): 0 takes each new lambda as
                            the minimiser of the quadratic model, as the paper
                            states it; 1 keeps it within [0.1, 0.5] of the
                            previous lambda (the usual safeguard of quadratic
                            backtracking)                                    */
    int external_workspace; /* 0: grim_create allocates the device memory;
                            1: it allocates none, and the caller hands over
                            grim_workspace_bytes(cfg) bytes of device memory
                            with grim_bind_workspace before any other call  */
    int stage_block;     /* threads per block of the one-kernel stage of 2-D
                            Minkowski grids: 0 chooses (512 while every tile
                            fits the device at once, else 256), 256 or 512
                            forces that size (for tests of both)             */
    int full_system;     /* GRIM_SYSTEM_REDUCED: Newton over the non-magnetic
                            primitives, B at its explicit update (5x5 / 7x7,
                            Sec. 8.2); GRIM_SYSTEM_FULL: over all nvar
                            primitives (8x8 / 10x10), B started at that update.
                            The same root.                                   */
    int riemann;         /* GRIM_RIEMANN_LLF or GRIM_RIEMANN_HLLE (Sec. 2.4.2) */
    int recon;           /* GRIM_RECON_PLM (generalized minmod), _WENO5 or _PPM
                            (Sec. 2.3, 2.4.1); the last two read three cells on
                            each side of a face: ng = 3 required              */
    int closure;         /* 0: chi and nu are the constants above; 1: per
                            state, chi = phi cs^2 tau_R and nu = psi cs^2 tau_R
                            (Sec. 4, closing paragraph), chi and nu unused    */
    double phi, psi;     /* closure constants (> 0 with closure = 1)          */
    int dp_saturation;   /* 1 (needs closure = 1): each zone's tau_R, taken at
                            P^E, is reduced smoothly where DeltaP passes the
                            firehose threshold -b^2 or the mirror threshold
                            b^2/2 (Sec. 8.1, Sec. 9): with x the anisotropy
                            over its threshold, tau = tau_R / (1 + ((x - 1) /
                            sat_width)^2) for x > 1, at least 1e-6 tau_R    */
    double sat_width;    /* > 0 with dp_saturation = 1                        */
} grim_config_t;

/* Per-call solver statistics (a13).  mean_iters is per zone per stage. */
typedef struct {
    double mean_iters[2];   /* stage 1 (half step), stage 2 (full step)      */
    int32_t max_iters;
    int32_t pad;
    int64_t n_fail;         /* zones flagged NOT_CONVERGED, SINGULAR or NONFINITE */
    int64_t n_ls_exhausted;
    int64_t n_unphysical;
    double max_resid;       /* largest final scaled residual norm            */
    int64_t zone_stages;    /* zones x stages accumulated                    */
    int64_t n_resid_calls;  /* residual evaluations R(P), summed over zones  */
    int64_t n_fallback;     /* zones whose learned guess was rejected        */
    int64_t n_f64_retry;    /* zones solved again with the FP64 Jacobian     */
    int64_t n_backtracks;   /* rejected line-search trials, summed over zones */
} grim_stats_t;

/* Adam training of the learned-guess network. */
typedef struct {
    int epochs;
    int batch;           /* rows per step                                     */
    int n_used;          /* outputs that enter the loss (5 ideal, 7 EMHD)     */
    int pad;
    double lr, beta1, beta2, eps;
    uint64_t seed;       /* shuffling                                         */
} grim_train_cfg_t;

/* Create a context: validates cfg, takes the device memory of the workspace
 * (ghosted primitive arrays of the state, the half step and the test hooks,
 * face fluxes, stage right-hand sides and EMHD coefficients, per-zone
 * results, statistics, metric tables of the grid of Sec. 2.1, the network's
 * parameters and per-zone features) in one allocation, and builds the metric
 * tables (a1).  With cfg->external_workspace = 1 it allocates no device
 * memory: the context is unusable (GRIM_E_STATE) until grim_bind_workspace.
 * hip_stream: a hipStream_t owned by the caller, or NULL.
 * Errors: GRIM_E_INVALID_ARG (bad sizes or parameters), GRIM_E_OOM, GRIM_E_HIP. */
int grim_create(const grim_config_t* cfg, void* hip_stream, grim_ctx_t** out);
int grim_destroy(grim_ctx_t* ctx);
const char* grim_last_error(const grim_ctx_t* ctx);
const char* grim_last_global_error(void);

/* Bytes of device memory the workspace of a context for cfg needs (the grid
 * of Sec. 2.1 with its ghost layers, Sec. 5.3), or 0 if cfg is invalid (the
 * reason in grim_last_global_error).  Training the network (grim_mlp_train,
 * grim_mlp_backward) allocates its batch buffers separately. */
size_t grim_workspace_bytes(const grim_config_t* cfg);

/* Hand a context created with cfg.external_workspace = 1 its workspace:
 * dev_ptr is device memory of at least grim_workspace_bytes(cfg) bytes,
 * aligned to 256 bytes, owned by the caller (e.g. a PyTorch tensor), which
 * must keep it alive and untouched until grim_destroy.  Clears the state,
 * builds the metric tables and synchronises.  Once per context.
 * Errors: GRIM_E_INVALID_ARG (null, misaligned or too small), GRIM_E_STATE
 * (the context allocates its own workspace, or one is already bound). */
int grim_bind_workspace(grim_ctx_t* ctx, void* dev_ptr, size_t bytes);

/* Device bytes the context holds or has been given (for capacity planning). */
size_t grim_device_bytes(const grim_ctx_t* ctx);

/* Copy the interior primitives in (set) or out (get).  on_device != 0 means P
 * is device memory.  Synchronises the stream. */
int grim_set_prims(grim_ctx_t* ctx, const double* P, int on_device);
int grim_get_prims(grim_ctx_t* ctx, double* P, int on_device);

/* dt = cfl * min over zones of 1 / sum_d (c_max^d / dX^d), with c_max^d the
 * largest |grid-frame speed| of the zone-centre state (Sec. 4.1).
 * Synchronises the stream. */
int grim_cfl_dt(grim_ctx_t* ctx, double cfl, double* dt);

/* Advance nsteps full steps of size dt (Sec. 2.3: half step with P^E = P_n,
 * dt' = dt/2, then full step with P^E = P_{n+1/2}, dt' = dt; both Newton
 * solves start from P_n with B at its explicit update).  Asynchronous unless
 * stats != NULL, in which case the statistics of these steps are returned.
 * use_graph != 0 replays captured HIP graphs of sixteen steps (and of one
 * step for the remainder), captured on the first call for this dt. */
int grim_run(grim_ctx_t* ctx, double dt, int nsteps, int use_graph, grim_stats_t* stats);

/* Test hook for a8: the residual R(P) of every interior zone for a stage with
 * P_n, P^E and dt' (eqs. half_step_residual / full_step), all nvar rows, and
 * the scaled Newton norm ||R|| = sqrt(sum_v (dt' R_v)^2) / U_rho(P_n) over
 * the rows of the Newton system (the non-magnetic rows, Sec. 8.2).  All
 * pointers device, interior layout; rnorm may be NULL. */
int grim_residual(grim_ctx_t* ctx, const double* Pn, const double* PE, double dtp,
                  const double* P, double* R, double* rnorm);

/* Test hook for a2-a12: one stage.  Flux stage on P^E, then the Newton solve
 * from guess (NULL: P_n) with B at its explicit update.  Outputs per zone:
 * P_out (interior layout), iterations, final scaled norm, flags and the
 * rejected line-search trials (Sec. 3.2); any of iters / resid / flags /
 * backtracks may be NULL.  All those pointers device.  stats (host, may be
 * NULL) receives the statistics of this stage (in mean_iters[0]). */
int grim_stage_solve(grim_ctx_t* ctx, const double* Pn, const double* PE, double dtp,
                     const double* guess, double* P_out, int32_t* iters, double* resid,
                     uint8_t* flags, int32_t* backtracks, grim_stats_t* stats);

/* Test hook for a2-a6: divF (eq. fvm_formulation, with flux-CT), the explicit
 * geometric source sqrt(-g) T^k_l Gamma^l_{nu k} at P^E (eq. divT_explicit)
 * and, for EMHD, the three P^E-only source parts per zone (spatial-derivative
 * and connection parts of the q0 and DeltaP0 targets and of div u).
 * divF, srcE: [nvar][zones]; emhd_sp: [zones][3] or NULL.  Device pointers. */
int grim_explicit(grim_ctx_t* ctx, const double* PE, double* divF, double* srcE,
                  double* emhd_sp);

/* Per-zone flags (GRIM_FLAG_*) and iteration counts of the last stage-2
 * solve (or last grim_stage_solve).  on_device as for grim_set_prims. */
int grim_get_zone_results(grim_ctx_t* ctx, uint8_t* flags, int32_t* iters, int on_device);

/* Kernel timing for the roofline measurement.  While enabled, grim_run
 * enqueues steps eagerly (no graph) and brackets every launch group with HIP
 * events on the context's stream.  grim_kernel_times synchronises and returns,
 * per kernel group, the summed device time in ms and the number of launches,
 * then clears the records.  Groups: 0 ghost fill (no longer launched inside
 * a step: the Newton kernel writes the ghosts), 1 face fluxes (all
 * directions, one launch), 2 flux-CT EMFs (now evaluated inside the stage
 * right-hand side: always empty), 3 stage right-hand side, 4 Newton solve,
 * 5 network inference (n = 6 entries). */
int grim_profile(grim_ctx_t* ctx, int enable);
int grim_kernel_times(grim_ctx_t* ctx, double* ms, int64_t* launches, int n);

/* ---- learned initial guess (spec: learned part) -------------------
 * Network 32 -> 128 -> 128 -> 16 with GELU, parameters one FP32 vector of
 * GRIM_MLP_PARAMS values: W1 [32][128], b1, W2 [128][128], b2, W3 [128][16],
 * b3, x_mean [32], x_istd [32], y_scale [16];
 *   y = (gelu(gelu(((x - x_mean) x_istd) W1 + b1) W2 + b2) W3 + b3) y_scale.
 * Inputs per zone (dimensionless): (dt' rhs_v - U_v(P_n)) / U_rho(P_n) for
 * every row v, u/rho, utilde^i, B^i/sqrt(rho), q/u, DP/u (EMHD), and the lapse,
 * g^{01}, g^{11} in the last three slots.  Outputs: (rho - rho_n)/rho_n,
 * (u - u_n)/u_n, utilde - utilde_n, (q - q_n)/u_n, (DP - DP_n)/u_n.
 * With cfg.guess = GRIM_GUESS_MLP each stage evaluates the network (BF16
 * matrix cores, FP32 accumulation) and each zone starts Newton from the
 * prediction if its residual norm is below that of P_n, and falls back to P_n
 * otherwise or if the solve from the prediction fails (stats.n_fallback).
 * Errors: GRIM_E_STATE if the guess is requested before weights are set. */

/* Copy n = GRIM_MLP_PARAMS FP32 values in from / out to host memory. */
int grim_mlp_set_weights(grim_ctx_t* ctx, const float* w, size_t n);
int grim_mlp_get_weights(grim_ctx_t* ctx, float* w, size_t n);

/* Inference on n rows: X [n][32] -> Y [n][16], device pointers, BF16 matrix
 * cores with FP32 accumulation (the path the solver uses).  Synchronises. */
int grim_mlp_forward(grim_ctx_t* ctx, const float* X, int64_t n, float* Y);

/* FP32 gradient of sum(dY * y(X)) with respect to all parameters (zero for the
 * normalisation entries).  X [n][32], dY [n][16], dW [GRIM_MLP_PARAMS], device
 * pointers.  Synchronises. */
int grim_mlp_backward(grim_ctx_t* ctx, const float* X, const float* dY, int64_t n, float* dW);

/* The gradient of grim_mlp_backward for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving or training loops,
 * harnesses that forbid hipMalloc): same arguments and result, but it calls
 * no allocating routine.  Its work buffers live in a device array of the
 * library (about 6.9 MB on each GPU it runs on, held until the process
 * ends) that holds at most 2048 rows: n must be in [1, 2048]
 * (GRIM_E_INVALID_ARG beyond).  Asynchronous: enqueued on the context's
 * stream, with no synchronisation, so it may be captured; dW is ready when
 * that stream has reached it.  Every call on one GPU shares that array,
 * whatever the context: calls that overlap on one GPU (two streams, or two
 * host threads) race, and the caller must order them.  Errors as for
 * grim_mlp_backward. */
int grim_mlp_backward_noalloc(grim_ctx_t* ctx, const float* X, const float* dY, int64_t n, float* dW);

/* Adam on the mean squared error over the first n_used outputs, on n pairs
 * X [n][32], T [n][16] (device); shuffled each epoch; FP32 master weights,
 * normalisation entries fixed.  loss_hist (host, cfg->epochs doubles, may be
 * NULL) receives the mean training loss of every epoch.  Synchronises. */
int grim_mlp_train(grim_ctx_t* ctx, const float* X, const float* T, int64_t n, const grim_train_cfg_t* cfg,
                   double* loss_hist);

/* Normalisation of the network from n training pairs X [n][32], T [n][16]
 * (device): x_mean[c] and the unbiased standard deviation s_c of every input
 * column, x_istd[c] = 1/s_c (0 for a column that is constant over the pairs),
 * and y_scale[c] = the unbiased standard deviation of target column c for
 * c < n_used, 0 otherwise (an output constant over the pairs or unused is held
 * at exactly zero).  Sums in FP64, in a fixed order (deterministic).  Output
 * arrays are host memory of 32, 32 and 16 doubles.  Synchronises.
 * Errors: GRIM_E_INVALID_ARG (n < 2, n_used outside [1, 16], null pointers). */
int grim_mlp_normalisation(grim_ctx_t* ctx, const float* X, const float* T, int64_t n, int n_used,
                           double* x_mean, double* x_istd, double* y_scale);

/* Training pairs from the plain FP64 solver: run nsteps full steps of size dt
 * (eager, guess P_n) and after every stage store the network inputs and the
 * scaled target (P - P_n) of the zones z = phase (mod stride), phase advancing
 * by one per stage, into X [cap][32], T [cap][16] (device).  *count receives
 * the number of pairs produced (those beyond cap are dropped).  Advances the
 * state. */
int grim_collect_pairs(grim_ctx_t* ctx, double dt, int nsteps, int stride, float* X, float* T, int64_t cap,
                       int64_t* count);

/* STREAM c = a + b over n doubles (the sustained-bandwidth yardstick of
 * Sec. 7.2).  a, b, c device pointers.  Enqueued, not timed. */
int grim_stream_add(grim_ctx_t* ctx, const double* a, const double* b, double* c, size_t n);

/* Test hook for the arithmetic of the hot loops: for each x[i] (device, n
 * doubles) writes the library's reciprocal, inverse square root and square
 * root (the hardware estimates refined by two Newton-Raphson steps) to
 * out[3i], out[3i + 1], out[3i + 2] (device).  Synchronises. */
int grim_math_probe(grim_ctx_t* ctx, const double* x, double* out, size_t n);

#ifdef __cplusplus
}
#endif
#endif
