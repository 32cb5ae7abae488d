/*
 * Plain FP64 CPU oracle of the grim method (Chandra, Foucart & Gammie,
 * "grim: A Flexible, Conservative Scheme for Relativistic Fluid Theories").
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU
 * baseline leg of the benchmark are the only code that may load this
 * library.  The GPU library neither links nor includes anything from here,
 * and nothing here includes anything from the GPU library.
 *
 * Arrays of primitives are structure-of-arrays, [nvar][n3][n2][n1] for the
 * interior-only API, i fastest.  Primitive order (Sec. 4, closing summary):
 *   0 rho, 1 u, 2..4 normal-observer four-velocity utilde^i, 5..7 B^i,
 *   8 q, 9 DeltaP (EMHD only).
 */
#ifndef GRIM_ORACLE_H
#define GRIM_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int ndim;              /* 1, 2 or 3 active directions (X1, X1-X2, X1-X3) */
    int n1, n2, n3;        /* interior zones (inactive directions: 1)       */
    int ng;                /* ghost layers on each side of active directions */
    int nvar;              /* 8 ideal MHD, 10 EMHD                            */
    int metric;            /* 0 Minkowski Cartesian, 1 modified Kerr-Schild  */
    int bc1, bc2, bc3;     /* 0 periodic, 1 outflow copy, 2 polar reflection */
    double x1s, x2s, x3s;  /* start of the domain in X^i                      */
    double dx1, dx2, dx3;  /* zone widths in X^i                              */
    double spin, hslope;   /* Kerr spin a, mid-plane refinement h             */
    double gam;            /* adiabatic index                                 */
    double tau_R, chi, nu; /* EMHD relaxation time and diffusivities          */
    double theta_plm;      /* generalized-minmod parameter                    */
    double tol, eps, eps_bt;
    int k_max, ls_max;
    int ls_safeguard;      /* 0: the update of Sec. 3.2 as printed; 1: each new
                              lambda kept in [0.1, 0.5] of the previous one  */
    int floors;            /* 1: rho >= rho_fl r^-3/2, u >= u_fl r^-5/2        */
    double rho_fl, u_fl;
    int nthreads;          /* OpenMP threads, 0 = runtime default             */
    int full_system;       /* 0: Newton over the non-magnetic unknowns (5x5 /
                              7x7, Sec. 8.2); 1: over all nvar primitives     */
    int riemann;           /* 0 LLF, 1 HLLE (Sec. 2.4.2)                       */
    int recon;             /* 0 PLM (generalized minmod), 1 WENO5, 2 PPM
                              (Sec. 2.3; the last two need ng >= 3)          */
    int closure;           /* 0: chi, nu as given; 1: chi = phi cs^2 tau_R,
                              nu = psi cs^2 tau_R (Sec. 4, closing paragraph) */
    double phi, psi;
    int dp_saturation;     /* 1: tau_R reduced smoothly where DeltaP leaves
                              [-b^2, b^2/2] (Sec. 8.1 firehose, Sec. 9); needs
                              closure = 1                                    */
    double sat_width;      /* relative overshoot that halves tau_R            */
} ocfg_t;

typedef struct {
    double iters_sum[2];   /* per stage: sum of Newton iterations            */
    int64_t zones;         /* interior zones per stage                       */
    int32_t max_iters;
    int64_t n_fail;        /* zones with NOT_CONVERGED/SINGULAR/NONFINITE    */
    int64_t n_ls_exhausted;
    int64_t n_unphysical;
    double max_resid;
    int64_t n_backtracks;  /* rejected line-search trials, summed over zones */
} ostats_t;

/* per-zone flags */
#define OFLAG_NOT_CONVERGED 1
#define OFLAG_LS_EXHAUSTED  2
#define OFLAG_SINGULAR      4
#define OFLAG_UNPHYSICAL    8
#define OFLAG_NONFINITE     16

/* Face states of one variable between cells i-1 and i from the values of
 * cells i-3..i+2 (s[0..5]; PLM reads s[1..4]) with the configured
 * reconstruction. */
void   oracle_reconstruct(const ocfg_t* c, const double* s, double* left, double* right);
int    oracle_stage(const ocfg_t* c, const double* Pn, const double* PE,
                    double dtp, const double* guess, double* Pout,
                    int32_t* iters, double* resid, uint8_t* flags);
/* As oracle_stage, with P^E given on the ghosted grid ([nvar][N3][N2][N1],
 * N = n + 2 ng on active directions): its ghosts are used as they are, not
 * refilled from the boundary conditions, so a subdomain of a larger grid can
 * be advanced with the halo taken from that grid.  backtracks (may be NULL)
 * receives the rejected line-search trials of every zone. */
int    oracle_stage_ghosted(const ocfg_t* c, const double* Pn, const double* PEg,
                            double dtp, const double* guess, double* Pout,
                            int32_t* iters, double* resid, uint8_t* flags,
                            int32_t* backtracks);
int    oracle_step(const ocfg_t* c, double* P, double dt, ostats_t* st);
int    oracle_run(const ocfg_t* c, double* P, double dt, int nsteps, ostats_t* st);
/* As oracle_residual, with P^E given on the ghosted grid (ghosts as given). */
int    oracle_residual_ghosted(const ocfg_t* c, const double* Pn, const double* PEg, double dtp,
                               const double* P, double* R, double* rnorm);
int    oracle_residual(const ocfg_t* c, const double* Pn, const double* PE,
                       double dtp, const double* P, double* R, double* rnorm);
int    oracle_explicit(const ocfg_t* c, const double* PE, double* divF,
                       double* srcE, double* emhd_sp);
double oracle_cfl_dt(const ocfg_t* c, const double* P, double cfl);
void   oracle_geometry(const ocfg_t* c, const double* X, double* gcov,
                       double* gcon, double* gdet, double* alpha);
void   oracle_connection(const ocfg_t* c, const double* X, double* conn);
void   oracle_prim_to_flux(const ocfg_t* c, const double* P, const double* X,
                           int dir, double* out);
void   oracle_speeds(const ocfg_t* c, const double* P, const double* X, int dir,
                     double* lp, double* lm);
double oracle_vmax2(const ocfg_t* c, const double* P, const double* X);
int    oracle_solve(int n, const double* A, const double* b, double* x);
double oracle_ls_lambda(double f0, double f1, double lam);
typedef void (*oresid_fn)(void* ctx, const double* x, double* r);
int    oracle_newton_generic(int n, oresid_fn fn, void* ctx, double* x,
                             double nscale, double tol, double eps,
                             double eps_bt, int k_max, int ls_max,
                             int ls_safeguard, int32_t* iters, double* resid,
                             uint8_t* flags, int32_t* backtracks);
void   oracle_fd_jacobian(int n, oresid_fn fn, void* ctx, const double* x,
                          const double* R, double eps, double* J);
int    oracle_zone_jacobian(const ocfg_t* c, const double* Pn, const double* PE,
                            double dtp, const double* P, long z, double* J,
                            double* Rz);
/* Per zone, the FD Jacobian of the Newton system at P (J [nz][m][m],
 * m = nvar - 3) and U_rho(P_n), for a stage with ghost-filled P^E. */
int    oracle_system_jacobians_ghosted(const ocfg_t* c, const double* Pn, const double* PEg, double dtp,
                                       const double* P, double* J, double* urho);
/* Interior P [nvar][n3][n2][n1] -> ghosted Pg [nvar][N3][N2][N1] with the
 * ghosts filled by the boundary conditions of c. */
int    oracle_fill_ghosts(const ocfg_t* c, const double* Pint, double* Pg);
int    oracle_divb(const ocfg_t* c, const double* P, double* divb);
int    oracle_sum_U(const ocfg_t* c, const double* P, double* sums);

#ifdef __cplusplus
}
#endif
#endif
