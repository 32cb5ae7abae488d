/*
 * Plain FP64 CPU oracle of the grim method (Chandra, Foucart & Gammie,
 * "grim: A Flexible, Conservative Scheme for Relativistic Fluid Theories").
 *
 * TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU
 * baseline leg of the benchmark are the only code that may load this
 * library.  It shares no source with the GPU library.
 *
 * The code is deliberately plain: one zone at a time, no blocking, no
 * fusion, geometry recomputed wherever it is needed.  Each routine names the
 * passage of the paper it follows.  Where the paper is silent, garbled or
 * inconsistent, the reading taken is stated beside the code and listed in
 * the design notes of the repository.
 */
#include "grim_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { RHO = 0, UU = 1, U1 = 2, U2 = 3, U3 = 4, B1 = 5, B2 = 6, B3 = 7, QQ = 8, DP = 9 };
#define NVMAX 10

/* ------------------------------------------------------------------------ */
/* grid layout                                                               */
/* ------------------------------------------------------------------------ */

typedef struct {
    int N[3];   /* ghosted extents */
    int g[3];   /* ghost offsets (0 for inactive directions) */
    int n[3];   /* interior extents */
    size_t cells;
} olay_t;

static olay_t o_layout(const ocfg_t* c)
{
    olay_t L;
    L.n[0] = c->n1;
    L.n[1] = c->ndim >= 2 ? c->n2 : 1;
    L.n[2] = c->ndim >= 3 ? c->n3 : 1;
    for (int d = 0; d < 3; ++d) {
        L.g[d] = (d < c->ndim) ? c->ng : 0;
        L.N[d] = L.n[d] + 2 * L.g[d];
    }
    L.cells = (size_t)L.N[0] * L.N[1] * L.N[2];
    return L;
}

static size_t o_cell(const olay_t* L, int i, int j, int k)
{
    return ((size_t)k * L->N[1] + j) * L->N[0] + i;
}

static size_t o_zones(const olay_t* L)
{
    return (size_t)L->n[0] * L->n[1] * L->n[2];
}

static void o_zone_X(const ocfg_t* c, const olay_t* L, int i, int j, int k, double X[4])
{
    X[0] = 0.0;
    X[1] = c->x1s + (i - L->g[0] + 0.5) * c->dx1;
    X[2] = c->x2s + (j - L->g[1] + 0.5) * c->dx2;
    X[3] = c->x3s + (k - L->g[2] + 0.5) * c->dx3;
}

static double o_dx(const ocfg_t* c, int d)
{
    return d == 0 ? c->dx1 : (d == 1 ? c->dx2 : c->dx3);
}

/* ------------------------------------------------------------------------ */
/* geometry (Sec. 2.1, eq. theta_transform and the matrix L)                 */
/* ------------------------------------------------------------------------ */

typedef struct {
    double gcov[4][4], gcon[4][4], gdet, alpha;
} ogeom_t;

/* Inverse and determinant of a 4x4 matrix by Gauss-Jordan elimination with
 * partial pivoting. */
static double o_inv4(const double A[4][4], double Ai[4][4])
{
    double M[4][8];
    double det = 1.0;
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 8; ++j) M[i][j] = (j < 4) ? A[i][j] : (j - 4 == i ? 1.0 : 0.0);
    for (int k = 0; k < 4; ++k) {
        int p = k;
        for (int i = k + 1; i < 4; ++i)
            if (fabs(M[i][k]) > fabs(M[p][k])) p = i;
        if (p != k) {
            for (int j = 0; j < 8; ++j) { double t = M[k][j]; M[k][j] = M[p][j]; M[p][j] = t; }
            det = -det;
        }
        double piv = M[k][k];
        det *= piv;
        for (int j = 0; j < 8; ++j) M[k][j] /= piv;
        for (int i = 0; i < 4; ++i) {
            if (i == k) continue;
            double f = M[i][k];
            for (int j = 0; j < 8; ++j) M[i][j] -= f * M[k][j];
        }
    }
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) Ai[i][j] = M[i][j + 4];
    return det;
}

/* Covariant metric at coordinate point X.
 * Minkowski: diag(-1, 1, 1, 1) in Cartesian X^i.
 * Modified Kerr-Schild: Kerr in Kerr-Schild (t, r, theta, phi), mapped with
 * r = exp(X1), theta = pi X2 + (1-h)/2 sin(2 pi X2), phi = X3 (Sec. 2.1),
 * g_{mu nu}(X) = g_{ab}(x) L^a_mu L^b_nu with L = diag(1, r, dtheta/dX2, 1).
 * Reading: near the axis sin^2(theta) is kept >= 1e-24 so that the inverse
 * metric stays finite on the polar faces; theta itself is not clamped, so
 * ghost zones across the axis see the mirror image of the metric. */
static void o_metric_cov(const ocfg_t* c, const double X[4], double g[4][4])
{
    memset(g, 0, sizeof(double) * 16);
    if (c->metric == 0) {
        g[0][0] = -1.0; g[1][1] = 1.0; g[2][2] = 1.0; g[3][3] = 1.0;
        return;
    }
    const double a = c->spin, h = c->hslope;
    double r = exp(X[1]);
    double th = M_PI * X[2] + 0.5 * (1.0 - h) * sin(2.0 * M_PI * X[2]);
    double dr_dX1 = r;
    double dth_dX2 = M_PI * (1.0 + (1.0 - h) * cos(2.0 * M_PI * X[2]));
    double cth = cos(th), sth = sin(th), s2 = sth * sth;
    if (s2 < 1e-24) s2 = 1e-24;
    double Sig = r * r + a * a * cth * cth;
    double ks[4][4];
    memset(ks, 0, sizeof(ks));
    ks[0][0] = -(1.0 - 2.0 * r / Sig);
    ks[0][1] = ks[1][0] = 2.0 * r / Sig;
    ks[0][3] = ks[3][0] = -2.0 * a * r * s2 / Sig;
    ks[1][1] = 1.0 + 2.0 * r / Sig;
    ks[1][3] = ks[3][1] = -a * s2 * (1.0 + 2.0 * r / Sig);
    ks[2][2] = Sig;
    ks[3][3] = s2 * (Sig + a * a * s2 * (1.0 + 2.0 * r / Sig));
    double Ld[4] = {1.0, dr_dX1, dth_dX2, 1.0};
    for (int m = 0; m < 4; ++m)
        for (int n = 0; n < 4; ++n) g[m][n] = ks[m][n] * Ld[m] * Ld[n];
}

static void o_geom(const ocfg_t* c, const double X[4], ogeom_t* G)
{
    o_metric_cov(c, X, G->gcov);
    double det = o_inv4(G->gcov, G->gcon);
    G->gdet = sqrt(fabs(det));
    G->alpha = 1.0 / sqrt(-G->gcon[0][0]);
}

/* Christoffel symbols conn[l][a][b] = Gamma^l_{ab}
 * = 1/2 g^{lk} (d_a g_kb + d_b g_ka - d_k g_ab).  Reading: the paper does not
 * say how the metric is differentiated; here each d_k g_ab is the
 * fourth-order central difference with step 1e-3 in X^k,
 *   (8 (g(X+h) - g(X-h)) - (g(X+2h) - g(X-2h))) / (12 h),
 * whose truncation (~h^4) and rounding (~eps/h) errors are both ~1e-12
 * relative here. */
static void o_conn(const ocfg_t* c, const double X[4], double conn[4][4][4])
{
    const double del = 1e-3;
    double dg[4][4][4]; /* dg[k][a][b] = d_k g_ab */
    for (int k = 0; k < 4; ++k) {
        double g[4][4][4]; /* metric at X + s del e_k, s = -2, -1, 1, 2 */
        const int sh[4] = {-2, -1, 1, 2};
        for (int q = 0; q < 4; ++q) {
            double Xs[4];
            for (int m = 0; m < 4; ++m) Xs[m] = X[m];
            Xs[k] += sh[q] * del;
            o_metric_cov(c, Xs, g[q]);
        }
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b)
                dg[k][a][b] = (8.0 * (g[2][a][b] - g[1][a][b]) - (g[3][a][b] - g[0][a][b])) / (12.0 * del);
    }
    ogeom_t G;
    o_geom(c, X, &G);
    for (int l = 0; l < 4; ++l)
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) {
                double s = 0.0;
                for (int k = 0; k < 4; ++k)
                    s += G.gcon[l][k] * (dg[a][k][b] + dg[b][k][a] - dg[k][a][b]);
                conn[l][a][b] = 0.5 * s;
            }
}

/* ------------------------------------------------------------------------ */
/* derived quantities of a primitive state (Sec. 4)                          */
/* ------------------------------------------------------------------------ */

typedef struct {
    double ucon[4], ucov[4], bcon[4], bcov[4];
    double bhcon[4], bhcov[4];
    double bsq, pg, gamL;
} ostate_t;

/* The velocity primitives are read as the normal-observer four-velocity
 * utilde^i (the paper inherits the harm convention); they equal u^i in
 * Minkowski.  b^t = B^i u_i, b^i = (B^i + b^t u^i)/u^t (Sec. 4), P = (gamma-1)u.
 * The unit vector bhat = b / sqrt(b^2) is set to zero when b^2 < 1e-30. */
static void o_state(const ocfg_t* c, const double* P, const ogeom_t* G, ostate_t* S)
{
    double qsq = 0.0;
    for (int i = 1; i < 4; ++i)
        for (int j = 1; j < 4; ++j) qsq += G->gcov[i][j] * P[U1 + i - 1] * P[U1 + j - 1];
    S->gamL = sqrt(1.0 + qsq);
    S->ucon[0] = S->gamL / G->alpha;
    for (int i = 1; i < 4; ++i)
        S->ucon[i] = P[U1 + i - 1] - S->gamL * G->alpha * G->gcon[0][i];
    for (int m = 0; m < 4; ++m) {
        S->ucov[m] = 0.0;
        for (int n = 0; n < 4; ++n) S->ucov[m] += G->gcov[m][n] * S->ucon[n];
    }
    S->bcon[0] = 0.0;
    for (int i = 1; i < 4; ++i) S->bcon[0] += P[B1 + i - 1] * S->ucov[i];
    for (int i = 1; i < 4; ++i)
        S->bcon[i] = (P[B1 + i - 1] + S->bcon[0] * S->ucon[i]) / S->ucon[0];
    for (int m = 0; m < 4; ++m) {
        S->bcov[m] = 0.0;
        for (int n = 0; n < 4; ++n) S->bcov[m] += G->gcov[m][n] * S->bcon[n];
    }
    S->bsq = 0.0;
    for (int m = 0; m < 4; ++m) S->bsq += S->bcon[m] * S->bcov[m];
    S->pg = (c->gam - 1.0) * P[UU];
    if (S->bsq > 1e-30) {
        double bm = sqrt(S->bsq);
        for (int m = 0; m < 4; ++m) { S->bhcon[m] = S->bcon[m] / bm; S->bhcov[m] = S->bcov[m] / bm; }
    } else {
        for (int m = 0; m < 4; ++m) { S->bhcon[m] = 0.0; S->bhcov[m] = 0.0; }
    }
}

/* Mixed stress tensor T^mu_nu (eq. fullSEtens with q^mu = q bhat^mu and
 * Pi^{mu nu} = -DeltaP (bhat^mu bhat^nu - h^{mu nu}/3)).  Expanding
 * h = g + u u turns the first two terms into
 * (rho + u + P + b^2) u^mu u_nu + (P + b^2/2) delta^mu_nu. */
static void o_tmunu(const ocfg_t* c, const double* P, const ostate_t* S, double T[4][4])
{
    double w = P[RHO] + P[UU] + S->pg + S->bsq;
    double pt = S->pg + 0.5 * S->bsq;
    for (int m = 0; m < 4; ++m)
        for (int n = 0; n < 4; ++n) {
            double t = w * S->ucon[m] * S->ucov[n] + (m == n ? pt : 0.0) - S->bcon[m] * S->bcov[n];
            if (c->nvar == 10) {
                double hmn = (m == n ? 1.0 : 0.0) + S->ucon[m] * S->ucov[n];
                t += P[QQ] * (S->bhcon[m] * S->ucov[n] + S->ucon[m] * S->bhcov[n]);
                t -= P[DP] * (S->bhcon[m] * S->bhcov[n] - hmn / 3.0);
            }
            T[m][n] = t;
        }
}

/* Sound speed squared of a state, cs^2 = gamma (gamma-1) u / (rho + gamma u)
 * (Sec. 4.1, below eq. modcs). */
static double o_cs2(const ocfg_t* c, const double* P)
{
    return c->gam * (c->gam - 1.0) * P[UU] / (P[RHO] + c->gam * P[UU]);
}

/* chi / tau_R and nu / tau_R of a state.  Without the closure both are the
 * given constants over the given tau_R; with the closure of Sec. 4 (closing
 * paragraph), chi = phi cs^2 tau_R and nu = psi cs^2 tau_R, so the ratios
 * are phi cs^2 and psi cs^2 whatever tau_R is. */
static void o_diff_over_tau(const ocfg_t* c, const double* P, double* chi_t, double* nu_t)
{
    if (c->closure) {
        double cs2 = o_cs2(c, P);
        *chi_t = c->phi * cs2;
        *nu_t = c->psi * cs2;
    } else {
        *chi_t = c->chi / c->tau_R;
        *nu_t = c->nu / c->tau_R;
    }
}

/* Rescaled dissipative variables, eqs. (q) and (dP):
 * qtilde = q sqrt(tau_R / (chi rho Theta^2)), DPtilde = DP sqrt(tau_R / (nu rho Theta)),
 * with Theta = P/rho, chi and nu those of the state itself. */
static void o_rescaled(const ocfg_t* c, const double* P, const ostate_t* S, double* qt, double* dpt)
{
    double theta = S->pg / P[RHO];
    if (c->closure) {
        double chi_t, nu_t;
        o_diff_over_tau(c, P, &chi_t, &nu_t);
        *qt = P[QQ] * sqrt(1.0 / (chi_t * P[RHO] * theta * theta));
        *dpt = P[DP] * sqrt(1.0 / (nu_t * P[RHO] * theta));
    } else {
        *qt = P[QQ] * sqrt(c->tau_R / (c->chi * P[RHO] * theta * theta));
        *dpt = P[DP] * sqrt(c->tau_R / (c->nu * P[RHO] * theta));
    }
}

/* The relaxation time of a zone's stage, taken at P^E.  Without saturation
 * it is tau_R.  With it (reading: the paper saturates DeltaP at the firehose
 * threshold -b^2 and the mirror threshold b^2/2 by reducing tau_R smoothly,
 * Sec. 8.1 and Sec. 9, and gives no formula): x = -DeltaP/b^2 for DeltaP < 0
 * and x = 2 DeltaP/b^2 for DeltaP > 0 measure the anisotropy against its
 * threshold, and tau = tau_R for x <= 1, tau = tau_R / (1 + ((x-1)/w)^2)
 * beyond (w = sat_width, a C^1 switch), never below 1e-6 tau_R; b^2 is
 * floored at 1e-30.  With the closure chi and nu scale with tau, so DeltaP_0
 * shrinks with it and the relaxation toward it speeds up. */
static double o_tau_eff(const ocfg_t* c, const double* P, const ostate_t* S)
{
    if (!c->dp_saturation) return c->tau_R;
    double b2 = S->bsq > 1e-30 ? S->bsq : 1e-30;
    double x = P[DP] < 0.0 ? -P[DP] / b2 : 2.0 * P[DP] / b2;
    double f = 1.0;
    if (x > 1.0) {
        double y = (x - 1.0) / c->sat_width;
        f = 1.0 / (1.0 + y * y);
        if (f < 1e-6) f = 1e-6;
    }
    return c->tau_R * f;
}

/* dir = 0: conserved vector U; dir = d in 1..3: flux F^d.
 * Rows: sqrt(-g) (rho u^dir, T^dir_nu (nu = 0..3), induction, qtilde u^dir,
 * DPtilde u^dir) (eqs. divN_explicit, divT_explicit, induction_eqn,
 * q_evol_eqn_rescaled, dP_evol_eqn_rescaled).
 * Reading: the induction flux is F^j_{B^i} = sqrt(-g)(b^i u^j - b^j u^i).
 * The paper prints the opposite sign, which would advect B against the flow
 * (and turns Alfven waves unstable); the sign here is the one that follows
 * from the divergence of the dual field tensor with B^i = *F^{it}.  For
 * dir = 0 the row reduces to sqrt(-g) B^i. */
static void o_flux_from_state(const ocfg_t* c, const double* P, const ogeom_t* G, const ostate_t* S,
                              int dir, double* out)
{
    double T[4][4];
    o_tmunu(c, P, S, T);
    out[RHO] = G->gdet * P[RHO] * S->ucon[dir];
    for (int n = 0; n < 4; ++n) out[UU + n] = G->gdet * T[dir][n];
    for (int i = 1; i < 4; ++i)
        out[B1 + i - 1] = G->gdet * (S->bcon[i] * S->ucon[dir] - S->bcon[dir] * S->ucon[i]);
    if (c->nvar == 10) {
        double qt, dpt;
        o_rescaled(c, P, S, &qt, &dpt);
        out[QQ] = G->gdet * qt * S->ucon[dir];
        out[DP] = G->gdet * dpt * S->ucon[dir];
    }
}

/* Upper bound on the fluid-frame wave speed (Sec. 4.1, eq. modcs):
 * v_max^2 = ct^2 + vA^2 - ct^2 vA^2, vA^2 = b^2/(rho + gamma u + b^2),
 * cs^2 = gamma (gamma-1) u/(rho + gamma u),
 * ct^2 = (cs^2 + vq^2 + sqrt(cs^4 + vq^4))/2 + vdP^2,
 * vq^2 = (gamma-1) chi/tau_R, vdP^2 = 4 nu/(3 tau_R), chi and nu those of the
 * state (o_diff_over_tau).  Ideal MHD: ct = cs. */
static double o_vmax2_state(const ocfg_t* c, const double* P, const ostate_t* S)
{
    double g = c->gam;
    double cs2 = g * (g - 1.0) * P[UU] / (P[RHO] + g * P[UU]);
    double va2 = S->bsq / (P[RHO] + g * P[UU] + S->bsq);
    double ct2 = cs2;
    if (c->nvar == 10) {
        double vq2, vd2;
        if (c->closure) {
            vq2 = (g - 1.0) * c->phi * cs2;
            vd2 = 4.0 * c->psi * cs2 / 3.0;
        } else {
            vq2 = (g - 1.0) * c->chi / c->tau_R;
            vd2 = 4.0 * c->nu / (3.0 * c->tau_R);
        }
        ct2 = 0.5 * (cs2 + vq2 + sqrt(cs2 * cs2 + vq2 * vq2)) + vd2;
    }
    return ct2 + va2 - ct2 * va2;
}

/* Grid-frame speeds of waves moving at +-v_max in the fluid frame along
 * direction dir (Sec. 4.1).  A wave covector k = (-lambda, e_dir) at fluid-frame
 * phase speed v satisfies (k.u)^2 = v^2 (k.k + (k.u)^2), a quadratic in
 * lambda. */
static void o_speeds_state(const ocfg_t* c, const double* P, const ogeom_t* G, const ostate_t* S,
                           int dir, double* lp, double* lm)
{
    double v2 = o_vmax2_state(c, P, S);
    double u0 = S->ucon[0], ud = S->ucon[dir];
    double A = (1.0 - v2) * u0 * u0 - v2 * G->gcon[0][0];
    double B = -2.0 * ((1.0 - v2) * u0 * ud - v2 * G->gcon[0][dir]);
    double C = (1.0 - v2) * ud * ud - v2 * G->gcon[dir][dir];
    double disc = B * B - 4.0 * A * C;
    if (disc < 0.0) disc = 0.0;
    double sq = sqrt(disc);
    double x1 = (-B + sq) / (2.0 * A), x2 = (-B - sq) / (2.0 * A);
    *lp = x1 > x2 ? x1 : x2;
    *lm = x1 > x2 ? x2 : x1;
}

/* ------------------------------------------------------------------------ */
/* reconstruction and Riemann solver (Sec. 2.4)                              */
/* ------------------------------------------------------------------------ */

/* generalized minmod slope minmod(theta a, (a+b)/2, theta b) */
static double o_gmm(double a, double b, double th)
{
    double x = th * a, y = 0.5 * (a + b), z = th * b;
    if (x > 0.0 && y > 0.0 && z > 0.0) return fmin(x, fmin(y, z));
    if (x < 0.0 && y < 0.0 && z < 0.0) return fmax(x, fmax(y, z));
    return 0.0;
}

static size_t o_stride(const olay_t* L, int d)
{
    return d == 0 ? 1 : (d == 1 ? (size_t)L->N[0] : (size_t)L->N[0] * L->N[1]);
}

/* WENO5 (Jiang & Shu's fifth-order weighted essentially non-oscillatory
 * interpolation, the scheme Sec. 2.3 names): the value at the right face of
 * the middle cell of the five equally spaced cell values a..e, as the
 * weighted mean of the three third-order values of the stencils (a,b,c),
 * (b,c,d), (c,d,e), with ideal weights 1/10, 6/10, 3/10 and the
 * smoothness indicators of that method; epsilon = 1e-6 (reading: the paper
 * gives none). */
static double o_weno5(double a, double b, double cc, double d, double e)
{
    double q0 = (2.0 * a - 7.0 * b + 11.0 * cc) / 6.0;
    double q1 = (-b + 5.0 * cc + 2.0 * d) / 6.0;
    double q2 = (2.0 * cc + 5.0 * d - e) / 6.0;
    double s0 = 13.0 / 12.0 * (a - 2.0 * b + cc) * (a - 2.0 * b + cc) + 0.25 * (a - 4.0 * b + 3.0 * cc) * (a - 4.0 * b + 3.0 * cc);
    double s1 = 13.0 / 12.0 * (b - 2.0 * cc + d) * (b - 2.0 * cc + d) + 0.25 * (b - d) * (b - d);
    double s2 = 13.0 / 12.0 * (cc - 2.0 * d + e) * (cc - 2.0 * d + e) + 0.25 * (3.0 * cc - 4.0 * d + e) * (3.0 * cc - 4.0 * d + e);
    const double eps = 1e-6;
    double w0 = 0.1 / ((eps + s0) * (eps + s0));
    double w1 = 0.6 / ((eps + s1) * (eps + s1));
    double w2 = 0.3 / ((eps + s2) * (eps + s2));
    return (w0 * q0 + w1 * q1 + w2 * q2) / (w0 + w1 + w2);
}

/* PPM (Colella & Woodward's piecewise parabolic method, the other scheme
 * Sec. 2.3 names): face values of the middle cell of a..e.  Each face value
 * starts as the fourth-order interpolant 7/12 (sum of the two neighbours) -
 * 1/12 (sum of the next two), bounded by its two neighbouring cell values;
 * then the parabola is made monotone: at a local extremum both face values
 * become the cell value, and where the parabola would overshoot, the far
 * face value is moved so that its extremum sits on the near face. */
static void o_ppm(double a, double b, double cc, double d, double e, double* left, double* right)
{
    double l = 7.0 / 12.0 * (b + cc) - 1.0 / 12.0 * (a + d);
    double r = 7.0 / 12.0 * (cc + d) - 1.0 / 12.0 * (b + e);
    l = fmin(fmax(l, fmin(b, cc)), fmax(b, cc));
    r = fmin(fmax(r, fmin(cc, d)), fmax(cc, d));
    if ((r - cc) * (cc - l) <= 0.0) {
        l = cc;
        r = cc;
    } else {
        double dd = r - l, m6 = 6.0 * (cc - 0.5 * (l + r));
        if (dd * m6 > dd * dd) l = 3.0 * cc - 2.0 * r;
        else if (-dd * dd > dd * m6) r = 3.0 * cc - 2.0 * l;
    }
    *left = l;
    *right = r;
}

/* Left and right states of one variable at the face between cells i-1 and
 * i, from the cell values s[0..5] of cells i-3..i+2 (PLM reads s[1..4]):
 * the left state is cell i-1's value at its right face, the right state
 * cell i's value at its left face (the mirrored stencil) (Sec. 2.4.1). */
static void o_recon(const ocfg_t* c, const double* s, double* left, double* right)
{
    if (c->recon == 0) {
        double sl = o_gmm(s[2] - s[1], s[3] - s[2], c->theta_plm);
        double sr = o_gmm(s[3] - s[2], s[4] - s[3], c->theta_plm);
        *left = s[2] + 0.5 * sl;
        *right = s[3] - 0.5 * sr;
    } else if (c->recon == 1) {
        *left = o_weno5(s[0], s[1], s[2], s[3], s[4]);
        *right = o_weno5(s[5], s[4], s[3], s[2], s[1]);
    } else {
        double l0, r0, l1, r1;
        o_ppm(s[0], s[1], s[2], s[3], s[4], &l0, &r0);
        o_ppm(s[1], s[2], s[3], s[4], s[5], &l1, &r1);
        *left = r0;
        *right = l1;
    }
}

void oracle_reconstruct(const ocfg_t* c, const double* s, double* left, double* right)
{
    o_recon(c, s, left, right);
}

/* Flux through the face on the low side of cell (i,j,k) in direction d:
 * reconstruction (Sec. 2.4.1; PLM with the generalized minmod slope, or the
 * five-point WENO5 / PPM operators, which read three cells on each side),
 * then the LLF or the HLLE flux (Sec. 2.4.2). */
static void o_face_flux(const ocfg_t* c, const olay_t* L, const double* Pg, int d, int i, int j, int k,
                        double* F)
{
    const int nv = c->nvar;
    size_t st = o_stride(L, d);
    size_t m = o_cell(L, i, j, k);
    double PL[NVMAX], PR[NVMAX];
    for (int v = 0; v < nv; ++v) {
        const double* a = Pg + (size_t)v * L->cells;
        double s6[6] = {0.0, a[m - 2 * st], a[m - st], a[m], a[m + st], 0.0};
        if (c->recon != 0) {
            s6[0] = a[m - 3 * st];
            s6[5] = a[m + 2 * st];
        }
        o_recon(c, s6, &PL[v], &PR[v]);
    }
    double X[4];
    o_zone_X(c, L, i, j, k, X);
    X[d + 1] -= 0.5 * o_dx(c, d);
    ogeom_t G;
    o_geom(c, X, &G);
    ostate_t SL, SR;
    o_state(c, PL, &G, &SL);
    o_state(c, PR, &G, &SR);
    double UL[NVMAX], UR[NVMAX], FL[NVMAX], FR[NVMAX];
    o_flux_from_state(c, PL, &G, &SL, 0, UL);
    o_flux_from_state(c, PR, &G, &SR, 0, UR);
    o_flux_from_state(c, PL, &G, &SL, d + 1, FL);
    o_flux_from_state(c, PR, &G, &SR, d + 1, FR);
    double lpL, lmL, lpR, lmR;
    o_speeds_state(c, PL, &G, &SL, d + 1, &lpL, &lmL);
    o_speeds_state(c, PR, &G, &SR, d + 1, &lpR, &lmR);
    if (c->riemann == 1) {
        /* HLLE: cR >= max(right-going speeds, 0), cL >= max(-left-going, 0) */
        double cR = fmax(0.0, fmax(lpL, lpR)), cL = fmax(0.0, fmax(-lmL, -lmR));
        for (int v = 0; v < nv; ++v)
            F[v] = (cR * FL[v] + cL * FR[v] - cR * cL * (UR[v] - UL[v])) / (cL + cR);
        return;
    }
    double cmax = fmax(fmax(fabs(lpL), fabs(lmL)), fmax(fabs(lpR), fabs(lmR)));
    for (int v = 0; v < nv; ++v) F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * cmax * (UR[v] - UL[v]);
}

/* ------------------------------------------------------------------------ */
/* boundary conditions                                                       */
/* ------------------------------------------------------------------------ */

/* Ghost fill, direction by direction (X1 on interior rows, then X2 on all X1
 * cells, then X3 on everything) so that edges and corners are filled.
 * periodic: wrap; outflow: copy the nearest interior zone; polar reflection:
 * mirror across the axis with utilde^2 and B^2 negated. */
static void o_fill_ghosts(const ocfg_t* c, const olay_t* L, double* Pg)
{
    const int bcs[3] = {c->bc1, c->bc2, c->bc3};
    for (int d = 0; d < c->ndim; ++d) {
        int g = L->g[d], n = L->n[d];
        int lo[3], hi[3];
        for (int e = 0; e < 3; ++e) {
            if (e < d) { lo[e] = 0; hi[e] = L->N[e]; }
            else { lo[e] = L->g[e]; hi[e] = L->g[e] + L->n[e]; }
        }
        for (int v = 0; v < c->nvar; ++v) {
            double* a = Pg + (size_t)v * L->cells;
            double sgn = 1.0;
            if (bcs[d] == 2 && d == 1 && (v == U2 || v == B2)) sgn = -1.0;
            for (int k = (d == 2 ? 0 : lo[2]); k < (d == 2 ? L->N[2] : hi[2]); ++k)
                for (int j = (d == 1 ? 0 : lo[1]); j < (d == 1 ? L->N[1] : hi[1]); ++j)
                    for (int i = (d == 0 ? 0 : lo[0]); i < (d == 0 ? L->N[0] : hi[0]); ++i) {
                        int idx[3] = {i, j, k};
                        int p = idx[d];
                        if (p >= g && p < g + n) continue;
                        int src;
                        double s = 1.0;
                        if (bcs[d] == 0) {
                            src = p < g ? p + n : p - n;
                        } else if (bcs[d] == 1) {
                            src = p < g ? g : g + n - 1;
                        } else {
                            src = p < g ? 2 * g - 1 - p : 2 * (g + n) - 1 - p;
                            s = sgn;
                        }
                        int sidx[3] = {i, j, k};
                        sidx[d] = src;
                        a[o_cell(L, i, j, k)] = s * a[o_cell(L, sidx[0], sidx[1], sidx[2])];
                    }
        }
    }
}

static void o_to_ghosted(const ocfg_t* c, const olay_t* L, const double* Pint, double* Pg)
{
    size_t nz = o_zones(L);
    for (int v = 0; v < c->nvar; ++v)
        for (int k = 0; k < L->n[2]; ++k)
            for (int j = 0; j < L->n[1]; ++j)
                for (int i = 0; i < L->n[0]; ++i)
                    Pg[(size_t)v * L->cells + o_cell(L, i + L->g[0], j + L->g[1], k + L->g[2])] =
                        Pint[(size_t)v * nz + ((size_t)k * L->n[1] + j) * L->n[0] + i];
    o_fill_ghosts(c, L, Pg);
}

static void o_get_cell(const ocfg_t* c, const olay_t* L, const double* Pg, size_t m, double* P)
{
    for (int v = 0; v < c->nvar; ++v) P[v] = Pg[(size_t)v * L->cells + m];
}

/* ------------------------------------------------------------------------ */
/* explicit stage: fluxes, flux-CT, divergence, explicit sources             */
/* ------------------------------------------------------------------------ */

/* Zone-centred quantities for the EMHD sources that depend only on P^E:
 * the spatial-derivative and connection parts of the q, DeltaP relaxation
 * targets (eqs. q0def, dP0def) and of div u. */
typedef struct {
    double sq_sp;   /* bhat^i d_i Theta + Theta (bhat^mu u^i d_i u_mu - bhat^mu Gamma^l_{n mu} u^n u_l) */
    double sdiv_sp; /* d_i u^i + Gamma^mu_{mu l} u^l                                                   */
    double sdp_sp;  /* bhat^i bhat^n d_i u_n - bhat^mu bhat^n Gamma^l_{mu n} u_l                         */
} oemhd_sp_t;

/* For every interior zone: divF (eq. fvm_formulation), the explicit
 * geometric source sqrt(-g) T^k_l Gamma^l_{nu k} at P^E (eq. divT_explicit),
 * and for EMHD the P^E-only parts of the relaxation sources.
 * Pg must be ghost-filled.  divF, srcE: [nvar][zones]; sp: [zones]. */
static void o_explicit_stage(const ocfg_t* c, const olay_t* L, const double* Pg, double* divF,
                             double* srcE, oemhd_sp_t* sp)
{
    const int nv = c->nvar;
    const int nd = c->ndim;
    double* Fd[3] = {NULL, NULL, NULL};
    for (int d = 0; d < nd; ++d) Fd[d] = (double*)calloc((size_t)nv * L->cells, sizeof(double));

    /* face fluxes: along d the faces of every interior cell; across the other
     * active directions one extra row on each side (needed by flux-CT). */
    for (int d = 0; d < nd; ++d) {
        int lo[3], hi[3];
        for (int e = 0; e < 3; ++e) {
            if (e == d) { lo[e] = L->g[e]; hi[e] = L->g[e] + L->n[e] + 1; }
            else if (e < nd) { lo[e] = L->g[e] - 1; hi[e] = L->g[e] + L->n[e] + 1; }
            else { lo[e] = 0; hi[e] = 1; }
        }
#pragma omp parallel for collapse(2) schedule(static)
        for (int k = lo[2]; k < hi[2]; ++k)
            for (int j = lo[1]; j < hi[1]; ++j)
                for (int i = lo[0]; i < hi[0]; ++i) {
                    double F[NVMAX];
                    o_face_flux(c, L, Pg, d, i, j, k, F);
                    size_t m = o_cell(L, i, j, k);
                    for (int v = 0; v < nv; ++v) Fd[d][(size_t)v * L->cells + m] = F[v];
                }
    }

    /* The flux of B^d through faces normal to d is zero in the continuum;
     * it is set to exactly zero (flux-CT does this in 2D and 3D). */
    for (int d = 0; d < nd; ++d)
        for (size_t m = 0; m < L->cells; ++m) Fd[d][(size_t)(B1 + d) * L->cells + m] = 0.0;

    /* flux-CT (Sec. 4.2): average face EMFs to edges, edges back to faces. */
    if (nd >= 2) {
        size_t C = L->cells;
        double* E1 = (double*)calloc(C, sizeof(double));
        double* E2 = (double*)calloc(C, sizeof(double));
        double* E3 = (double*)calloc(C, sizeof(double));
        const int g1 = L->g[0], g2 = L->g[1], g3 = L->g[2];
        const int n1 = L->n[0], n2 = L->n[1], n3 = L->n[2];
        const size_t s1 = 1, s2 = L->N[0], s3 = (size_t)L->N[0] * L->N[1];
        double* F1B2 = Fd[0] + (size_t)B2 * C;
        double* F1B3 = Fd[0] + (size_t)B3 * C;
        double* F2B1 = Fd[1] + (size_t)B1 * C;
        double* F2B3 = Fd[1] + (size_t)B3 * C;
        double* F3B1 = nd >= 3 ? Fd[2] + (size_t)B1 * C : NULL;
        double* F3B2 = nd >= 3 ? Fd[2] + (size_t)B2 * C : NULL;
        /* E3 on X3-edges at (i-1/2, j-1/2, k) */
        for (int k = g3; k < g3 + n3; ++k)
            for (int j = g2; j <= g2 + n2; ++j)
                for (int i = g1; i <= g1 + n1; ++i) {
                    size_t m = o_cell(L, i, j, k);
                    E3[m] = 0.25 * (F1B2[m] + F1B2[m - s2] - F2B1[m] - F2B1[m - s1]);
                }
        if (nd >= 3) {
            /* E1 on X1-edges at (i, j-1/2, k-1/2) */
            for (int k = g3; k <= g3 + n3; ++k)
                for (int j = g2; j <= g2 + n2; ++j)
                    for (int i = g1; i < g1 + n1; ++i) {
                        size_t m = o_cell(L, i, j, k);
                        E1[m] = 0.25 * (F2B3[m] + F2B3[m - s3] - F3B2[m] - F3B2[m - s2]);
                    }
            /* E2 on X2-edges at (i-1/2, j, k-1/2) */
            for (int k = g3; k <= g3 + n3; ++k)
                for (int j = g2; j < g2 + n2; ++j)
                    for (int i = g1; i <= g1 + n1; ++i) {
                        size_t m = o_cell(L, i, j, k);
                        E2[m] = 0.25 * (F3B1[m] + F3B1[m - s1] - F1B3[m] - F1B3[m - s3]);
                    }
        }
        /* X1 faces */
        for (int k = g3; k < g3 + n3; ++k)
            for (int j = g2; j < g2 + n2; ++j)
                for (int i = g1; i <= g1 + n1; ++i) {
                    size_t m = o_cell(L, i, j, k);
                    F1B2[m] = 0.5 * (E3[m] + E3[m + s2]);
                    if (nd >= 3) F1B3[m] = -0.5 * (E2[m] + E2[m + s3]);
                }
        /* X2 faces */
        for (int k = g3; k < g3 + n3; ++k)
            for (int j = g2; j <= g2 + n2; ++j)
                for (int i = g1; i < g1 + n1; ++i) {
                    size_t m = o_cell(L, i, j, k);
                    F2B1[m] = -0.5 * (E3[m] + E3[m + s1]);
                    if (nd >= 3) F2B3[m] = 0.5 * (E1[m] + E1[m + s3]);
                }
        /* X3 faces */
        if (nd >= 3)
            for (int k = g3; k <= g3 + n3; ++k)
                for (int j = g2; j < g2 + n2; ++j)
                    for (int i = g1; i < g1 + n1; ++i) {
                        size_t m = o_cell(L, i, j, k);
                        F3B1[m] = 0.5 * (E2[m] + E2[m + s1]);
                        F3B2[m] = -0.5 * (E1[m] + E1[m + s2]);
                    }
        free(E1);
        free(E2);
        free(E3);
    }

    /* divergence of the fluxes, explicit sources, EMHD spatial parts */
    const size_t nz = o_zones(L);
#pragma omp parallel for collapse(2) schedule(static)
    for (int kk = 0; kk < L->n[2]; ++kk)
        for (int jj = 0; jj < L->n[1]; ++jj)
            for (int ii = 0; ii < L->n[0]; ++ii) {
                int i = ii + L->g[0], j = jj + L->g[1], k = kk + L->g[2];
                size_t z = ((size_t)kk * L->n[1] + jj) * L->n[0] + ii;
                size_t m = o_cell(L, i, j, k);
                for (int v = 0; v < nv; ++v) {
                    double s = 0.0;
                    for (int d = 0; d < nd; ++d) {
                        size_t st = o_stride(L, d);
                        s += (Fd[d][(size_t)v * L->cells + m + st] - Fd[d][(size_t)v * L->cells + m]) / o_dx(c, d);
                    }
                    divF[(size_t)v * nz + z] = s;
                }
                double X[4], P[NVMAX], conn[4][4][4], T[4][4];
                o_zone_X(c, L, i, j, k, X);
                ogeom_t G;
                o_geom(c, X, &G);
                o_conn(c, X, conn);
                o_get_cell(c, L, Pg, m, P);
                ostate_t S;
                o_state(c, P, &G, &S);
                o_tmunu(c, P, &S, T);
                for (int v = 0; v < nv; ++v) srcE[(size_t)v * nz + z] = 0.0;
                for (int n = 0; n < 4; ++n) {
                    double s = 0.0;
                    for (int kap = 0; kap < 4; ++kap)
                        for (int lam = 0; lam < 4; ++lam) s += T[kap][lam] * conn[lam][n][kap];
                    srcE[(size_t)(UU + n) * nz + z] = G.gdet * s;
                }
                if (nv == 10) {
                    /* limited slopes of Theta, u_mu, u^i at P^E (Sec. 2.3: spatial
                     * derivatives in the sources use the generalized minmod slope) */
                    double dth[3] = {0, 0, 0}, ducov[3][4], ducon[3][4];
                    memset(ducov, 0, sizeof(ducov));
                    memset(ducon, 0, sizeof(ducon));
                    for (int d = 0; d < nd; ++d) {
                        size_t st = o_stride(L, d);
                        double Xq[3][9];
                        for (int o = -1; o <= 1; ++o) {
                            double Xn[4], Pnb[NVMAX];
                            int idx[3] = {i, j, k};
                            idx[d] += o;
                            o_zone_X(c, L, idx[0], idx[1], idx[2], Xn);
                            ogeom_t Gn;
                            o_geom(c, Xn, &Gn);
                            o_get_cell(c, L, Pg, (size_t)((long)m + o * (long)st), Pnb);
                            ostate_t Sn;
                            o_state(c, Pnb, &Gn, &Sn);
                            Xq[o + 1][0] = Sn.pg / Pnb[RHO];
                            for (int mu = 0; mu < 4; ++mu) Xq[o + 1][1 + mu] = Sn.ucov[mu];
                            for (int mu = 1; mu < 4; ++mu) Xq[o + 1][4 + mu] = Sn.ucon[mu];
                        }
                        double dxd = o_dx(c, d);
                        double sl[8];
                        for (int q = 0; q < 8; ++q)
                            sl[q] = o_gmm(Xq[1][q] - Xq[0][q], Xq[2][q] - Xq[1][q], c->theta_plm) / dxd;
                        dth[d] = sl[0];
                        for (int mu = 0; mu < 4; ++mu) ducov[d][mu] = sl[1 + mu];
                        for (int mu = 1; mu < 4; ++mu) ducon[d][mu] = sl[4 + mu];
                    }
                    double theta = S.pg / P[RHO];
                    double a1 = 0.0, a2 = 0.0, divs = 0.0, b1 = 0.0, b2 = 0.0;
                    for (int d = 0; d < nd; ++d) {
                        a1 += S.bhcon[d + 1] * dth[d];
                        for (int mu = 0; mu < 4; ++mu) {
                            a2 += S.bhcon[mu] * S.ucon[d + 1] * ducov[d][mu];
                            b1 += S.bhcon[d + 1] * S.bhcon[mu] * ducov[d][mu];
                        }
                        divs += ducon[d][d + 1];
                    }
                    double gam_a = 0.0, gam_div = 0.0, gam_b = 0.0;
                    for (int mu = 0; mu < 4; ++mu)
                        for (int n = 0; n < 4; ++n)
                            for (int l = 0; l < 4; ++l) {
                                gam_a += S.bhcon[mu] * conn[l][n][mu] * S.ucon[n] * S.ucov[l];
                                gam_b += S.bhcon[mu] * S.bhcon[n] * conn[l][mu][n] * S.ucov[l];
                            }
                    for (int mu = 0; mu < 4; ++mu)
                        for (int l = 0; l < 4; ++l) gam_div += conn[mu][mu][l] * S.ucon[l];
                    (void)b2;
                    sp[z].sq_sp = a1 + theta * (a2 - gam_a);
                    sp[z].sdiv_sp = divs + gam_div;
                    sp[z].sdp_sp = b1 - gam_b;
                } else {
                    sp[z].sq_sp = sp[z].sdiv_sp = sp[z].sdp_sp = 0.0;
                }
            }
    for (int d = 0; d < nd; ++d) free(Fd[d]);
}

/* ------------------------------------------------------------------------ */
/* linear solve and Newton driver (Sec. 3)                                   */
/* ------------------------------------------------------------------------ */

/* Solve A x = b (A row-major n x n) by Gaussian elimination with partial
 * pivoting (the factorisation LAPACK's dgesv performs).  Returns 1 on an
 * exactly zero pivot. */
int oracle_solve(int n, const double* A, const double* b, double* x)
{
    double M[16][17];
    if (n > 16) return 2;
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) M[i][j] = A[i * n + j];
        M[i][n] = b[i];
    }
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (fabs(M[i][k]) > fabs(M[p][k])) p = i;
        if (M[p][k] == 0.0) return 1;
        if (p != k)
            for (int j = 0; j <= n; ++j) { double t = M[k][j]; M[k][j] = M[p][j]; M[p][j] = t; }
        for (int i = k + 1; i < n; ++i) {
            double f = M[i][k] / M[k][k];
            for (int j = k; j <= n; ++j) M[i][j] -= f * M[k][j];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = M[i][n];
        for (int j = i + 1; j < n; ++j) s -= M[i][j] * x[j];
        x[i] = s / M[i][i];
    }
    return 0;
}

/* Quadratic backtracking step (Sec. 3.2, eq. linesearch_residual and the
 * update that follows it): model f(lam) as a quadratic with f'(0) = -2 f(0). */
double oracle_ls_lambda(double f0, double f1, double lam)
{
    return f0 * lam * lam / (f1 + (2.0 * lam - 1.0) * f0);
}

static double o_norm(int n, const double* r, double nscale)
{
    double s = 0.0;
    for (int v = 0; v < n; ++v) s += r[v] * r[v];
    return nscale * sqrt(s);
}

/* Numerical Jacobian (Sec. 3.1, eq. numerical_jacobian and the perturbation
 * rule that follows): row i = residual component, column j = perturbed
 * primitive,  J_ij = (R_i(P_eps,j) - R_i(P)) / (P_eps,j - P_j), where only P_j
 * is perturbed: P_eps = (1+eps) P (1 - small) + eps small, small = [|P| < 5 eps].
 * Reading: if the perturbation is exactly zero, P_j + eps is used.
 * R must hold R(x) on entry; J is row-major n x n. */
void oracle_fd_jacobian(int n, oresid_fn fn, void* ctx, const double* x, const double* R, double eps, double* J)
{
    double xp[16], Rp[16];
    for (int j = 0; j < n; ++j) {
        for (int q = 0; q < n; ++q) xp[q] = x[q];
        double pj = x[j];
        double small = fabs(pj) < 5.0 * eps ? 1.0 : 0.0;
        double pe = (1.0 + eps) * pj * (1.0 - small) + eps * small;
        double h = pe - pj;
        if (h == 0.0) { pe = pj + eps; h = pe - pj; }
        xp[j] = pe;
        fn(ctx, xp, Rp);
        for (int i = 0; i < n; ++i) J[i * n + j] = (Rp[i] - R[i]) / h;
    }
}

/* Newton iteration with a numerical Jacobian and backtracking (Sec. 3,
 * eqs. newton_iters and numerical_jacobian, Sec. 3.1, Sec. 3.2), one system.
 *  - norm: ||R|| = nscale * sqrt(sum R_v^2)
 *  - stop when ||R|| < tol (iters = number of linear solves), or at k_max
 *  - Jacobian by oracle_fd_jacobian
 *  - line search (Sec. 3.2): lambda = 1; accept if
 *    ||R(P + lam dP)|| < ||R(P)|| (1 - eps_bt lam); otherwise lambda becomes
 *    the minimiser of the quadratic model (oracle_ls_lambda) and the trial is
 *    repeated.  Readings where the paper is silent: a non-finite trial halves
 *    lambda; after ls_max trials the last finite trial is taken (flag
 *    LS_EXHAUSTED).  ls_safeguard = 1 keeps each new lambda in [0.1, 0.5] of
 *    the previous one (the usual safeguard of quadratic backtracking); 0
 *    applies the printed update unchanged.
 *  - backtracks: the rejected trials, summed over the iterations. */
int oracle_newton_generic(int n, oresid_fn fn, void* ctx, double* x, double nscale, double tol, double eps,
                          double eps_bt, int k_max, int ls_max, int ls_safeguard, int32_t* iters, double* resid,
                          uint8_t* flags, int32_t* backtracks)
{
    double R[16], J[256], dx[16], xt[16], Rt[16], negR[16];
    uint8_t fl = 0;
    int k = 0, nbt = 0;
    if (n > 16) return 2;
    fn(ctx, x, R);
    double r = o_norm(n, R, nscale);
    for (;;) {
        if (!isfinite(r)) { fl |= OFLAG_NONFINITE; break; }
        if (r < tol) break;
        if (k >= k_max) { fl |= OFLAG_NOT_CONVERGED; break; }
        oracle_fd_jacobian(n, fn, ctx, x, R, eps, J);
        for (int i = 0; i < n; ++i) negR[i] = -R[i];
        if (oracle_solve(n, J, negR, dx) != 0) { fl |= OFLAG_SINGULAR; break; }
        double f0 = r * r, lam = 1.0, rt = 0.0;
        int accepted = 0, have_finite = 0;
        double xf[16], Rf[16], rf = 0.0;
        for (int t = 0; t < ls_max; ++t) {
            for (int q = 0; q < n; ++q) xt[q] = x[q] + lam * dx[q];
            fn(ctx, xt, Rt);
            rt = o_norm(n, Rt, nscale);
            if (isfinite(rt)) {
                have_finite = 1;
                for (int q = 0; q < n; ++q) { xf[q] = xt[q]; Rf[q] = Rt[q]; }
                rf = rt;
                if (rt < r * (1.0 - eps_bt * lam)) { accepted = 1; break; }
                double ln = oracle_ls_lambda(f0, rt * rt, lam);
                if (ls_safeguard) {
                    if (!(ln >= 0.1 * lam)) ln = 0.1 * lam;
                    if (ln > 0.5 * lam) ln = 0.5 * lam;
                }
                lam = ln;
            } else {
                lam *= 0.5;
            }
            ++nbt;
        }
        if (!accepted) {
            fl |= OFLAG_LS_EXHAUSTED;
            if (!have_finite) { fl |= OFLAG_NONFINITE; ++k; break; }
        }
        for (int q = 0; q < n; ++q) { x[q] = xf[q]; R[q] = Rf[q]; }
        r = rf;
        ++k;
    }
    if (iters) *iters = k;
    if (resid) *resid = r;
    if (flags) *flags = fl;
    if (backtracks) *backtracks = nbt;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* the per-zone residual (Sec. 2.3 eqs. half_step, full_step; Sec. 3        */
/* eq. half_step_residual; Sec. 4 relaxation equations)                      */
/* ------------------------------------------------------------------------ */

typedef struct {
    const ocfg_t* c;
    ogeom_t G;
    double dtp;
    double Un[NVMAX];     /* U(P_n)                                         */
    double expl[NVMAX];   /* -divF(P^E) + S^E(P^E)                           */
    /* EMHD: time level n */
    double theta_n, ucov_n[4], u0_n, qt_n, dpt_n;
    /* EMHD: quantities frozen at P^E, with the stage's relaxation time and
     * diffusivities (o_tau_eff, o_diff_over_tau at P^E) */
    double rhoE, thetaE, u0E, qtE, dptE, bhE[4];
    double tauE, chiE, nuE;
    oemhd_sp_t sp;
} ozone_t;

/* R(P) = (U(P) - U(P_n))/dtp + divF(P^E) - S^E(P^E) - [implicit q, DP sources].
 * EMHD relaxation rows (eqs. q_evol_eqn_rescaled, dP_evol_eqn_rescaled with
 * the IMEX split of Sec. 2.3), reading of the relaxation sign as -(X-X0)/tau:
 *   S_q = sqrt(-g) [ -(qt(P) + qt(P_n))/(2 tau) + qt0s / tau + qt(P^E)/2 divus ]
 * where qt0s = q0s sqrt(tau/(chi rho Theta^2)) at P^E and
 *   q0s   = -rho chi [ bhat^0 dTheta/dt + Theta bhat^mu u^0 du_mu/dt + sq_sp ]
 *   DP0s  = 3 rho nu [ bhat^0 bhat^nu du_nu/dt + sdp_sp - divus / 3 ]
 *   divus = du^0/dt + sdiv_sp
 * with d X/dt = (X(P) - X(P_n))/dtp (reading of A^t dP/dt: the derived X in
 * {Theta, u_mu, u^0} is differenced against P_n) and every coefficient,
 * spatial derivative and connection term frozen at P^E. */
static void o_zone_residual(void* ctx, const double* P, double* R)
{
    ozone_t* z = (ozone_t*)ctx;
    const ocfg_t* c = z->c;
    const int nv = c->nvar;
    ostate_t S;
    o_state(c, P, &z->G, &S);
    double U[NVMAX];
    o_flux_from_state(c, P, &z->G, &S, 0, U);
    for (int v = 0; v < nv; ++v) R[v] = (U[v] - z->Un[v]) / z->dtp - z->expl[v];
    if (nv == 10) {
        double dtp = z->dtp;
        double theta = S.pg / P[RHO];
        double qt, dpt;
        o_rescaled(c, P, &S, &qt, &dpt);
        double dtheta = (theta - z->theta_n) / dtp;
        double du0 = (S.ucon[0] - z->u0_n) / dtp;
        double bdu = 0.0;
        for (int mu = 0; mu < 4; ++mu) bdu += z->bhE[mu] * (S.ucov[mu] - z->ucov_n[mu]) / dtp;
        double divu = du0 + z->sp.sdiv_sp;
        double q0 = -z->rhoE * z->chiE * (z->bhE[0] * dtheta + z->thetaE * z->u0E * bdu + z->sp.sq_sp);
        double dp0 = 3.0 * z->rhoE * z->nuE * (z->bhE[0] * bdu + z->sp.sdp_sp - divu / 3.0);
        double qt0 = q0 * sqrt(z->tauE / (z->chiE * z->rhoE * z->thetaE * z->thetaE));
        double dpt0 = dp0 * sqrt(z->tauE / (z->nuE * z->rhoE * z->thetaE));
        double tau = z->tauE;
        double Sq = z->G.gdet * (-(qt + z->qt_n) / (2.0 * tau) + qt0 / tau + 0.5 * z->qtE * divu);
        double Sd = z->G.gdet * (-(dpt + z->dpt_n) / (2.0 * tau) + dpt0 / tau + 0.5 * z->dptE * divu);
        R[QQ] -= Sq;
        R[DP] -= Sd;
    }
}

/* The Newton unknowns are the non-magnetic primitives (Sec. 8.2: a 5x5
 * Jacobian over {rho, u, u^1, u^2, u^3} for ideal MHD, 7x7 with q and DP for
 * EMHD).  B is held at its explicit update, the root of the induction rows,
 * which depend on B alone; the system is the residual's non-magnetic rows. */
static const int o_unknown[7] = {RHO, UU, U1, U2, U3, QQ, DP};
/* With full_system = 1 the unknowns are every primitive (an 8x8 / 10x10
 * system, B among them, still started from its explicit update): the same
 * root, since the B rows depend on B alone and are solved by that update. */
static const int o_all[NVMAX] = {RHO, UU, U1, U2, U3, B1, B2, B3, QQ, DP};

static int o_sys_size(const ocfg_t* c) { return c->full_system ? c->nvar : c->nvar - 3; }
static const int* o_sys_map(const ocfg_t* c) { return c->full_system ? o_all : o_unknown; }

typedef struct {
    ozone_t* z;
    double P[NVMAX]; /* full primitive vector; entries outside the system fixed */
    int m;           /* number of unknowns */
    const int* map;  /* unknown i is primitive map[i] */
} oreduced_t;

static void o_reduced_residual(void* ctx, const double* x, double* R)
{
    oreduced_t* q = (oreduced_t*)ctx;
    double P[NVMAX], Rf[NVMAX];
    for (int v = 0; v < NVMAX; ++v) P[v] = q->P[v];
    for (int i = 0; i < q->m; ++i) P[q->map[i]] = x[i];
    o_zone_residual(q->z, P, Rf);
    for (int i = 0; i < q->m; ++i) R[i] = Rf[q->map[i]];
}

static void o_zone_setup(const ocfg_t* c, const double X[4], const double* Pn, const double* PE,
                         const double* divF_z, const double* srcE_z, const oemhd_sp_t* sp, double dtp,
                         ozone_t* z)
{
    z->c = c;
    o_geom(c, X, &z->G);
    z->dtp = dtp;
    ostate_t Sn;
    o_state(c, Pn, &z->G, &Sn);
    o_flux_from_state(c, Pn, &z->G, &Sn, 0, z->Un);
    for (int v = 0; v < c->nvar; ++v) z->expl[v] = -divF_z[v] + srcE_z[v];
    if (c->nvar == 10) {
        z->theta_n = Sn.pg / Pn[RHO];
        for (int mu = 0; mu < 4; ++mu) z->ucov_n[mu] = Sn.ucov[mu];
        z->u0_n = Sn.ucon[0];
        o_rescaled(c, Pn, &Sn, &z->qt_n, &z->dpt_n);
        ostate_t SE;
        o_state(c, PE, &z->G, &SE);
        z->rhoE = PE[RHO];
        z->thetaE = SE.pg / PE[RHO];
        z->u0E = SE.ucon[0];
        o_rescaled(c, PE, &SE, &z->qtE, &z->dptE);
        for (int mu = 0; mu < 4; ++mu) z->bhE[mu] = SE.bhcon[mu];
        z->sp = *sp;
        if (c->closure) {
            double chi_t, nu_t;
            o_diff_over_tau(c, PE, &chi_t, &nu_t);
            z->tauE = o_tau_eff(c, PE, &SE);
            z->chiE = chi_t * z->tauE;
            z->nuE = nu_t * z->tauE;
        } else {
            z->tauE = c->tau_R;
            z->chiE = c->chi;
            z->nuE = c->nu;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* one stage of the two-stage scheme                                         */
/* ------------------------------------------------------------------------ */

/* One stage (Sec. 2.3) on a ghost-filled P^E: the explicit stage, then the
 * Newton solve of every interior zone from P_n (or the supplied guess). */
static int o_stage_core(const ocfg_t* c, const olay_t* Lp, const double* Pn, const double* PEg, double dtp,
                        const double* guess, double* Pout, int32_t* iters, double* resid, uint8_t* flags,
                        int32_t* backtracks)
{
    olay_t L = *Lp;
    const int nv = c->nvar;
    const size_t nz = o_zones(&L);
    double* divF = (double*)calloc((size_t)nv * nz, sizeof(double));
    double* srcE = (double*)calloc((size_t)nv * nz, sizeof(double));
    oemhd_sp_t* sp = (oemhd_sp_t*)calloc(nz, sizeof(oemhd_sp_t));
    if (!divF || !srcE || !sp) { free(divF); free(srcE); free(sp); return -1; }
    o_explicit_stage(c, &L, PEg, divF, srcE, sp);

#pragma omp parallel for collapse(2) schedule(static)
    for (int kk = 0; kk < L.n[2]; ++kk)
        for (int jj = 0; jj < L.n[1]; ++jj)
            for (int ii = 0; ii < L.n[0]; ++ii) {
                size_t z = ((size_t)kk * L.n[1] + jj) * L.n[0] + ii;
                size_t m = o_cell(&L, ii + L.g[0], jj + L.g[1], kk + L.g[2]);
                double X[4], pn[NVMAX], pe[NVMAX], dz[NVMAX], sz[NVMAX], P[NVMAX];
                o_zone_X(c, &L, ii + L.g[0], jj + L.g[1], kk + L.g[2], X);
                for (int v = 0; v < nv; ++v) {
                    pn[v] = Pn[(size_t)v * nz + z];
                    pe[v] = PEg[(size_t)v * L.cells + m];
                    dz[v] = divF[(size_t)v * nz + z];
                    sz[v] = srcE[(size_t)v * nz + z];
                }
                ozone_t Z;
                o_zone_setup(c, X, pn, pe, dz, sz, &sp[z], dtp, &Z);
                /* initial guess: P_n (or the supplied guess) with B set to the
                 * explicit update, which is the exact root of the B rows */
                for (int v = 0; v < nv; ++v) P[v] = guess ? guess[(size_t)v * nz + z] : pn[v];
                for (int i = 0; i < 3; ++i)
                    P[B1 + i] = (Z.Un[B1 + i] + dtp * Z.expl[B1 + i]) / Z.G.gdet;
                double urho_n = Z.Un[RHO];
                int32_t it = 0, bt = 0;
                double rr = 0.0;
                uint8_t fl = 0;
                oreduced_t Q;
                Q.z = &Z;
                Q.m = o_sys_size(c);
                Q.map = o_sys_map(c);
                for (int v = 0; v < NVMAX; ++v) Q.P[v] = v < nv ? P[v] : 0.0;
                double x[NVMAX];
                for (int i = 0; i < Q.m; ++i) x[i] = P[Q.map[i]];
                oracle_newton_generic(Q.m, o_reduced_residual, &Q, x, dtp / urho_n, c->tol, c->eps, c->eps_bt,
                                      c->k_max, c->ls_max, c->ls_safeguard, &it, &rr, &fl, &bt);
                for (int i = 0; i < Q.m; ++i) P[Q.map[i]] = x[i];
                if (!(P[RHO] > 0.0) || !(P[UU] > 0.0)) fl |= OFLAG_UNPHYSICAL;
                if (c->floors) {
                    double r = exp(X[1]);
                    double rf = c->rho_fl * pow(r, -1.5), uf = c->u_fl * pow(r, -2.5);
                    if (!(P[RHO] >= rf)) P[RHO] = rf;
                    if (!(P[UU] >= uf)) P[UU] = uf;
                }
                for (int v = 0; v < nv; ++v) Pout[(size_t)v * nz + z] = P[v];
                if (iters) iters[z] = it;
                if (resid) resid[z] = rr;
                if (flags) flags[z] = fl;
                if (backtracks) backtracks[z] = bt;
            }
    free(divF);
    free(srcE);
    free(sp);
    return 0;
}

int oracle_stage(const ocfg_t* c, const double* Pn, const double* PE, double dtp, const double* guess,
                 double* Pout, int32_t* iters, double* resid, uint8_t* flags)
{
#ifdef _OPENMP
    if (c->nthreads > 0) omp_set_num_threads(c->nthreads);
#endif
    olay_t L = o_layout(c);
    double* PEg = (double*)calloc((size_t)c->nvar * L.cells, sizeof(double));
    if (!PEg) return -1;
    o_to_ghosted(c, &L, PE, PEg);
    int rc = o_stage_core(c, &L, Pn, PEg, dtp, guess, Pout, iters, resid, flags, NULL);
    free(PEg);
    return rc;
}

int oracle_stage_ghosted(const ocfg_t* c, const double* Pn, const double* PEg, double dtp, const double* guess,
                         double* Pout, int32_t* iters, double* resid, uint8_t* flags, int32_t* backtracks)
{
#ifdef _OPENMP
    if (c->nthreads > 0) omp_set_num_threads(c->nthreads);
#endif
    olay_t L = o_layout(c);
    return o_stage_core(c, &L, Pn, PEg, dtp, guess, Pout, iters, resid, flags, backtracks);
}

static void o_accumulate(ostats_t* st, int stage, size_t nz, const int32_t* it, const double* rr,
                         const uint8_t* fl, const int32_t* bt)
{
    if (!st) return;
    st->zones = (int64_t)nz;
    for (size_t z = 0; z < nz; ++z) {
        st->iters_sum[stage] += it[z];
        if (it[z] > st->max_iters) st->max_iters = it[z];
        if (fl[z] & (OFLAG_NOT_CONVERGED | OFLAG_SINGULAR | OFLAG_NONFINITE)) st->n_fail++;
        if (fl[z] & OFLAG_LS_EXHAUSTED) st->n_ls_exhausted++;
        if (fl[z] & OFLAG_UNPHYSICAL) st->n_unphysical++;
        if (rr[z] > st->max_resid || !isfinite(rr[z])) st->max_resid = rr[z];
        st->n_backtracks += bt[z];
    }
}

/* One full step (Sec. 2.3): half step P_n -> P_{n+1/2} with P^E = P_n and
 * dtp = dt/2, then full step P_n -> P_{n+1} with P^E = P_{n+1/2}, dtp = dt.
 * Both solves start from P_n. */
int oracle_step(const ocfg_t* c, double* P, double dt, ostats_t* st)
{
#ifdef _OPENMP
    if (c->nthreads > 0) omp_set_num_threads(c->nthreads);
#endif
    olay_t L = o_layout(c);
    const size_t nz = o_zones(&L);
    const size_t nvz = (size_t)c->nvar * nz;
    double* Ph = (double*)malloc(nvz * sizeof(double));
    double* P1 = (double*)malloc(nvz * sizeof(double));
    double* Pg = (double*)calloc((size_t)c->nvar * L.cells, sizeof(double));
    int32_t* it = (int32_t*)malloc(nz * sizeof(int32_t));
    int32_t* bt = (int32_t*)malloc(nz * sizeof(int32_t));
    double* rr = (double*)malloc(nz * sizeof(double));
    uint8_t* fl = (uint8_t*)malloc(nz);
    int rc = -1;
    if (Ph && P1 && Pg && it && bt && rr && fl) {
        o_to_ghosted(c, &L, P, Pg);
        rc = o_stage_core(c, &L, P, Pg, 0.5 * dt, NULL, Ph, it, rr, fl, bt);
        o_accumulate(st, 0, nz, it, rr, fl, bt);
        if (rc == 0) {
            o_to_ghosted(c, &L, Ph, Pg);
            rc = o_stage_core(c, &L, P, Pg, dt, NULL, P1, it, rr, fl, bt);
        }
        o_accumulate(st, 1, nz, it, rr, fl, bt);
        if (rc == 0) memcpy(P, P1, nvz * sizeof(double));
    }
    free(Ph);
    free(P1);
    free(Pg);
    free(it);
    free(bt);
    free(rr);
    free(fl);
    return rc;
}

int oracle_run(const ocfg_t* c, double* P, double dt, int nsteps, ostats_t* st)
{
    for (int s = 0; s < nsteps; ++s) {
        int rc = oracle_step(c, P, dt, st);
        if (rc) return rc;
    }
    return 0;
}

/* The residual of every interior zone at the state P, for a stage with the
 * given P_n, ghost-filled P^E and dtp; also the scaled norm used by the
 * solver. */
static int o_residual_core(const ocfg_t* c, const olay_t* Lp, const double* Pn, const double* PEg, double dtp,
                           const double* P, double* R, double* rnorm)
{
    olay_t L = *Lp;
    const int nv = c->nvar;
    const size_t nz = o_zones(&L);
    double* divF = (double*)calloc((size_t)nv * nz, sizeof(double));
    double* srcE = (double*)calloc((size_t)nv * nz, sizeof(double));
    oemhd_sp_t* sp = (oemhd_sp_t*)calloc(nz, sizeof(oemhd_sp_t));
    if (!divF || !srcE || !sp) { free(divF); free(srcE); free(sp); return -1; }
    o_explicit_stage(c, &L, PEg, divF, srcE, sp);
#pragma omp parallel for collapse(2) schedule(static)
    for (int kk = 0; kk < L.n[2]; ++kk)
        for (int jj = 0; jj < L.n[1]; ++jj)
            for (int ii = 0; ii < L.n[0]; ++ii) {
                size_t z = ((size_t)kk * L.n[1] + jj) * L.n[0] + ii;
                size_t m = o_cell(&L, ii + L.g[0], jj + L.g[1], kk + L.g[2]);
                double X[4], pn[NVMAX], pe[NVMAX], dz[NVMAX], sz[NVMAX], p[NVMAX], r[NVMAX];
                o_zone_X(c, &L, ii + L.g[0], jj + L.g[1], kk + L.g[2], X);
                for (int v = 0; v < nv; ++v) {
                    pn[v] = Pn[(size_t)v * nz + z];
                    pe[v] = PEg[(size_t)v * L.cells + m];
                    dz[v] = divF[(size_t)v * nz + z];
                    sz[v] = srcE[(size_t)v * nz + z];
                    p[v] = P[(size_t)v * nz + z];
                }
                ozone_t Z;
                o_zone_setup(c, X, pn, pe, dz, sz, &sp[z], dtp, &Z);
                o_zone_residual(&Z, p, r);
                for (int v = 0; v < nv; ++v) R[(size_t)v * nz + z] = r[v];
                if (rnorm) {
                    /* the Newton norm: over the system rows (without the B
                     * rows unless the system is the full one) */
                    double rs[NVMAX];
                    const int* map = o_sys_map(c);
                    for (int i = 0; i < o_sys_size(c); ++i) rs[i] = r[map[i]];
                    rnorm[z] = o_norm(o_sys_size(c), rs, dtp / Z.Un[RHO]);
                }
            }
    free(divF);
    free(srcE);
    free(sp);
    return 0;
}

int oracle_residual(const ocfg_t* c, const double* Pn, const double* PE, double dtp, const double* P, double* R,
                    double* rnorm)
{
    olay_t L = o_layout(c);
    double* PEg = (double*)calloc((size_t)c->nvar * L.cells, sizeof(double));
    if (!PEg) return -1;
    o_to_ghosted(c, &L, PE, PEg);
    int rc = o_residual_core(c, &L, Pn, PEg, dtp, P, R, rnorm);
    free(PEg);
    return rc;
}

int oracle_residual_ghosted(const ocfg_t* c, const double* Pn, const double* PEg, double dtp, const double* P,
                            double* R, double* rnorm)
{
#ifdef _OPENMP
    if (c->nthreads > 0) omp_set_num_threads(c->nthreads);
#endif
    olay_t L = o_layout(c);
    return o_residual_core(c, &L, Pn, PEg, dtp, P, R, rnorm);
}

/* divF, the explicit geometric source and the EMHD P^E-only source parts
 * (sq_sp, sdiv_sp, sdp_sp per zone) for a state PE. */
int oracle_explicit(const ocfg_t* c, const double* PE, double* divF, double* srcE, double* emhd_sp)
{
    olay_t L = o_layout(c);
    const size_t nz = o_zones(&L);
    double* PEg = (double*)calloc((size_t)c->nvar * L.cells, sizeof(double));
    oemhd_sp_t* sp = (oemhd_sp_t*)calloc(nz, sizeof(oemhd_sp_t));
    o_to_ghosted(c, &L, PE, PEg);
    o_explicit_stage(c, &L, PEg, divF, srcE, sp);
    if (emhd_sp)
        for (size_t z = 0; z < nz; ++z) {
            emhd_sp[3 * z + 0] = sp[z].sq_sp;
            emhd_sp[3 * z + 1] = sp[z].sdiv_sp;
            emhd_sp[3 * z + 2] = sp[z].sdp_sp;
        }
    free(PEg);
    free(sp);
    return 0;
}

/* Time step from the CFL condition on zone-centre speeds:
 * dt = cfl * min_zones 1 / sum_d (c_max^d / dX^d). */
double oracle_cfl_dt(const ocfg_t* c, const double* P, double cfl)
{
    olay_t L = o_layout(c);
    const size_t nz = o_zones(&L);
    double best = 1e300;
    for (int kk = 0; kk < L.n[2]; ++kk)
        for (int jj = 0; jj < L.n[1]; ++jj)
            for (int ii = 0; ii < L.n[0]; ++ii) {
                size_t z = ((size_t)kk * L.n[1] + jj) * L.n[0] + ii;
                double X[4], p[NVMAX];
                o_zone_X(c, &L, ii + L.g[0], jj + L.g[1], kk + L.g[2], X);
                for (int v = 0; v < c->nvar; ++v) p[v] = P[(size_t)v * nz + z];
                ogeom_t G;
                o_geom(c, X, &G);
                ostate_t S;
                o_state(c, p, &G, &S);
                double s = 0.0;
                for (int d = 0; d < c->ndim; ++d) {
                    double lp, lm;
                    o_speeds_state(c, p, &G, &S, d + 1, &lp, &lm);
                    s += fmax(fabs(lp), fabs(lm)) / o_dx(c, d);
                }
                double t = 1.0 / s;
                if (t < best) best = t;
            }
    return cfl * best;
}

/* Corner-centred divergence of sqrt(-g) B (the discrete constraint flux-CT
 * preserves, Sec. 4.2) at every interior corner (i-1/2, j-1/2[, k-1/2]),
 * i.e. for i in [1, n1), j in [1, n2)[, k in [1, n3)] of the interior grid:
 * divb has n1*n2*n3 entries, the entries with a zero index are set to 0. */
int oracle_divb(const ocfg_t* c, const double* P, double* divb)
{
    olay_t L = o_layout(c);
    const size_t nz = o_zones(&L);
    const int nd = c->ndim;
    if (nd < 2) return 1;
    for (int k = 0; k < L.n[2]; ++k)
        for (int j = 0; j < L.n[1]; ++j)
            for (int i = 0; i < L.n[0]; ++i) {
                size_t z = ((size_t)k * L.n[1] + j) * L.n[0] + i;
                divb[z] = 0.0;
                if (i == 0 || j == 0 || (nd == 3 && k == 0)) continue;
                double s = 0.0;
                int nk = nd == 3 ? 2 : 1;
                for (int d = 0; d < nd; ++d) {
                    double acc = 0.0;
                    for (int ok = 0; ok < nk; ++ok)
                        for (int oj = 0; oj < 2; ++oj)
                            for (int oi = 0; oi < 2; ++oi) {
                                int ci = i - 1 + oi, cj = j - 1 + oj, ck = nd == 3 ? k - 1 + ok : k;
                                int o[3] = {oi, oj, ok};
                                double sgn = o[d] ? 1.0 : -1.0;
                                double X[4];
                                o_zone_X(c, &L, ci + L.g[0], cj + L.g[1], ck + L.g[2], X);
                                ogeom_t G;
                                o_geom(c, X, &G);
                                size_t zz = ((size_t)ck * L.n[1] + cj) * L.n[0] + ci;
                                acc += sgn * G.gdet * P[(size_t)(B1 + d) * nz + zz];
                            }
                    s += acc / ((nd == 3 ? 4.0 : 2.0) * o_dx(c, d));
                }
                divb[z] = s;
            }
    return 0;
}

/* Sum over interior zones of U(P) (times the zone volume in X). */
int oracle_sum_U(const ocfg_t* c, const double* P, double* sums)
{
    olay_t L = o_layout(c);
    const size_t nz = o_zones(&L);
    double vol = c->dx1 * (c->ndim >= 2 ? c->dx2 : 1.0) * (c->ndim >= 3 ? c->dx3 : 1.0);
    for (int v = 0; v < c->nvar; ++v) sums[v] = 0.0;
    for (int k = 0; k < L.n[2]; ++k)
        for (int j = 0; j < L.n[1]; ++j)
            for (int i = 0; i < L.n[0]; ++i) {
                size_t z = ((size_t)k * L.n[1] + j) * L.n[0] + i;
                double X[4], p[NVMAX], U[NVMAX];
                o_zone_X(c, &L, i + L.g[0], j + L.g[1], k + L.g[2], X);
                for (int v = 0; v < c->nvar; ++v) p[v] = P[(size_t)v * nz + z];
                ogeom_t G;
                o_geom(c, X, &G);
                ostate_t S;
                o_state(c, p, &G, &S);
                o_flux_from_state(c, p, &G, &S, 0, U);
                for (int v = 0; v < c->nvar; ++v) sums[v] += U[v] * vol;
            }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* point functions exported for the pins                                     */
/* ------------------------------------------------------------------------ */

/* Interior primitives -> ghosted grid with every ghost cell filled by the
 * boundary conditions (o_fill_ghosts). */
int oracle_fill_ghosts(const ocfg_t* c, const double* Pint, double* Pg)
{
    olay_t L = o_layout(c);
    o_to_ghosted(c, &L, Pint, Pg);
    return 0;
}

void oracle_geometry(const ocfg_t* c, const double* X, double* gcov, double* gcon, double* gdet, double* alpha)
{
    ogeom_t G;
    o_geom(c, X, &G);
    for (int m = 0; m < 4; ++m)
        for (int n = 0; n < 4; ++n) {
            gcov[4 * m + n] = G.gcov[m][n];
            gcon[4 * m + n] = G.gcon[m][n];
        }
    *gdet = G.gdet;
    *alpha = G.alpha;
}

void oracle_connection(const ocfg_t* c, const double* X, double* conn)
{
    double C[4][4][4];
    o_conn(c, X, C);
    memcpy(conn, C, sizeof(C));
}

void oracle_prim_to_flux(const ocfg_t* c, const double* P, const double* X, int dir, double* out)
{
    ogeom_t G;
    o_geom(c, X, &G);
    ostate_t S;
    o_state(c, P, &G, &S);
    o_flux_from_state(c, P, &G, &S, dir, out);
}

void oracle_speeds(const ocfg_t* c, const double* P, const double* X, int dir, double* lp, double* lm)
{
    ogeom_t G;
    o_geom(c, X, &G);
    ostate_t S;
    o_state(c, P, &G, &S);
    o_speeds_state(c, P, &G, &S, dir, lp, lm);
}

double oracle_vmax2(const ocfg_t* c, const double* P, const double* X)
{
    ogeom_t G;
    o_geom(c, X, &G);
    ostate_t S;
    o_state(c, P, &G, &S);
    return o_vmax2_state(c, P, &S);
}

/* Finite-difference Jacobian of the residual of one interior zone (index z in
 * the interior ordering) at state P, for a stage with P_n, P^E and dtp. */
/* For every interior zone, the finite-difference Jacobian of the Newton
 * system (the non-magnetic rows and unknowns, Sec. 3.1 and 8.2) at the state
 * P, for a stage with P_n, ghost-filled P^E and dtp: J[z][i][j] (m x m,
 * m = nvar - 3), and U_rho(P_n) of the zone, the scale of the Newton norm.
 * It bounds how far two states whose residual norms are below the tolerance
 * can lie apart: P_a - P_b = J^-1 (R_a - R_b) to first order. */
int oracle_system_jacobians_ghosted(const ocfg_t* c, const double* Pn, const double* PEg, double dtp,
                                    const double* P, double* J, double* urho)
{
#ifdef _OPENMP
    if (c->nthreads > 0) omp_set_num_threads(c->nthreads);
#endif
    olay_t L = o_layout(c);
    const int nv = c->nvar, m = nv - 3;
    const size_t nz = o_zones(&L);
    double* divF = (double*)calloc((size_t)nv * nz, sizeof(double));
    double* srcE = (double*)calloc((size_t)nv * nz, sizeof(double));
    oemhd_sp_t* sp = (oemhd_sp_t*)calloc(nz, sizeof(oemhd_sp_t));
    if (!divF || !srcE || !sp) { free(divF); free(srcE); free(sp); return -1; }
    o_explicit_stage(c, &L, PEg, divF, srcE, sp);
#pragma omp parallel for collapse(2) schedule(static)
    for (int kk = 0; kk < L.n[2]; ++kk)
        for (int jj = 0; jj < L.n[1]; ++jj)
            for (int ii = 0; ii < L.n[0]; ++ii) {
                size_t z = ((size_t)kk * L.n[1] + jj) * L.n[0] + ii;
                size_t cm = o_cell(&L, ii + L.g[0], jj + L.g[1], kk + L.g[2]);
                double X[4], pn[NVMAX], pe[NVMAX], dz[NVMAX], sz[NVMAX];
                o_zone_X(c, &L, ii + L.g[0], jj + L.g[1], kk + L.g[2], X);
                for (int v = 0; v < nv; ++v) {
                    pn[v] = Pn[(size_t)v * nz + z];
                    pe[v] = PEg[(size_t)v * L.cells + cm];
                    dz[v] = divF[(size_t)v * nz + z];
                    sz[v] = srcE[(size_t)v * nz + z];
                }
                ozone_t Z;
                o_zone_setup(c, X, pn, pe, dz, sz, &sp[z], dtp, &Z);
                oreduced_t Q;
                Q.z = &Z;
                Q.m = m;
                Q.map = o_unknown;
                for (int v = 0; v < NVMAX; ++v) Q.P[v] = v < nv ? P[(size_t)v * nz + z] : 0.0;
                double x[7], R[7];
                for (int i = 0; i < m; ++i) x[i] = Q.P[o_unknown[i]];
                o_reduced_residual(&Q, x, R);
                oracle_fd_jacobian(m, o_reduced_residual, &Q, x, R, c->eps, J + z * (size_t)m * m);
                urho[z] = Z.Un[RHO];
            }
    free(divF);
    free(srcE);
    free(sp);
    return 0;
}

int oracle_zone_jacobian(const ocfg_t* c, const double* Pn, const double* PE, double dtp, const double* P,
                         long z, double* J, double* Rz)
{
    olay_t L = o_layout(c);
    const int nv = c->nvar;
    const size_t nz = o_zones(&L);
    if (z < 0 || (size_t)z >= nz) return 1;
    double* PEg = (double*)calloc((size_t)nv * L.cells, sizeof(double));
    double* divF = (double*)calloc((size_t)nv * nz, sizeof(double));
    double* srcE = (double*)calloc((size_t)nv * nz, sizeof(double));
    oemhd_sp_t* sp = (oemhd_sp_t*)calloc(nz, sizeof(oemhd_sp_t));
    o_to_ghosted(c, &L, PE, PEg);
    o_explicit_stage(c, &L, PEg, divF, srcE, sp);
    int ii = (int)(z % L.n[0]), jj = (int)((z / L.n[0]) % L.n[1]), kk = (int)(z / ((size_t)L.n[0] * L.n[1]));
    double X[4], pn[NVMAX], pe[NVMAX], dz[NVMAX], sz[NVMAX], p[NVMAX];
    o_zone_X(c, &L, ii + L.g[0], jj + L.g[1], kk + L.g[2], X);
    for (int v = 0; v < nv; ++v) {
        pn[v] = Pn[(size_t)v * nz + z];
        pe[v] = PE[(size_t)v * nz + z];
        dz[v] = divF[(size_t)v * nz + z];
        sz[v] = srcE[(size_t)v * nz + z];
        p[v] = P[(size_t)v * nz + z];
    }
    ozone_t Z;
    o_zone_setup(c, X, pn, pe, dz, sz, &sp[z], dtp, &Z);
    o_zone_residual(&Z, p, Rz);
    oracle_fd_jacobian(nv, o_zone_residual, &Z, p, Rz, c->eps, J);
    free(PEg);
    free(divF);
    free(srcE);
    free(sp);
    return 0;
}
