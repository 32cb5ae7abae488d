// Device-side physics of the grim method for gfx950: metric access, derived
// fluid quantities, conserved variables, fluxes and wave speeds.  Everything
// here is __forceinline__ register code; the kernels that use it live in
// kernels.hip and newton.hip.
//
// Metric access is templated on a geometry type.  Each type declares at
// compile time which entries of g_{mu nu} and g^{mu nu} are structurally
// nonzero (nzc / nzn), so that after unrolling the Minkowski path carries no
// metric arithmetic at all and the Kerr-Schild path skips the theta-decoupled
// zeros (g_{0 2} = g_{1 2} = g_{2 3} = 0).  IEEE rules forbid the compiler
// from folding 0*x or 0+x itself, so the sparsity is made explicit here.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace grim {

enum : int { RHO = 0, UU = 1, U1 = 2, U2 = 3, U3 = 4, B1 = 5, B2 = 6, B3 = 7, QQ = 8, DP = 9 };

// Packed index of a symmetric 4x4 entry (m, n).
__host__ __device__ constexpr int sidx(int m, int n)
{
    return m <= n ? m * 4 - m * (m - 1) / 2 + n - m : n * 4 - n * (n - 1) / 2 + m - n;
}

// Reciprocal, inverse square root and square root for the hot loops: the
// hardware estimate (relative error below 2^-22 in double precision) refined
// by Newton-Raphson steps, each of which squares the relative error
// (Newton's iteration for 1/x and 1/sqrt(x); P. Markstein, IBM J. Res. Dev.
// 34 (1990) 111).  Two steps give about one unit in the last place at half the
// instructions and a much shorter dependency chain than the correctly rounded
// sequences.  Where a step is not finite (zero, infinite or NaN argument) the
// estimate, which is then the IEEE result, is returned.
__device__ __forceinline__ double rcp_nr(double x)
{
    const double r0 = __builtin_amdgcn_rcp(x);
    const double r1 = fma(fma(-x, r0, 1.0), r0, r0);
    const double r2 = fma(fma(-x, r1, 1.0), r1, r1);
    return __builtin_isfinite(r2) ? r2 : r0;
}

__device__ __forceinline__ float rcp_nr(float x)
{
    // the single-precision estimate is within 1 ulp already; one step
    const float r0 = __builtin_amdgcn_rcpf(x);
    const float r1 = fmaf(fmaf(-x, r0, 1.0f), r0, r0);
    return __builtin_isfinite(r1) ? r1 : r0;
}

__device__ __forceinline__ double rsq_nr(double x)
{
    // y <- y + (y/2)(1 - x y^2)
    const double y0 = __builtin_amdgcn_rsq(x);
    const double y1 = fma(0.5 * y0, fma(-x * y0, y0, 1.0), y0);
    const double y2 = fma(0.5 * y1, fma(-x * y1, y1, 1.0), y1);
    return __builtin_isfinite(y2) ? y2 : y0;
}

// sqrt(x) = x / sqrt(x), exact 0 for x = 0 (the clamp turns 0 * inf into
// 0 * DBL_MAX) and NaN for x < 0 (the clamp lets NaN through, which fmin
// would not); +inf gives NaN.  (A select on x == 0 instead costs the stage
// kernels 30-90 registers.)
__device__ __forceinline__ double sqrt_nr(double x)
{
    const double y = rsq_nr(x);
    return x * (y > 1.7976931348623157e308 ? 1.7976931348623157e308 : y);
}

// Physical constants shared by every kernel of one context.
struct Phys {
    double gam;      // adiabatic index
    double gm1;      // gamma - 1
    double kq, kd;   // sqrt(tau_R/chi), sqrt(tau_R/nu): EMHD rescaling (eqs. q, dP)
    double vq2, vd2; // (gamma-1) chi/tau_R, 4 nu/(3 tau_R) (Sec. 4.1)
    double tau, chi, nu;
    double theta;    // generalized-minmod parameter
    int closure;     // 1: chi = phi cs^2 tau_R, nu = psi cs^2 tau_R per state (Sec. 4)
    int sat;         // 1: DeltaP saturation through tau_R (Sec. 8.1, 9)
    double phi, psi, sat_w;
    int riemann;     // 0 LLF, 1 HLLE
    int recon;       // 0 PLM, 1 WENO5, 2 PPM
};

// Whether a configuration uses any option beyond the plain method (HLLE, a
// five-point reconstruction, the closure, the DeltaP saturation).  Kernels
// are instantiated for X = false (plain) and X = true; a plain instance
// clears the option fields of its own copy of Phys, so every option branch
// folds away at compile time and its registers match the method without
// options.
__host__ __device__ inline bool uses_options(const Phys& ph)
{
    return ph.closure || ph.sat || ph.riemann || ph.recon;
}
template <bool X>
__device__ __forceinline__ void plain_options(Phys& ph)
{
    if constexpr (!X) {
        ph.closure = 0;
        ph.sat = 0;
        ph.riemann = 0;
        ph.recon = 0;
    }
}

// ---------------------------------------------------------------- geometry

// Flat space in Cartesian coordinates.
struct GeoMink {
    static constexpr bool kFlat = true;
    __device__ __forceinline__ static constexpr bool nzc(int m, int n) { return m == n; }
    __device__ __forceinline__ static constexpr bool nzn(int m, int n) { return m == n; }
    __device__ __forceinline__ constexpr double gcov(int m, int n) const { return m == 0 && n == 0 ? -1.0 : 1.0; }
    __device__ __forceinline__ constexpr double gcon(int m, int n) const { return m == 0 && n == 0 ? -1.0 : 1.0; }
    __device__ __forceinline__ constexpr double gdet() const { return 1.0; }
    __device__ __forceinline__ constexpr double alpha() const { return 1.0; }
};

// Kerr in modified Kerr-Schild coordinates: stationary, axisymmetric, with
// X2 decoupled from the other coordinates.  Seven nonzero entries each for
// g_{mu nu} and g^{mu nu}: (0,0) (0,1) (0,3) (1,1) (1,3) (2,2) (3,3).
struct GeoKS {
    static constexpr bool kFlat = false;
    double c[7];  // g_{mu nu}
    double u[7];  // g^{mu nu}
    double gd, al;
    __device__ __forceinline__ static constexpr bool nzc(int m, int n)
    {
        return !((m == 2) ^ (n == 2));
    }
    __device__ __forceinline__ static constexpr bool nzn(int m, int n) { return nzc(m, n); }
    __device__ __forceinline__ static constexpr int k7(int m, int n)
    {
        // (0,0)->0 (0,1)->1 (0,3)->2 (1,1)->3 (1,3)->4 (2,2)->5 (3,3)->6
        const int a = m < n ? m : n, b = m < n ? n : m;
        return a == 0 ? (b == 0 ? 0 : (b == 1 ? 1 : 2)) : (a == 1 ? (b == 1 ? 3 : 4) : (a == 2 ? 5 : 6));
    }
    __device__ __forceinline__ double gcov(int m, int n) const { return c[k7(m, n)]; }
    __device__ __forceinline__ double gcon(int m, int n) const { return u[k7(m, n)]; }
    __device__ __forceinline__ double gdet() const { return gd; }
    __device__ __forceinline__ double alpha() const { return al; }
};

// Number of doubles per point in a Kerr-Schild metric table: 7 + 7 + gdet + alpha.
constexpr int kGeoDoubles = 16;

// Load the metric of table point p from an SoA table [kGeoDoubles][stride].
__device__ __forceinline__ void load_geo(GeoKS& g, const double* __restrict__ t, size_t p, size_t stride)
{
#pragma unroll
    for (int q = 0; q < 7; ++q) g.c[q] = t[q * stride + p];
#pragma unroll
    for (int q = 0; q < 7; ++q) g.u[q] = t[(7 + q) * stride + p];
    g.gd = t[14 * stride + p];
    g.al = t[15 * stride + p];
}

// dn_m = g_{m n} up^n, structural zeros skipped.
template <class G>
__device__ __forceinline__ void lower(const G& g, const double* up, double* dn)
{
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        double acc = 0.0;
        bool first = true;
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            if (G::nzc(m, n)) {
                const double t = g.gcov(m, n) * up[n];
                acc = first ? t : acc + t;
                first = false;
            }
        }
        dn[m] = acc;
    }
}

// ---------------------------------------------------------------- fluid state

template <int NV>
struct St {
    double ucon[4], ucov[4], bcon[4], bcov[4];
    double bsq, pg;
    double bh[4], bhc[4];  // unit b (EMHD only)
};

// Derived quantities of primitive state P (Sec. 4): gamma = sqrt(1 + g_ij
// ut^i ut^j), u^0 = gamma/alpha, u^i = ut^i - gamma alpha g^{0i};
// b^0 = B^i u_i, b^i = (B^i + b^0 u^i)/u^0; P = (gamma-1) u; bhat = b/|b|
// (zero for b^2 < 1e-30).
// kSelect: 1/|b| is computed unconditionally and selected, which keeps the
// caller's code in one basic block (the Minkowski kernels and every residual
// evaluation gain from it); otherwise a branch skips it where a whole wave
// has b^2 = 0 (field-free Kerr atmosphere), which the Kerr explicit-stage
// kernels gain from.
template <int NV, class G, bool kSelect = G::kFlat>
__device__ __forceinline__ void derive(const double* P, const G& g, const Phys& ph, St<NV>& s)
{
    double q2 = 0.0;
    bool first = true;
#pragma unroll
    for (int i = 1; i < 4; ++i)
#pragma unroll
        for (int j = 1; j < 4; ++j)
            if (G::nzc(i, j)) {
                const double t = g.gcov(i, j) * P[1 + i] * P[1 + j];
                q2 = first ? t : q2 + t;
                first = false;
            }
    const double gl2 = 1.0 + q2;
    const double igl = rsq_nr(gl2);  // 1/gamma
    const double gl = gl2 * igl;
    double iu0;
    if constexpr (G::kFlat) {
        s.ucon[0] = gl;
        iu0 = igl;
#pragma unroll
        for (int i = 1; i < 4; ++i) s.ucon[i] = P[1 + i];
    } else {
        s.ucon[0] = gl * rcp_nr(g.alpha());
        iu0 = g.alpha() * igl;
        const double ga = gl * g.alpha();
#pragma unroll
        for (int i = 1; i < 4; ++i) s.ucon[i] = P[1 + i] - ga * g.gcon(0, i);
    }
    lower(g, s.ucon, s.ucov);
    const double b0 = P[B1] * s.ucov[1] + P[B2] * s.ucov[2] + P[B3] * s.ucov[3];
    s.bcon[0] = b0;
#pragma unroll
    for (int i = 1; i < 4; ++i) s.bcon[i] = (P[B1 + i - 1] + b0 * s.ucon[i]) * iu0;
    lower(g, s.bcon, s.bcov);
    s.bsq = s.bcon[0] * s.bcov[0] + s.bcon[1] * s.bcov[1] + s.bcon[2] * s.bcov[2] + s.bcon[3] * s.bcov[3];
    s.pg = ph.gm1 * P[UU];
    if constexpr (NV == 10) {
        double ib;
        if constexpr (kSelect) {
            const double r = rsq_nr(s.bsq);
            ib = s.bsq > 1e-30 ? r : 0.0;
        } else {
            ib = s.bsq > 1e-30 ? rsq_nr(s.bsq) : 0.0;
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            s.bh[m] = s.bcon[m] * ib;
            s.bhc[m] = s.bcov[m] * ib;
        }
    }
}

// Row DIR of the mixed stress tensor T^DIR_nu (eq. fullSEtens), for nu = 0..3:
// (rho + u + P + b^2) u^DIR u_nu + (P + b^2/2) delta^DIR_nu - b^DIR b_nu
//  + q (bhat^DIR u_nu + u^DIR bhat_nu) - DP (bhat^DIR bhat_nu - (delta^DIR_nu + u^DIR u_nu)/3)
template <int NV, int DIR>
__device__ __forceinline__ void trow(const double* P, const St<NV>& s, double* T)
{
    const double w = P[RHO] + P[UU] + s.pg + s.bsq;
    const double pt = s.pg + 0.5 * s.bsq;
    const double wu = w * s.ucon[DIR];
    const double bd = s.bcon[DIR];
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        double t = wu * s.ucov[n] - bd * s.bcov[n];
        if (n == DIR) t += pt;
        if constexpr (NV == 10) {
            const double q = P[QQ], dp = P[DP];
            double h = s.ucon[DIR] * s.ucov[n];
            if (n == DIR) h += 1.0;
            t += q * (s.bh[DIR] * s.ucov[n] + s.ucon[DIR] * s.bhc[n]);
            t -= dp * (s.bh[DIR] * s.bhc[n] - h * (1.0 / 3.0));
        }
        T[n] = t;
    }
}

// Sound speed squared cs^2 = gamma (gamma-1) u / (rho + gamma u) (Sec. 4.1).
__device__ __forceinline__ double sound2(const double* P, const Phys& ph)
{
    return ph.gam * ph.gm1 * P[UU] * rcp_nr(P[RHO] + ph.gam * P[UU]);
}

// EMHD rescaled variables (eqs. q and dP): qt = q sqrt(tau/(chi rho Theta^2)),
// DPt = DP sqrt(tau/(nu rho Theta)), Theta = P/rho; written as
// qt = q sqrt(tau/chi) sqrt(rho)/P and DPt = DP sqrt(tau/nu)/sqrt(P).  With
// the closure (chi = phi cs^2 tau, nu = psi cs^2 tau of the state itself)
// sqrt(tau/chi) = 1/sqrt(phi cs^2) and sqrt(tau/nu) = 1/sqrt(psi cs^2).
template <int NV>
__device__ __forceinline__ void rescaled(const double* P, const St<NV>& s, const Phys& ph, double& qt, double& dpt)
{
    const double isp = rsq_nr(s.pg);  // 1/sqrt(P)
    if (ph.closure) {
        const double cs2 = sound2(P, ph);
        qt = P[QQ] * rsq_nr(ph.phi * cs2) * sqrt_nr(P[RHO]) * (isp * isp);
        dpt = P[DP] * rsq_nr(ph.psi * cs2) * isp;
    } else {
        qt = P[QQ] * ph.kq * sqrt_nr(P[RHO]) * (isp * isp);
        dpt = P[DP] * ph.kd * isp;
    }
}

// The relaxation time of a zone's stage at P^E (state P, derived s): tau_R,
// or with saturation tau_R / (1 + ((x - 1)/w)^2) where the anisotropy x =
// -DP/b^2 (DP < 0) or 2 DP/b^2 (DP > 0) exceeds 1 (firehose and mirror
// thresholds, Sec. 8.1 and 9), at least 1e-6 tau_R; b^2 floored at 1e-30.
template <int NV>
__device__ __forceinline__ double tau_eff(const double* P, const St<NV>& s, const Phys& ph)
{
    if (!ph.sat) return ph.tau;
    const double ib2 = rcp_nr(fmax(s.bsq, 1e-30));
    const double x = P[DP] < 0.0 ? -P[DP] * ib2 : 2.0 * P[DP] * ib2;
    const double y = (x - 1.0) * rcp_nr(ph.sat_w);
    const double f = x > 1.0 ? fmax(rcp_nr(1.0 + y * y), 1e-6) : 1.0;
    return ph.tau * f;
}

// Conserved vector U (Sec. 4: sqrt(-g) times rho u^0, T^0_nu, B^i, qt u^0, DPt u^0).
template <int NV, class G>
__device__ __forceinline__ void conserved(const double* P, const G& g, const St<NV>& s, const Phys& ph, double* U)
{
    double T[4];
    trow<NV, 0>(P, s, T);
    const double gd = g.gdet();
    U[RHO] = gd * P[RHO] * s.ucon[0];
#pragma unroll
    for (int n = 0; n < 4; ++n) U[UU + n] = gd * T[n];
#pragma unroll
    for (int i = 0; i < 3; ++i) U[B1 + i] = gd * P[B1 + i];
    if constexpr (NV == 10) {
        double qt, dpt;
        rescaled<NV>(P, s, ph, qt, dpt);
        U[QQ] = gd * qt * s.ucon[0];
        U[DP] = gd * dpt * s.ucon[0];
    }
}

// Flux along DIR (1..3): sqrt(-g) times rho u^d, T^d_nu, b^i u^d - b^d u^i,
// qt u^d, DPt u^d.  The induction flux takes the sign that follows from
// d_mu(sqrt(-g) *F^{mu i}) = 0 with B^i = *F^{i t}.
template <int NV, int DIR, class G>
__device__ __forceinline__ void flux(const double* P, const G& g, const St<NV>& s, const Phys& ph, double* F)
{
    double T[4];
    trow<NV, DIR>(P, s, T);
    const double gd = g.gdet();
    F[RHO] = gd * P[RHO] * s.ucon[DIR];
#pragma unroll
    for (int n = 0; n < 4; ++n) F[UU + n] = gd * T[n];
#pragma unroll
    for (int i = 1; i < 4; ++i) F[B1 + i - 1] = (i == DIR) ? 0.0 : gd * (s.bcon[i] * s.ucon[DIR] - s.bcon[DIR] * s.ucon[i]);
    if constexpr (NV == 10) {
        double qt, dpt;
        rescaled<NV>(P, s, ph, qt, dpt);
        F[QQ] = gd * qt * s.ucon[DIR];
        F[DP] = gd * dpt * s.ucon[DIR];
    }
}

// v_max^2 (Sec. 4.1, eq. modcs).
// With the closure vq^2 = (gamma-1) phi cs^2 and vdP^2 = 4 psi cs^2/3 of the
// state; otherwise the constants (gamma-1) chi/tau_R and 4 nu/(3 tau_R).
template <int NV>
__device__ __forceinline__ double vmax2(const double* P, const St<NV>& s, const Phys& ph)
{
    const double e = P[RHO] + ph.gam * P[UU];
    const double cs2 = ph.gam * ph.gm1 * P[UU] * rcp_nr(e);
    const double va2 = s.bsq * rcp_nr(e + s.bsq);
    double ct2 = cs2;
    if constexpr (NV == 10) {
        if (ph.closure) {
            const double vq2 = ph.gm1 * ph.phi * cs2;
            ct2 = 0.5 * (cs2 + vq2 + sqrt_nr(cs2 * cs2 + vq2 * vq2)) + (4.0 / 3.0) * ph.psi * cs2;
        } else {
            ct2 = 0.5 * (cs2 + ph.vq2 + sqrt_nr(cs2 * cs2 + ph.vq2 * ph.vq2)) + ph.vd2;
        }
    }
    return ct2 + va2 - ct2 * va2;
}

// Largest |grid-frame speed| along DIR of waves at +-v_max in the fluid frame:
// the roots of (1-v^2)(u^d - l u^0)^2 - v^2 (g^00 l^2 - 2 g^0d l + g^dd) = 0;
// max|root| = (|B| + sqrt(B^2 - 4AC)) / (2|A|).
template <int NV, int DIR, class G>
__device__ __forceinline__ double cmax(const double* P, const G& g, const St<NV>& s, const Phys& ph)
{
    const double v2 = vmax2<NV>(P, s, ph);
    const double a = 1.0 - v2;
    const double u0 = s.ucon[0], ud = s.ucon[DIR];
    const double A = a * u0 * u0 - v2 * g.gcon(0, 0);
    double B = a * u0 * ud;
    if (G::nzn(0, DIR)) B -= v2 * g.gcon(0, DIR);
    B *= -2.0;
    const double C = a * ud * ud - v2 * g.gcon(DIR, DIR);
    const double disc = fmax(B * B - 4.0 * A * C, 0.0);
    return (fabs(B) + sqrt_nr(disc)) * rcp_nr(2.0 * fabs(A));
}

// Both grid-frame speeds along DIR of waves at +-v_max in the fluid frame
// (the roots of the quadratic of cmax; A > 0 for any timelike u):
// lp = (-B + sqrt(disc)) / (2A) >= lm = (-B - sqrt(disc)) / (2A).
template <int NV, int DIR, class G>
__device__ __forceinline__ void speeds(const double* P, const G& g, const St<NV>& s, const Phys& ph, double& lp,
                                       double& lm)
{
    const double v2 = vmax2<NV>(P, s, ph);
    const double a = 1.0 - v2;
    const double u0 = s.ucon[0], ud = s.ucon[DIR];
    const double A = a * u0 * u0 - v2 * g.gcon(0, 0);
    double B = a * u0 * ud;
    if (G::nzn(0, DIR)) B -= v2 * g.gcon(0, DIR);
    B *= -2.0;
    const double C = a * ud * ud - v2 * g.gcon(DIR, DIR);
    const double sq = sqrt_nr(fmax(B * B - 4.0 * A * C, 0.0));
    const double i2a = rcp_nr(2.0 * A);
    lp = (sq - B) * i2a;
    lm = (-B - sq) * i2a;
}

// Generalized minmod slope minmod(theta a, (a+b)/2, theta b) (Sec. 2.3, 2.4.1).
__device__ __forceinline__ double gmm(double a, double b, double th)
{
    const double x = th * a, y = 0.5 * (a + b), z = th * b;
    const double mn = fmin(x, fmin(y, z)), mx = fmax(x, fmax(y, z));
    return mn > 0.0 ? mn : (mx < 0.0 ? mx : 0.0);
}

// WENO5 (Jiang and Shu's fifth-order weighted interpolation, one of the two
// five-point schemes Sec. 2.3 names): the value at the right face of the
// middle cell of a..e, the weighted mean of the third-order values of the
// stencils (a,b,c), (b,c,d), (c,d,e) with ideal weights 1/10, 6/10, 3/10,
// their smoothness indicators and epsilon = 1e-6.
__device__ __forceinline__ double weno5(double a, double b, double c, double d, double e)
{
    const double q0 = (2.0 * a - 7.0 * b + 11.0 * c) * (1.0 / 6.0);
    const double q1 = (-b + 5.0 * c + 2.0 * d) * (1.0 / 6.0);
    const double q2 = (2.0 * c + 5.0 * d - e) * (1.0 / 6.0);
    const double t0 = a - 2.0 * b + c, u0 = a - 4.0 * b + 3.0 * c;
    const double t1 = b - 2.0 * c + d, u1 = b - d;
    const double t2 = c - 2.0 * d + e, u2 = 3.0 * c - 4.0 * d + e;
    const double s0 = 1e-6 + (13.0 / 12.0) * t0 * t0 + 0.25 * u0 * u0;
    const double s1 = 1e-6 + (13.0 / 12.0) * t1 * t1 + 0.25 * u1 * u1;
    const double s2 = 1e-6 + (13.0 / 12.0) * t2 * t2 + 0.25 * u2 * u2;
    const double w0 = 0.1 * rcp_nr(s0 * s0), w1 = 0.6 * rcp_nr(s1 * s1), w2 = 0.3 * rcp_nr(s2 * s2);
    return (w0 * q0 + w1 * q1 + w2 * q2) * rcp_nr(w0 + w1 + w2);
}

// PPM (Colella and Woodward's piecewise parabolic method, the other scheme
// Sec. 2.3 names): the left and right face values of the middle cell of
// a..e.  Face values start as 7/12 (sum of the two neighbours) - 1/12 (sum of
// the next two), bounded by the neighbouring cell values; at a local
// extremum both become the cell value, and a parabola that would overshoot
// has its far face value moved so that the extremum sits on the near face.
__device__ __forceinline__ void ppm(double a, double b, double c, double d, double e, double& l, double& r)
{
    l = (7.0 / 12.0) * (b + c) - (1.0 / 12.0) * (a + d);
    r = (7.0 / 12.0) * (c + d) - (1.0 / 12.0) * (b + e);
    l = fmin(fmax(l, fmin(b, c)), fmax(b, c));
    r = fmin(fmax(r, fmin(c, d)), fmax(c, d));
    const double dd = r - l, m6 = 6.0 * (c - 0.5 * (l + r));
    const bool flat = (r - c) * (c - l) <= 0.0;
    const bool lo = !flat && dd * m6 > dd * dd;
    const bool hi = !flat && !lo && -dd * dd > dd * m6;
    const double l2 = flat ? c : (lo ? 3.0 * c - 2.0 * r : l);
    const double r2 = flat ? c : (hi ? 3.0 * c - 2.0 * l : r);
    l = l2;
    r = r2;
}

}  // namespace grim
