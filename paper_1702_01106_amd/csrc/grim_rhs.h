// The stage right-hand side of one zone (Sec. 2.3, eqs. half_step,
// full_step; Sec. 4.2 flux-CT; Sec. 4 EMHD sources) from the face fluxes and
// P_n, P^E: used by the right-hand-side kernel, which stores it for the
// Newton kernel, and by the Newton kernel's fused form, which computes it in
// registers and never stores it.
#pragma once

#include "grim_device.h"
#include "grim_internal.h"

namespace grim {

// Flux of every variable through one face normal to DIR (Sec. 2.4): left
// and right states by reconstruction along DIR, then LLF (c_max the largest
// |speed| of either state) or, with ph.riemann, HLLE (cR the largest
// right-going speed and cL the largest left-going one, both at least zero).
// cell(v, o) is variable v of the cell at offset o from the face's high
// cell: o in {-2, -1, 0, 1} for PLM (generalized minmod), and with kFive
// and ph.recon set also -3 and 2 for WENO5 / PPM (a grid with three ghost
// layers).  The normal B flux is exactly zero.
template <int NV, class G, int DIR, bool kFive = false, class Cell>
__device__ __forceinline__ void llf_face(const Phys& ph, const G& g, const Cell& cell, double* f)
{
    const double th = ph.theta;
    double PL[NV], PR[NV];
    if (!kFive || ph.recon == 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double pm2 = cell(v, -2), pm1 = cell(v, -1), p0 = cell(v, 0), pp1 = cell(v, 1);
            PL[v] = pm1 + 0.5 * gmm(pm1 - pm2, p0 - pm1, th);
            PR[v] = p0 - 0.5 * gmm(p0 - pm1, pp1 - p0, th);
        }
    } else if (ph.recon == 1) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double a = cell(v, -3), b = cell(v, -2), c = cell(v, -1), d = cell(v, 0), e = cell(v, 1),
                         h = cell(v, 2);
            PL[v] = weno5(a, b, c, d, e);
            PR[v] = weno5(h, e, d, c, b);
        }
    } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double a = cell(v, -3), b = cell(v, -2), c = cell(v, -1), d = cell(v, 0), e = cell(v, 1),
                         h = cell(v, 2);
            double l0, r0, l1, r1;
            ppm(a, b, c, d, e, l0, r0);
            ppm(b, c, d, e, h, l1, r1);
            PL[v] = r0;
            PR[v] = l1;
        }
    }
    St<NV> sL, sR;
    derive<NV>(PL, g, ph, sL);
    derive<NV>(PR, g, ph, sR);
    double UL[NV], UR[NV], FL[NV], FR[NV];
    conserved<NV>(PL, g, sL, ph, UL);
    conserved<NV>(PR, g, sR, ph, UR);
    flux<NV, DIR>(PL, g, sL, ph, FL);
    flux<NV, DIR>(PR, g, sR, ph, FR);
    if (ph.riemann) {
        double lpL, lmL, lpR, lmR;
        speeds<NV, DIR>(PL, g, sL, ph, lpL, lmL);
        speeds<NV, DIR>(PR, g, sR, ph, lpR, lmR);
        const double cR = fmax(0.0, fmax(lpL, lpR)), cL = fmax(0.0, fmax(-lmL, -lmR));
        const double is = rcp_nr(cL + cR), cRL = cR * cL;
#pragma unroll
        for (int v = 0; v < NV; ++v)
            f[v] = (v == B1 + DIR - 1) ? 0.0 : (cR * FL[v] + cL * FR[v] - cRL * (UR[v] - UL[v])) * is;
        return;
    }
    const double c = fmax(cmax<NV, DIR>(PL, g, sL, ph), cmax<NV, DIR>(PR, g, sR, ph));
#pragma unroll
    for (int v = 0; v < NV; ++v) f[v] = (v == B1 + DIR - 1) ? 0.0 : 0.5 * (FL[v] + FR[v]) - 0.5 * c * (UR[v] - UL[v]);
}

// Exchange a double with the other lane of its pair (lanes 2m and 2m + 1):
// DPP quad permutation [1, 0, 3, 2].  Every lane of the wave must be active.
__device__ __forceinline__ double pair_swap(double x)
{
    constexpr int kSwapPairs = 0xb1;
    const unsigned long long u = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)u, (int)(unsigned)u, kSwapPairs, 0xf, 0xf, false);
    const unsigned hi =
        (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)(u >> 32), (int)(unsigned)(u >> 32), kSwapPairs, 0xf, 0xf, false);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// The LLF flux of one face normal to DIR computed by a pair of lanes (Sec.
// 2.4): the even lane builds the left state and the odd lane the right one
// (PLM, derived state, wave speed, U and F, each exactly as llf_face builds
// it), the pair swaps c_max, U and F, and the even lane combines them in
// llf_face's order; the odd lane's f is not meaningful.  cell(v, o) is as
// for llf_face.  Every lane of the wave must take part (the swaps are
// cross-lane).
template <int NV, class G, int DIR, class Cell>
__device__ __forceinline__ void llf_pair(const Phys& ph, const G& g, const Cell& cell, bool right, double* f)
{
    const double th = ph.theta;
    const int o = right ? -1 : -2;
    double P[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const double x0 = cell(v, o), x1 = cell(v, o + 1), x2 = cell(v, o + 2);
        const double h = 0.5 * gmm(x1 - x0, x2 - x1, th);
        P[v] = right ? x1 - h : x1 + h;
    }
    St<NV> st;
    derive<NV>(P, g, ph, st);
    double U[NV], F[NV];
    conserved<NV>(P, g, st, ph, U);
    flux<NV, DIR>(P, g, st, ph, F);
    if (ph.riemann) {
        // HLLE, as llf_face: the even lane's state is the left one
        double lp, lm;
        speeds<NV, DIR>(P, g, st, ph, lp, lm);
        const double cR = fmax(0.0, fmax(lp, pair_swap(lp))), cL = fmax(0.0, fmax(-lm, -pair_swap(lm)));
        const double is = rcp_nr(cL + cR), cRL = cR * cL;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double Fo = pair_swap(F[v]), Uo = pair_swap(U[v]);
            f[v] = (v == B1 + DIR - 1) ? 0.0 : (cR * F[v] + cL * Fo - cRL * (Uo - U[v])) * is;
        }
        return;
    }
    const double c = cmax<NV, DIR>(P, g, st, ph);
    const double cc = fmax(c, pair_swap(c));
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const double Fo = pair_swap(F[v]), Uo = pair_swap(U[v]);
        f[v] = (v == B1 + DIR - 1) ? 0.0 : 0.5 * (F[v] + Fo) - 0.5 * cc * (Uo - U[v]);
    }
}

// Where zone_rhs reads the face fluxes, P^E and P_n: F(d, v, m, o) is the
// flux of variable v through the face normal to d on the low side of the cell
// at offset o = (o1, o2, o3) from cell m; PE(v, m, o) is P^E there; Pn(v, m)
// is P_n of cell m.  SrcGlobal reads the stage buffers; the tiled stage
// kernel reads its LDS tile and the P_n it loaded ahead.  A source with
// kNbrX also hands over the EMHD slope points of the zone's six neighbours
// (emhd_point, nbr_x(d, below, above)) instead of their P^E.
struct SrcGlobal {
    static constexpr bool kNbrX = false;
    const StageArgs& a;
    __device__ __forceinline__ long at(long m, int o1, int o2, int o3) const
    {
        return m + o1 + (long)o2 * a.L.N[0] + (long)o3 * a.L.N[0] * a.L.N[1];
    }
    __device__ __forceinline__ double F(int d, int v, long m, int o1, int o2, int o3) const
    {
        return a.F[d][(long)v * a.L.cells + at(m, o1, o2, o3)];
    }
    __device__ __forceinline__ double PE(int v, long m, int o1, int o2, int o3) const
    {
        return a.PE[(long)v * a.L.cells + at(m, o1, o2, o3)];
    }
    __device__ __forceinline__ double Pn(int v, long m) const { return a.Pn[(long)v * a.L.cells + m]; }
    // Kerr: the centre metric and connection of table point p = j N1 + i
    template <class G>
    __device__ __forceinline__ void centre(G& g, size_t p) const
    {
        if constexpr (!G::kFlat) load_geo(g, a.geo.centre, p, a.geo.stride);
    }
    __device__ __forceinline__ double conn(int q, size_t p) const { return a.geo.conn[(size_t)q * a.geo.stride + p]; }
};

// Flux-CT (Sec. 4.2): the edge EMF as the average of the four face B-fluxes
// around the edge.  E (index e) at the cell at offset o from m: E3 on
// (i-1/2, j-1/2, k), E1 on (i, j-1/2, k-1/2), E2 on (i-1/2, j, k-1/2).
// Evaluated where the stage right-hand side needs it, from the face fluxes.
template <int E, class Src>
__device__ __forceinline__ double edge_emf(const Src& f, long m, int o1, int o2, int o3)
{
    if constexpr (E == 2)
        return 0.25 * (f.F(0, B2, m, o1, o2, o3) + f.F(0, B2, m, o1, o2 - 1, o3) - f.F(1, B1, m, o1, o2, o3) -
                       f.F(1, B1, m, o1 - 1, o2, o3));
    else if constexpr (E == 0)
        return 0.25 * (f.F(1, B3, m, o1, o2, o3) + f.F(1, B3, m, o1, o2, o3 - 1) - f.F(2, B2, m, o1, o2, o3) -
                       f.F(2, B2, m, o1, o2 - 1, o3));
    else
        return 0.25 * (f.F(2, B1, m, o1, o2, o3) + f.F(2, B1, m, o1 - 1, o2, o3) - f.F(0, B3, m, o1, o2, o3) -
                       f.F(0, B3, m, o1, o2, o3 - 1));
}

// ------------------------------------------------------------------ stage rhs

// Generalized-minmod slope of the derived quantities used by the EMHD
// sources: Theta, u_0..u_3, u^1..u^3 (8 values).
template <int NV, class G>
__device__ __forceinline__ void emhd_point(const double* P, const G& g, const Phys& ph, double* X)
{
    St<NV> s;
    derive<NV>(P, g, ph, s);
    X[0] = s.pg * rcp_nr(P[RHO]);
#pragma unroll
    for (int m = 0; m < 4; ++m) X[1 + m] = s.ucov[m];
#pragma unroll
    for (int m = 1; m < 4; ++m) X[4 + m] = s.ucon[m];
}

template <int NV>
__device__ __forceinline__ void load_cell(const double* P, long cells, long m, double* out)
{
#pragma unroll
    for (int v = 0; v < NV; ++v) out[v] = P[(long)v * cells + m];
}

// The stage right-hand side of interior zone z:
//   rhs_v = U_v(P_n)/dt' - divF_v(P^E) + S^E_v(P^E)
// plus, for EMHD, every P-independent part of the relaxation sources folded
// into rhs_q, rhs_DP, and the kEmhdCoef coefficients co[] the Newton residual
// needs (bhat^mu of P^E, Theta(P_n), u^0(P_n), bhat.u(P_n), aq1, aq2, aq3,
// ad2, ad3, chalf).  g returns the zone's metric.  With kOut the optional
// outputs of a (learned-guess features, test-hook arrays) are written too.
template <int NV, class G, int ND, bool kOut, class Src>
__device__ __forceinline__ void zone_rhs(const StageArgs& a, long z, double* rhs, double* co, G& g, const Src& in)
{
    const Layout& L = a.L;
    int ii, jj, kk;
    zone_ijk(L, z, ii, jj, kk);
    const int i = ii + L.g[0], j = jj + L.g[1], k = kk + L.g[2];
    const long m = L.cell(i, j, k);
    const long C = L.cells;
    constexpr int nd = ND;

    // divergence of the face fluxes, B rows from the flux-CT EMFs
    double divF[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        double s = 0.0;
#pragma unroll
        for (int d = 0; d < nd; ++d) {
            // offset of the high face's cell
            const int e1 = d == 0, e2 = d == 1, e3 = d == 2;
            double fr, fl;
            const bool ct = nd >= 2 && v >= B1 && v <= B3 && (nd == 3 || v != B3);
            if (!ct) {
                fr = in.F(d, v, m, e1, e2, e3);
                fl = in.F(d, v, m, 0, 0, 0);
            } else {
                const int b = v - B1;
                // face B^b flux through the face normal to d of the cell at
                // offset o, from the edge EMFs
                auto face = [&](int o1, int o2, int o3) -> double {
                    if (b == d) return 0.0;
                    if (d == 0 && b == 1)
                        return 0.5 * (edge_emf<2>(in, m, o1, o2, o3) + edge_emf<2>(in, m, o1, o2 + 1, o3));
                    if (d == 0 && b == 2)
                        return -0.5 * (edge_emf<1>(in, m, o1, o2, o3) + edge_emf<1>(in, m, o1, o2, o3 + 1));
                    if (d == 1 && b == 0)
                        return -0.5 * (edge_emf<2>(in, m, o1, o2, o3) + edge_emf<2>(in, m, o1 + 1, o2, o3));
                    if (d == 1 && b == 2)
                        return 0.5 * (edge_emf<0>(in, m, o1, o2, o3) + edge_emf<0>(in, m, o1, o2, o3 + 1));
                    if (d == 2 && b == 0)
                        return 0.5 * (edge_emf<1>(in, m, o1, o2, o3) + edge_emf<1>(in, m, o1 + 1, o2, o3));
                    return -0.5 * (edge_emf<0>(in, m, o1, o2, o3) + edge_emf<0>(in, m, o1, o2 + 1, o3));  // d == 2, b == 1
                };
                fr = face(e1, e2, e3);
                fl = face(0, 0, 0);
            }
            s += (fr - fl) * (1.0 / L.dx[d]);
        }
        divF[v] = s;
    }

    if constexpr (!G::kFlat) in.centre(g, (size_t)((long)j * L.N[0] + i));
    const double idt = 1.0 / a.dtp;
    double Pn[NV], PE[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        Pn[v] = in.Pn(v, m);
        PE[v] = in.PE(v, m, 0, 0, 0);
    }
    St<NV> sn, sE;
    derive<NV>(Pn, g, a.ph, sn);
    derive<NV>(PE, g, a.ph, sE);
    double Un[NV];
    conserved<NV>(Pn, g, sn, a.ph, Un);

    // explicit geometric source sqrt(-g) T^k_l Gamma^l_{nu k} at P^E, and for
    // EMHD the connection parts of the q0, DP0 and div u terms at P^E:
    //   ga = bhat^mu Gamma^l_{n mu} u^n u_l,  gb = bhat^mu bhat^n Gamma^l_{mu n} u_l,
    //   gdv = Gamma^mu_{mu l} u^l.
    // Gamma is read one upper index l at a time (16 values), so at most 16 of
    // its 64 entries are live in registers.
    double src[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) src[v] = 0.0;
    double ga = 0.0, gb = 0.0, gdv = 0.0;
    if constexpr (!G::kFlat) {
        const size_t p = (size_t)((long)j * L.N[0] + i);
        double T[4][4];
        trow<NV, 0>(PE, sE, T[0]);
        trow<NV, 1>(PE, sE, T[1]);
        trow<NV, 2>(PE, sE, T[2]);
        trow<NV, 3>(PE, sE, T[3]);
        double s4[4] = {0.0, 0.0, 0.0, 0.0};
        // ga and gb as sums over l of u_l times Gamma^l contracted with the
        // tensors wa^{n mu} = u^n bhat^mu and wb^{mu n} = bhat^mu bhat^n
        double wa[4][4], wb[4][4];
        if constexpr (NV == 10) {
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    wa[a][b] = sE.ucon[a] * sE.bh[b];
                    wb[a][b] = sE.bh[a] * sE.bh[b];
                }
        }
#pragma unroll
        for (int l = 0; l < 4; ++l) {
            double c[4][4];  // Gamma^l_{a b}
#pragma unroll
            for (int q = 0; q < 16; ++q) c[q / 4][q % 4] = in.conn(l * 16 + q, p);
#pragma unroll
            for (int n = 0; n < 4; ++n)
#pragma unroll
                for (int kap = 0; kap < 4; ++kap) s4[n] += T[kap][l] * c[n][kap];
            if constexpr (NV == 10) {
                double ta = 0.0, tb = 0.0;
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 4; ++b) {
                        ta = fma(c[a][b], wa[a][b], ta);
                        tb = fma(c[a][b], wb[a][b], tb);
                    }
                ga = fma(ta, sE.ucov[l], ga);
                gb = fma(tb, sE.ucov[l], gb);
#pragma unroll
                for (int n = 0; n < 4; ++n) gdv += c[l][n] * sE.ucon[n];
            }
        }
#pragma unroll
        for (int n = 0; n < 4; ++n) src[UU + n] = g.gdet() * s4[n];
    }

#pragma unroll
    for (int v = 0; v < NV; ++v) rhs[v] = Un[v] * idt - divF[v] + src[v];

    double sq = 0.0, sdiv = 0.0, sdp = 0.0;
    if constexpr (NV == 10) {
        // limited slopes of Theta, u_mu, u^i of P^E (Sec. 2.3), folded into
        // the sums a1 = bhat^d dTheta/dx^d, a2 = bhat^mu u^d du_mu/dx^d,
        // b1 = bhat^d bhat^mu du_mu/dx^d and divs = du^d/dx^d one direction
        // at a time
        double X0[8];
        emhd_point<NV>(PE, g, a.ph, X0);
        double a1 = 0.0, a2 = 0.0, b1 = 0.0, divs = 0.0;
#pragma unroll
        for (int d = 0; d < nd; ++d) {
            const double bhd = sE.bh[d + 1], ud = sE.ucon[d + 1];
            double Xm[8], Xp[8];
            if constexpr (Src::kNbrX) {
                in.nbr_x(d, Xm, Xp);
            } else {
                const int e1 = d == 0, e2 = d == 1, e3 = d == 2;
                double Pm[NV], Pp[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    Pm[v] = in.PE(v, m, -e1, -e2, -e3);
                    Pp[v] = in.PE(v, m, e1, e2, e3);
                }
                G gm, gp;
                if constexpr (!G::kFlat) {
                    const int im = d == 0 ? i - 1 : i, jm = d == 1 ? j - 1 : j;
                    const int ip = d == 0 ? i + 1 : i, jp = d == 1 ? j + 1 : j;
                    load_geo(gm, a.geo.centre, (size_t)((long)jm * L.N[0] + im), a.geo.stride);
                    load_geo(gp, a.geo.centre, (size_t)((long)jp * L.N[0] + ip), a.geo.stride);
                }
                emhd_point<NV>(Pm, gm, a.ph, Xm);
                emhd_point<NV>(Pp, gp, a.ph, Xp);
            }
            const double idx = 1.0 / L.dx[d];
            double dX[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) dX[q] = gmm(X0[q] - Xm[q], Xp[q] - X0[q], a.ph.theta) * idx;
            a1 += bhd * dX[0];
#pragma unroll
            for (int mu = 0; mu < 4; ++mu) {
                a2 += sE.bh[mu] * ud * dX[1 + mu];
                b1 += bhd * sE.bh[mu] * dX[1 + mu];
            }
            divs += dX[4 + d + 1];
        }
        const double theta = X0[0];
        sq = a1 + theta * (a2 - ga);
        sdiv = divs + gdv;
        sdp = b1 - gb;

        // fold the P-independent parts of the relaxation sources, with the
        // stage's relaxation time and diffusivities taken at P^E: tau_R (or
        // its saturated value) and chi, nu (or phi cs^2 tau, psi cs^2 tau of
        // P^E with the closure, when tau/chi = 1/(phi cs^2), tau/nu =
        // 1/(psi cs^2))
        const Phys& ph = a.ph;
        const double gd = g.gdet();
        const double rhoE = PE[RHO], thE = sE.pg * rcp_nr(PE[RHO]), u0E = sE.ucon[0];
        double qtE, dptE, qtn, dptn;
        rescaled<NV>(PE, sE, ph, qtE, dptE);
        rescaled<NV>(Pn, sn, ph, qtn, dptn);
        double tau = ph.tau, chiE = ph.chi, nuE = ph.nu, kq = ph.kq, kd = ph.kd;
        if (ph.closure) {
            const double cs2 = sound2(PE, ph);
            tau = tau_eff<NV>(PE, sE, ph);
            chiE = ph.phi * cs2 * tau;
            nuE = ph.psi * cs2 * tau;
            kq = rsq_nr(ph.phi * cs2);
            kd = rsq_nr(ph.psi * cs2);
        }
        const double itau = 1.0 / tau;
        // sqrt(tau/(chi rho Theta^2)) and sqrt(tau/(nu rho Theta)) at P^E
        const double kqE = kq * rsq_nr(rhoE * thE * thE);
        const double kdE = kd * rsq_nr(rhoE * thE);
        const double cq = (kqE * itau) * (-rhoE * chiE);
        const double cd = (kdE * itau) * (3.0 * rhoE * nuE);
        const double thn = sn.pg * rcp_nr(Pn[RHO]);
        const double u0n = sn.ucon[0];
        const double cbun = sE.bh[0] * sn.ucov[0] + sE.bh[1] * sn.ucov[1] + sE.bh[2] * sn.ucov[2] + sE.bh[3] * sn.ucov[3];
        rhs[QQ] += gd * (-qtn * (0.5 * itau) + cq * sq + 0.5 * qtE * sdiv);
        rhs[DP] += gd * (-dptn * (0.5 * itau) + cd * (sdp - sdiv * (1.0 / 3.0)) + 0.5 * dptE * sdiv);
#pragma unroll
        for (int mu = 0; mu < 4; ++mu) co[mu] = sE.bh[mu];
        co[4] = thn;
        co[5] = u0n;
        co[6] = cbun;
        co[7] = gd * cq * sE.bh[0] * idt;
        co[8] = gd * cq * thE * u0E * idt;
        co[9] = gd * 0.5 * qtE * idt;
        co[10] = gd * cd * sE.bh[0] * idt;
        co[11] = gd * (-(kdE * itau) * rhoE * nuE + 0.5 * dptE) * idt;
        co[12] = gd * (0.5 * itau);
    }
    if constexpr (!kOut) return;
    if (a.mlp_x) {
        // learned-guess features (dimensionless): the change of U the stage
        // asks for, relative to U_rho(P_n); the P_n state; lapse and g^{01},
        // g^{11} (constant in Minkowski)
        float x[kMlpIn];
#pragma unroll
        for (int q = 0; q < kMlpIn; ++q) x[q] = 0.0f;
        const double ur = Un[RHO];
#pragma unroll
        for (int v = 0; v < NV; ++v) x[v] = (float)((rhs[v] * a.dtp - Un[v]) / ur);
        x[NV] = (float)(Pn[UU] / Pn[RHO]);
#pragma unroll
        for (int i = 0; i < 3; ++i) x[NV + 1 + i] = (float)Pn[U1 + i];
        const double isr = 1.0 / sqrt(Pn[RHO]);
#pragma unroll
        for (int i = 0; i < 3; ++i) x[NV + 4 + i] = (float)(Pn[B1 + i] * isr);
        if constexpr (NV == 10) {
            x[NV + 7] = (float)(Pn[QQ] / Pn[UU]);
            x[NV + 8] = (float)(Pn[DP] / Pn[UU]);
        }
        x[kMlpIn - 3] = (float)g.alpha();
        x[kMlpIn - 2] = G::nzn(0, 1) ? (float)g.gcon(0, 1) : 0.0f;
        x[kMlpIn - 1] = (float)g.gcon(1, 1);
        float* xo = a.mlp_x + z * kMlpIn;
#pragma unroll
        for (int q = 0; q < kMlpIn; ++q) xo[q] = x[q];
    }
    if (a.dbg_divF) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            a.dbg_divF[(long)v * L.nz + z] = divF[v];
            a.dbg_src[(long)v * L.nz + z] = src[v];
        }
        if (a.dbg_sp) {
            a.dbg_sp[3 * z + 0] = sq;
            a.dbg_sp[3 * z + 1] = sdiv;
            a.dbg_sp[3 * z + 2] = sdp;
        }
    }
}

}  // namespace grim
