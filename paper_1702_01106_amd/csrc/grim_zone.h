// Per-zone data of one stage solve and the stage residual R(P) (Sec. 3,
// eq. half_step_residual), evaluated in registers.  Shared by the Newton
// kernel and the residual test hook.
//
// Every term of R that does not depend on the unknown P is folded by the
// rhs kernel into rhs[v] (and, for EMHD, into the coefficient bundle), so
// one residual evaluation is: derive the state of P, build U(P), and for
// EMHD add the implicit relaxation terms:
//   R_v  = U_v(P)/dt' - rhs_v
//   R_q  += chalf qt(P) - aq1 (Theta - Theta_n) - aq2 (bhat.u - bhat.u_n) - aq3 (u^0 - u^0_n)
//   R_DP += chalf DPt(P) - ad2 (bhat.u - bhat.u_n) - ad3 (u^0 - u^0_n)
// where bhat.u = bhat_E^mu u_mu(P): the IMEX split of Sec. 2.3 with the
// time derivatives of Theta, u_mu and u^0 differenced against P_n and every
// coefficient frozen at P^E.
#pragma once

#include "grim_device.h"
#include "grim_internal.h"

namespace grim {

template <int NV, class G>
struct ZoneC {
    G g;
    double rhs[NV];
    double idt;
    double bh[4], thn, u0n, cbun, aq1, aq2, aq3, ad2, ad3, chalf;  // EMHD only
};

// Interior zone index z -> ghosted cell index.
__device__ __forceinline__ long zone_cell(const Layout& L, long z)
{
    int i, j, k;
    zone_ijk(L, z, i, j, k);
    return L.cell(i + L.g[0], j + L.g[1], k + L.g[2]);
}

template <int NV, class G>
__device__ __forceinline__ void load_zone(const StageArgs& a, long z, long cell, ZoneC<NV, G>& zc)
{
    if constexpr (!G::kFlat) {
        const long p = cell % ((long)a.L.N[0] * a.L.N[1]);
        load_geo(zc.g, a.geo.centre, (size_t)p, a.geo.stride);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) zc.rhs[v] = a.rhs[(long)v * a.L.nz + z];
    zc.idt = 1.0 / a.dtp;
    if constexpr (NV == 10) {
        const double* c = a.coef;
        const long nz = a.L.nz;
#pragma unroll
        for (int m = 0; m < 4; ++m) zc.bh[m] = c[m * nz + z];
        zc.thn = c[4 * nz + z];
        zc.u0n = c[5 * nz + z];
        zc.cbun = c[6 * nz + z];
        zc.aq1 = c[7 * nz + z];
        zc.aq2 = c[8 * nz + z];
        zc.aq3 = c[9 * nz + z];
        zc.ad2 = c[10 * nz + z];
        zc.ad3 = c[11 * nz + z];
        zc.chalf = c[12 * nz + z];
    }
}

// ZoneC from a zone's stage right-hand side and EMHD coefficients computed in
// registers (the same fields load_zone reads from memory).
template <int NV, class G>
__device__ __forceinline__ void zone_from_rhs(const StageArgs& a, const double* co, ZoneC<NV, G>& zc)
{
    zc.idt = 1.0 / a.dtp;
    if constexpr (NV == 10) {
#pragma unroll
        for (int m = 0; m < 4; ++m) zc.bh[m] = co[m];
        zc.thn = co[4];
        zc.u0n = co[5];
        zc.cbun = co[6];
        zc.aq1 = co[7];
        zc.aq2 = co[8];
        zc.aq3 = co[9];
        zc.ad2 = co[10];
        zc.ad3 = co[11];
        zc.chalf = co[12];
    }
}

template <int NV, class G>
__device__ __forceinline__ void zone_residual(const double* P, const ZoneC<NV, G>& zc, const Phys& ph, double* R)
{
    St<NV> s;
    derive<NV, G, true>(P, zc.g, ph, s);
    double T[4];
    trow<NV, 0>(P, s, T);
    const double gd = zc.g.gdet();
    const double gi = gd * zc.idt;
    R[RHO] = gi * P[RHO] * s.ucon[0] - zc.rhs[RHO];
#pragma unroll
    for (int n = 0; n < 4; ++n) R[UU + n] = gi * T[n] - zc.rhs[UU + n];
#pragma unroll
    for (int i = 0; i < 3; ++i) R[B1 + i] = gi * P[B1 + i] - zc.rhs[B1 + i];
    if constexpr (NV == 10) {
        double qt, dpt;
        rescaled<NV>(P, s, ph, qt, dpt);
        const double th = s.pg * rcp_nr(P[RHO]);
        const double bu = zc.bh[0] * s.ucov[0] + zc.bh[1] * s.ucov[1] + zc.bh[2] * s.ucov[2] + zc.bh[3] * s.ucov[3];
        const double dbu = bu - zc.cbun;
        const double du0 = s.ucon[0] - zc.u0n;
        R[QQ] = gi * qt * s.ucon[0] - zc.rhs[QQ] + zc.chalf * qt - zc.aq1 * (th - zc.thn) - zc.aq2 * dbu -
                zc.aq3 * du0;
        R[DP] = gi * dpt * s.ucon[0] - zc.rhs[DP] + zc.chalf * dpt - zc.ad2 * dbu - zc.ad3 * du0;
    }
}

// The Newton system.  The paper's (Sec. 8.2: 5x5 for ideal MHD, 7x7 for
// EMHD) is over the non-magnetic primitives; B stays at its explicit update,
// the root of the induction rows, which depend on B alone.  With FULL the
// system is over all NV primitives (8x8 / 10x10), B started at that update:
// the same root.  Unknown i is primitive unk<FULL>(i).
template <int NV, bool FULL = false>
struct Sys {
    static constexpr int N = FULL ? NV : NV - 3;
};
template <bool FULL = false>
__device__ __forceinline__ constexpr int unk(int i) { return FULL ? i : (i < B1 ? i : i + 3); }

// sum of squares of the system rows of a residual vector
template <int NV, bool FULL = false>
__device__ __forceinline__ double sumsq(const double* R)
{
    double s = R[0] * R[0];
#pragma unroll
    for (int i = 1; i < Sys<NV, FULL>::N; ++i) s = fma(R[unk<FULL>(i)], R[unk<FULL>(i)], s);
    return s;
}

}  // namespace grim
