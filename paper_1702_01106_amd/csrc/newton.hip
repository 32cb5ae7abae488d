// The per-zone Newton-Raphson solve of grim (Sec. 3) for gfx950: one zone per
// lane, everything in registers.
//
//   R(P) FP64 always (a8).  Jacobian by forward differences with the
//   perturbation rule of Sec. 3.1 (a9): column j = (R(P_eps,j) - R(P))/h_j,
//   h_j = P_eps,j - P_j.  Dense LU with threshold partial pivoting (a10): row swaps are
//   branch-free selects so J never leaves registers.  Quadratic backtracking
//   line search (a11, Sec. 3.2): each new lambda is the minimiser of the
//   quadratic model, or with the safeguard option that minimiser kept in
//   [0.1, 0.5] of the previous lambda.  Converged lanes go idle; the wave
//   leaves the loop when every lane has (a12).  Statistics are reduced across
//   the wave with DPP moves and ballots and accumulated with one atomic per
//   wave and counter (a13).
//
// JT selects the precision of the difference quotients, the stored Jacobian
// and the LU: double (the plain method) or float (mixed precision; the
// residual, conserved variables, metric and Lorentz factor stay FP64).  In
// mixed precision a zone whose FP32 solve fails (in badly scaled zones the
// FP32 Newton direction can be too inaccurate to converge) is marked, and a
// second launch of the FP64 kernel solves only the marked zones from P_n.
#include <hip/hip_runtime.h>

#include "grim_internal.h"
#include "grim_rhs.h"
#include "grim_zone.h"

namespace grim {

namespace {

constexpr int kWave = 64;

// Solve A x = b in place (x returned in b) by Gaussian elimination with
// threshold partial pivoting: at step k the row of the column's largest
// entry is swapped in only when the diagonal entry is below kPivotThreshold
// of it (each multiplier then stays below 1/kPivotThreshold in size).  On
// the Kerr torus partial pivoting swaps rows in about a third of the zones
// although their diagonal entries are not small; with the threshold 0.2%
// of the zones swap, and on sampled Jacobians the largest entry of U stays
// the largest of A (growth factor 1).  Returns false on an exactly zero
// pivot column.
constexpr double kPivotThreshold = 0.1;
template <int N, typename T>
__device__ __forceinline__ bool lu_solve(T (&A)[N][N], T (&b)[N])
{
    bool ok = true;
    T inv[N];  // reciprocal pivots
#pragma unroll
    for (int k = 0; k < N; ++k) {
        T best = fabs(A[k][k]);
        int p = k;
#pragma unroll
        for (int i = k + 1; i < N; ++i) {
            const T v = fabs(A[i][k]);
            const bool gt = v > best;
            best = gt ? v : best;
            p = gt ? i : p;
        }
        ok = ok && (best != T(0));
        p = fabs(A[k][k]) < T(kPivotThreshold) * best ? p : k;
        // swap rows k and p with selects (J stays in registers), skipped
        // when no active lane of the wave needs a swap at this step
        if (k < N - 1 && __ballot(p != k) != 0ull) {
#pragma unroll
            for (int i = k + 1; i < N; ++i) {
                const bool s = (p == i);
#pragma unroll
                for (int j = k; j < N; ++j) {
                    const T tk = A[k][j], ti = A[i][j];
                    A[k][j] = s ? ti : tk;
                    A[i][j] = s ? tk : ti;
                }
                const T tk = b[k], ti = b[i];
                b[k] = s ? ti : tk;
                b[i] = s ? tk : ti;
            }
        }
        inv[k] = rcp_nr(A[k][k]);
#pragma unroll
        for (int i = k + 1; i < N; ++i) {
            const T f = A[i][k] * inv[k];
#pragma unroll
            for (int j = k + 1; j < N; ++j) A[i][j] = fma(-f, A[k][j], A[i][j]);
            b[i] = fma(-f, b[k], b[i]);
        }
    }
#pragma unroll
    for (int i = N - 1; i >= 0; --i) {
        T s = b[i];
#pragma unroll
        for (int j = i + 1; j < N; ++j) s = fma(-A[i][j], b[j], s);
        b[i] = s * inv[i];
    }
    return ok;
}

// Wave-wide reductions with DPP row shifts and row broadcasts (no LDS): an
// inclusive scan within each row of 16 lanes (shifts 1, 2, 4, 8), then row 0's
// total into row 1 and row 2's into row 3 (broadcast of lane 15), then the
// first two rows' total into rows 2 and 3 (broadcast of lane 31); lane 63
// ends with the whole wave.  Lanes a DPP move cannot source get the
// identity.  Inactive lanes must hold the identity too.
template <int Ctrl, int RowMask = 0xf>
__device__ __forceinline__ unsigned long long dpp64(unsigned long long x, unsigned long long id)
{
    const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)id, (int)(unsigned)x, Ctrl, RowMask, 0xf, false);
    const unsigned hi =
        (unsigned)__builtin_amdgcn_update_dpp((int)(unsigned)(id >> 32), (int)(unsigned)(x >> 32), Ctrl, RowMask, 0xf, false);
    return ((unsigned long long)hi << 32) | lo;
}

template <class Op>
__device__ __forceinline__ unsigned long long wave_reduce64(unsigned long long x, unsigned long long id, Op op)
{
    x = op(x, dpp64<0x111>(x, id));        // row_shr:1
    x = op(x, dpp64<0x112>(x, id));        // row_shr:2
    x = op(x, dpp64<0x114>(x, id));        // row_shr:4
    x = op(x, dpp64<0x118>(x, id));        // row_shr:8
    x = op(x, dpp64<0x142, 0xa>(x, id));   // row_bcast:15 into rows 1, 3
    x = op(x, dpp64<0x143, 0xc>(x, id));   // row_bcast:31 into rows 2, 3
    const unsigned lo = __builtin_amdgcn_readlane((unsigned)x, 63), hi = __builtin_amdgcn_readlane((unsigned)(x >> 32), 63);
    return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long wave_sumu64(unsigned long long x)
{
    return wave_reduce64(x, 0ull, [](unsigned long long a, unsigned long long b) { return a + b; });
}

__device__ __forceinline__ unsigned long long wave_maxu64(unsigned long long x)
{
    return wave_reduce64(x, 0ull, [](unsigned long long a, unsigned long long b) { return a > b ? a : b; });
}

__device__ __forceinline__ int wave_max(int x)
{
    return (int)wave_maxu64((unsigned long long)(unsigned)(x > 0 ? x : 0));
}

// Candidate guess from the network output y: rho, u relative to P_n,
// utilde absolute, q and DP relative to u_n; B is set by the caller.
template <int NV>
__device__ __forceinline__ void Pc_from_net(const double* pn, const float* y, double* P)
{
#pragma unroll
    for (int v = 0; v < NV; ++v) P[v] = pn[v];
    P[RHO] = pn[RHO] * (1.0 + (double)y[0]);
    P[UU] = pn[UU] * (1.0 + (double)y[1]);
#pragma unroll
    for (int i = 0; i < 3; ++i) P[U1 + i] = pn[U1 + i] + (double)y[2 + i];
    if constexpr (NV == 10) {
        P[QQ] = pn[QQ] + pn[UU] * (double)y[5];
        P[DP] = pn[DP] + pn[UU] * (double)y[6];
    }
}

// The Newton direction dP (zero in the B entries) at P, whose residual is R:
// the finite-difference Jacobian over the system's unknowns, column by
// column, then LU with threshold partial pivoting.  The energy row of the linear
// system is taken as energy + mass (both sides), which removes the rest-mass
// energy from it: an elementary row operation, so dP is unchanged, but the
// mass row's rho entry (u^0) no longer competes with the energy row's
// (about -(u^0)^2) for the first pivot, a near tie that made partial
// pivoting swap the two rows in about 40% of slow-flow zones.  Returns false
// on an exactly zero pivot.
template <int NV, class G, typename JT, bool FULL>
__device__ __forceinline__ bool newton_dir(const double* P, const double* R, const ZoneC<NV, G>& zc,
                                           const Phys& ph, double eps, double* dP)
{
    constexpr int N = Sys<NV, FULL>::N;
#pragma unroll
    for (int v = 0; v < NV; ++v) dP[v] = 0.0;
    JT J[N][N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        double Pe[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) Pe[q] = P[q];
        const double pj = P[unk<FULL>(j)];
        const bool small = fabs(pj) < 5.0 * eps;
        double pe = small ? eps : (1.0 + eps) * pj;
        double h = pe - pj;
        if (h == 0.0) {
            pe = pj + eps;
            h = pe - pj;
        }
        Pe[unk<FULL>(j)] = pe;
        double Re[NV];
        zone_residual<NV, G>(Pe, zc, ph, Re);
        const double ih = rcp_nr(h);
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const double d = Re[unk<FULL>(i)] - R[unk<FULL>(i)];
            J[i][j] = (JT)((i == 1 ? d + (Re[RHO] - R[RHO]) : d) * ih);
        }
    }
    static_assert(unk<FULL>(0) == RHO && unk<FULL>(1) == UU, "mass and energy rows come first");
    JT x[N];
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = (JT)(i == 1 ? -(R[UU] + R[RHO]) : -R[unk<FULL>(i)]);
    if (!lu_solve<N, JT>(J, x)) return false;
#pragma unroll
    for (int i = 0; i < N; ++i) dP[unk<FULL>(i)] = (double)x[i];
    return true;
}

// Ghosted coordinates along one direction that take their value from
// ghosted index p of an interior cell: p itself and up to two ghost images,
// the inverses of the ghost maps (periodic wrap, outflow clamp, polar mirror)
// for n >= Ng, which the host enforces.  Held in registers (an array indexed
// by a per-lane count would be placed in LDS or scratch).
struct GhostSlots {
    int cnt;     // 1 + number of images
    int q1, q2;  // the images (q2 only when cnt == 3); outflow: the images
                 // are the Ng consecutive cells from q1
    bool run;
};

__device__ __forceinline__ GhostSlots ghost_slots(int p, int g, int n, int bc)
{
    GhostSlots s;
    s.run = bc == 1;
    if (bc == 0) {
        // periodic: lower ghost p - n (p >= n), upper ghost p + n (p < 2g)
        const bool lo = p >= n, hi = p < 2 * g;
        s.cnt = 1 + (int)lo + (int)hi;
        s.q1 = lo ? p - n : p + n;
        s.q2 = p + n;
    } else if (bc == 1) {
        // outflow: the first interior cell fills every lower ghost, the last
        // every upper one
        const bool lo = p == g, hi = p == g + n - 1;
        s.cnt = (lo || hi) ? 1 + g : 1;
        s.q1 = lo ? 0 : g + n;
        s.q2 = s.q1 + 1;
    } else {
        // polar mirror about each face: 2g - 1 - p (p < 2g), 2(g + n) - 1 - p (p >= n)
        const bool lo = p < 2 * g, hi = p >= n;
        s.cnt = 1 + (int)lo + (int)hi;
        s.q1 = lo ? 2 * g - 1 - p : 2 * (g + n) - 1 - p;
        s.q2 = 2 * (g + n) - 1 - p;
    }
    return s;
}

__device__ __forceinline__ int slot(int a, int p, const GhostSlots& s)
{
    return a == 0 ? p : (s.run ? s.q1 + a - 1 : (a == 1 ? s.q1 : s.q2));
}

// Store a zone's primitives at its cell and at every ghost cell that maps to
// it (the composite map is the product of the per-direction maps; a polar
// image in X2 negates utilde^2 and B^2).  (i, j, k) are interior coordinates.
template <int NV>
__device__ __forceinline__ void store_with_ghosts(const Layout& L, const int* bc, int i, int j, int k, const double* P,
                                                  double* out)
{
    const int p0 = i + L.g[0], p1 = j + L.g[1], p2 = k + L.g[2];
    const GhostSlots s0 = ghost_slots(p0, L.g[0], L.n[0], bc[0]);
    GhostSlots s1{1, 0, 0, false}, s2{1, 0, 0, false};
    if (L.ndim > 1) s1 = ghost_slots(p1, L.g[1], L.n[1], bc[1]);
    if (L.ndim > 2) s2 = ghost_slots(p2, L.g[2], L.n[2], bc[2]);
    const bool polar = bc[1] == 2;
    const long C = L.cells;
    for (int a2 = 0; a2 < s2.cnt; ++a2) {
        const int q2 = slot(a2, p2, s2);
        for (int a1 = 0; a1 < s1.cnt; ++a1) {
            const int q1 = slot(a1, p1, s1);
            const bool flip = polar && a1 > 0;
            for (int a0 = 0; a0 < s0.cnt; ++a0) {
                double* o = out + L.cell(slot(a0, p0, s0), q1, q2);
#pragma unroll
                for (int v = 0; v < NV; ++v) o[(long)v * C] = (flip && (v == U2 || v == B2)) ? -P[v] : P[v];
            }
        }
    }
}

// Per-lane state of one zone's solve.
template <int NV, class G>
struct ZoneSolve {
    ZoneC<NV, G> zc;
    double P[NV], R[NV];
    double r, nscale, fB;
    long z, cell;
    int k, iters, ncalls, nbt, fallback;
    bool from_net;
    uint8_t fl;
};

// Start zone z: its constants (read from the rhs kernel's output, or for
// ND > 0 computed here from the face fluxes), P_n (or the caller's guess) with
// B at its explicit update (the exact root of the B rows), the learned
// candidate if one is given and its residual is smaller, and the initial
// residual.
template <int NV, class G, int ND, bool FULL, class Src = SrcGlobal>
__device__ __forceinline__ void zs_begin(const NewtonArgs& a, long z, const double* guess, const float* mlp_y,
                                         ZoneSolve<NV, G>& s, const Src* in = nullptr)
{
    const Layout& L = a.s.L;
    const Phys& ph = a.s.ph;
    s.z = z;
    s.cell = zone_cell(L, z);
    if constexpr (ND == 0) {
        load_zone<NV, G>(a.s, z, s.cell, s.zc);
    } else {
        double co[kEmhdCoef];
        if constexpr (__is_same(Src, SrcGlobal))
            zone_rhs<NV, G, ND, false>(a.s, z, s.zc.rhs, co, s.zc.g, SrcGlobal{a.s});
        else
            zone_rhs<NV, G, ND, false>(a.s, z, s.zc.rhs, co, s.zc.g, *in);
        zone_from_rhs<NV, G>(a.s, co, s.zc);
    }
    s.fB = a.s.dtp / s.zc.g.gdet();
    s.k = 0;
    s.iters = 0;
    s.ncalls = 0;
    s.nbt = 0;
    s.fallback = 0;
    s.from_net = false;
    s.fl = 0;
    double P_alt[NV];
    {
        double pn[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if constexpr (__is_same(Src, SrcGlobal))
                pn[v] = a.s.Pn[(long)v * L.cells + s.cell];
            else
                pn[v] = in->Pn(v, s.cell);
        }
        St<NV> sn;
        derive<NV>(pn, s.zc.g, ph, sn);
        // scaled norm: ||R|| = dt' sqrt(sum R^2) / U_rho(P_n)
        s.nscale = a.s.dtp / (s.zc.g.gdet() * pn[RHO] * sn.ucon[0]);
#pragma unroll
        for (int v = 0; v < NV; ++v) s.P[v] = guess ? guess[(long)v * L.nz + z] : pn[v];
        if (mlp_y) Pc_from_net<NV>(pn, mlp_y + z * kMlpOut, P_alt);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) s.P[B1 + i] = s.zc.rhs[B1 + i] * s.fB;
    zone_residual<NV, G>(s.P, s.zc, ph, s.R);
    ++s.ncalls;
    s.r = s.nscale * sqrt_nr(sumsq<NV, FULL>(s.R));
    if (mlp_y) {
        // keep the learned guess only if its residual is smaller
#pragma unroll
        for (int i = 0; i < 3; ++i) P_alt[B1 + i] = s.zc.rhs[B1 + i] * s.fB;
        double Rc[NV];
        zone_residual<NV, G>(P_alt, s.zc, ph, Rc);
        ++s.ncalls;
        const double rc = s.nscale * sqrt_nr(sumsq<NV, FULL>(Rc));
        if (rc < s.r) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                s.P[v] = P_alt[v];
                s.R[v] = Rc[v];
            }
            s.r = rc;
            s.from_net = true;
        } else {
            s.fallback = 1;
        }
    }
}

// One step of the solve: the convergence tests, then one Newton iteration
// with its line search.  Returns true once the solve has ended (converged, or
// failed with the flags set).  A failed solve from the learned guess starts
// again from P_n instead of ending.
template <int NV, class G, typename JT, bool FULL>
__device__ __forceinline__ bool zs_step(const NewtonArgs& a, ZoneSolve<NV, G>& s)
{
    constexpr int N = Sys<NV, FULL>::N;
    const Phys& ph = a.s.ph;
    bool ended = false;
    if (!isfinite(s.r)) {
        s.fl |= 16;
        ended = true;
    } else if (s.r < a.tol) {
        return true;
    } else if (s.k >= a.k_max) {
        s.fl |= 1;
        ended = true;
    } else {
        double dP[NV];
        const bool ok = newton_dir<NV, G, JT, FULL>(s.P, s.R, s.zc, ph, a.eps, dP);
        s.ncalls += N;
        if (!ok) {
            s.fl |= 4;
            ended = true;
        } else {
            // quadratic backtracking line search
            const double r = s.r, f0 = r * r;
            double lam = 1.0;
            bool accepted = false, have = false;
            double Pf[NV], Rf[NV], rf = 0.0;
            for (int tr = 0; tr < a.ls_max; ++tr) {
                double Pt[NV], Rt[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) Pt[v] = fma(lam, dP[v], s.P[v]);
                zone_residual<NV, G>(Pt, s.zc, ph, Rt);
                ++s.ncalls;
                const double rt = s.nscale * sqrt_nr(sumsq<NV, FULL>(Rt));
                if (isfinite(rt)) {
                    have = true;
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        Pf[v] = Pt[v];
                        Rf[v] = Rt[v];
                    }
                    rf = rt;
                    if (rt < r * (1.0 - a.eps_bt * lam)) {
                        accepted = true;
                        break;
                    }
                    // minimiser of the quadratic model f(0) - 2 f(0) lam + c lam^2
                    // through f(lam) (eq. linesearch_residual), optionally kept
                    // within [0.1, 0.5] of the previous lambda
                    const double ln = f0 * lam * lam / (rt * rt + (2.0 * lam - 1.0) * f0);
                    lam = a.ls_safeguard ? fmin(fmax(ln, 0.1 * lam), 0.5 * lam) : ln;
                } else {
                    lam *= 0.5;
                }
                ++s.nbt;  // a rejected trial
            }
            ++s.iters;
            ++s.k;
            if (!accepted) {
                s.fl |= 2;
                if (!have) {
                    s.fl |= 16;
                    ended = true;
                }
            }
            if (have) {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    s.P[v] = Pf[v];
                    s.R[v] = Rf[v];
                }
                s.r = rf;
            }
        }
    }
    if (!ended) return false;
    if (!(s.from_net && (s.fl & (1 | 4 | 16)))) return true;
    // the solve from the learned guess failed: start again from P_n
    const Layout& L = a.s.L;
    s.from_net = false;
    s.fallback = 1;
    s.fl = 0;
    s.k = 0;
#pragma unroll
    for (int v = 0; v < NV; ++v) s.P[v] = a.s.Pn[(long)v * L.cells + s.cell];
#pragma unroll
    for (int i = 0; i < 3; ++i) s.P[B1 + i] = s.zc.rhs[B1 + i] * s.fB;
    zone_residual<NV, G>(s.P, s.zc, ph, s.R);
    ++s.ncalls;
    s.r = s.nscale * sqrt_nr(sumsq<NV, FULL>(s.R));
    return false;
}

// Per-lane accumulators of the statistics over the zones a lane finishes.
struct LaneStats {
    int iters = 0, nc = 0, nbt = 0;  // Newton iterations, residual evaluations, rejected trials
    bool nf = false, nl = false, nu = false, na = false, nfb = false, nrt = false;
    unsigned long long rb = 0;  // bits of the final residual (ordered like the value)
};

// Floors, flags, outputs and statistics of a finished zone.
template <int NV, class G>
__device__ __forceinline__ void zs_finish(const NewtonArgs& a, ZoneSolve<NV, G>& s, bool retry, LaneStats& ls)
{
    const Layout& L = a.s.L;
    const long z = s.z;
    if (!(s.P[RHO] > 0.0) || !(s.P[UU] > 0.0)) s.fl |= 8;
    if ((a.pass == 1 && (s.fl & (1 | 4 | 16))) || retry) s.fl |= kFlagRetry;
    if (a.s.floors) {
        const int ii = (int)((unsigned)z % (unsigned)L.n[0]);
        const double r1 = exp(L.xs[0] + (ii + 0.5) * L.dx[0]);
        const double rf = a.s.rho_fl * pow(r1, -1.5), uf = a.s.u_fl * pow(r1, -2.5);
        if (!(s.P[RHO] >= rf)) s.P[RHO] = rf;
        if (!(s.P[UU] >= uf)) s.P[UU] = uf;
    }
    if (a.out_ghosted && a.write_ghosts) {
        int i, j, k;
        zone_ijk(L, z, i, j, k);
        store_with_ghosts<NV>(L, a.bc, i, j, k, s.P, a.out);
    } else if (a.out_ghosted) {
#pragma unroll
        for (int v = 0; v < NV; ++v) a.out[(long)v * L.cells + s.cell] = s.P[v];
    } else {
#pragma unroll
        for (int v = 0; v < NV; ++v) a.out[(long)v * L.nz + z] = s.P[v];
    }
    if (a.iters) {
        // the retry pass adds to the FP32 pass's count (the read sits in its
        // own branch so the first pass does not wait for its stores)
        if (retry)
            a.iters[z] += s.iters;
        else
            a.iters[z] = s.iters;
    }
    if (a.backtracks) {
        if (retry)
            a.backtracks[z] += s.nbt;
        else
            a.backtracks[z] = s.nbt;
    }
    if (a.resid) a.resid[z] = s.r;
    if (a.flags) a.flags[z] = s.fl;
    // a zone marked for the FP64 retry contributes only its work (iterations,
    // residual calls) to the FP32 pass; the retry pass reports its outcome
    const bool final_ = !(a.pass == 1 && (s.fl & kFlagRetry));
    ls.iters = s.iters;
    ls.nc = s.ncalls;
    ls.nbt = s.nbt;
    ls.nfb = s.fallback != 0;
    ls.na = !retry;
    ls.nrt = retry;
    if (final_) {
        ls.nf = (s.fl & (1 | 4 | 16)) != 0;
        ls.nl = (s.fl & 2) != 0;
        ls.nu = (s.fl & 8) != 0;
        const unsigned long long b =
            isfinite(s.r) ? (unsigned long long)__double_as_longlong(s.r) : 0x7FF0000000000000ull;
        ls.rb = b > ls.rb ? b : ls.rb;
    }
}

// Wave reduction of the lane statistics, one atomic per wave and counter:
// the 0/1 counters are popcounts of ballots; the iteration, residual-call and
// rejected-trial counts share one 64-bit sum in 21-bit fields (the host caps
// k_max at 100 and ls_max at 64, so a wave's sums stay below 2^20).
constexpr int kPack = 21;
constexpr unsigned long long kPackMask = (1ull << kPack) - 1;
__device__ __forceinline__ void flush_stats(const NewtonArgs& a, const LaneStats& ls)
{
    const unsigned long long all = wave_sumu64(((unsigned long long)(unsigned)ls.nbt << (2 * kPack)) |
                                               ((unsigned long long)(unsigned)ls.nc << kPack) | (unsigned)ls.iters);
    const int mit = wave_max(ls.iters);
    const unsigned long long rb = wave_maxu64(ls.rb);
    const unsigned long long nf = __popcll(__ballot(ls.nf)), nl = __popcll(__ballot(ls.nl)),
                             nu = __popcll(__ballot(ls.nu)), na = __popcll(__ballot(ls.na)),
                             nfb = __popcll(__ballot(ls.nfb)), nrt = __popcll(__ballot(ls.nrt));
    DevStats* ds = a.stats + (blockIdx.x & (kStatCopies - 1));
    if ((threadIdx.x & (kWave - 1)) == 0) {
        atomicAdd(&ds->iters[a.stage], all & kPackMask);
        atomicMax(&ds->max_iters, (unsigned)mit);
        if (nf > 0) atomicAdd(&ds->n_fail, nf);
        if (nl > 0) atomicAdd(&ds->n_ls, nl);
        if (nu > 0) atomicAdd(&ds->n_unphys, nu);
        if (na > 0) atomicAdd(&ds->zone_stages, na);
        if (nrt > 0) atomicAdd(&ds->n_retry, nrt);
        atomicAdd(&ds->resid_calls, (all >> kPack) & kPackMask);
        const unsigned long long nbt = all >> (2 * kPack);
        if (nbt > 0) atomicAdd(&ds->n_bt, nbt);
        if (nfb > 0) atomicAdd(&ds->n_fallback, nfb);
        atomicMax(&ds->max_resid_bits, rb);
    }
}

// Zones of a 3-D grid in bricks of kBrickI x kBrickJ x kBrickK, one brick a
// wave: a wave runs as long as its slowest zone, and the zones that need an
// extra Newton iteration come in clusters, which a compact brick meets with
// fewer waves than a row of 64.
constexpr int kBrickI = 8, kBrickJ = 4, kBrickK = 2;
static_assert(kBrickI * kBrickJ * kBrickK == kWave, "a brick per wave");
inline long brick_count(const Layout& L)
{
    return (long)((L.n[0] + kBrickI - 1) / kBrickI) * ((L.n[1] + kBrickJ - 1) / kBrickJ) *
           ((L.n[2] + kBrickK - 1) / kBrickK);
}
__device__ __forceinline__ bool brick_zone(const Layout& L, unsigned b, unsigned lane, long& z)
{
    const unsigned nbi = ((unsigned)L.n[0] + kBrickI - 1) / kBrickI, nbj = ((unsigned)L.n[1] + kBrickJ - 1) / kBrickJ;
    const unsigned r = b / nbi, bk = r / nbj;
    const unsigned i = (b - r * nbi) * kBrickI + lane % kBrickI;
    const unsigned j = (r - bk * nbj) * kBrickJ + (lane / kBrickI) % kBrickJ;
    const unsigned k = bk * kBrickK + lane / (kBrickI * kBrickJ);
    z = ((long)k * L.n[1] + j) * L.n[0] + i;
    return i < (unsigned)L.n[0] && j < (unsigned)L.n[1] && k < (unsigned)L.n[2];
}

// A zone per lane: the wave runs until its slowest zone has finished.  ND > 0:
// fused with the stage right-hand side of an ND-dimensional grid.  (A
// work-queue variant, where a lane that finished took the next zone of its
// wave's range, ran 20-45% slower on every workload measured and was
// dropped.)
template <int NV, class G, typename JT, int ND, bool FULL, bool X>
__global__ __launch_bounds__(kWave) void k_newton(NewtonArgs a)
{
    plain_options<X>(a.s.ph);
    // (the plane-interleaved order of the Kerr flux kernel made this one
    // 4-6% slower on the Kerr tori)
    // (the column order of the Kerr rhs kernel, with or without the XCD
    // renumbering, made this one 7% slower on the 192x192x96 torus)
    const unsigned wb = xcd_block(blockIdx.x, gridDim.x);
    long z;
    bool active;
    if (ND == 0 && a.s.L.ndim == 3) {
        active = brick_zone(a.s.L, wb, threadIdx.x, z);
    } else {
        z = (long)wb * kWave + threadIdx.x;
        active = z < a.s.L.nz;
    }
    const bool retry = a.pass == 2;
    if (retry) {
        active = active && (a.flags[z] & kFlagRetry);
        if (__ballot(active) == 0ull) return;  // wave-uniform exit
    }
    LaneStats ls;
    if (active) {
        ZoneSolve<NV, G> s;
        zs_begin<NV, G, ND, FULL>(a, z, retry ? nullptr : a.guess, retry ? nullptr : a.mlp_y, s);
        while (!zs_step<NV, G, JT, FULL>(a, s)) {
        }
        zs_finish<NV, G>(a, s, retry, ls);
    }
    if (a.stats) flush_stats(a, ls);
}

// ------------------------------------------------------------------ tiled stage
//
// One kernel per stage for 1- and 2-D Minkowski grids: a block of 256 threads
// owns a tile of TX x TY zones (16 x 16 in 2-D, 256 in 1-D).  It stages the
// tile's P^E with a two-cell halo in LDS, computes into LDS every face flux
// its zones need (the x-faces of rows -1..TY, for the corner EMFs of
// flux-CT, and the y-faces of columns -1..TX), then solves one zone per
// thread, reading fluxes and P^E from LDS.
// Fluxes never go to global memory and the stage is one launch; the price is
// recomputing the faces shared with neighbouring tiles (2.4 faces per zone in
// 2-D against 2.0).
template <int ND>
struct Tile {
    static constexpr int TX = ND == 1 ? 256 : 16, TY = ND == 1 ? 1 : 16;
    static constexpr int HY = ND == 1 ? 0 : 2;                     // P^E halo rows per side
    static constexpr int PX = TX + 4, PY = TY + 2 * HY;            // P^E tile, origin at (-2, -HY)
    static constexpr int XX = TX + 1, XY = ND == 1 ? 1 : TY + 2;   // x-faces: columns 0..TX, rows -1..TY
    static constexpr int XR = ND == 1 ? 0 : 1;                     // row offset of the x-face tile
    static constexpr int YX = TX + 2, YY = ND == 1 ? 0 : TY + 1;   // y-faces: columns -1..TX, rows 0..TY
    static constexpr int kThreads = TX * TY;
    template <int NV>
    static constexpr int words() { return NV * (PX * PY + XX * XY + YX * YY); }
};

template <int NV, int ND>
struct SrcTile {
    static constexpr bool kNbrX = false;
    using T = Tile<ND>;
    const double* pe;  // [NV][PY][PX]
    const double* fx;  // [NV][XY][XX]
    const double* fy;  // [NV][YY][YX]
    const double* pn;  // P_n of the zone (registers)
    int lx, ly;        // the zone in the tile
    __device__ __forceinline__ double F(int d, int v, long, int o1, int o2, int) const
    {
        if (d == 0) return fx[(v * T::XY + ly + o2 + T::XR) * T::XX + lx + o1];
        return fy[(v * T::YY + ly + o2) * T::YX + lx + o1 + 1];
    }
    __device__ __forceinline__ double PE(int v, long, int o1, int o2, int) const
    {
        return pe[(v * T::PY + ly + o2 + T::HY) * T::PX + lx + o1 + 2];
    }
    __device__ __forceinline__ double Pn(int v, long) const { return pn[v]; }
};

// Held to 256 registers (two waves per SIMD): with 79 KiB of LDS a block,
// two tiles then share a CU whenever the grid has more tiles than CUs.  When
// every tile fits at once (one per CU), 2-D blocks have kBlock = 512 threads
// instead: waves 4-7 stage P^E and compute the y-faces beside waves 0-3 (the
// x-faces), so the face phase runs two waves per SIMD, and then leave the
// zones to waves 0-3.
template <int NV, int ND, typename JT, int kBlock, bool FULL>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) void k_stage(NewtonArgs a)
{
    plain_options<false>(a.s.ph);  // the tiled stage runs the plain method only
    static_assert(kBlock == Tile<ND>::kThreads || (ND == 2 && kBlock == 2 * Tile<ND>::kThreads), "block size");
    using T = Tile<ND>;
    __shared__ double lds[T::template words<NV>()];
    double* pe = lds;
    double* fx = pe + NV * T::PY * T::PX;
    double* fy = fx + NV * T::XY * T::XX;
    const Layout& L = a.s.L;
    const long C = L.cells;
    const int tid = threadIdx.x;
    const unsigned tb = xcd_block(blockIdx.x, gridDim.x);
    const unsigned ntx = (unsigned)((L.n[0] + T::TX - 1) / T::TX);
    const int x0 = (int)(tb % ntx) * T::TX, y0 = (int)(tb / ntx) * T::TY;  // interior coordinates
    const int w = min(T::TX, L.n[0] - x0), h = ND == 1 ? 1 : min(T::TY, L.n[1] - y0);
    const int lx = tid % T::TX, ly = tid / T::TX;
    const bool active = lx < w && ly < h;
    const long z = (long)(y0 + ly) * L.n[0] + x0 + lx;
    // P^E of the tile and its halo, every read issued before the first LDS
    // write; cells past the ghosted grid (ragged tiles) are not needed.  A
    // thread takes whole cells (all NV variables at one address plus a
    // stride), so each load costs an add, not a division chain.  The zone's
    // P_n (needed only by the solve) is read after them: loads complete in
    // order, so the face phase waits for P^E alone and P_n arrives behind it
    double pn[NV];
    {
        const int gi0 = x0 + L.g[0] - 2, gj0 = y0 + L.g[1] - T::HY;
        constexpr int cells = T::PY * T::PX, rounds = (cells + kBlock - 1) / kBlock;
        double b[rounds][NV];
#pragma unroll
        for (int r = 0; r < rounds; ++r) {
            // a cell outside the tile or the grid reads cell 0 instead and is
            // multiplied by zero: no load sits in a branch, whose end would
            // have to wait for it
            const int cq = tid + r * kBlock;
            const int gi = gi0 + cq % T::PX, gj = gj0 + cq / T::PX;
            const bool in = cq < cells && gi < L.N[0] && gj < L.N[1];
            const double keep = in ? 1.0 : 0.0;
            const double* src = a.s.PE + (in ? L.cell(gi, gj, 0) : 0L);
#pragma unroll
            for (int v = 0; v < NV; ++v) b[r][v] = src[(long)v * C] * keep;
        }
        {
            // a lane without a zone (ragged tile) reads cell 0 and never uses it
            const long m = active ? L.cell(x0 + lx + L.g[0], y0 + ly + L.g[1], 0) : 0L;
#pragma unroll
            for (int v = 0; v < NV; ++v) pn[v] = a.s.Pn[(long)v * C + m];
        }
#pragma unroll
        for (int r = 0; r < rounds; ++r) {
            const int cq = tid + r * kBlock;
            if (r < rounds - 1 || cq < cells) {
#pragma unroll
                for (int v = 0; v < NV; ++v) pe[v * cells + cq] = b[r][v];
            }
        }
    }
    __syncthreads();

    // the tile's face fluxes.  First every thread computes x-face t and
    // y-face t together: two independent chains per lane in one basic block,
    // both stored unconditionally after both are computed (a conditional
    // store would let the compiler sink each chain into its own branch).  In
    // a ragged tile a face past the tile's zones reads defined LDS (zeros
    // past the grid) and lands in a slot that no zone reads.  The remaining
    // faces (100 of 612 in 2-D) are then computed by lane pairs, so every
    // wave's third round is half a face's chain instead of two waves doing
    // a whole face while the other two wait at the barrier.
    constexpr int nxf = T::XX * T::XY, nyf = T::YX * T::YY;
    static_assert(nxf >= T::kThreads && (ND == 1 || nyf >= T::kThreads), "every thread has a first face");
    const Phys& ph = a.s.ph;
    const GeoMink g{};
    auto xface = [&](int q, double* f) {
        const int cx = q % T::XX, cy = q / T::XX - T::XR;
        const double* p = pe + (cy + T::HY) * T::PX + cx + 2;
        llf_face<NV, GeoMink, 1>(ph, g, [&](int v, int o) { return p[v * T::PY * T::PX + o]; }, f);
    };
    auto xstore = [&](int q, const double* f) {
        const int cx = q % T::XX, cy = q / T::XX - T::XR;
#pragma unroll
        for (int v = 0; v < NV; ++v) fx[(v * T::XY + cy + T::XR) * T::XX + cx] = f[v];
    };
    auto yface = [&](int q, double* f) {
        const int ex = q % T::YX - 1, ey = q / T::YX;
        const double* p = pe + (ey + T::HY) * T::PX + ex + 2;
        llf_face<NV, GeoMink, 2>(ph, g, [&](int v, int o) { return p[v * T::PY * T::PX + o * T::PX]; }, f);
    };
    auto ystore = [&](int q, const double* f) {
        const int ex = q % T::YX - 1, ey = q / T::YX;
#pragma unroll
        for (int v = 0; v < NV; ++v) fy[(v * T::YY + ey) * T::YX + ex + 1] = f[v];
    };
    if constexpr (ND >= 2) {
        if constexpr (kBlock == T::kThreads) {
            double f0[NV], f1[NV];
            xface(tid, f0);
            yface(tid, f1);
            xstore(tid, f0);
            ystore(tid, f1);
        } else {
            // waves 0-3 the x-faces, waves 4-7 the y-faces (wave-uniform)
            double f0[NV];
            if (tid < T::kThreads) {
                xface(tid, f0);
                xstore(tid, f0);
            } else {
                yface(tid - T::kThreads, f0);
                ystore(tid - T::kThreads, f0);
            }
        }
        // the remaining faces, each by a pair of lanes (half a face's chain
        // per lane): waves 0-1 take the x-faces and waves 2-3 the y-faces, a
        // wave-uniform choice; lanes past the last face repeat it and do
        // not store
        static_assert(2 * (nxf - T::kThreads) <= T::kThreads / 2 && 2 * (nyf - T::kThreads) <= T::kThreads / 2,
                      "pair split");
        const int e = tid & (T::kThreads / 2 - 1);
        const bool right = (e & 1) != 0;
        double f2[NV];
        if (tid < T::kThreads / 2) {
            const int q = T::kThreads + min(e >> 1, nxf - T::kThreads - 1);
            const int cx = q % T::XX, cy = q / T::XX - T::XR;
            const double* p = pe + (cy + T::HY) * T::PX + cx + 2;
            llf_pair<NV, GeoMink, 1>(ph, g, [&](int v, int o) { return p[v * T::PY * T::PX + o]; }, right, f2);
            if (!right && (e >> 1) < nxf - T::kThreads) xstore(q, f2);
        } else if (tid < T::kThreads) {
            const int q = T::kThreads + min(e >> 1, nyf - T::kThreads - 1);
            const int ex = q % T::YX - 1, ey = q / T::YX;
            const double* p = pe + (ey + T::HY) * T::PX + ex + 2;
            llf_pair<NV, GeoMink, 2>(ph, g, [&](int v, int o) { return p[v * T::PY * T::PX + o * T::PX]; }, right, f2);
            if (!right && (e >> 1) < nyf - T::kThreads) ystore(q, f2);
        }
    } else {
        double f0[NV];
        xface(tid, f0);
        xstore(tid, f0);
        if (tid < nxf - T::kThreads) {
            xface(T::kThreads + tid, f0);
            xstore(T::kThreads + tid, f0);
        }
    }
    __syncthreads();

    // one zone per thread; a wave is four rows of 16 zones (2-D)
    LaneStats ls;
    if (active) {
        const SrcTile<NV, ND> in{pe, fx, fy, pn, lx, ly};
        ZoneSolve<NV, GeoMink> s;
        zs_begin<NV, GeoMink, ND, FULL>(a, z, a.guess, nullptr, s, &in);
        while (!zs_step<NV, GeoMink, JT, FULL>(a, s)) {
        }
        bool retried = false;
        if constexpr (!__is_same(JT, double)) {
            // a failed FP32-Jacobian solve is solved again from P_n with the
            // FP64 Jacobian in the same lane (the two-pass kernels do this in
            // a second launch); iterations and residual calls of both count
            if (s.fl & (1 | 4 | 16)) {
                const int it = s.iters, nc = s.ncalls, nb = s.nbt;
                zs_begin<NV, GeoMink, ND, FULL>(a, z, nullptr, nullptr, s, &in);
                while (!zs_step<NV, GeoMink, double, FULL>(a, s)) {
                }
                s.iters += it;
                s.ncalls += nc;
                s.nbt += nb;
                s.fl |= kFlagRetry;
                retried = true;
            }
        }
        zs_finish<NV, GeoMink>(a, s, false, ls);
        ls.nrt = retried;
    }
    if (a.stats && tid < T::kThreads) flush_stats(a, ls);  // waves 4-7 solve no zone
}

template <int NV, int ND, bool FULL>
hipError_t stage_tiled(const NewtonArgs& a, int jac_f32, hipStream_t st)
{
    using T = Tile<ND>;
    const long tiles = (long)((a.s.L.n[0] + T::TX - 1) / T::TX) * ((a.s.L.n[1] + T::TY - 1) / T::TY);
    NewtonArgs b = a;
    b.pass = 0;
    // 512-thread blocks (face phase at two waves per SIMD) while every tile
    // fits the device at once; past that, 256-thread blocks two to a CU
    constexpr int kWide = ND == 2 ? 2 * T::kThreads : T::kThreads;
    const bool wide = ND == 2 && (a.block == 512 || (a.block == 0 && a.cus > 0 && tiles <= a.cus));
    const dim3 grid((unsigned)tiles);
    if (jac_f32) {
        if (wide) hipLaunchKernelGGL((k_stage<NV, ND, float, kWide, FULL>), grid, dim3(kWide), 0, st, b);
        else hipLaunchKernelGGL((k_stage<NV, ND, float, T::kThreads, FULL>), grid, dim3(T::kThreads), 0, st, b);
    } else {
        if (wide) hipLaunchKernelGGL((k_stage<NV, ND, double, kWide, FULL>), grid, dim3(kWide), 0, st, b);
        else hipLaunchKernelGGL((k_stage<NV, ND, double, T::kThreads, FULL>), grid, dim3(T::kThreads), 0, st, b);
    }
    return hipGetLastError();
}

template <int NV, class G, int ND, bool FULL, bool X>
hipError_t newton_nd(const NewtonArgs& a, int jac_f32, hipStream_t st)
{
    const long waves = ND == 0 && a.s.L.ndim == 3 ? brick_count(a.s.L) : (a.s.L.nz + kWave - 1) / kWave;
    const dim3 grid((unsigned)waves), blk(kWave);
    NewtonArgs b = a;
    if (jac_f32) {
        // FP32 pass, then the FP64 retry of the zones it marks (needs flags)
        if (!a.flags) return hipErrorInvalidValue;
        b.pass = 1;
        hipLaunchKernelGGL((k_newton<NV, G, float, ND, FULL, X>), grid, blk, 0, st, b);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        b.pass = 2;
        hipLaunchKernelGGL((k_newton<NV, G, double, ND, FULL, X>), grid, blk, 0, st, b);
    } else {
        b.pass = 0;
        hipLaunchKernelGGL((k_newton<NV, G, double, ND, FULL, X>), grid, blk, 0, st, b);
    }
    return hipGetLastError();
}

// The fused form exists for Minkowski only: with the Kerr tables (16 metric
// and 64 connection values per zone) the fused kernel needs more registers
// than the Newton solve alone and spills (measured on the 192x192x96 torus:
// 4.74 ms per step in the fused Newton kernel against 1.61 + 1.72 ms for
// the rhs and Newton kernels).
template <int NV, class G, bool FULL, bool X>
hipError_t newton_t(const NewtonArgs& a, int jac_f32, hipStream_t st)
{
    if constexpr (G::kFlat) {
        if constexpr (!X) {
            if (a.fused && a.tiled && !a.mlp_y && a.s.L.ndim <= 2)
                return a.s.L.ndim == 1 ? stage_tiled<NV, 1, FULL>(a, jac_f32, st)
                                       : stage_tiled<NV, 2, FULL>(a, jac_f32, st);
        }
        if (a.fused) {
            switch (a.s.L.ndim) {
                case 1: return newton_nd<NV, G, 1, FULL, X>(a, jac_f32, st);
                case 2: return newton_nd<NV, G, 2, FULL, X>(a, jac_f32, st);
                default: return newton_nd<NV, G, 3, FULL, X>(a, jac_f32, st);
            }
        }
    }
    return newton_nd<NV, G, 0, FULL, X>(a, jac_f32, st);
}

// The full system runs the plain method; a configuration with options runs
// the paper's reduced system (the host rejects both at once).
template <int NV, class G>
hipError_t newton_sys(const NewtonArgs& a, int jac_f32, hipStream_t st)
{
    if (uses_options(a.s.ph)) {
        if (a.full) return hipErrorInvalidValue;
        return newton_t<NV, G, false, true>(a, jac_f32, st);
    }
    return a.full ? newton_t<NV, G, true, false>(a, jac_f32, st) : newton_t<NV, G, false, false>(a, jac_f32, st);
}

}  // namespace

hipError_t launch_newton(const NewtonArgs& a, int nvar, int metric, int jac_f32, hipStream_t st)
{
    if (nvar == 8) return metric == 0 ? newton_sys<8, GeoMink>(a, jac_f32, st) : newton_sys<8, GeoKS>(a, jac_f32, st);
    return metric == 0 ? newton_sys<10, GeoMink>(a, jac_f32, st) : newton_sys<10, GeoKS>(a, jac_f32, st);
}

}  // namespace grim
