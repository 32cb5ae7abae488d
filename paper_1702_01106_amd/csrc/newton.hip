// The per-zone Newton-Raphson solve of grim (Sec. 3) for gfx950: one zone per
// lane, everything in registers.
//
//   R(P) FP64 always (a8).  Jacobian by forward differences with the
//   perturbation rule of Sec. 3.1 (a9): column j = (R(P_eps,j) - R(P))/h_j,
//   h_j = P_eps,j - P_j.  Dense LU with partial pivoting (a10): row swaps are
//   branch-free selects so J never leaves registers.  Quadratic backtracking
//   line search (a11, Sec. 3.2), each new lambda kept in [0.1, 0.5] of the
//   previous one.  Converged lanes go idle; the wave leaves
//   the loop when every lane has (a12).  Statistics are reduced across the
//   wave with shuffles and accumulated with one atomic per wave (a13).
//
// JT selects the precision of the difference quotients, the stored Jacobian
// and the LU: double (the plain method) or float (mixed precision; the
// residual, conserved variables, metric and Lorentz factor stay FP64).  In
// mixed precision a zone whose FP32 solve fails (in badly scaled zones the
// FP32 Newton direction can be too inaccurate to converge) is marked, and a
// second launch of the FP64 kernel solves only the marked zones from P_n.
#include <hip/hip_runtime.h>

#include "grim_internal.h"
#include "grim_zone.h"

namespace grim {

namespace {

constexpr int kWave = 64;

// Solve A x = b in place (x returned in b) by Gaussian elimination with
// partial pivoting.  Returns false on an exactly zero pivot.
template <int N, typename T>
__device__ __forceinline__ bool lu_solve(T (&A)[N][N], T (&b)[N])
{
    bool ok = true;
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
        // swap rows k and p with selects (J stays in registers)
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
        const T inv = T(1) / A[k][k];
#pragma unroll
        for (int i = k + 1; i < N; ++i) {
            const T f = A[i][k] * inv;
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
        b[i] = s / A[i][i];
    }
    return ok;
}

__device__ __forceinline__ double wave_sum(double x)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    return x;
}

__device__ __forceinline__ int wave_max(int x)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o, kWave));
    return x;
}

__device__ __forceinline__ unsigned long long wave_maxu64(unsigned long long x)
{
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(x, o, kWave);
        x = y > x ? y : x;
    }
    return x;
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
// column, then LU with partial pivoting.  Returns false on an exactly zero
// pivot.
template <int NV, class G, typename JT>
__device__ __forceinline__ bool newton_dir(const double* P, const double* R, const ZoneC<NV, G>& zc,
                                           const Phys& ph, double eps, double* dP)
{
    constexpr int N = Sys<NV>::N;
#pragma unroll
    for (int v = 0; v < NV; ++v) dP[v] = 0.0;
    JT J[N][N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        double Pe[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) Pe[q] = P[q];
        const double pj = P[unk(j)];
        const bool small = fabs(pj) < 5.0 * eps;
        double pe = small ? eps : (1.0 + eps) * pj;
        double h = pe - pj;
        if (h == 0.0) {
            pe = pj + eps;
            h = pe - pj;
        }
        Pe[unk(j)] = pe;
        double Re[NV];
        zone_residual<NV, G>(Pe, zc, ph, Re);
        const double ih = 1.0 / h;
#pragma unroll
        for (int i = 0; i < N; ++i) J[i][j] = (JT)((Re[unk(i)] - R[unk(i)]) * ih);
    }
    JT x[N];
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = (JT)(-R[unk(i)]);
    if (!lu_solve<N, JT>(J, x)) return false;
#pragma unroll
    for (int i = 0; i < N; ++i) dP[unk(i)] = (double)x[i];
    return true;
}

// Ghosted coordinates along one direction that take their value from
// interior index p (p itself first): the inverses of the ghost maps
// (periodic wrap, outflow clamp, polar mirror, Ng = 2).  Returns the count;
// mirror[m] marks a polar image.
__device__ __forceinline__ int ghost_images(int p, int g, int n, int bc, int* q, bool* mirror)
{
    int c = 0;
    q[c] = p;
    mirror[c++] = false;
    if (bc == 0) {
        if (p >= n) { q[c] = p - n; mirror[c++] = false; }          // lower ghost p - n in [0, g)
        if (p < 2 * g) { q[c] = p + n; mirror[c++] = false; }       // upper ghost in [g + n, 2g + n)
    } else if (bc == 1) {
        if (p == g)
            for (int m = 0; m < g; ++m) { q[c] = m; mirror[c++] = false; }
        if (p == g + n - 1)
            for (int m = 0; m < g; ++m) { q[c] = g + n + m; mirror[c++] = false; }
    } else {
        if (p < 2 * g) { q[c] = 2 * g - 1 - p; mirror[c++] = true; }
        if (p >= n) { q[c] = 2 * (g + n) - 1 - p; mirror[c++] = true; }
    }
    return c;
}

// Store a zone's primitives at its cell and at every ghost cell that maps to
// it (the composite map is the product of the per-direction maps; a polar
// image in X2 negates utilde^2 and B^2).
template <int NV>
__device__ __forceinline__ void store_with_ghosts(const Layout& L, const int* bc, long z, const double* P, double* out)
{
    const int p[3] = {(int)(z % L.n[0]) + L.g[0], (int)((z / L.n[0]) % L.n[1]) + L.g[1],
                      (int)(z / ((long)L.n[0] * L.n[1])) + L.g[2]};
    int q[3][5];
    bool mir[3][5];
    int cnt[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (d < L.ndim) {
            cnt[d] = ghost_images(p[d], L.g[d], L.n[d], bc[d], q[d], mir[d]);
        } else {
            cnt[d] = 1;
            q[d][0] = p[d];
            mir[d][0] = false;
        }
    }
    for (int c2 = 0; c2 < cnt[2]; ++c2)
        for (int c1 = 0; c1 < cnt[1]; ++c1)
            for (int c0 = 0; c0 < cnt[0]; ++c0) {
                const long cell = L.cell(q[0][c0], q[1][c1], q[2][c2]);
                const bool flip = mir[1][c1];
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    out[(long)v * L.cells + cell] = (flip && (v == U2 || v == B2)) ? -P[v] : P[v];
            }
}

template <int NV, class G, typename JT>
__global__ __launch_bounds__(kWave) void k_newton(NewtonArgs a)
{
    constexpr int N = Sys<NV>::N;
    const long z = (long)blockIdx.x * kWave + threadIdx.x;
    const Layout& L = a.s.L;
    const bool retry = a.pass == 2;
    bool active = z < L.nz;
    if (retry) {
        active = active && (a.flags[z] & kFlagRetry);
        if (__ballot(active) == 0ull) return;  // wave-uniform exit
    }
    const double* guess = retry ? nullptr : a.guess;
    const float* mlp_y = retry ? nullptr : a.mlp_y;
    int iters = 0, ncalls = 0, fallback = 0;
    uint8_t fl = 0;
    double rr = 0.0;

    if (active) {
        const long cell = zone_cell(L, z);
        ZoneC<NV, G> zc;
        load_zone<NV, G>(a.s, z, cell, zc);
        const Phys& ph = a.s.ph;
        double P_alt[NV];

        // initial guess: P_n (or the caller's guess) with B at its explicit
        // update, the exact root of the B rows
        const double fB = a.s.dtp / zc.g.gdet();
        double P[NV];
        double nscale;
        {
            double pn[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) pn[v] = a.s.Pn[(long)v * L.cells + cell];
            St<NV> sn;
            derive<NV>(pn, zc.g, ph, sn);
            // scaled norm: ||R|| = dt' sqrt(sum R^2) / U_rho(P_n)
            nscale = a.s.dtp / (zc.g.gdet() * pn[RHO] * sn.ucon[0]);
#pragma unroll
            for (int v = 0; v < NV; ++v) P[v] = guess ? guess[(long)v * L.nz + z] : pn[v];
            if (mlp_y) {
                // learned candidate: P = P_n + scaled network output
                const float* y = mlp_y + z * kMlpOut;
                Pc_from_net<NV>(pn, y, P_alt);
            }
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) P[B1 + i] = zc.rhs[B1 + i] * fB;

        double R[NV];
        zone_residual<NV, G>(P, zc, ph, R);
        ++ncalls;
        double r = nscale * sqrt(sumsq<NV>(R));
        bool from_net = false;
        if (mlp_y) {
            // keep the learned guess only if its residual is smaller
#pragma unroll
            for (int i = 0; i < 3; ++i) P_alt[B1 + i] = zc.rhs[B1 + i] * fB;
            double Rc[NV];
            zone_residual<NV, G>(P_alt, zc, ph, Rc);
            ++ncalls;
            const double rc = nscale * sqrt(sumsq<NV>(Rc));
            if (rc < r) {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    P[v] = P_alt[v];
                    R[v] = Rc[v];
                }
                r = rc;
                from_net = true;
            } else {
                fallback = 1;
            }
        }
        const double eps = a.eps;
        for (int attempt = 0; attempt < 2; ++attempt) {
            fl = 0;
            int k = 0;
            for (;;) {
                if (!isfinite(r)) { fl |= 16; break; }
                if (r < a.tol) break;
                if (k >= a.k_max) { fl |= 1; break; }
                double dP[NV];
                const bool ok = newton_dir<NV, G, JT>(P, R, zc, ph, eps, dP);
                ncalls += N;
                if (!ok) { fl |= 4; break; }

                // quadratic backtracking line search
                const double f0 = r * r;
                double lam = 1.0;
                bool accepted = false, have = false;
                double Pf[NV], Rf[NV], rf = 0.0;
                for (int tr = 0; tr < a.ls_max; ++tr) {
                    double Pt[NV], Rt[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) Pt[v] = fma(lam, dP[v], P[v]);
                    zone_residual<NV, G>(Pt, zc, ph, Rt);
                    ++ncalls;
                    const double rt = nscale * sqrt(sumsq<NV>(Rt));
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
                        // minimiser of the quadratic model f(0) - 2 f(0) lam + c lam^2,
                        // kept within [0.1, 0.5] of the previous lambda
                        const double ln = f0 * lam * lam / (rt * rt + (2.0 * lam - 1.0) * f0);
                        lam = fmin(fmax(ln, 0.1 * lam), 0.5 * lam);
                    } else {
                        lam *= 0.5;
                    }
                }
                if (!accepted) {
                    fl |= 2;
                    if (!have) {
                        fl |= 16;
                        ++iters;
                        ++k;
                        break;
                    }
                }
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    P[v] = Pf[v];
                    R[v] = Rf[v];
                }
                r = rf;
                ++iters;
                ++k;
            }
            if (!(from_net && (fl & (1 | 4 | 16)))) break;
            // the solve from the learned guess failed: start again from P_n
            from_net = false;
            fallback = 1;
#pragma unroll
            for (int v = 0; v < NV; ++v) P[v] = a.s.Pn[(long)v * L.cells + cell];
#pragma unroll
            for (int i = 0; i < 3; ++i) P[B1 + i] = zc.rhs[B1 + i] * fB;
            zone_residual<NV, G>(P, zc, ph, R);
            ++ncalls;
            r = nscale * sqrt(sumsq<NV>(R));
        }
        rr = r;
        if (!(P[RHO] > 0.0) || !(P[UU] > 0.0)) fl |= 8;
        if ((a.pass == 1 && (fl & (1 | 4 | 16))) || retry) fl |= kFlagRetry;
        if (a.s.floors) {
            const int ii = (int)(z % L.n[0]);
            const double r1 = exp(L.xs[0] + (ii + 0.5) * L.dx[0]);
            const double rf = a.s.rho_fl * pow(r1, -1.5), uf = a.s.u_fl * pow(r1, -2.5);
            if (!(P[RHO] >= rf)) P[RHO] = rf;
            if (!(P[UU] >= uf)) P[UU] = uf;
        }
        {
            if (a.out_ghosted && a.write_ghosts) {
                store_with_ghosts<NV>(L, a.bc, z, P, a.out);
            } else if (a.out_ghosted) {
#pragma unroll
                for (int v = 0; v < NV; ++v) a.out[(long)v * L.cells + cell] = P[v];
            } else {
#pragma unroll
                for (int v = 0; v < NV; ++v) a.out[(long)v * L.nz + z] = P[v];
            }
            if (a.iters) a.iters[z] = (retry ? a.iters[z] : 0) + iters;
            if (a.resid) a.resid[z] = rr;
            if (a.flags) a.flags[z] = fl;
        }
    }

    // wave-level statistics, one atomic per wave.  A zone marked for the
    // FP64 retry contributes only its work (iterations, residual calls) to the
    // FP32 pass; the retry pass reports its outcome.
    if (a.stats) {
        const bool mine = active;
        const bool final_ = mine && !(a.pass == 1 && (fl & kFlagRetry));
        const double sit = wave_sum(mine ? (double)iters : 0.0);
        const int mit = wave_max(mine ? iters : 0);
        const double nf = wave_sum(final_ && (fl & (1 | 4 | 16)) ? 1.0 : 0.0);
        const double nl = wave_sum(final_ && (fl & 2) ? 1.0 : 0.0);
        const double nu = wave_sum(final_ && (fl & 8) ? 1.0 : 0.0);
        const double na = wave_sum(mine && !retry ? 1.0 : 0.0);
        const double nc = wave_sum(mine ? (double)ncalls : 0.0);
        const double nfb = wave_sum(mine ? (double)fallback : 0.0);
        const double nrt = wave_sum(mine && retry ? 1.0 : 0.0);
        unsigned long long rb = 0;
        if (final_) rb = isfinite(rr) ? (unsigned long long)__double_as_longlong(rr) : 0x7FF0000000000000ull;
        rb = wave_maxu64(rb);
        if (threadIdx.x == 0) {
            atomicAdd(&a.stats->iters[a.stage], (unsigned long long)sit);
            atomicMax(&a.stats->max_iters, (unsigned)mit);
            if (nf > 0) atomicAdd(&a.stats->n_fail, (unsigned long long)nf);
            if (nl > 0) atomicAdd(&a.stats->n_ls, (unsigned long long)nl);
            if (nu > 0) atomicAdd(&a.stats->n_unphys, (unsigned long long)nu);
            if (na > 0) atomicAdd(&a.stats->zone_stages, (unsigned long long)na);
            if (nrt > 0) atomicAdd(&a.stats->n_retry, (unsigned long long)nrt);
            atomicAdd(&a.stats->resid_calls, (unsigned long long)nc);
            if (nfb > 0) atomicAdd(&a.stats->n_fallback, (unsigned long long)nfb);
            atomicMax(&a.stats->max_resid_bits, rb);
        }
    }
}

template <int NV, class G>
hipError_t newton_t(const NewtonArgs& a, int jac_f32, hipStream_t st)
{
    const dim3 grid((unsigned)((a.s.L.nz + kWave - 1) / kWave)), blk(kWave);
    if (jac_f32) {
        // FP32 pass, then the FP64 retry of the zones it marks (needs flags)
        if (!a.flags) return hipErrorInvalidValue;
        NewtonArgs b = a;
        b.pass = 1;
        hipLaunchKernelGGL((k_newton<NV, G, float>), grid, blk, 0, st, b);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        b.pass = 2;
        hipLaunchKernelGGL((k_newton<NV, G, double>), grid, blk, 0, st, b);
    } else {
        NewtonArgs b = a;
        b.pass = 0;
        hipLaunchKernelGGL((k_newton<NV, G, double>), grid, blk, 0, st, b);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_newton(const NewtonArgs& a, int nvar, int metric, int jac_f32, hipStream_t st)
{
    if (nvar == 8) return metric == 0 ? newton_t<8, GeoMink>(a, jac_f32, st) : newton_t<8, GeoKS>(a, jac_f32, st);
    return metric == 0 ? newton_t<10, GeoMink>(a, jac_f32, st) : newton_t<10, GeoKS>(a, jac_f32, st);
}

}  // namespace grim
