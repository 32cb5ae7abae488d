// Explicit-stage kernels of libgrim for gfx950: ghost fill (a2), PLM + LLF
// face fluxes (a3, a4), flux-CT edge EMFs (a5), the stage right-hand side
// with explicit sources and the EMHD coefficient bundle (a6), the CFL time
// step, the residual test hook, and small utility kernels.
#include <hip/hip_runtime.h>

#include "grim_internal.h"
#include "grim_rhs.h"
#include "grim_zone.h"

namespace grim {

namespace {

constexpr int kBlock = 256;

inline unsigned nblocks(long n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

// ------------------------------------------------------------------ ghosts

// Every ghost cell takes its value from one interior cell: the per-direction
// maps (periodic wrap, outflow clamp, polar mirror) are independent, so the
// composite map equals filling X1, X2, X3 ghosts in turn.  Polar mirroring
// negates utilde^2 and B^2.
__global__ __launch_bounds__(kBlock) void k_fill_ghosts(Layout L, int nvar, int bc0, int bc1, int bc2, double* P)
{
    const long c = (long)blockIdx.x * kBlock + threadIdx.x;
    if (c >= L.cells) return;
    int idx[3];
    idx[0] = (int)(c % L.N[0]);
    idx[1] = (int)((c / L.N[0]) % L.N[1]);
    idx[2] = (int)(c / ((long)L.N[0] * L.N[1]));
    const int bc[3] = {bc0, bc1, bc2};
    int src[3];
    bool ghost = false, flip = false;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int p = idx[d], g = L.g[d], n = L.n[d];
        if (d >= L.ndim || (p >= g && p < g + n)) {
            src[d] = p;
            continue;
        }
        ghost = true;
        if (bc[d] == 0) {
            src[d] = p < g ? p + n : p - n;
        } else if (bc[d] == 1) {
            src[d] = p < g ? g : g + n - 1;
        } else {
            src[d] = p < g ? 2 * g - 1 - p : 2 * (g + n) - 1 - p;
            if (d == 1) flip = !flip;
        }
    }
    if (!ghost) return;
    const long s = L.cell(src[0], src[1], src[2]);
    for (int v = 0; v < nvar; ++v) {
        const double x = P[(long)v * L.cells + s];
        P[(long)v * L.cells + c] = (flip && (v == U2 || v == B2)) ? -x : x;
    }
}

// ------------------------------------------------------------------ fluxes

// The face on the low side of cell (i, j, k) in direction DIR (llf_face),
// read from and stored to the stage buffers.
template <int NV, class G, int DIR, bool X>
__device__ __forceinline__ void face_flux(const StageArgs& a, int i, int j, int k)
{
    const Layout& L = a.L;
    const long m = L.cell(i, j, k);
    const long st = L.stride(DIR - 1);
    G g;
    if constexpr (!G::kFlat) load_geo(g, a.geo.face[DIR - 1], (size_t)((long)j * L.N[0] + i), a.geo.stride);
    double f[NV];
    llf_face<NV, G, DIR, X>(a.ph, g, [&](int v, int o) { return a.PE[(long)v * L.cells + m + o * st]; }, f);
    double* F = a.F[DIR - 1];
#pragma unroll
    for (int v = 0; v < NV; ++v) F[(long)v * L.cells + m] = f[v];
}

// Face ranges of every active direction in one launch: blocks
// [first[d], first[d + 1]) take the faces normal to direction d, so each
// block (and wave) works on one direction.
struct FaceRanges {
    int lo[3][3];
    unsigned cnt[3][3];
    unsigned first[4];
};

template <int NV, class G, bool X>
__global__ __launch_bounds__(kBlock) void k_fluxes(StageArgs a, FaceRanges r)
{
    plain_options<X>(a.ph);
    // Minkowski: each XCD takes a contiguous eighth of the faces.  Kerr:
    // plane-interleaved order (plane_blocks), so the blocks in flight share
    // the 2-D face metric tables of a few rows (2.8x faster than the plain
    // order on the 128x128x64 and 192x192x96 tori).  Ideal MHD also takes
    // the XCD renumbering, which gives each XCD whole columns of planes
    // (6% faster on the 128x128x64 torus; the EMHD faces ran 7% slower)
    const unsigned b = (G::kFlat || NV == 8) ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
    const int d = b < r.first[1] ? 0 : (b < r.first[2] ? 1 : 2);
    const unsigned* cnt = r.cnt[d];
    const int* lo = r.lo[d];
    int i, j, k;
    if constexpr (G::kFlat) {
        // face counts per direction stay below 2^32 (the host limits zones to 2e9)
        const unsigned t = (b - r.first[d]) * kBlock + threadIdx.x;
        if (t >= cnt[0] * cnt[1] * cnt[2]) return;
        const unsigned q = t / cnt[0], kk = q / cnt[1];
        i = lo[0] + (int)(t - q * cnt[0]);
        j = lo[1] + (int)(q - kk * cnt[1]);
        k = lo[2] + (int)kk;
    } else {
        const unsigned bb = b - r.first[d], kk = bb % cnt[2];
        const unsigned t = (bb / cnt[2]) * kBlock + threadIdx.x;
        if (t >= cnt[0] * cnt[1]) return;
        const unsigned q = t / cnt[0];
        i = lo[0] + (int)(t - q * cnt[0]);
        j = lo[1] + (int)q;
        k = lo[2] + (int)kk;
    }
    if (d == 0) face_flux<NV, G, 1, X>(a, i, j, k);
    else if (d == 1) face_flux<NV, G, 2, X>(a, i, j, k);
    else face_flux<NV, G, 3, X>(a, i, j, k);
}

// The faces of a 3-D Kerr grid by cells: a thread takes the low x-, y- and
// z-faces of one cell of the box one cell wider each side than the
// interior, as flux-CT needs.  The x- and y-faces are computed for every
// cell of the box (those at the box's low i and j edge are faces no kernel
// reads; their stencils stay inside the array), so both are one basic block;
// a block is one plane, and the z-face waits for the planes above the first.
// EMHD on the 192x192x96 torus: 1.22 -> 1.14 ms a step against k_fluxes.
template <int NV, class G, bool X>
__global__ __launch_bounds__(kBlock) void k_fluxes_cell(StageArgs a)
{
    plain_options<X>(a.ph);
    const Layout& L = a.L;
    const unsigned c0 = L.n[0] + 2, c1 = L.n[1] + 2, c2 = L.n[2] + 2;
    const unsigned b = blockIdx.x, kk = b % c2;
    const unsigned t = (b / c2) * kBlock + threadIdx.x;
    if (t >= c0 * c1) return;
    const unsigned q = t / c0;
    const int i = L.g[0] - 1 + (int)(t - q * c0), j = L.g[1] - 1 + (int)q, k = L.g[2] - 1 + (int)kk;
    face_flux<NV, G, 1, X>(a, i, j, k);
    face_flux<NV, G, 2, X>(a, i, j, k);
    if (k >= L.g[2]) face_flux<NV, G, 3, X>(a, i, j, k);
}

// One thread per interior zone: the stage right-hand side (zone_rhs), stored
// for the Newton kernel.
template <int NV, class G, int ND, bool X>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 3))) void k_rhs(StageArgs a)
{
    plain_options<X>(a.ph);
    // Kerr 3-D: column order (column_zone), the block's four waves in four
    // successive planes of one row segment, so they share its metric and
    // connection table points (5% faster on both tori than the plain order;
    // adding the XCD renumbering made it slower again)
    long z;
    if constexpr (!G::kFlat && ND == 3) {
        if (!column_zone(a.L, blockIdx.x * (kBlock / 64) + threadIdx.x / 64, threadIdx.x % 64, z)) return;
    } else {
        z = (long)blockIdx.x * kBlock + threadIdx.x;
    }
    if (z >= a.L.nz) return;
    double rhs[NV], co[kEmhdCoef];
    G g;
    zone_rhs<NV, G, ND, true>(a, z, rhs, co, g, SrcGlobal{a});
    const long nz = a.L.nz;
#pragma unroll
    for (int v = 0; v < NV; ++v) a.rhs[(long)v * nz + z] = rhs[v];
    if constexpr (NV == 10) {
#pragma unroll
        for (int q = 0; q < kEmhdCoef; ++q) a.coef[(long)q * nz + z] = co[q];
    }
}

// EMHD on the 3-D Kerr grid: the stage right-hand side by columns.  A block
// takes a tile of kMarchTI x kMarchTJ columns (i, j) (one wave a row) and
// marches up a chunk of planes k.  The slopes of the EMHD sources need the
// slope point X (emhd_point) of the zone's six neighbours: the block shares
// X of each plane through LDS, the waves at the tile's edges computing X of
// the halo cells (wave 0 row j0-1, wave 3 row j0+4, waves 1 and 2 the columns
// i0-1 and i0+64), and each lane keeps X of its own column one plane below
// and above in registers, with the column's metric.  Every cell's X is then
// derived once a plane (plus one halo cell a wave) instead of six times, and
// the neighbours' P^E and metrics are never read.  The column's connection
// (40 distinct Gamma^l_{m n}, the table being symmetric in m, n) is read once
// a chunk into the lane's own slots of LDS.  Same arithmetic as k_rhs up to
// the compiler's contraction of products into fused multiply-adds.
constexpr int kMarchTI = 64, kMarchTJ = 4;

// Slot of Gamma^l_{m n} (q = 16 l + 4 m + n) among the 40 with m <= n.
__device__ __forceinline__ constexpr int conn_slot(int q)
{
    const int l = q / 16, a = (q / 4) % 4, b = q % 4;
    const int m = a < b ? a : b, n = a < b ? b : a;
    return l * 10 + m * (7 - m) / 2 + n;
}
static_assert(kBlock == kMarchTI * kMarchTJ, "one wave per tile row");

struct SrcMarch {
    static constexpr bool kNbrX = true;
    SrcGlobal gl;
    const GeoKS& g0;      // metric of the zone's column
    const double* pe;     // P^E of the zone
    const double* xm;     // X one plane below and above
    const double* xp;
    const double (*xl)[kMarchTJ + 2][kMarchTI + 2];  // X of the plane [q][row][col]
    const double (*cs)[kBlock];                      // connection slots [40][thread]
    int r, c;             // the zone's row and column in xl
    __device__ __forceinline__ double F(int d, int v, long m, int o1, int o2, int o3) const
    {
        return gl.F(d, v, m, o1, o2, o3);
    }
    __device__ __forceinline__ double PE(int v, long m, int o1, int o2, int o3) const
    {
        return (o1 | o2 | o3) == 0 ? pe[v] : gl.PE(v, m, o1, o2, o3);
    }
    __device__ __forceinline__ double Pn(int v, long m) const { return gl.Pn(v, m); }
    template <class G>
    __device__ __forceinline__ void centre(G& g, size_t) const { g = g0; }
    __device__ __forceinline__ double conn(int q, size_t) const { return cs[conn_slot(q)][threadIdx.x]; }
    __device__ __forceinline__ void nbr_x(int d, double* Xm, double* Xp) const
    {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            Xm[q] = d == 0 ? xl[q][r][c - 1] : (d == 1 ? xl[q][r - 1][c] : xm[q]);
            Xp[q] = d == 0 ? xl[q][r][c + 1] : (d == 1 ? xl[q][r + 1][c] : xp[q]);
        }
    }
};

template <bool X>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(1, 3))) void k_rhs_march(StageArgs a, int kc)
{
    constexpr int NV = 10;
    plain_options<X>(a.ph);
    __shared__ double xs[2][8][kMarchTJ + 2][kMarchTI + 2];
    __shared__ double gs[40][kBlock];
    const Layout& L = a.L;
    const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
    const int nti = (L.n[0] + kMarchTI - 1) / kMarchTI, ntj = (L.n[1] + kMarchTJ - 1) / kMarchTJ;
    const int t = blockIdx.x % (nti * ntj), ch = blockIdx.x / (nti * ntj);
    const int i0 = (t % nti) * kMarchTI, j0 = (t / nti) * kMarchTJ;
    const int k0 = ch * kc, k1 = min(k0 + kc, L.n[2]);
    const int i = i0 + lane, j = j0 + w;  // interior indices of the lane's column
    const bool act = i < L.n[0] && j < L.n[1];
    // the column's cell and this lane's halo cell (ghost-inclusive), clamped
    // into the grid where a tile overhangs it; no active zone reads those
    const int ci = min(i + L.g[0], L.N[0] - 1), cj = min(j + L.g[1], L.N[1] - 1);
    int hi, hj, hr, hc;
    bool hon = true;
    if (w == 0 || w == kMarchTJ - 1) {
        hi = i;
        hj = w == 0 ? j0 - 1 : j0 + kMarchTJ;
        hr = w == 0 ? 0 : kMarchTJ + 1;
        hc = lane + 1;
    } else {
        hi = w == 1 ? i0 - 1 : i0 + kMarchTI;
        hj = j0 + lane;
        hr = lane + 1;
        hc = w == 1 ? 0 : kMarchTI + 1;
        hon = lane < kMarchTJ;
    }
    const int hci = min(max(hi + L.g[0], 0), L.N[0] - 1), hcj = min(max(hj + L.g[1], 0), L.N[1] - 1);
    GeoKS g0, gh;
    load_geo(g0, a.geo.centre, (size_t)((long)cj * L.N[0] + ci), a.geo.stride);
    load_geo(gh, a.geo.centre, (size_t)((long)hcj * L.N[0] + hci), a.geo.stride);
#pragma unroll
    for (int l = 0; l < 4; ++l)
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = m; n < 4; ++n) {
                const int q = l * 16 + m * 4 + n;
                gs[conn_slot(q)][threadIdx.x] = a.geo.conn[(size_t)q * a.geo.stride + (size_t)((long)cj * L.N[0] + ci)];
            }
    const long C = L.cells;
    double pe[NV], xm[8], xc[8];
    {
        double p0[NV];
        load_cell<NV>(a.PE, C, L.cell(ci, cj, k0 + L.g[2] - 1), p0);
        emhd_point<NV>(p0, g0, a.ph, xm);
    }
    load_cell<NV>(a.PE, C, L.cell(ci, cj, k0 + L.g[2]), pe);
    emhd_point<NV>(pe, g0, a.ph, xc);
    const long nz = L.nz;
    int buf = 0;
    for (int kk = k0; kk < k1; ++kk) {
        const int ck = kk + L.g[2];
        double pu[NV], xp[8];
        load_cell<NV>(a.PE, C, L.cell(ci, cj, ck + 1), pu);
        emhd_point<NV>(pu, g0, a.ph, xp);
        if (hon) {
            double ph[NV], xh[8];
            load_cell<NV>(a.PE, C, L.cell(hci, hcj, ck), ph);
            emhd_point<NV>(ph, gh, a.ph, xh);
#pragma unroll
            for (int q = 0; q < 8; ++q) xs[buf][q][hr][hc] = xh[q];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) xs[buf][q][w + 1][lane + 1] = xc[q];
        __syncthreads();
        if (act) {
            const long z = ((long)kk * L.n[1] + j) * L.n[0] + i;
            double rhs[NV], co[kEmhdCoef];
            GeoKS g;
            zone_rhs<NV, GeoKS, 3, true>(a, z, rhs, co, g,
                                         SrcMarch{SrcGlobal{a}, g0, pe, xm, xp, xs[buf], gs, w + 1, lane + 1});
#pragma unroll
            for (int v = 0; v < NV; ++v) a.rhs[(long)v * nz + z] = rhs[v];
#pragma unroll
            for (int q = 0; q < kEmhdCoef; ++q) a.coef[(long)q * nz + z] = co[q];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            xm[q] = xc[q];
            xc[q] = xp[q];
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) pe[v] = pu[v];
        buf ^= 1;
    }
}

// Planes per block of k_rhs_march.
constexpr int kMarchPlanes = 8;

// Ideal MHD on the 3-D Kerr grid: the stage right-hand side by columns, a
// lane per (i, j) column marching up a chunk of planes with the column's
// metric in registers and its 40 distinct connection entries in the lane's
// own LDS slots (read once a chunk instead of once a zone).
struct SrcColumn {
    static constexpr bool kNbrX = false;
    SrcGlobal gl;
    const GeoKS& g0;
    const double (*cs)[kBlock];
    __device__ __forceinline__ double F(int d, int v, long m, int o1, int o2, int o3) const
    {
        return gl.F(d, v, m, o1, o2, o3);
    }
    __device__ __forceinline__ double PE(int v, long m, int o1, int o2, int o3) const { return gl.PE(v, m, o1, o2, o3); }
    __device__ __forceinline__ double Pn(int v, long m) const { return gl.Pn(v, m); }
    template <class G>
    __device__ __forceinline__ void centre(G& g, size_t) const { g = g0; }
    __device__ __forceinline__ double conn(int q, size_t) const { return cs[conn_slot(q)][threadIdx.x]; }
};

template <bool X>
__global__ __launch_bounds__(kBlock) void k_rhs_column(StageArgs a, int kc)
{
    constexpr int NV = 8;
    plain_options<X>(a.ph);
    __shared__ double gs[40][kBlock];
    const Layout& L = a.L;
    const unsigned ncol = (unsigned)L.n[0] * (unsigned)L.n[1];
    const unsigned nb = (ncol + kBlock - 1) / kBlock;
    const unsigned b = blockIdx.x % nb, ch = blockIdx.x / nb;
    const unsigned c = b * kBlock + threadIdx.x;
    if (c >= ncol) return;  // no barrier below
    const int j = (int)(c / (unsigned)L.n[0]), i = (int)(c - (unsigned)j * (unsigned)L.n[0]);
    const size_t p = (size_t)((long)(j + L.g[1]) * L.N[0] + i + L.g[0]);
    GeoKS g0;
    load_geo(g0, a.geo.centre, p, a.geo.stride);
#pragma unroll
    for (int l = 0; l < 4; ++l)
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int n = m; n < 4; ++n) {
                const int q = l * 16 + m * 4 + n;
                gs[conn_slot(q)][threadIdx.x] = a.geo.conn[(size_t)q * a.geo.stride + p];
            }
    const int k0 = (int)ch * kc, k1 = min(k0 + kc, L.n[2]);
    const long nz = L.nz;
    for (int kk = k0; kk < k1; ++kk) {
        const long z = ((long)kk * L.n[1] + j) * L.n[0] + i;
        double rhs[NV], co[kEmhdCoef];
        GeoKS g;
        zone_rhs<NV, GeoKS, 3, true>(a, z, rhs, co, g, SrcColumn{SrcGlobal{a}, g0, gs});
#pragma unroll
        for (int v = 0; v < NV; ++v) a.rhs[(long)v * nz + z] = rhs[v];
    }
}

// ------------------------------------------------------------------ math hook

__global__ __launch_bounds__(kBlock) void k_math_probe(const double* x, double* out, size_t n)
{
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double v = x[i];
    out[3 * i] = rcp_nr(v);
    out[3 * i + 1] = rsq_nr(v);
    out[3 * i + 2] = sqrt_nr(v);
}

// ------------------------------------------------------------------ residual hook

template <int NV, class G, bool X>
__global__ __launch_bounds__(kBlock) void k_residual(StageArgs a, const double* P, double* R, double* rnorm)
{
    plain_options<X>(a.ph);
    const long z = (long)blockIdx.x * kBlock + threadIdx.x;
    if (z >= a.L.nz) return;
    const long cell = zone_cell(a.L, z);
    ZoneC<NV, G> zc;
    load_zone<NV, G>(a, z, cell, zc);
    double p[NV], r[NV], pn[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        p[v] = P[(long)v * a.L.nz + z];
        pn[v] = a.Pn[(long)v * a.L.cells + cell];
    }
    zone_residual<NV, G>(p, zc, a.ph, r);
#pragma unroll
    for (int v = 0; v < NV; ++v) R[(long)v * a.L.nz + z] = r[v];
    if (rnorm) {
        St<NV> sn;
        derive<NV>(pn, zc.g, a.ph, sn);
        const double urho = zc.g.gdet() * pn[RHO] * sn.ucon[0];
        rnorm[z] = a.dtp * sqrt(a.full ? sumsq<NV, true>(r) : sumsq<NV, false>(r)) / urho;
    }
}

// ------------------------------------------------------------------ CFL

template <int NV, class G, bool X>
__global__ __launch_bounds__(kBlock) void k_cfl(Layout L, Phys ph, GeoTables geo, const double* P,
                                                unsigned long long* out)
{
    plain_options<X>(ph);
    __shared__ double red[kBlock];
    const long z = (long)blockIdx.x * kBlock + threadIdx.x;
    double t = 1e300;
    if (z < L.nz) {
        const long cell = zone_cell(L, z);
        double p[NV];
        load_cell<NV>(P, L.cells, cell, p);
        G g;
        if constexpr (!G::kFlat) load_geo(g, geo.centre, (size_t)(cell % ((long)L.N[0] * L.N[1])), geo.stride);
        St<NV> s;
        derive<NV>(p, g, ph, s);
        double acc = cmax<NV, 1>(p, g, s, ph) / L.dx[0];
        if (L.ndim >= 2) acc += cmax<NV, 2>(p, g, s, ph) / L.dx[1];
        if (L.ndim >= 3) acc += cmax<NV, 3>(p, g, s, ph) / L.dx[2];
        t = 1.0 / acc;
    }
    red[threadIdx.x] = t;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + o]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMin(out, (unsigned long long)__double_as_longlong(red[0]));
}

// ------------------------------------------------------------------ utilities

// clears every field of every copy: block b takes copy b, as 8-byte words,
// one lane per word
__global__ void k_zero_stats(DevStats* s)
{
    static_assert(sizeof(DevStats) % 8 == 0 && sizeof(DevStats) / 8 <= 64, "DevStats layout");
    unsigned long long* w = reinterpret_cast<unsigned long long*>(s + blockIdx.x);
    if (threadIdx.x < sizeof(DevStats) / 8) w[threadIdx.x] = 0ull;
}

__global__ __launch_bounds__(kBlock) void k_stream_add(const double* __restrict__ a, const double* __restrict__ b,
                                                       double* __restrict__ c, size_t n)
{
    size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * kBlock;
    for (; i < n; i += stride) c[i] = a[i] + b[i];
}

// Training pairs: for zones z = phase (mod stride), copy the features and
// write the target (P - P_n) scaled as the guess expects:
// rho, u relative; utilde absolute; q, DP relative to u_n.
template <int NV>
__global__ __launch_bounds__(kBlock) void k_collect(Layout L, const double* Pn, const double* Pout, int og,
                                                    const float* X, int stride, int phase, float* Xo, float* To,
                                                    long base, long cap)
{
    const long j = (long)blockIdx.x * kBlock + threadIdx.x;
    const long z = j * stride + phase;
    if (z >= L.nz) return;
    const long idx = base + j;
    if (idx >= cap) return;
    const long cell = zone_cell(L, z);
    double pn[NV], p[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        pn[v] = Pn[(long)v * L.cells + cell];
        p[v] = og ? Pout[(long)v * L.cells + cell] : Pout[(long)v * L.nz + z];
    }
    for (int q = 0; q < kMlpIn; ++q) Xo[idx * kMlpIn + q] = X[z * kMlpIn + q];
    float t[kMlpOut];
#pragma unroll
    for (int q = 0; q < kMlpOut; ++q) t[q] = 0.0f;
    t[0] = (float)((p[RHO] - pn[RHO]) / pn[RHO]);
    t[1] = (float)((p[UU] - pn[UU]) / pn[UU]);
#pragma unroll
    for (int i = 0; i < 3; ++i) t[2 + i] = (float)(p[U1 + i] - pn[U1 + i]);
    if constexpr (NV == 10) {
        t[5] = (float)((p[QQ] - pn[QQ]) / pn[UU]);
        t[6] = (float)((p[DP] - pn[DP]) / pn[UU]);
    }
#pragma unroll
    for (int q = 0; q < kMlpOut; ++q) To[idx * kMlpOut + q] = t[q];
}

__global__ __launch_bounds__(kBlock) void k_copy_interior(Layout L, int nvar, const double* src, int sg, double* dst,
                                                          int dg)
{
    const long z = (long)blockIdx.x * kBlock + threadIdx.x;
    if (z >= L.nz) return;
    const long cell = zone_cell(L, z);
    for (int v = 0; v < nvar; ++v) {
        const double x = src[(long)v * (sg ? L.cells : L.nz) + (sg ? cell : z)];
        dst[(long)v * (dg ? L.cells : L.nz) + (dg ? cell : z)] = x;
    }
}

template <int NV, class G>
hipError_t fluxes_t(const StageArgs& a, hipStream_t st)
{
    const Layout& L = a.L;
    const int nd = L.ndim;
    // face ranges: along d the n_d + 1 faces of interior cells; across the
    // other active directions one extra row each side (flux-CT needs them)
    // (a lane pair per face, as the tiled stage computes its last faces, ran
    // 33% slower than a lane per face on the 192x192x96 and 128x128x64 tori)
    const int per = kBlock;
    FaceRanges r{};
    unsigned blocks = 0;
    for (int d = 0; d < 3; ++d) {
        r.first[d] = blocks;
        if (d >= nd) continue;
        for (int e = 0; e < 3; ++e) {
            if (e == d) { r.lo[d][e] = L.g[e]; r.cnt[d][e] = L.n[e] + 1; }
            else if (e < nd) { r.lo[d][e] = L.g[e] - 1; r.cnt[d][e] = L.n[e] + 2; }
            else { r.lo[d][e] = 0; r.cnt[d][e] = 1; }
        }
        blocks += G::kFlat ? nblocks((long)r.cnt[d][0] * r.cnt[d][1] * r.cnt[d][2], per)
                           : plane_blocks((long)r.cnt[d][0] * r.cnt[d][1], r.cnt[d][2], per);
    }
    r.first[3] = blocks;
    for (int d = nd; d < 3; ++d) r.first[d] = blocks;
    if constexpr (!G::kFlat && NV == 10) {
        // (ideal MHD: 5% slower than the plane-interleaved faces with the XCD
        // renumbering on the 128x128x64 torus)
        if (nd == 3 && !uses_options(a.ph)) {
            const unsigned cb = plane_blocks((long)(L.n[0] + 2) * (L.n[1] + 2), L.n[2] + 2, kBlock);
            hipLaunchKernelGGL((k_fluxes_cell<NV, G, false>), dim3(cb), dim3(kBlock), 0, st, a);
            return hipGetLastError();
        }
    }
    if (uses_options(a.ph)) hipLaunchKernelGGL((k_fluxes<NV, G, true>), dim3(blocks), dim3(kBlock), 0, st, a, r);
    else hipLaunchKernelGGL((k_fluxes<NV, G, false>), dim3(blocks), dim3(kBlock), 0, st, a, r);
    return hipGetLastError();
}

template <int NV, class G, bool X>
hipError_t rhs_x(const StageArgs& a, hipStream_t st)
{
    if constexpr (NV == 8 && !G::kFlat && !X) {
        if (a.L.ndim == 3) {
            const long nb = ((long)a.L.n[0] * a.L.n[1] + kBlock - 1) / kBlock;
            const int nc = (a.L.n[2] + kMarchPlanes - 1) / kMarchPlanes;
            hipLaunchKernelGGL((k_rhs_column<X>), dim3((unsigned)(nb * nc)), dim3(kBlock), 0, st, a, kMarchPlanes);
            return hipGetLastError();
        }
    }
    if constexpr (NV == 10 && !G::kFlat && !X) {
        if (a.L.ndim == 3) {
            const int nt = ((a.L.n[0] + kMarchTI - 1) / kMarchTI) * ((a.L.n[1] + kMarchTJ - 1) / kMarchTJ);
            const int nc = (a.L.n[2] + kMarchPlanes - 1) / kMarchPlanes;
            hipLaunchKernelGGL((k_rhs_march<X>), dim3(nt * nc), dim3(kBlock), 0, st, a, kMarchPlanes);
            return hipGetLastError();
        }
    }
    const bool col = !G::kFlat && a.L.ndim == 3;
    const dim3 grid(col ? nblocks(column_waves(a.L), kBlock / 64) : nblocks(a.L.nz)), blk(kBlock);
    if (a.L.ndim == 1) hipLaunchKernelGGL((k_rhs<NV, G, 1, X>), grid, blk, 0, st, a);
    else if (a.L.ndim == 2) hipLaunchKernelGGL((k_rhs<NV, G, 2, X>), grid, blk, 0, st, a);
    else hipLaunchKernelGGL((k_rhs<NV, G, 3, X>), grid, blk, 0, st, a);
    return hipGetLastError();
}

template <int NV, class G>
hipError_t rhs_t(const StageArgs& a, hipStream_t st)
{
    return uses_options(a.ph) ? rhs_x<NV, G, true>(a, st) : rhs_x<NV, G, false>(a, st);
}

template <int NV, class G>
hipError_t explicit_stage_t(const StageArgs& a, hipStream_t st)
{
    hipError_t e = fluxes_t<NV, G>(a, st);
    if (e == hipSuccess) e = rhs_t<NV, G>(a, st);
    return e;
}

}  // namespace

hipError_t launch_fill_ghosts(const Layout& L, int nvar, const int bc[3], double* P, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_ghosts, dim3(nblocks(L.cells)), dim3(kBlock), 0, st, L, nvar, bc[0], bc[1], bc[2], P);
    return hipGetLastError();
}

hipError_t launch_explicit_stage(const StageArgs& a, int nvar, int metric, hipStream_t st)
{
    if (nvar == 8) return metric == 0 ? explicit_stage_t<8, GeoMink>(a, st) : explicit_stage_t<8, GeoKS>(a, st);
    return metric == 0 ? explicit_stage_t<10, GeoMink>(a, st) : explicit_stage_t<10, GeoKS>(a, st);
}

hipError_t launch_fluxes(const StageArgs& a, int nvar, int metric, hipStream_t st)
{
    if (nvar == 8) return metric == 0 ? fluxes_t<8, GeoMink>(a, st) : fluxes_t<8, GeoKS>(a, st);
    return metric == 0 ? fluxes_t<10, GeoMink>(a, st) : fluxes_t<10, GeoKS>(a, st);
}

hipError_t launch_rhs(const StageArgs& a, int nvar, int metric, hipStream_t st)
{
    if (nvar == 8) return metric == 0 ? rhs_t<8, GeoMink>(a, st) : rhs_t<8, GeoKS>(a, st);
    return metric == 0 ? rhs_t<10, GeoMink>(a, st) : rhs_t<10, GeoKS>(a, st);
}

hipError_t launch_residual(const StageArgs& a, int nvar, int metric, const double* P, double* R, double* rnorm,
                           hipStream_t st)
{
    const dim3 grid(nblocks(a.L.nz)), blk(kBlock);
    const bool x = uses_options(a.ph);
    if (nvar == 8) {
        if (metric == 0) hipLaunchKernelGGL((k_residual<8, GeoMink, false>), grid, blk, 0, st, a, P, R, rnorm);
        else hipLaunchKernelGGL((k_residual<8, GeoKS, false>), grid, blk, 0, st, a, P, R, rnorm);
    } else if (!x) {
        if (metric == 0) hipLaunchKernelGGL((k_residual<10, GeoMink, false>), grid, blk, 0, st, a, P, R, rnorm);
        else hipLaunchKernelGGL((k_residual<10, GeoKS, false>), grid, blk, 0, st, a, P, R, rnorm);
    } else {
        if (metric == 0) hipLaunchKernelGGL((k_residual<10, GeoMink, true>), grid, blk, 0, st, a, P, R, rnorm);
        else hipLaunchKernelGGL((k_residual<10, GeoKS, true>), grid, blk, 0, st, a, P, R, rnorm);
    }
    return hipGetLastError();
}

hipError_t launch_cfl(const Layout& L, const Phys& ph, const GeoTables& geo, int nvar, int metric, const double* P,
                      unsigned long long* out_bits, hipStream_t st)
{
    // the time step depends on the closure (through v_max) only
    const dim3 grid(nblocks(L.nz)), blk(kBlock);
    if (nvar == 8) {
        if (metric == 0) hipLaunchKernelGGL((k_cfl<8, GeoMink, false>), grid, blk, 0, st, L, ph, geo, P, out_bits);
        else hipLaunchKernelGGL((k_cfl<8, GeoKS, false>), grid, blk, 0, st, L, ph, geo, P, out_bits);
    } else {
        if (metric == 0) hipLaunchKernelGGL((k_cfl<10, GeoMink, true>), grid, blk, 0, st, L, ph, geo, P, out_bits);
        else hipLaunchKernelGGL((k_cfl<10, GeoKS, true>), grid, blk, 0, st, L, ph, geo, P, out_bits);
    }
    return hipGetLastError();
}

hipError_t launch_zero_stats(DevStats* s, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_stats, dim3(kStatCopies), dim3(64), 0, st, s);
    return hipGetLastError();
}

hipError_t launch_math_probe(const double* x, double* out, size_t n, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_math_probe, dim3((unsigned)((n + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, x, out, n);
    return hipGetLastError();
}

hipError_t launch_stream_add(const double* a, const double* b, double* c, size_t n, hipStream_t st)
{
    const long blocks = (long)std::min<size_t>((n + kBlock - 1) / kBlock, (size_t)256 * 64);
    hipLaunchKernelGGL(k_stream_add, dim3((unsigned)std::max<long>(blocks, 1)), dim3(kBlock), 0, st, a, b, c, n);
    return hipGetLastError();
}

hipError_t launch_collect(const StageArgs& a, int nvar, const double* Pout, int out_ghosted, int stride, int phase,
                          float* Xo, float* To, long base, long cap, hipStream_t st)
{
    const long cnt = phase < a.L.nz ? (a.L.nz - 1 - phase) / stride + 1 : 0;
    if (cnt <= 0) return hipSuccess;
    if (nvar == 8)
        hipLaunchKernelGGL((k_collect<8>), dim3(nblocks(cnt)), dim3(kBlock), 0, st, a.L, a.Pn, Pout, out_ghosted,
                           a.mlp_x, stride, phase, Xo, To, base, cap);
    else
        hipLaunchKernelGGL((k_collect<10>), dim3(nblocks(cnt)), dim3(kBlock), 0, st, a.L, a.Pn, Pout, out_ghosted,
                           a.mlp_x, stride, phase, Xo, To, base, cap);
    return hipGetLastError();
}

hipError_t launch_copy_interior(const Layout& L, int nvar, const double* src, int src_ghosted, double* dst,
                                int dst_ghosted, hipStream_t st)
{
    hipLaunchKernelGGL(k_copy_interior, dim3(nblocks(L.nz)), dim3(kBlock), 0, st, L, nvar, src, src_ghosted, dst,
                       dst_ghosted);
    return hipGetLastError();
}

}  // namespace grim
