// Internal declarations of libgrim: grid layout, kernel argument blocks and
// the host-side launchers implemented in kernels.hip and newton.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "grim.h"
#include "grim_device.h"

namespace grim {

// Ghosted structure-of-arrays grid: cell (i, j, k) of variable v sits at
// v * cells + (k * N2 + j) * N1 + i, with interior cells i in [g1, g1 + n1).
struct Layout {
    int ndim;
    int n[3];  // interior extents (1 for inactive directions)
    int g[3];  // ghost offsets (0 for inactive directions)
    int N[3];  // ghosted extents
    long cells;
    long nz;   // interior zones
    double xs[3], dx[3];
    __host__ __device__ long cell(int i, int j, int k) const { return ((long)k * N[1] + j) * N[0] + i; }
    __host__ __device__ long stride(int d) const { return d == 0 ? 1L : (d == 1 ? (long)N[0] : (long)N[0] * N[1]); }
};

// Interior zone index z -> interior coordinates (i, j, k).  The host limits
// a grid to 2e9 zones, so 32-bit unsigned division is exact (a 64-bit one
// is several times longer).
__device__ __forceinline__ void zone_ijk(const Layout& L, long z, int& i, int& j, int& k)
{
    const unsigned u = (unsigned)z, n0 = (unsigned)L.n[0], n1 = (unsigned)L.n[1];
    const unsigned r = u / n0;
    const unsigned kk = r / n1;
    i = (int)(u - r * n0);
    j = (int)(r - kk * n1);
    k = (int)kk;
}

// Workgroups are dispatched round-robin over the eight XCDs (workgroup b runs
// on XCD b mod 8), and each XCD has its own L2.  xcd_block renumbers them so
// that every XCD takes one contiguous eighth of the logical blocks: zones
// whose stencils overlap then meet in the same L2 instead of being fetched
// by several XCDs.  A bijection on [0, nb) for any nb.
constexpr unsigned kXcds = 8;
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nb)
{
    const unsigned per = nb / kXcds, rem = nb % kXcds;  // XCDs x < rem take per + 1
    const unsigned x = b % kXcds, i = b / kXcds;
    return x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}

// Column order of the zones of a 3-D grid (the Kerr metric tables depend on
// (i, j) only): logical wave w covers 64 consecutive i of row j in plane k,
// with k fastest, so successive waves read the same table points.  Total
// waves: ceil(n1 / 64) * n2 * n3.  Returns false for lanes past the row's end
// and for waves past the last.
__device__ __forceinline__ bool column_zone(const Layout& L, unsigned w, unsigned lane, long& z)
{
    const unsigned nic = ((unsigned)L.n[0] + 63u) / 64u, nk = (unsigned)L.n[2];
    const unsigned k = w % nk, r = w / nk, ic = r % nic, j = r / nic;
    const unsigned i = ic * 64u + lane;
    z = ((long)k * L.n[1] + j) * L.n[0] + i;
    return i < (unsigned)L.n[0] && j < (unsigned)L.n[1];
}
inline long column_waves(const Layout& L) { return (long)((L.n[0] + 63) / 64) * L.n[1] * L.n[2]; }

// Block order of the Kerr flux kernel, which reads 2-D (i, j) face metric
// tables shared by every plane k: block b covers the points
// [chunk * width, chunk * width + width) of plane k, with k = b % planes and
// chunk = b / planes, so consecutive blocks take the same points in
// successive planes and the blocks in flight share the tables of a few rows,
// instead of every plane fetching the whole plane's tables again.
__host__ __device__ inline unsigned plane_blocks(long points, unsigned planes, unsigned width)
{
    return (unsigned)((points + width - 1) / width) * planes;
}

// Device-side accumulators of the solver statistics.  kStatCopies copies,
// one 128-byte line each: a wave adds into copy (block index mod copies), so
// no address sees more than 1/kStatCopies of the waves' atomics (atomics to
// one address serialise in its L2 channel, which cost more than the Newton
// iterations themselves at 4,096 waves).  The host sums the copies.
constexpr int kStatCopies = 256;
struct alignas(128) DevStats {
    unsigned long long iters[2];
    unsigned long long n_fail, n_ls, n_unphys, zone_stages, resid_calls, n_fallback, n_retry, n_bt;
    unsigned long long max_resid_bits;
    unsigned int max_iters;
    unsigned int pad;
};

// Sum (max for the maxima) of the statistics copies, on the host.
inline DevStats sum_stats(const DevStats* s, int n)
{
    DevStats d{};
    for (int i = 0; i < n; ++i) {
        d.iters[0] += s[i].iters[0];
        d.iters[1] += s[i].iters[1];
        d.n_fail += s[i].n_fail;
        d.n_ls += s[i].n_ls;
        d.n_unphys += s[i].n_unphys;
        d.zone_stages += s[i].zone_stages;
        d.resid_calls += s[i].resid_calls;
        d.n_fallback += s[i].n_fallback;
        d.n_retry += s[i].n_retry;
        d.n_bt += s[i].n_bt;
        d.max_resid_bits = s[i].max_resid_bits > d.max_resid_bits ? s[i].max_resid_bits : d.max_resid_bits;
        d.max_iters = s[i].max_iters > d.max_iters ? s[i].max_iters : d.max_iters;
    }
    return d;
}

// Metric tables (Kerr-Schild only).  Centre and face tables depend on
// (i, j) only: the metric is independent of X3.  Layout [kGeoDoubles][N2*N1];
// the face table of direction d holds the metric at the low face of the
// cell in direction d.  conn: Gamma^l_{m n} at centres, [64][N2*N1].
struct GeoTables {
    const double* centre;
    const double* face[3];
    const double* conn;
    size_t stride;  // N1 * N2
};

// Learned-guess network: 32 -> 128 -> 128 -> 16 (FP32 master parameters).
constexpr int kMlpIn = 32, kMlpHidden = 128, kMlpOut = 16;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpIn * kMlpHidden;
constexpr int kOffW2 = kOffB1 + kMlpHidden;
constexpr int kOffB2 = kOffW2 + kMlpHidden * kMlpHidden;
constexpr int kOffW3 = kOffB2 + kMlpHidden;
constexpr int kOffB3 = kOffW3 + kMlpHidden * kMlpOut;
constexpr int kOffXm = kOffB3 + kMlpOut;   // input mean      (fixed during training)
constexpr int kOffXs = kOffXm + kMlpIn;    // input 1/std     (fixed)
constexpr int kOffYs = kOffXs + kMlpIn;    // output scale    (fixed)
constexpr int kMlpParams = kOffYs + kMlpOut;
constexpr int kMlpTrainable = kOffXm;

// FP32 training work buffers for batches of up to `cap` rows.
struct MlpWork {
    float *xh, *tb, *z1, *h1, *z2, *h2, *o, *d_o, *dh, *dh1;
    int cap;
};

// Per-zone EMHD coefficients frozen at P^E (count and order shared by the
// rhs and Newton kernels).
constexpr int kEmhdCoef = 13;  // bh[4], thn, u0n, cbun, aq1, aq2, aq3, ad2, ad3, chalf

struct StageArgs {
    Layout L;
    Phys ph;
    GeoTables geo;
    const double* Pn;   // ghosted P_n
    const double* PE;   // ghosted P^E (ghosts filled)
    double* F[3];       // face fluxes per active direction, ghosted layout
    double* rhs;        // [nvar][nz]
    double* coef;       // [kEmhdCoef][nz] (EMHD)
    double dtp;
    int floors;
    int full;           // Newton over all nvar primitives (else the non-magnetic ones)
    double rho_fl, u_fl;
    // optional outputs of the explicit stage (test hook), [nvar][nz] / [nz][3]
    double* dbg_divF;
    double* dbg_src;
    double* dbg_sp;
    float* mlp_x;       // if set: learned-guess input features, [nz][kMlpIn]
};

struct NewtonArgs {
    StageArgs s;
    const double* guess;   // interior layout or null (then P_n)
    double* out;           // output primitives
    int out_ghosted;       // 1: out is a ghosted array, 0: interior layout
    int32_t* iters;
    double* resid;
    uint8_t* flags;
    DevStats* stats;
    int stage;             // 0 or 1 (statistics slot)
    const float* mlp_y;    // if set: network output per zone [nz][kMlpOut] -> candidate guess
    double tol, eps, eps_bt;
    int k_max, ls_max;
    int ls_safeguard;      // 1: each new lambda kept in [0.1, 0.5] of the previous
    int full;              // 1: the 8x8 / 10x10 system (B among the unknowns)
    int32_t* backtracks;   // if set: rejected line-search trials per zone
    // 0: one solve; 1: FP32 pass that marks failed zones kFlagRetry instead
    // of counting them; 2: FP64 solve from P_n of the marked zones only
    int pass;
    // with out_ghosted: also write every ghost cell whose boundary map
    // (bc per direction: 0 periodic, 1 outflow, 2 polar) takes its value from
    // this zone, so the output needs no separate ghost fill
    int write_ghosts;
    int bc[3];
    // 1: compute each zone's stage right-hand side in the Newton kernel from
    // the face fluxes (fused), instead of reading what the rhs kernel stored
    // (Minkowski only; ignored for Kerr)
    int fused;
    // with fused, 1- and 2-D and no network: one kernel per stage that
    // computes a tile's face fluxes into LDS, then solves its zones (the flux
    // kernel is not launched; FP32-Jacobian failures are retried in FP64 in
    // the same lane)
    int tiled;
    // compute units of the device (0 if unknown): a 2-D tiled stage whose
    // tiles all fit at once runs 512-thread blocks (see k_stage)
    int cus;
    // 0: block size of the 2-D tiled stage chosen from cus; 256 or 512: forced
    int block;
};
constexpr uint8_t kFlagRetry = 32;

// Host helpers of the C ABI (abi.hip): configuration check (non-zero and a
// reason if invalid), grid layout, physical constants, and the message that
// grim_last_global_error returns on this thread.
int check_config(const grim_config_t* cfg, std::string& why);
Layout grid_layout(const grim_config_t* cfg);
Phys physics(const grim_config_t* cfg);
void set_global_error(const std::string& msg);

// launchers (return hipSuccess or the launch error)
hipError_t launch_fill_ghosts(const Layout& L, int nvar, const int bc[3], double* P, hipStream_t st);
hipError_t launch_explicit_stage(const StageArgs& a, int nvar, int metric, hipStream_t st);
hipError_t launch_fluxes(const StageArgs& a, int nvar, int metric, hipStream_t st);
hipError_t launch_rhs(const StageArgs& a, int nvar, int metric, hipStream_t st);
hipError_t launch_newton(const NewtonArgs& a, int nvar, int metric, int jac_f32, hipStream_t st);
hipError_t launch_residual(const StageArgs& a, int nvar, int metric, const double* P, double* R, double* rnorm,
                           hipStream_t st);
hipError_t launch_cfl(const Layout& L, const Phys& ph, const GeoTables& geo, int nvar, int metric, const double* P,
                      unsigned long long* out_bits, hipStream_t st);
hipError_t launch_zero_stats(DevStats* s, hipStream_t st);
hipError_t launch_stream_add(const double* a, const double* b, double* c, size_t n, hipStream_t st);
hipError_t launch_math_probe(const double* x, double* out, size_t n, hipStream_t st);
hipError_t launch_copy_interior(const Layout& L, int nvar, const double* src, int src_ghosted, double* dst,
                                int dst_ghosted, hipStream_t st);
hipError_t launch_collect(const StageArgs& a, int nvar, const double* Pout, int out_ghosted, int stride, int phase,
                          float* Xo, float* To, long base, long cap, hipStream_t st);
hipError_t mlp_pack(const float* params, unsigned short* w1t, unsigned short* w2t, unsigned short* w3t,
                    hipStream_t st);
hipError_t mlp_infer(const float* X, long n, const float* params, const unsigned short* w1t,
                     const unsigned short* w2t, const unsigned short* w3t, float* Y, hipStream_t st);
hipError_t mlp_batch_grad(const MlpWork& w, const float* X, const float* T, const float* dY, const int* idx,
                          long off, int nbatch, int n_used, float inv_count, const float* p, float* grad, int acc,
                          double* loss, hipStream_t st);
hipError_t mlp_fill(float* p, long n, float v, hipStream_t st);
hipError_t mlp_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                    int step, hipStream_t st);
// Means and unbiased variances of the 32 input and 16 target columns of n
// training pairs, into work[nblocks * 48 ..] (means) and the 48 doubles after
// them (variances); work holds (nblocks + 2) * 48 doubles.
hipError_t mlp_norm_stats(const float* X, const float* T, long n, double* work, int nblocks, hipStream_t st);
hipError_t build_geometry(const Layout& L, double spin, double h, double* centre, double* face[3], double* conn,
                          hipStream_t st);

}  // namespace grim
