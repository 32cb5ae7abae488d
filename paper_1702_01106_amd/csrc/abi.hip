// Host side of libgrim's C ABI (declared in include/grim.h): context
// lifetime, buffer management, the two-stage step and the test hooks.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <new>
#include <type_traits>
#include <mutex>
#include <random>
#include <string>
#include <vector>

#include "grim.h"
#include "grim_internal.h"

using grim::DevStats;
using grim::Layout;
using grim::NewtonArgs;
using grim::Phys;
using grim::StageArgs;

struct grim_ctx {
    grim_config_t cfg{};
    Layout L{};
    Phys ph{};
    int nvar = 0;
    hipStream_t st = nullptr;       // work stream (caller's, or owned)
    bool own_st = false;
    hipStream_t cap = nullptr;      // private stream used only for graph capture
    double* P[2] = {nullptr, nullptr};  // ghosted state buffers (ping-pong)
    double* H = nullptr;                // ghosted half-step state P_{n+1/2}
    int cur = 0;                         // buffer holding the current state
    double* F[3] = {nullptr, nullptr, nullptr};
    double* rhs = nullptr;
    double* coef = nullptr;
    double* interior = nullptr;          // staging buffer, interior layout
    double* hookP[2] = {nullptr, nullptr};
    double* nrm = nullptr;               // partial sums of grim_mlp_normalisation
    int32_t* iters = nullptr;
    double* resid = nullptr;
    uint8_t* flags = nullptr;
    DevStats* stats = nullptr;
    unsigned long long* u64 = nullptr;
    double* geo_centre = nullptr;
    double* geo_face[3] = {nullptr, nullptr, nullptr};
    double* geo_conn = nullptr;
    // learned guess
    float* mlp_p = nullptr;              // FP32 parameters
    unsigned short* mlp_w[3] = {nullptr, nullptr, nullptr};  // transposed BF16 weights
    float* mlp_x = nullptr;              // per-zone inputs [nz][32]
    float* mlp_y = nullptr;              // per-zone outputs [nz][16]
    bool mlp_set = false;
    grim::MlpWork work{};
    float* mlp_grad = nullptr;
    float* adam_m = nullptr;
    float* adam_v = nullptr;
    int* mlp_idx = nullptr;
    long mlp_idx_cap = 0;
    double* dloss = nullptr;
    char* ws = nullptr;                  // the workspace every buffer above is carved from
    bool own_ws = false;                 // allocated by grim_create (else bound by the caller)
    size_t ws_bytes = 0;
    size_t bytes = 0;                    // device bytes held: workspace + training buffers
    // graph[p]: one step from state buffer p; graph[2 + p]: kGraphSteps steps
    // from buffer p (an even count, so the step after it starts from p again)
    hipGraphExec_t graph[4] = {nullptr, nullptr, nullptr, nullptr};
    double graph_dt = 0.0;
    int cus = 0;  // compute units of the device (0 if the query failed)
    float* scratch = nullptr;  // this device's copy of the no-allocation scratch array
    bool timing = false;
    struct Mark {
        int group;
        hipEvent_t a, b;
    };
    std::vector<Mark> marks;
    std::string err;
};

namespace {

thread_local std::string g_last_error;

int fail(grim_ctx* c, int code, const std::string& msg)
{
    if (c) c->err = msg;
    else g_last_error = msg;
    return code;
}

int hip_fail(grim_ctx* c, hipError_t e, const char* what)
{
    return fail(c, GRIM_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

// ---- scratch of the no-allocation gradient call (grim_mlp_backward_noalloc)
//
// The ten per-row work buffers of one gradient pass (network input and
// target, the two hidden layers before and after GELU, the output, its
// gradient and the two hidden gradients: 848 floats a row) for up to
// kNoAllocRows rows, then one double for the loss accumulator the kernels
// take.  A file-scope device array, so the call allocates nothing; each GPU
// holds its own copy (about 6.9 MB) until the process ends.  Host code never
// names the array itself (on the host its name is a stand-in, not a device
// address): grim_create resolves its address on the context's device with
// hipGetSymbolAddress, once per device, and every launch takes that pointer.
constexpr int kNoAllocRows = 2048;
constexpr int kRowFloats = grim::kMlpIn + grim::kMlpOut + 6 * grim::kMlpHidden + 2 * grim::kMlpOut;
static_assert(kRowFloats == 848, "work buffer widths");
constexpr size_t kScratchFloats = (size_t)kNoAllocRows * kRowFloats + 64;
static __device__ __align__(256) float scratch[kScratchFloats];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_dev[kMaxDevices] = {};

// The current device's address of `scratch` (resolved on first use on that
// device); hipSuccess or the error of the lookup.
hipError_t scratch_address(float** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_dev[dev] = static_cast<float*>(p);
    }
    *out = g_scratch_dev[dev];
    return hipSuccess;
}

// A context whose device memory is in place (create allocated it, or a
// workspace was bound).
int usable(grim_ctx* c)
{
    if (!c) return fail(nullptr, GRIM_E_INVALID_ARG, "null context");
    if (!c->ws) return fail(c, GRIM_E_STATE, "no workspace bound (grim_bind_workspace)");
    return GRIM_OK;
}

#define HIP_TRY(c, expr)                                        \
    do {                                                        \
        hipError_t e_ = (expr);                                 \
        if (e_ != hipSuccess) return hip_fail((c), e_, #expr);  \
    } while (0)

template <typename T>
int dalloc(grim_ctx* c, T** p, size_t count)
{
    const size_t b = count * sizeof(T);
    hipError_t e = hipMalloc((void**)p, b);
    if (e != hipSuccess) {
        *p = nullptr;
        return fail(c, e == hipErrorOutOfMemory ? GRIM_E_OOM : GRIM_E_HIP,
                    std::string("hipMalloc(") + std::to_string(b) + " bytes): " + hipGetErrorString(e));
    }
    c->bytes += b;
    return GRIM_OK;
}

void release(grim_ctx* c)
{
    for (auto& m : c->marks) {
        hipEventDestroy(m.a);
        hipEventDestroy(m.b);
    }
    c->marks.clear();
    for (int i = 0; i < 4; ++i)
        if (c->graph[i]) hipGraphExecDestroy(c->graph[i]);
    if (c->cap) hipStreamDestroy(c->cap);
    if (c->own_st && c->st) hipStreamDestroy(c->st);
    // the workspace buffers are carved from c->ws; the training buffers are
    // allocated one by one
    void* ptrs[] = {c->mlp_grad, c->adam_m, c->adam_v, c->mlp_idx, c->dloss, c->work.xh, c->work.tb,
                    c->work.z1, c->work.h1, c->work.z2, c->work.h2, c->work.o, c->work.d_o, c->work.dh,
                    c->work.dh1};
    for (void* p : ptrs)
        if (p) hipFree(p);
    if (c->own_ws && c->ws) hipFree(c->ws);
}

int validate(const grim_config_t* g, std::string& why)
{
    if (g->ndim < 1 || g->ndim > 3) return why = "ndim must be 1, 2 or 3", 1;
    const int n[3] = {g->n1, g->n2, g->n3};
    for (int d = 0; d < 3; ++d) {
        if (d < g->ndim && n[d] < 1) return why = "active direction with no zones", 1;
        if (d >= g->ndim && n[d] != 1) return why = "inactive direction must have n = 1", 1;
    }
    if (g->ng != 2 && g->ng != 3) return why = "ng must be 2 or 3", 1;
    if (g->recon < GRIM_RECON_PLM || g->recon > GRIM_RECON_PPM) return why = "unknown reconstruction", 1;
    if (g->recon != GRIM_RECON_PLM && g->ng < 3)
        return why = "WENO5 and PPM read three cells on each side of a face: ng = 3", 1;
    if (g->riemann != GRIM_RIEMANN_LLF && g->riemann != GRIM_RIEMANN_HLLE) return why = "unknown Riemann solver", 1;
    if (g->full_system != 0 && g->full_system != 1) return why = "full_system must be 0 or 1", 1;
    if (g->closure != 0 && g->closure != 1) return why = "closure must be 0 or 1", 1;
    if (g->dp_saturation != 0 && g->dp_saturation != 1) return why = "dp_saturation must be 0 or 1", 1;
    if (g->dp_saturation && !g->closure) return why = "dp_saturation needs closure = 1", 1;
    if (g->dp_saturation && !(g->sat_width > 0)) return why = "sat_width must be positive", 1;
    if (g->full_system && (g->riemann || g->recon || (g->model == GRIM_EMHD && (g->closure || g->dp_saturation))))
        return why = "the full system runs the plain method (LLF, PLM, constant chi and nu)", 1;
    if (g->model != GRIM_IDEAL_MHD && g->model != GRIM_EMHD) return why = "model must be 8 or 10", 1;
    if (g->metric != GRIM_MINKOWSKI && g->metric != GRIM_MKS_KERR) return why = "unknown metric", 1;
    if (g->metric == GRIM_MKS_KERR && g->ndim < 2) return why = "Kerr needs ndim >= 2", 1;
    for (int d = 0; d < 3; ++d) {
        if (g->bc[d] < 0 || g->bc[d] > 2) return why = "unknown boundary condition", 1;
        if (g->bc[d] == GRIM_BC_POLAR && d != 1) return why = "polar boundary only in X2", 1;
        if (d < g->ndim && !(g->x_end[d] > g->x_start[d])) return why = "empty domain", 1;
        if (d < g->ndim && n[d] < g->ng)
            return why = "active directions need n >= ng (ghost maps read interior)", 1;
    }
    if (!(g->gamma > 1.0)) return why = "gamma must exceed 1", 1;
    if (g->model == GRIM_EMHD && !(g->tau_R > 0)) return why = "EMHD needs tau_R > 0", 1;
    if (g->model == GRIM_EMHD && !g->closure && !(g->chi > 0 && g->nu > 0))
        return why = "EMHD needs chi, nu > 0", 1;
    if (g->model == GRIM_EMHD && g->closure && !(g->phi > 0 && g->psi > 0))
        return why = "the closure needs phi, psi > 0", 1;
    if (!(g->tol > 0) || !(g->eps_fd > 0) || !(g->eps_bt >= 0)) return why = "bad tolerances", 1;
    // the solver statistics pack per-wave sums into 21-bit fields
    if (g->k_max < 0 || g->k_max > 100 || g->ls_max < 1 || g->ls_max > 64)
        return why = "k_max in [0, 100] and ls_max in [1, 64] required", 1;
    if (g->ls_safeguard != 0 && g->ls_safeguard != 1) return why = "ls_safeguard must be 0 or 1", 1;
    if (g->external_workspace != 0 && g->external_workspace != 1)
        return why = "external_workspace must be 0 or 1", 1;
    if (g->stage_block != 0 && g->stage_block != 256 && g->stage_block != 512)
        return why = "stage_block must be 0, 256 or 512", 1;
    if (g->jac_precision != GRIM_JAC_F64 && g->jac_precision != GRIM_JAC_F32) return why = "bad jac_precision", 1;
    if (g->guess != GRIM_GUESS_PN && g->guess != GRIM_GUESS_MLP) return why = "bad guess", 1;

    const double zones = (double)n[0] * n[1] * n[2];
    if (zones > 2.0e9) return why = "too many zones", 1;
    return 0;
}

// Grid layout of a configuration (ghost layers on active directions only).
Layout layout_of(const grim_config_t* cfg)
{
    Layout L{};
    L.ndim = cfg->ndim;
    const int n[3] = {cfg->n1, cfg->n2, cfg->n3};
    for (int d = 0; d < 3; ++d) {
        L.n[d] = n[d];
        L.g[d] = d < cfg->ndim ? cfg->ng : 0;
        L.N[d] = n[d] + 2 * L.g[d];
        L.xs[d] = cfg->x_start[d];
        L.dx[d] = d < cfg->ndim ? (cfg->x_end[d] - cfg->x_start[d]) / n[d] : 1.0;
    }
    L.cells = (long)L.N[0] * L.N[1] * L.N[2];
    L.nz = (long)n[0] * n[1] * n[2];
    return L;
}

// Physical constants of a configuration, with the EMHD rescaling factors
// sqrt(tau_R / chi), sqrt(tau_R / nu) and the squared diffusion speeds.
Phys phys_of(const grim_config_t* cfg)
{
    Phys ph{};
    ph.gam = cfg->gamma;
    ph.gm1 = cfg->gamma - 1.0;
    ph.tau = cfg->tau_R;
    ph.chi = cfg->chi;
    ph.nu = cfg->nu;
    ph.theta = cfg->plm_theta;
    if (cfg->model == GRIM_EMHD && !cfg->closure) {
        ph.kq = std::sqrt(cfg->tau_R / cfg->chi);
        ph.kd = std::sqrt(cfg->tau_R / cfg->nu);
        ph.vq2 = (cfg->gamma - 1.0) * cfg->chi / cfg->tau_R;
        ph.vd2 = 4.0 * cfg->nu / (3.0 * cfg->tau_R);
    }
    ph.closure = cfg->model == GRIM_EMHD ? cfg->closure : 0;
    ph.phi = cfg->phi;
    ph.psi = cfg->psi;
    ph.sat = cfg->model == GRIM_EMHD ? cfg->dp_saturation : 0;
    ph.sat_w = cfg->sat_width;
    ph.riemann = cfg->riemann;
    ph.recon = cfg->recon;
    return ph;
}

constexpr int kNormBlocks = 256;  // partial sums of the normalisation kernel
constexpr int kNormCols = grim::kMlpIn + grim::kMlpOut;

// Lay every device buffer of a context out in one workspace, each on a
// 256-byte boundary, and return its size.  With c and base set, the
// context's pointers are set into base; with c null only the size is
// computed.
size_t carve(const grim_config_t* cfg, grim_ctx* c, char* base)
{
    const Layout L = layout_of(cfg);
    const size_t nv = (size_t)cfg->model, cells = (size_t)L.cells, nz = (size_t)L.nz;
    size_t off = 0;
    auto take = [&](auto** p, size_t count) {
        using T = std::remove_reference_t<decltype(**p)>;
        off = (off + 255) & ~(size_t)255;
        if (c && base) *p = reinterpret_cast<T*>(base + off);
        off += count * sizeof(T);
    };
    grim_ctx dummy;
    grim_ctx* t = c ? c : &dummy;
    take(&t->P[0], nv * cells);
    take(&t->P[1], nv * cells);
    take(&t->H, nv * cells);
    for (int d = 0; d < cfg->ndim; ++d) take(&t->F[d], nv * cells);
    take(&t->rhs, nv * nz);
    if (cfg->model == GRIM_EMHD) take(&t->coef, (size_t)grim::kEmhdCoef * nz);
    take(&t->interior, nv * nz);
    take(&t->hookP[0], nv * cells);
    take(&t->hookP[1], nv * cells);
    take(&t->iters, nz);
    take(&t->resid, nz);
    take(&t->flags, nz);
    take(&t->stats, (size_t)grim::kStatCopies);
    take(&t->u64, 4);
    take(&t->nrm, (size_t)(kNormBlocks + 2) * kNormCols);
    take(&t->mlp_p, (size_t)grim::kMlpParams);
    take(&t->mlp_w[0], (size_t)grim::kMlpHidden * grim::kMlpIn);
    take(&t->mlp_w[1], (size_t)grim::kMlpHidden * grim::kMlpHidden);
    take(&t->mlp_w[2], (size_t)32 * grim::kMlpHidden);
    take(&t->mlp_x, nz * grim::kMlpIn);
    take(&t->mlp_y, nz * grim::kMlpOut);
    if (cfg->metric == GRIM_MKS_KERR) {
        const size_t s2 = (size_t)L.N[0] * L.N[1];
        take(&t->geo_centre, grim::kGeoDoubles * s2);
        for (int d = 0; d < 3; ++d) take(&t->geo_face[d], grim::kGeoDoubles * s2);
        take(&t->geo_conn, 64 * s2);
    }
    return (off + 255) & ~(size_t)255;
}

// Carve the context's buffers from its workspace, clear the state buffers
// and build the metric tables (a1); synchronises.
int init_workspace(grim_ctx* c, char* base, size_t bytes)
{
    c->ws = base;
    c->ws_bytes = bytes;
    c->bytes += bytes;
    carve(&c->cfg, c, base);
    const size_t nv = (size_t)c->nvar, cells = (size_t)c->L.cells;
    double* zero[] = {c->P[0], c->P[1], c->H, c->F[0], c->F[1], c->F[2], c->hookP[0], c->hookP[1]};
    for (double* p : zero)
        if (p) HIP_TRY(c, hipMemsetAsync(p, 0, sizeof(double) * nv * cells, c->st));
    if (c->cfg.metric == GRIM_MKS_KERR)
        HIP_TRY(c, grim::build_geometry(c->L, c->cfg.spin_a, c->cfg.mks_h, c->geo_centre, c->geo_face, c->geo_conn,
                                        c->st));
    HIP_TRY(c, hipStreamSynchronize(c->st));
    return GRIM_OK;
}

// Whether stage solves compute the right-hand side inside the Newton kernel.
bool fused_rhs(const grim_ctx* c) { return c->cfg.metric == GRIM_MINKOWSKI; }

// Whether a fused stage runs as the one tiled kernel (fluxes in LDS): every
// 1- and 2-D grid.  Two tiles fit a CU (79 KiB of LDS and at most 256
// registers each), so past 256 tiles a SIMD holds two waves.  Measured on
// the 2-D EMHD workload: 24 us per stage against 33 us for the flux and
// Newton kernels at 256^2, and 71 against 91 us at 512^2.
bool tiled_stage(const grim_ctx* c)
{
    // the tiled kernel runs the plain method (PLM: its P^E halo is two cells)
    return fused_rhs(c) && c->cfg.ndim <= 2 && !grim::uses_options(c->ph);
}

StageArgs stage_args(grim_ctx* c, const double* Pn, const double* PE, double dtp)
{
    StageArgs a{};
    a.L = c->L;
    a.ph = c->ph;
    a.geo.centre = c->geo_centre;
    for (int d = 0; d < 3; ++d) a.geo.face[d] = c->geo_face[d];
    a.geo.conn = c->geo_conn;
    a.geo.stride = (size_t)c->L.N[0] * c->L.N[1];
    a.Pn = Pn;
    a.PE = PE;
    for (int d = 0; d < 3; ++d) a.F[d] = c->F[d];
    a.rhs = c->rhs;
    a.coef = c->coef;
    a.dtp = dtp;
    a.floors = c->cfg.floors;
    a.full = c->cfg.full_system;
    a.rho_fl = c->cfg.rho_floor;
    a.u_fl = c->cfg.u_floor;
    return a;
}

NewtonArgs newton_args(grim_ctx* c, const StageArgs& s)
{
    NewtonArgs a{};
    a.cus = c->cus;
    a.block = c->cfg.stage_block;
    a.s = s;
    a.tol = c->cfg.tol;
    a.eps = c->cfg.eps_fd;
    a.eps_bt = c->cfg.eps_bt;
    a.k_max = c->cfg.k_max;
    a.ls_max = c->cfg.ls_max;
    a.ls_safeguard = c->cfg.ls_safeguard;
    a.full = c->cfg.full_system;
    a.iters = c->iters;
    a.resid = c->resid;
    a.flags = c->flags;
    a.stats = c->stats;
    for (int d = 0; d < 3; ++d) a.bc[d] = c->cfg.bc[d];
    return a;
}

// Event bracket around a launch group when kernel timing is on.
struct Timed {
    grim_ctx* c;
    int group;
    hipStream_t st;
    hipEvent_t a = nullptr, b = nullptr;
    Timed(grim_ctx* c_, int g, hipStream_t s) : c(c_), group(g), st(s)
    {
        if (c->timing && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
            hipEventRecord(a, st);
    }
    ~Timed()
    {
        if (a && b) {
            hipEventRecord(b, st);
            c->marks.push_back({group, a, b});
        }
    }
};

// Where a stage stores training pairs (grim_collect_pairs).
struct Collect {
    int stride;
    int phase;
    float* X;
    float* T;
    long cap;
    long count;
};

// One stage: flux stage on PE (ghosts of PE must be filled), then Newton
// (from the learned guess when cfg.guess asks for it).
int enqueue_stage(grim_ctx* c, double* Pn, double* PE, double dtp, double* out, int stage, hipStream_t st,
                  Collect* col = nullptr)
{
    StageArgs s = stage_args(c, Pn, PE, dtp);
    const bool net = c->cfg.guess == GRIM_GUESS_MLP && !col;
    if (net || col) s.mlp_x = c->mlp_x;
    // Minkowski without the network's features: the Newton kernel computes
    // each zone's right-hand side itself (no rhs kernel, no rhs round trip)
    const bool fused = fused_rhs(c) && !net && !col;
    const bool tiled = fused && tiled_stage(c);
    if (!tiled) {
        Timed t(c, 1, st);
        HIP_TRY(c, grim::launch_fluxes(s, c->nvar, c->cfg.metric, st));
    }
    if (!fused) {
        Timed t(c, 3, st);
        HIP_TRY(c, grim::launch_rhs(s, c->nvar, c->cfg.metric, st));
    }
    if (net) {
        Timed t(c, 5, st);
        HIP_TRY(c, grim::mlp_infer(c->mlp_x, c->L.nz, c->mlp_p, c->mlp_w[0], c->mlp_w[1], c->mlp_w[2], c->mlp_y, st));
    }
    NewtonArgs n = newton_args(c, s);
    n.out = out;
    n.out_ghosted = 1;
    n.write_ghosts = 1;  // the output's ghosts are written with it
    n.fused = fused ? 1 : 0;
    n.tiled = tiled ? 1 : 0;
    n.stage = stage;
    n.mlp_y = net ? c->mlp_y : nullptr;
    {
        Timed t(c, 4, st);
        HIP_TRY(c, grim::launch_newton(n, c->nvar, c->cfg.metric, c->cfg.jac_precision, st));
    }
    if (col) {
        HIP_TRY(c, grim::launch_collect(s, c->nvar, out, 1, col->stride, col->phase, col->X, col->T, col->count,
                                        col->cap, st));
        const long nz = c->L.nz;
        col->count += col->phase < nz ? (nz - 1 - col->phase) / col->stride + 1 : 0;
        col->phase = (col->phase + 1) % col->stride;
    }
    return GRIM_OK;
}

// One full step from buffer `from` into the other buffer, enqueued on st:
// stage 1 from P_n into H (P_{n+1/2}), stage 2 with P^E = H into the other
// buffer.  No stage writes a buffer it reads: the Newton kernel reads P^E
// when it computes the right-hand side itself, so writing P_{n+1} over
// P_{n+1/2} would race with other waves' reads of their neighbours.  The
// state buffers always hold valid ghosts: grim_set_prims fills them, and each
// stage's Newton kernel writes the ghost images of every zone it solves.
int enqueue_step(grim_ctx* c, int from, double dt, hipStream_t st, Collect* col = nullptr)
{
    double* A = c->P[from];
    double* B = c->P[1 - from];
    int rc = enqueue_stage(c, A, A, 0.5 * dt, c->H, 0, st, col);
    if (rc) return rc;
    return enqueue_stage(c, A, c->H, dt, B, 1, st, col);
}

int ensure_mlp_train_buffers(grim_ctx* c, int cap)
{
    grim::MlpWork& w = c->work;
    if (w.cap < cap) {
        float** bufs[] = {&w.xh, &w.tb, &w.z1, &w.h1, &w.z2, &w.h2, &w.o, &w.d_o, &w.dh, &w.dh1};
        const int widths[] = {grim::kMlpIn, grim::kMlpOut, grim::kMlpHidden, grim::kMlpHidden, grim::kMlpHidden,
                              grim::kMlpHidden, grim::kMlpOut, grim::kMlpOut, grim::kMlpHidden, grim::kMlpHidden};
        for (int i = 0; i < 10; ++i) {
            if (*bufs[i]) {
                hipFree(*bufs[i]);
                *bufs[i] = nullptr;
            }
            int rc = dalloc(c, bufs[i], (size_t)cap * widths[i]);
            if (rc) return rc;
        }
        w.cap = cap;
    }
    int rc = GRIM_OK;
    if (!c->mlp_grad) rc = dalloc(c, &c->mlp_grad, (size_t)grim::kMlpParams);
    if (!rc && !c->adam_m) rc = dalloc(c, &c->adam_m, (size_t)grim::kMlpTrainable);
    if (!rc && !c->adam_v) rc = dalloc(c, &c->adam_v, (size_t)grim::kMlpTrainable);
    if (!rc && !c->dloss) rc = dalloc(c, &c->dloss, 1);
    return rc;
}

// Stage the hook inputs P_n (interior) and P^E (interior) into ghosted
// buffers and run the explicit stage.
int hook_setup(grim_ctx* c, const double* Pn, const double* PE, double dtp, StageArgs* out, double* dbg_divF,
               double* dbg_src, double* dbg_sp)
{
    if (!Pn || !PE) return fail(c, GRIM_E_INVALID_ARG, "null input pointer");
    if (!(dtp > 0.0) || !std::isfinite(dtp)) return fail(c, GRIM_E_INVALID_ARG, "dt' must be positive");
    HIP_TRY(c, grim::launch_copy_interior(c->L, c->nvar, Pn, 0, c->hookP[0], 1, c->st));
    HIP_TRY(c, grim::launch_copy_interior(c->L, c->nvar, PE, 0, c->hookP[1], 1, c->st));
    const int bc[3] = {c->cfg.bc[0], c->cfg.bc[1], c->cfg.bc[2]};
    HIP_TRY(c, grim::launch_fill_ghosts(c->L, c->nvar, bc, c->hookP[1], c->st));
    StageArgs s = stage_args(c, c->hookP[0], c->hookP[1], dtp);
    s.dbg_divF = dbg_divF;
    s.dbg_src = dbg_src;
    s.dbg_sp = dbg_sp;
    HIP_TRY(c, grim::launch_explicit_stage(s, c->nvar, c->cfg.metric, c->st));
    *out = s;
    return GRIM_OK;
}

// Sum the statistics copies on the host into stats; `per_stage` stages of
// every zone were accumulated into each stage slot.  Synchronises.
int read_stats(grim_ctx* c, int per_stage, grim_stats_t* stats)
{
    std::vector<DevStats> copies(grim::kStatCopies);
    HIP_TRY(c, hipMemcpyAsync(copies.data(), c->stats, sizeof(DevStats) * grim::kStatCopies, hipMemcpyDeviceToHost,
                              c->st));
    HIP_TRY(c, hipStreamSynchronize(c->st));
    const DevStats d = grim::sum_stats(copies.data(), grim::kStatCopies);
    const double zs = (double)c->L.nz * (double)per_stage;
    stats->mean_iters[0] = (double)d.iters[0] / zs;
    stats->mean_iters[1] = (double)d.iters[1] / zs;
    stats->max_iters = (int32_t)d.max_iters;
    stats->pad = 0;
    stats->n_fail = (int64_t)d.n_fail;
    stats->n_ls_exhausted = (int64_t)d.n_ls;
    stats->n_unphysical = (int64_t)d.n_unphys;
    double mr;
    std::memcpy(&mr, &d.max_resid_bits, sizeof(mr));
    stats->max_resid = mr;
    stats->zone_stages = (int64_t)d.zone_stages;
    stats->n_resid_calls = (int64_t)d.resid_calls;
    stats->n_fallback = (int64_t)d.n_fallback;
    stats->n_f64_retry = (int64_t)d.n_retry;
    stats->n_backtracks = (int64_t)d.n_bt;
    return GRIM_OK;
}

}  // namespace

extern "C" {

const char* grim_last_global_error(void) { return g_last_error.c_str(); }

const char* grim_last_error(const grim_ctx_t* ctx) { return ctx ? ctx->err.c_str() : g_last_error.c_str(); }

size_t grim_device_bytes(const grim_ctx_t* ctx) { return ctx ? ctx->bytes : 0; }

int grim_create(const grim_config_t* cfg, void* hip_stream, grim_ctx_t** out)
{
    if (!cfg || !out) return fail(nullptr, GRIM_E_INVALID_ARG, "null argument");
    *out = nullptr;
    std::string why;
    if (validate(cfg, why)) return fail(nullptr, GRIM_E_INVALID_ARG, "invalid config: " + why);
    grim_ctx* c = new (std::nothrow) grim_ctx();
    if (!c) return fail(nullptr, GRIM_E_OOM, "host allocation failed");
    c->cfg = *cfg;
    c->st = (hipStream_t)hip_stream;
    {
        // NULL: an owned blocking stream (it orders itself with the legacy
        // default stream, which PyTorch uses by default).  Graphs are
        // captured on a private non-blocking stream and replayed on st.
        hipError_t e = hipSuccess;
        if (!c->st) {
            e = hipStreamCreateWithFlags(&c->st, hipStreamDefault);
            c->own_st = e == hipSuccess;
        }
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
        if (e != hipSuccess) {
            g_last_error = std::string("stream creation: ") + hipGetErrorString(e);
            release(c);
            delete c;
            return GRIM_E_HIP;
        }
    }
    {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&c->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            c->cus = 0;
    }
    {
        // this device's copy of the no-allocation scratch array
        const hipError_t e = scratch_address(&c->scratch);
        if (e != hipSuccess) {
            g_last_error = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            release(c);
            delete c;
            return GRIM_E_HIP;
        }
    }
    c->nvar = cfg->model;
    c->L = layout_of(cfg);
    c->ph = phys_of(cfg);
    if (!cfg->external_workspace) {
        // the whole workspace in one allocation
        const size_t bytes = carve(cfg, nullptr, nullptr);
        char* base = nullptr;
        hipError_t e = hipMalloc((void**)&base, bytes);
        int rc = GRIM_OK;
        if (e != hipSuccess) {
            rc = e == hipErrorOutOfMemory ? GRIM_E_OOM : GRIM_E_HIP;
            c->err = std::string("hipMalloc(") + std::to_string(bytes) + " bytes): " + hipGetErrorString(e);
        } else {
            c->own_ws = true;
            rc = init_workspace(c, base, bytes);
            if (rc) c->err = "device initialisation: " + c->err;
        }
        if (rc) {
            g_last_error = c->err;
            release(c);
            delete c;
            return rc;
        }
    }
    *out = c;
    return GRIM_OK;
}

size_t grim_workspace_bytes(const grim_config_t* cfg)
{
    if (!cfg) {
        fail(nullptr, GRIM_E_INVALID_ARG, "null config");
        return 0;
    }
    std::string why;
    if (validate(cfg, why)) {
        fail(nullptr, GRIM_E_INVALID_ARG, "invalid config: " + why);
        return 0;
    }
    return carve(cfg, nullptr, nullptr);
}

int grim_bind_workspace(grim_ctx_t* c, void* dev_ptr, size_t bytes)
{
    if (!c) return fail(nullptr, GRIM_E_INVALID_ARG, "null context");
    if (!c->cfg.external_workspace) return fail(c, GRIM_E_STATE, "the context allocated its own workspace");
    if (c->ws) return fail(c, GRIM_E_STATE, "a workspace is already bound");
    if (!dev_ptr || ((uintptr_t)dev_ptr & 255u)) return fail(c, GRIM_E_INVALID_ARG, "null or not 256-byte aligned");
    const size_t need = carve(&c->cfg, nullptr, nullptr);
    if (bytes < need)
        return fail(c, GRIM_E_INVALID_ARG,
                    "workspace too small: " + std::to_string(bytes) + " < " + std::to_string(need) + " bytes");
    return init_workspace(c, (char*)dev_ptr, need);
}

int grim_destroy(grim_ctx_t* ctx)
{
    if (!ctx) return GRIM_OK;
    hipStreamSynchronize(ctx->st);
    release(ctx);
    delete ctx;
    return GRIM_OK;
}

int grim_set_prims(grim_ctx_t* c, const double* P, int on_device)
{
    if (int rc_ = usable(c)) return rc_;
    if (!P) return fail(c, GRIM_E_INVALID_ARG, "null P");
    const size_t bytes = sizeof(double) * c->nvar * c->L.nz;
    const double* src = P;
    if (!on_device) {
        HIP_TRY(c, hipMemcpyAsync(c->interior, P, bytes, hipMemcpyHostToDevice, c->st));
        src = c->interior;
    }
    HIP_TRY(c, grim::launch_copy_interior(c->L, c->nvar, src, 0, c->P[c->cur], 1, c->st));
    const int bc[3] = {c->cfg.bc[0], c->cfg.bc[1], c->cfg.bc[2]};
    HIP_TRY(c, grim::launch_fill_ghosts(c->L, c->nvar, bc, c->P[c->cur], c->st));
    HIP_TRY(c, hipStreamSynchronize(c->st));
    return GRIM_OK;
}

int grim_get_prims(grim_ctx_t* c, double* P, int on_device)
{
    if (int rc_ = usable(c)) return rc_;
    if (!P) return fail(c, GRIM_E_INVALID_ARG, "null P");
    const size_t bytes = sizeof(double) * c->nvar * c->L.nz;
    if (on_device) {
        HIP_TRY(c, grim::launch_copy_interior(c->L, c->nvar, c->P[c->cur], 1, P, 0, c->st));
    } else {
        HIP_TRY(c, grim::launch_copy_interior(c->L, c->nvar, c->P[c->cur], 1, c->interior, 0, c->st));
        HIP_TRY(c, hipMemcpyAsync(P, c->interior, bytes, hipMemcpyDeviceToHost, c->st));
    }
    HIP_TRY(c, hipStreamSynchronize(c->st));
    return GRIM_OK;
}

int grim_cfl_dt(grim_ctx_t* c, double cfl, double* dt)
{
    if (int rc_ = usable(c)) return rc_;
    if (!dt || !(cfl > 0.0)) return fail(c, GRIM_E_INVALID_ARG, "cfl must be positive and dt non-null");
    const unsigned long long init = 0x7FEFFFFFFFFFFFFFull;  // largest finite double
    HIP_TRY(c, hipMemcpyAsync(c->u64, &init, sizeof(init), hipMemcpyHostToDevice, c->st));
    grim::GeoTables geo{c->geo_centre, {c->geo_face[0], c->geo_face[1], c->geo_face[2]}, c->geo_conn,
                        (size_t)c->L.N[0] * c->L.N[1]};
    HIP_TRY(c, grim::launch_cfl(c->L, c->ph, geo, c->nvar, c->cfg.metric, c->P[c->cur], c->u64, c->st));
    unsigned long long bits = 0;
    HIP_TRY(c, hipMemcpyAsync(&bits, c->u64, sizeof(bits), hipMemcpyDeviceToHost, c->st));
    HIP_TRY(c, hipStreamSynchronize(c->st));
    double m;
    std::memcpy(&m, &bits, sizeof(m));
    if (!std::isfinite(m) || !(m > 0.0)) return fail(c, GRIM_E_STATE, "non-finite or zero time step (bad state?)");
    *dt = cfl * m;
    return GRIM_OK;
}

// Steps per launch of the multi-step graph (even: the buffers ping-pong).
constexpr int kGraphSteps = 16;

int grim_run(grim_ctx_t* c, double dt, int nsteps, int use_graph, grim_stats_t* stats)
{
    if (int rc_ = usable(c)) return rc_;
    if (!(dt > 0.0) || !std::isfinite(dt) || nsteps < 0) return fail(c, GRIM_E_INVALID_ARG, "bad dt or nsteps");
    if (c->cfg.guess == GRIM_GUESS_MLP && !c->mlp_set)
        return fail(c, GRIM_E_STATE, "learned guess requested but no network weights were set");
    HIP_TRY(c, grim::launch_zero_stats(c->stats, c->st));
    if (use_graph && nsteps > 0 && !c->timing) {
        if (c->graph_dt != dt || !c->graph[0]) {
            for (int i = 0; i < 4; ++i)
                if (c->graph[i]) {
                    hipGraphExecDestroy(c->graph[i]);
                    c->graph[i] = nullptr;
                }
            for (int i = 0; i < 4; ++i) {
                hipGraph_t g = nullptr;
                HIP_TRY(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeRelaxed));
                int rc = 0;
                for (int s = 0; s < (i < 2 ? 1 : kGraphSteps) && rc == 0; ++s)
                    rc = enqueue_step(c, (i + s) & 1, dt, c->cap);
                hipError_t e = hipStreamEndCapture(c->cap, &g);
                if (rc) {
                    if (g) hipGraphDestroy(g);
                    return rc;
                }
                if (e != hipSuccess) return hip_fail(c, e, "hipStreamEndCapture");
                e = hipGraphInstantiate(&c->graph[i], g, nullptr, nullptr, 0);
                hipGraphDestroy(g);
                if (e != hipSuccess) return hip_fail(c, e, "hipGraphInstantiate");
            }
            c->graph_dt = dt;
        }
        // each graph launch costs ~8 us of idle GPU between graphs, so
        // steps go kGraphSteps to a launch
        int s = 0;
        for (; s + kGraphSteps <= nsteps; s += kGraphSteps) HIP_TRY(c, hipGraphLaunch(c->graph[2 + c->cur], c->st));
        for (; s < nsteps; ++s) {
            HIP_TRY(c, hipGraphLaunch(c->graph[c->cur], c->st));
            c->cur = 1 - c->cur;
        }
    } else {
        for (int s = 0; s < nsteps; ++s) {
            int rc = enqueue_step(c, c->cur, dt, c->st);
            if (rc) return rc;
            c->cur = 1 - c->cur;
        }
    }
    if (stats) return read_stats(c, nsteps > 0 ? nsteps : 1, stats);
    return GRIM_OK;
}

int grim_residual(grim_ctx_t* c, const double* Pn, const double* PE, double dtp, const double* P, double* R,
                  double* rnorm)
{
    if (int rc_ = usable(c)) return rc_;
    if (!P || !R) return fail(c, GRIM_E_INVALID_ARG, "null P or R");
    StageArgs s;
    int rc = hook_setup(c, Pn, PE, dtp, &s, nullptr, nullptr, nullptr);
    if (rc) return rc;
    HIP_TRY(c, grim::launch_residual(s, c->nvar, c->cfg.metric, P, R, rnorm, c->st));
    HIP_TRY(c, hipStreamSynchronize(c->st));
    return GRIM_OK;
}

int grim_stage_solve(grim_ctx_t* c, const double* Pn, const double* PE, double dtp, const double* guess,
                     double* P_out, int32_t* iters, double* resid, uint8_t* flags, int32_t* backtracks,
                     grim_stats_t* stats)
{
    if (int rc_ = usable(c)) return rc_;
    if (!P_out) return fail(c, GRIM_E_INVALID_ARG, "null P_out");
    StageArgs s;
    int rc = hook_setup(c, Pn, PE, dtp, &s, nullptr, nullptr, nullptr);
    if (rc) return rc;
    HIP_TRY(c, grim::launch_zero_stats(c->stats, c->st));
    NewtonArgs n = newton_args(c, s);
    n.guess = guess;
    n.out = P_out;
    n.out_ghosted = 0;
    n.fused = fused_rhs(c) ? 1 : 0;  // the same Newton kernel grim_run uses
    n.tiled = tiled_stage(c) ? 1 : 0;
    n.stage = 0;
    if (iters) n.iters = iters;
    if (resid) n.resid = resid;
    if (flags) n.flags = flags;
    n.backtracks = backtracks;
    HIP_TRY(c, grim::launch_newton(n, c->nvar, c->cfg.metric, c->cfg.jac_precision, c->st));
    if (stats) return read_stats(c, 1, stats);
    HIP_TRY(c, hipStreamSynchronize(c->st));
    return GRIM_OK;
}

int grim_explicit(grim_ctx_t* c, const double* PE, double* divF, double* srcE, double* emhd_sp)
{
    if (int rc_ = usable(c)) return rc_;
    if (!divF || !srcE) return fail(c, GRIM_E_INVALID_ARG, "null divF or srcE");
    StageArgs s;
    int rc = hook_setup(c, PE, PE, 1.0, &s, divF, srcE, emhd_sp);
    if (rc) return rc;
    HIP_TRY(c, hipStreamSynchronize(c->st));
    return GRIM_OK;
}

int grim_get_zone_results(grim_ctx_t* c, uint8_t* flags, int32_t* iters, int on_device)
{
    if (int rc_ = usable(c)) return rc_;
    const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
    if (flags) HIP_TRY(c, hipMemcpyAsync(flags, c->flags, (size_t)c->L.nz, k, c->st));
    if (iters) HIP_TRY(c, hipMemcpyAsync(iters, c->iters, sizeof(int32_t) * c->L.nz, k, c->st));
    HIP_TRY(c, hipStreamSynchronize(c->st));
    return GRIM_OK;
}

int grim_profile(grim_ctx_t* c, int enable)
{
    if (!c) return fail(nullptr, GRIM_E_INVALID_ARG, "null context");
    c->timing = enable != 0;
    return GRIM_OK;
}

int grim_kernel_times(grim_ctx_t* c, double* ms, int64_t* launches, int n)
{
    if (!c) return fail(nullptr, GRIM_E_INVALID_ARG, "null context");
    if (!ms || !launches || n < 6) return fail(c, GRIM_E_INVALID_ARG, "need 6-entry output arrays");
    for (int i = 0; i < n; ++i) {
        ms[i] = 0.0;
        launches[i] = 0;
    }
    HIP_TRY(c, hipStreamSynchronize(c->st));
    for (auto& m : c->marks) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, m.a, m.b) == hipSuccess) {
            ms[m.group] += t;
            launches[m.group] += 1;
        }
        hipEventDestroy(m.a);
        hipEventDestroy(m.b);
    }
    c->marks.clear();
    return GRIM_OK;
}

int grim_mlp_set_weights(grim_ctx_t* c, const float* w, size_t n)
{
    if (int rc_ = usable(c)) return rc_;
    if (!w || n != (size_t)grim::kMlpParams) return fail(c, GRIM_E_INVALID_ARG, "need GRIM_MLP_PARAMS values");
    HIP_TRY(c, hipMemcpyAsync(c->mlp_p, w, sizeof(float) * n, hipMemcpyHostToDevice, c->st));
    HIP_TRY(c, grim::mlp_pack(c->mlp_p, c->mlp_w[0], c->mlp_w[1], c->mlp_w[2], c->st));
    HIP_TRY(c, hipStreamSynchronize(c->st));
    c->mlp_set = true;
    return GRIM_OK;
}

int grim_mlp_get_weights(grim_ctx_t* c, float* w, size_t n)
{
    if (int rc_ = usable(c)) return rc_;
    if (!w || n != (size_t)grim::kMlpParams) return fail(c, GRIM_E_INVALID_ARG, "need GRIM_MLP_PARAMS values");
    if (!c->mlp_set) return fail(c, GRIM_E_STATE, "no network weights set");
    HIP_TRY(c, hipMemcpyAsync(w, c->mlp_p, sizeof(float) * n, hipMemcpyDeviceToHost, c->st));
    HIP_TRY(c, hipStreamSynchronize(c->st));
    return GRIM_OK;
}

int grim_mlp_forward(grim_ctx_t* c, const float* X, int64_t n, float* Y)
{
    if (int rc_ = usable(c)) return rc_;
    if (!X || !Y || n < 0) return fail(c, GRIM_E_INVALID_ARG, "bad arguments");
    if (!c->mlp_set) return fail(c, GRIM_E_STATE, "no network weights set");
    HIP_TRY(c, grim::mlp_infer(X, (long)n, c->mlp_p, c->mlp_w[0], c->mlp_w[1], c->mlp_w[2], Y, c->st));
    HIP_TRY(c, hipStreamSynchronize(c->st));
    return GRIM_OK;
}

int grim_mlp_backward(grim_ctx_t* c, const float* X, const float* dY, int64_t n, float* dW)
{
    if (int rc_ = usable(c)) return rc_;
    if (!X || !dY || !dW || n <= 0) return fail(c, GRIM_E_INVALID_ARG, "bad arguments");
    if (!c->mlp_set) return fail(c, GRIM_E_STATE, "no network weights set");
    const int chunk = 4096;
    int rc = ensure_mlp_train_buffers(c, chunk);
    if (rc) return rc;
    HIP_TRY(c, hipMemsetAsync(dW, 0, sizeof(float) * grim::kMlpParams, c->st));
    for (long off = 0; off < n; off += chunk) {
        const int b = (int)std::min<long>(chunk, n - off);
        HIP_TRY(c, grim::mlp_batch_grad(c->work, X, nullptr, dY, nullptr, off, b, 0, 0.0f, c->mlp_p, dW,
                                        off > 0 ? 1 : 0, c->dloss, c->st));
    }
    HIP_TRY(c, hipStreamSynchronize(c->st));
    return GRIM_OK;
}

int grim_mlp_backward_noalloc(grim_ctx_t* c, const float* X, const float* dY, int64_t n, float* dW)
{
    if (int rc_ = usable(c)) return rc_;
    if (!X || !dY || !dW || n <= 0) return fail(c, GRIM_E_INVALID_ARG, "bad arguments");
    if (n > kNoAllocRows)
        return fail(c, GRIM_E_INVALID_ARG,
                    "n = " + std::to_string(n) + " rows exceeds the " + std::to_string(kNoAllocRows) +
                        " rows of the no-allocation scratch");
    if (!c->mlp_set) return fail(c, GRIM_E_STATE, "no network weights set");
    if (!c->scratch) return fail(c, GRIM_E_STATE, "no scratch address for this device");
    grim::MlpWork w{};
    float* q = c->scratch;
    float** bufs[] = {&w.xh, &w.tb, &w.z1, &w.h1, &w.z2, &w.h2, &w.o, &w.d_o, &w.dh, &w.dh1};
    const int widths[] = {grim::kMlpIn, grim::kMlpOut, grim::kMlpHidden, grim::kMlpHidden, grim::kMlpHidden,
                          grim::kMlpHidden, grim::kMlpOut, grim::kMlpOut, grim::kMlpHidden, grim::kMlpHidden};
    for (int i = 0; i < 10; ++i) {
        *bufs[i] = q;
        q += (size_t)kNoAllocRows * widths[i];
    }
    w.cap = kNoAllocRows;
    double* loss = reinterpret_cast<double*>(q);  // 256-byte aligned: every buffer is a multiple of it
    // every work buffer is written before it is read, and the layers' weight
    // and bias gradients are written, not accumulated (acc = 0); only the
    // normalisation entries of dW, which no kernel writes, are cleared (by
    // a fill kernel, so the call can be captured in a graph)
    HIP_TRY(c, grim::mlp_fill(dW + grim::kOffXm, grim::kMlpParams - grim::kOffXm, 0.0f, c->st));
    HIP_TRY(c, grim::mlp_batch_grad(w, X, nullptr, dY, nullptr, 0, (int)n, 0, 0.0f, c->mlp_p, dW, 0, loss, c->st));
    return GRIM_OK;
}

int grim_mlp_train(grim_ctx_t* c, const float* X, const float* T, int64_t n, const grim_train_cfg_t* cfg,
                   double* loss_hist)
{
    if (int rc_ = usable(c)) return rc_;
    if (!X || !T || !cfg || n <= 0 || cfg->epochs < 0 || cfg->batch <= 0 || cfg->n_used <= 0 ||
        cfg->n_used > grim::kMlpOut || !(cfg->lr > 0))
        return fail(c, GRIM_E_INVALID_ARG, "bad training arguments");
    if (!c->mlp_set) return fail(c, GRIM_E_STATE, "set initial weights (and normalisation) first");
    const int B = (int)std::min<int64_t>(cfg->batch, n);
    int rc = ensure_mlp_train_buffers(c, B);
    if (rc) return rc;
    if (c->mlp_idx_cap < n) {
        if (c->mlp_idx) hipFree(c->mlp_idx);
        c->mlp_idx = nullptr;
        rc = dalloc(c, &c->mlp_idx, (size_t)n);
        if (rc) return rc;
        c->mlp_idx_cap = n;
    }
    HIP_TRY(c, hipMemsetAsync(c->adam_m, 0, sizeof(float) * grim::kMlpTrainable, c->st));
    HIP_TRY(c, hipMemsetAsync(c->adam_v, 0, sizeof(float) * grim::kMlpTrainable, c->st));
    std::vector<int> perm((size_t)n);
    std::mt19937_64 rng(cfg->seed);
    int step = 0;
    const long nbatches = n / B;
    for (int e = 0; e < cfg->epochs; ++e) {
        for (long i = 0; i < n; ++i) perm[(size_t)i] = (int)i;
        std::shuffle(perm.begin(), perm.end(), rng);
        HIP_TRY(c, hipMemcpyAsync(c->mlp_idx, perm.data(), sizeof(int) * n, hipMemcpyHostToDevice, c->st));
        HIP_TRY(c, hipMemsetAsync(c->dloss, 0, sizeof(double), c->st));
        for (long bi = 0; bi < nbatches; ++bi) {
            HIP_TRY(c, grim::mlp_batch_grad(c->work, X, T, nullptr, c->mlp_idx, bi * B, B, cfg->n_used,
                                            1.0f / (float)(B * cfg->n_used), c->mlp_p, c->mlp_grad, 0, c->dloss,
                                            c->st));
            HIP_TRY(c, grim::mlp_adam(c->mlp_p, c->mlp_grad, c->adam_m, c->adam_v, grim::kMlpTrainable,
                                      (float)cfg->lr, (float)cfg->beta1, (float)cfg->beta2, (float)cfg->eps, ++step,
                                      c->st));
        }
        double lsum = 0.0;
        HIP_TRY(c, hipMemcpyAsync(&lsum, c->dloss, sizeof(double), hipMemcpyDeviceToHost, c->st));
        HIP_TRY(c, hipStreamSynchronize(c->st));
        if (loss_hist) loss_hist[e] = lsum / (double)std::max<long>(nbatches, 1);
    }
    HIP_TRY(c, grim::mlp_pack(c->mlp_p, c->mlp_w[0], c->mlp_w[1], c->mlp_w[2], c->st));
    HIP_TRY(c, hipStreamSynchronize(c->st));
    return GRIM_OK;
}

int grim_mlp_normalisation(grim_ctx_t* c, const float* X, const float* T, int64_t n, int n_used, double* x_mean,
                           double* x_istd, double* y_scale)
{
    if (int rc_ = usable(c)) return rc_;
    if (!X || !T || !x_mean || !x_istd || !y_scale || n < 2 || n_used < 1 || n_used > grim::kMlpOut)
        return fail(c, GRIM_E_INVALID_ARG, "bad arguments (n >= 2 and n_used in [1, 16] required)");
    HIP_TRY(c, grim::mlp_norm_stats(X, T, (long)n, c->nrm, kNormBlocks, c->st));
    double mv[2 * kNormCols];
    HIP_TRY(c, hipMemcpyAsync(mv, c->nrm + (size_t)kNormBlocks * kNormCols, sizeof(mv), hipMemcpyDeviceToHost, c->st));
    HIP_TRY(c, hipStreamSynchronize(c->st));
    const double* mean = mv;
    const double* var = mv + kNormCols;
    for (int i = 0; i < grim::kMlpIn; ++i) {
        x_mean[i] = mean[i];
        x_istd[i] = var[i] > 0.0 ? 1.0 / std::sqrt(var[i]) : 0.0;
    }
    for (int i = 0; i < grim::kMlpOut; ++i)
        y_scale[i] = (i < n_used && var[grim::kMlpIn + i] > 0.0) ? std::sqrt(var[grim::kMlpIn + i]) : 0.0;
    return GRIM_OK;
}

int grim_collect_pairs(grim_ctx_t* c, double dt, int nsteps, int stride, float* X, float* T, int64_t cap,
                       int64_t* count)
{
    if (int rc_ = usable(c)) return rc_;
    if (!X || !T || !count || stride < 1 || cap < 0 || nsteps < 0 || !(dt > 0.0))
        return fail(c, GRIM_E_INVALID_ARG, "bad arguments");
    int rc = GRIM_OK;
    Collect col{stride, 0, X, T, (long)cap, 0};
    for (int s = 0; s < nsteps; ++s) {
        rc = enqueue_step(c, c->cur, dt, c->st, &col);
        if (rc) return rc;
        c->cur = 1 - c->cur;
    }
    HIP_TRY(c, hipStreamSynchronize(c->st));
    *count = std::min<long>(col.count, (long)cap);
    return GRIM_OK;
}

int grim_math_probe(grim_ctx_t* c, const double* x, double* out, size_t n)
{
    if (int rc_ = usable(c)) return rc_;
    if (n > 0 && (!x || !out)) return fail(c, GRIM_E_INVALID_ARG, "null pointer");
    HIP_TRY(c, grim::launch_math_probe(x, out, n, c->st));
    HIP_TRY(c, hipStreamSynchronize(c->st));
    return GRIM_OK;
}

int grim_stream_add(grim_ctx_t* c, const double* a, const double* b, double* cc, size_t n)
{
    if (int rc_ = usable(c)) return rc_;
    if (!a || !b || !cc) return fail(c, GRIM_E_INVALID_ARG, "null pointer");
    HIP_TRY(c, grim::launch_stream_add(a, b, cc, n, c->st));
    return GRIM_OK;
}

}  // extern "C"

namespace grim {

int check_config(const grim_config_t* cfg, std::string& why) { return validate(cfg, why); }
Layout grid_layout(const grim_config_t* cfg) { return layout_of(cfg); }
Phys physics(const grim_config_t* cfg) { return phys_of(cfg); }
void set_global_error(const std::string& msg) { g_last_error = msg; }

}  // namespace grim
