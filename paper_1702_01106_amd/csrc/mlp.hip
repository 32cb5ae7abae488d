// The learned initial guess: a 32 -> 128 -> 128 -> 16 GELU network.
//
// Inference (a14) is BF16 on the matrix cores with FP32 accumulation
// (v_mfma_f32_32x32x8_bf16), one wave per 32 rows, evaluated transposed so the
// activations never leave registers; the transposed BF16 weights sit in LDS.  Training (a15) is FP32 on the vector units: a tiled
// GEMM, elementwise GELU / loss kernels and Adam on FP32 master weights.
//
// Parameter vector (FP32): W1 [32][128], b1, W2 [128][128], b2, W3 [128][16],
// b3, x_mean [32], x_istd [32], y_scale [16].
//   y = (gelu(gelu(((x - x_mean) * x_istd) W1 + b1) W2 + b2) W3 + b3) * y_scale
// with gelu(z) = z (1 + erf(z / sqrt 2)) / 2.
#include <hip/hip_runtime.h>

#include "grim_internal.h"

namespace grim {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int DI = kMlpIn, DH = kMlpHidden, DO = kMlpOut;

// float -> bfloat16 bits, round to nearest even (finite inputs)
__device__ __forceinline__ unsigned short to_bf16(float f)
{
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// ------------------------------------------------------------------ BF16 weights

// Transposed BF16 copies for the MFMA B operand: W1t [128][32], W2t [128][128],
// W3t [32][128] (output columns 16..31 zero).
__global__ void k_mlp_pack(const float* __restrict__ p, unsigned short* __restrict__ w1t,
                           unsigned short* __restrict__ w2t, unsigned short* __restrict__ w3t)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < DH * DI) {
        const int n = t / DI, k = t % DI;
        w1t[t] = to_bf16(p[kOffW1 + k * DH + n]);
    }
    if (t < DH * DH) {
        const int n = t / DH, k = t % DH;
        w2t[t] = to_bf16(p[kOffW2 + k * DH + n]);
    }
    if (t < 32 * DH) {
        const int n = t / DH, k = t % DH;
        w3t[t] = n < DO ? to_bf16(p[kOffW3 + k * DO + n]) : (unsigned short)0;
    }
}

// ------------------------------------------------------------------ inference

// The network is evaluated transposed, Z^T = W^T X^T, so that each wave's 32
// rows are the N dimension of v_mfma_f32_32x32x8_bf16.  Operand layouts of that
// instruction (lane l, e = 0..3): A[m = l%32][k = 4(l/32) + e],
// B[k = 4(l/32) + e][n = l%32]; accumulator element r of lane l is
// D[m = 8(r/4) + 4(l/32) + r%4][n = l%32].  A hidden layer's accumulator
// elements 4q..4q+3 of output tile t are therefore exactly the B operand of
// k-step 4t + q of the next layer: activations stay in registers, and only
// the transposed BF16 weights (the A operands) live in LDS.
constexpr int kRowsPerWave = 32;
constexpr int kWaves = 4;
// LDS row strides in bf16 elements: K + 4 puts the 8-byte reads of the 32
// lanes of a half-wave on distinct banks
constexpr int kS1 = DI + 4, kS2 = DH + 4;

// gelu(z) = z (1 + erf(z / sqrt 2)) / 2 with erf from Abramowitz & Stegun
// 7.1.26 (absolute error below 1.5e-7, far under the BF16 rounding that
// follows); the training path keeps erff.
__device__ __forceinline__ float gelu_fast(float z)
{
    const float ax = fabsf(z) * 0.70710678118654752f;
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.0f));
    float p = fmaf(t, 1.061405429f, -1.453152027f);
    p = fmaf(t, p, 1.421413741f);
    p = fmaf(t, p, -0.284496736f);
    p = fmaf(t, p, 0.254829592f);
    p *= t;
    const float e = 1.0f - p * __expf(-ax * ax);
    return 0.5f * z * (1.0f + copysignf(e, z));
}

// Four floats to bfloat16, round to nearest even: v_cvt_pk_bf16_f32 on gfx950
// (two values per instruction).
typedef __bf16 bfv2 __attribute__((ext_vector_type(2)));
typedef float fv2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ bf16x4 pack4(float a, float b, float c, float d)
{
    const fv2 lo = {a, b}, hi = {c, d};
    const unsigned l = __builtin_bit_cast(unsigned, __builtin_convertvector(lo, bfv2));
    const unsigned u = __builtin_bit_cast(unsigned, __builtin_convertvector(hi, bfv2));
    return __builtin_bit_cast(bf16x4, (unsigned long long)l | ((unsigned long long)u << 32));
}

__device__ __forceinline__ bf16x4 lds_a(const unsigned short* base)
{
    // 8-byte aligned: every row stride and k offset is a multiple of 4 elements
    return *reinterpret_cast<const bf16x4*>(base);
}

__global__ __launch_bounds__(kWaves * 64, 3) void k_mlp_infer(const float* __restrict__ X, long n,
                                                           const float* __restrict__ p,
                                                           const unsigned short* __restrict__ w1t,
                                                           const unsigned short* __restrict__ w2t,
                                                           const unsigned short* __restrict__ w3t,
                                                           float* __restrict__ Y)
{
    __shared__ __align__(16) unsigned short sW1[DH * kS1];
    __shared__ __align__(16) unsigned short sW2[DH * kS2];
    __shared__ __align__(16) unsigned short sW3[32 * kS2];
    __shared__ float sB1[DH], sB2[DH], sB3[32], sXm[DI], sXs[DI], sYs[32];

    const int tid = threadIdx.x;
    // stage the transposed weights, 4 bf16 (8 bytes) per access
    {
        const uint2* g1 = reinterpret_cast<const uint2*>(w1t);
        for (int i = tid; i < DH * DI / 4; i += kWaves * 64) {
            const int r = i / (DI / 4), c = 4 * (i % (DI / 4));
            *reinterpret_cast<uint2*>(&sW1[r * kS1 + c]) = g1[i];
        }
        const uint2* g2 = reinterpret_cast<const uint2*>(w2t);
        for (int i = tid; i < DH * DH / 4; i += kWaves * 64) {
            const int r = i / (DH / 4), c = 4 * (i % (DH / 4));
            *reinterpret_cast<uint2*>(&sW2[r * kS2 + c]) = g2[i];
        }
        const uint2* g3 = reinterpret_cast<const uint2*>(w3t);
        for (int i = tid; i < 32 * DH / 4; i += kWaves * 64) {
            const int r = i / (DH / 4), c = 4 * (i % (DH / 4));
            *reinterpret_cast<uint2*>(&sW3[r * kS2 + c]) = g3[i];
        }
    }
    if (tid < DH) {
        sB1[tid] = p[kOffB1 + tid];
        sB2[tid] = p[kOffB2 + tid];
    }
    if (tid < 32) {
        sB3[tid] = tid < DO ? p[kOffB3 + tid] : 0.0f;
        sYs[tid] = tid < DO ? p[kOffYs + tid] : 0.0f;
        sXm[tid] = p[kOffXm + tid];
        sXs[tid] = p[kOffXs + tid];
    }
    __syncthreads();

    // one 32-row tile per wave (no tile loop: the weight reads below would be
    // hoisted out of it as loop invariants and spilled)
    const int lane = tid & 63;
    const int c = lane & 31, h = lane >> 5;
    const long tile = (long)blockIdx.x * kWaves + (tid >> 6);
    {
        const long row = tile * kRowsPerWave + c;
        const bool live = row < n;

        // ---- layer 1, B = normalised X^T: k = 8s + 4h + e of row `row`
        bf16x4 bx[DI / 8];
#pragma unroll
        for (int s = 0; s < DI / 8; ++s) {
            const int k0 = 8 * s + 4 * h;
            float4 x = live ? *reinterpret_cast<const float4*>(X + row * DI + k0) : make_float4(0.f, 0.f, 0.f, 0.f);
            bx[s] = pack4((x.x - sXm[k0 + 0]) * sXs[k0 + 0], (x.y - sXm[k0 + 1]) * sXs[k0 + 1],
                          (x.z - sXm[k0 + 2]) * sXs[k0 + 2], (x.w - sXm[k0 + 3]) * sXs[k0 + 3]);
        }
        bf16x4 b2[DH / 8];
#pragma unroll
        for (int t = 0; t < DH / 32; ++t) {
            f32x16 acc = {};
#pragma unroll
            for (int s = 0; s < DI / 8; ++s)
                acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(lds_a(&sW1[(32 * t + c) * kS1 + 8 * s + 4 * h]), bx[s],
                                                              acc, 0, 0, 0);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = 32 * t + 8 * q + 4 * h;
                b2[4 * t + q] = pack4(gelu_fast(acc[4 * q + 0] + sB1[m + 0]), gelu_fast(acc[4 * q + 1] + sB1[m + 1]),
                                      gelu_fast(acc[4 * q + 2] + sB1[m + 2]), gelu_fast(acc[4 * q + 3] + sB1[m + 3]));
            }
        }
        // ---- layer 2: k-steps outer, the four output tiles inner
        f32x16 acc2[DH / 32];
#pragma unroll
        for (int t = 0; t < DH / 32; ++t) acc2[t] = f32x16{};
#pragma unroll
        for (int s = 0; s < DH / 8; ++s)
#pragma unroll
            for (int t = 0; t < DH / 32; ++t)
                acc2[t] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(lds_a(&sW2[(32 * t + c) * kS2 + 8 * s + 4 * h]),
                                                                  b2[s], acc2[t], 0, 0, 0);
        bf16x4 b3[DH / 8];
#pragma unroll
        for (int t = 0; t < DH / 32; ++t)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = 32 * t + 8 * q + 4 * h;
                b3[4 * t + q] = pack4(gelu_fast(acc2[t][4 * q + 0] + sB2[m + 0]), gelu_fast(acc2[t][4 * q + 1] + sB2[m + 1]),
                                      gelu_fast(acc2[t][4 * q + 2] + sB2[m + 2]), gelu_fast(acc2[t][4 * q + 3] + sB2[m + 3]));
            }
        // ---- layer 3: 32 output rows of which the first 16 are real
        f32x16 acc = {};
#pragma unroll
        for (int s = 0; s < DH / 8; ++s)
            acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(lds_a(&sW3[c * kS2 + 8 * s + 4 * h]), b3[s], acc, 0, 0, 0);
        if (live) {
            // elements 0..3: outputs 4h..4h+3; 4..7: outputs 8+4h..8+4h+3
#pragma unroll
            for (int g = 0; g < 2; ++g) {
                const int m0 = 8 * g + 4 * h;
                float4 y;
                y.x = (acc[4 * g + 0] + sB3[m0 + 0]) * sYs[m0 + 0];
                y.y = (acc[4 * g + 1] + sB3[m0 + 1]) * sYs[m0 + 1];
                y.z = (acc[4 * g + 2] + sB3[m0 + 2]) * sYs[m0 + 2];
                y.w = (acc[4 * g + 3] + sB3[m0 + 3]) * sYs[m0 + 3];
                *reinterpret_cast<float4*>(Y + row * DO + m0) = y;
            }
        }
    }
}

// ------------------------------------------------------------------ training (FP32)

constexpr int kT = 16;  // GEMM tile

// C[M][N] (+)= op(A)[M][K] * op(B)[K][N]; op(A)[m][k] = ta ? A[k*lda + m] : A[m*lda + k].
__global__ __launch_bounds__(kT* kT) void k_gemm(const float* __restrict__ A, int lda, int ta,
                                                 const float* __restrict__ B, int ldb, int tb, float* __restrict__ C,
                                                 int ldc, int M, int N, int K, int accumulate)
{
    __shared__ float sa[kT][kT + 1], sb[kT][kT + 1];
    const int tx = threadIdx.x % kT, ty = threadIdx.x / kT;
    const int m = blockIdx.y * kT + ty, nn = blockIdx.x * kT + tx;
    float acc = 0.0f;
    for (int k0 = 0; k0 < K; k0 += kT) {
        {
            const int mm = blockIdx.y * kT + ty, kk = k0 + tx;
            sa[ty][tx] = (mm < M && kk < K) ? (ta ? A[(long)kk * lda + mm] : A[(long)mm * lda + kk]) : 0.0f;
        }
        {
            const int kk = k0 + ty, cc = blockIdx.x * kT + tx;
            sb[ty][tx] = (kk < K && cc < N) ? (tb ? B[(long)cc * ldb + kk] : B[(long)kk * ldb + cc]) : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kT; ++k) acc = fmaf(sa[ty][k], sb[k][tx], acc);
        __syncthreads();
    }
    if (m < M && nn < N) C[(long)m * ldc + nn] = accumulate ? C[(long)m * ldc + nn] + acc : acc;
}

// gather a batch (optionally through an index list) and normalise the input
__global__ void k_gather(const float* __restrict__ X, const float* __restrict__ T, const int* __restrict__ idx,
                         long off, int nb, const float* __restrict__ p, float* __restrict__ XH, float* __restrict__ TB)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nb * DI) return;
    const int b = t / DI, k = t % DI;
    const long row = idx ? (long)idx[off + b] : off + b;
    XH[t] = (X[row * DI + k] - p[kOffXm + k]) * p[kOffXs + k];
    if (T && k < DO) TB[b * DO + k] = T[row * DO + k];
}

// z += bias (per column), h = gelu(z)
__global__ void k_bias_gelu(float* __restrict__ Z, float* __restrict__ Hh, const float* __restrict__ bias, int nb, int nc)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nb * nc) return;
    const float z = Z[t] + bias[t % nc];
    Z[t] = z;
    Hh[t] = gelu(z);
}

// output layer: dO = d loss / d(pre-scale output) for the MSE loss in
// normalised units, mean over rows and the first n_used outputs of
// ((y - t) / y_scale)^2; or, with dY given, for sum(dY * y).
__global__ void k_out_grad(const float* __restrict__ O, const float* __restrict__ b3, const float* __restrict__ ys,
                           const float* __restrict__ TB, const float* __restrict__ dY, int nb, int n_used,
                           float inv_count, float* __restrict__ dO, double* __restrict__ loss)
{
    // launched with 256 threads per block; the loss is summed per block
    // (wave shuffles, then LDS) and added with one atomic per block
    __shared__ double part[4];
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    double contrib = 0.0;
    if (t < nb * DO) {
        const int j = t % DO;
        float g = 0.0f;
        if (dY) {
            g = dY[t] * ys[j];
        } else if (j < n_used && ys[j] != 0.0f) {
            // loss in normalised output units: ((y - t) / y_scale)^2; an output
            // with y_scale 0 is held at zero and carries no loss
            const float d = (O[t] + b3[j]) - TB[t] / ys[j];
            g = 2.0f * d * inv_count;
            contrib = (double)d * (double)d * (double)inv_count;
        }
        dO[t] = g;
    }
    if (dY) return;  // block-uniform
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) contrib += __shfl_xor(contrib, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = contrib;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(loss, part[0] + part[1] + part[2] + part[3]);
}

__global__ void k_gelu_back(float* __restrict__ dH, const float* __restrict__ Z, int count)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) dH[t] *= gelu_grad(Z[t]);
}

// column sums: g[c] (+)= sum_b D[b][c]
__global__ void k_colsum(const float* __restrict__ D, int nb, int nc, float* __restrict__ g, int accumulate)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    float s = 0.0f;
    for (int b = 0; b < nb; ++b) s += D[(long)b * nc + c];
    g[c] = accumulate ? g[c] + s : s;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const float gg = g[t];
    const float mm = b1 * m[t] + (1.0f - b1) * gg;
    const float vv = b2 * v[t] + (1.0f - b2) * gg * gg;
    m[t] = mm;
    v[t] = vv;
    p[t] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

inline unsigned nb(long n, int b) { return (unsigned)((n + b - 1) / b); }

void gemm(const float* A, int lda, int ta, const float* B, int ldb, int tb, float* C, int ldc, int M, int N, int K,
          int acc, hipStream_t st)
{
    hipLaunchKernelGGL(k_gemm, dim3(nb(N, kT), nb(M, kT)), dim3(kT * kT), 0, st, A, lda, ta, B, ldb, tb, C, ldc, M,
                       N, K, acc);
}

// Column statistics of the training pairs (the network's normalisation):
// 48 columns, X's 32 then T's 16.  Block b of nb sums rows b, b + nb, ... of
// each column in FP64 (mode 0: x; mode 1: (x - mean)^2), its four row lanes
// are combined in a fixed order, and part[b][col] holds the block's sum, so
// the result does not depend on timing.
constexpr int kNormCols = DI + DO, kNormLanes = 4;
__global__ __launch_bounds__(kNormCols* kNormLanes) void k_norm_partial(const float* __restrict__ X,
                                                                       const float* __restrict__ T, long n,
                                                                       const double* __restrict__ mean, int mode,
                                                                       double* __restrict__ part)
{
    __shared__ double red[kNormLanes][kNormCols];
    const int col = threadIdx.x % kNormCols, lane = threadIdx.x / kNormCols;
    const double m = mode ? mean[col] : 0.0;
    double acc = 0.0;
    for (long r = (long)blockIdx.x * kNormLanes + lane; r < n; r += (long)gridDim.x * kNormLanes) {
        const double x = col < DI ? (double)X[r * DI + col] : (double)T[r * DO + col - DI];
        const double d = x - m;
        acc += mode ? d * d : x;
    }
    red[lane][col] = acc;
    __syncthreads();
    if (lane == 0) {
        double t = 0.0;
        for (int l = 0; l < kNormLanes; ++l) t += red[l][col];
        part[(long)blockIdx.x * kNormCols + col] = t;
    }
}

// out[col] = (sum over blocks of part[b][col], in block order) / denom.  A
// division, not a product with 1/denom: the mean of a constant column is
// then that constant exactly, and its deviations exactly zero.
__global__ void k_norm_final(const double* __restrict__ part, int nb, double denom, double* __restrict__ out)
{
    const int col = threadIdx.x;
    if (col >= kNormCols) return;
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += part[(long)b * kNormCols + col];
    out[col] = t / denom;
}

}  // namespace

hipError_t mlp_pack(const float* params, unsigned short* w1t, unsigned short* w2t, unsigned short* w3t, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_pack, dim3(nb(DH * DH, 256)), dim3(256), 0, st, params, w1t, w2t, w3t);
    return hipGetLastError();
}

hipError_t mlp_infer(const float* X, long n, const float* params, const unsigned short* w1t,
                     const unsigned short* w2t, const unsigned short* w3t, float* Y, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    // X rows and Y rows are read / written as 16-byte vectors
    if ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Y)) & 15) return hipErrorInvalidValue;
    const long tiles = (n + kRowsPerWave - 1) / kRowsPerWave;
    const long blocks = (tiles + kWaves - 1) / kWaves;
    if (blocks > 0x7FFFFFFFL) return hipErrorInvalidValue;
    const unsigned grid = (unsigned)blocks;
    hipLaunchKernelGGL(k_mlp_infer, dim3(grid), dim3(kWaves * 64), 0, st, X, n, params, w1t, w2t, w3t, Y);
    return hipGetLastError();
}

// Forward and backward of one batch in FP32.  With T the MSE loss over the
// first n_used outputs is differentiated (and accumulated into *loss); with dY
// the gradient of sum(dY * y) is taken.  Gradients are written (acc = 0) or
// added (acc = 1) into grad.
hipError_t mlp_batch_grad(const MlpWork& w, const float* X, const float* T, const float* dY, const int* idx, long off,
                          int nbatch, int n_used, float inv_count, const float* p, float* grad, int acc, double* loss,
                          hipStream_t st)
{
    const int B = nbatch;
    hipLaunchKernelGGL(k_gather, dim3(nb((long)B * DI, 256)), dim3(256), 0, st, X, T, idx, off, B, p, w.xh, w.tb);
    gemm(w.xh, DI, 0, p + kOffW1, DH, 0, w.z1, DH, B, DH, DI, 0, st);
    hipLaunchKernelGGL(k_bias_gelu, dim3(nb((long)B * DH, 256)), dim3(256), 0, st, w.z1, w.h1, p + kOffB1, B, DH);
    gemm(w.h1, DH, 0, p + kOffW2, DH, 0, w.z2, DH, B, DH, DH, 0, st);
    hipLaunchKernelGGL(k_bias_gelu, dim3(nb((long)B * DH, 256)), dim3(256), 0, st, w.z2, w.h2, p + kOffB2, B, DH);
    gemm(w.h2, DH, 0, p + kOffW3, DO, 0, w.o, DO, B, DO, DH, 0, st);
    hipLaunchKernelGGL(k_out_grad, dim3(nb((long)B * DO, 256)), dim3(256), 0, st, w.o, p + kOffB3, p + kOffYs, w.tb,
                       dY ? dY + off * DO : nullptr, B, n_used, inv_count, w.d_o, loss);
    // output layer
    gemm(w.h2, DH, 1, w.d_o, DO, 0, grad + kOffW3, DO, DH, DO, B, acc, st);
    hipLaunchKernelGGL(k_colsum, dim3(1), dim3(64), 0, st, w.d_o, B, DO, grad + kOffB3, acc);
    gemm(w.d_o, DO, 0, p + kOffW3, DO, 1, w.dh, DH, B, DH, DO, 0, st);
    hipLaunchKernelGGL(k_gelu_back, dim3(nb((long)B * DH, 256)), dim3(256), 0, st, w.dh, w.z2, B * DH);
    // hidden layer 2
    gemm(w.h1, DH, 1, w.dh, DH, 0, grad + kOffW2, DH, DH, DH, B, acc, st);
    hipLaunchKernelGGL(k_colsum, dim3(1), dim3(128), 0, st, w.dh, B, DH, grad + kOffB2, acc);
    gemm(w.dh, DH, 0, p + kOffW2, DH, 1, w.dh1, DH, B, DH, DH, 0, st);
    hipLaunchKernelGGL(k_gelu_back, dim3(nb((long)B * DH, 256)), dim3(256), 0, st, w.dh1, w.z1, B * DH);
    // hidden layer 1
    gemm(w.xh, DI, 1, w.dh1, DH, 0, grad + kOffW1, DH, DI, DH, B, acc, st);
    hipLaunchKernelGGL(k_colsum, dim3(1), dim3(128), 0, st, w.dh1, B, DH, grad + kOffB1, acc);
    return hipGetLastError();
}

static __global__ void k_fill(float* __restrict__ p, long n, float v)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t mlp_fill(float* p, long n, float v, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(nb(n, 256)), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}

hipError_t mlp_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                    int step, hipStream_t st)
{
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(nb(n, 256)), dim3(256), 0, st, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}


hipError_t mlp_norm_stats(const float* X, const float* T, long n, double* work, int nblocks, hipStream_t st)
{
    // work: nblocks x 48 partial sums, then the 48 means and 48 variances
    double* mean = work + (long)nblocks * kNormCols;
    double* var = mean + kNormCols;
    hipLaunchKernelGGL(k_norm_partial, dim3(nblocks), dim3(kNormCols * kNormLanes), 0, st, X, T, n, mean, 0, work);
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(64), 0, st, work, nblocks, (double)n, mean);
    hipLaunchKernelGGL(k_norm_partial, dim3(nblocks), dim3(kNormCols * kNormLanes), 0, st, X, T, n, mean, 1, work);
    hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(64), 0, st, work, nblocks, (double)(n - 1), var);
    return hipGetLastError();
}

}  // namespace grim
