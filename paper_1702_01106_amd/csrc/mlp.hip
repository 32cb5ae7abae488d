// The learned initial guess: a 32 -> 128 -> 128 -> 16 GELU network.
//
// Inference (a14) is BF16 on the matrix cores with FP32 accumulation
// (v_mfma_f32_32x32x8_bf16): a block of four waves takes 128 rows, each wave
// 32 rows; the transposed BF16 weights sit in LDS, and each hidden layer goes
// through LDS once to turn the MFMA result layout into the next layer's
// A-operand layout.  Training (a15) is FP32 on the vector units: a tiled
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

constexpr int kRowsPerWave = 32;
constexpr int kWaves = 4;
constexpr int kRowsPerBlock = kRowsPerWave * kWaves;
constexpr int kHStride = DH + 8;  // bf16 elements per LDS row (padding spreads banks)

// Accumulator element r of lane l sits at row 8 (r/4) + 4 (l/32) + r%4, column l%32.
__device__ __forceinline__ int acc_row(int r, int lane) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

__global__ __launch_bounds__(256) void k_mlp_infer(const float* __restrict__ X, long n, const float* __restrict__ p,
                                                   const unsigned short* __restrict__ w1t,
                                                   const unsigned short* __restrict__ w2t,
                                                   const unsigned short* __restrict__ w3t, float* __restrict__ Y)
{
    __shared__ unsigned short sW1[DH * DI];
    __shared__ unsigned short sW2[DH * DH];
    __shared__ unsigned short sW3[32 * DH];
    __shared__ unsigned short sH[kWaves][kRowsPerWave * kHStride];
    __shared__ float sB1[DH], sB2[DH], sB3[32], sXm[DI], sXs[DI], sYs[32];

    const int tid = threadIdx.x;
    for (int i = tid; i < DH * DI; i += 256) sW1[i] = w1t[i];
    for (int i = tid; i < DH * DH; i += 256) sW2[i] = w2t[i];
    for (int i = tid; i < 32 * DH; i += 256) sW3[i] = w3t[i];
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

    const int wave = tid >> 6, lane = tid & 63;
    const int col = lane & 31, half = lane >> 5;
    unsigned short* H = sH[wave];
    const long ntiles = (n + kRowsPerBlock - 1) / kRowsPerBlock;
    for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const long row0 = tile * kRowsPerBlock + (long)wave * kRowsPerWave;
        // ---- layer 1: A = normalised input rows (K = 32, four k-steps of 8)
        bf16x4 a1[4];
        {
            const long row = row0 + col;
#pragma unroll
            for (int s = 0; s < 4; ++s)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k = 8 * s + 4 * half + e;
                    const float x = row < n ? (X[row * DI + k] - sXm[k]) * sXs[k] : 0.0f;
                    a1[s][e] = (short)to_bf16(x);
                }
        }
#pragma unroll
        for (int t = 0; t < DH / 32; ++t) {
            f32x16 acc = {};
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                bf16x4 b;
#pragma unroll
                for (int e = 0; e < 4; ++e) b[e] = (short)sW1[(32 * t + col) * DI + 8 * s + 4 * half + e];
                acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a1[s], b, acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 16; ++r)
                H[acc_row(r, lane) * kHStride + 32 * t + col] = to_bf16(gelu(acc[r] + sB1[32 * t + col]));
        }
        __syncthreads();  // hidden activations visible in LDS
        // ---- layer 2: K = 128 (sixteen k-steps)
        f32x16 acc2[DH / 32];
#pragma unroll
        for (int t = 0; t < DH / 32; ++t) acc2[t] = f32x16{};
#pragma unroll
        for (int s = 0; s < DH / 8; ++s) {
            bf16x4 a;
#pragma unroll
            for (int e = 0; e < 4; ++e) a[e] = (short)H[col * kHStride + 8 * s + 4 * half + e];
#pragma unroll
            for (int t = 0; t < DH / 32; ++t) {
                bf16x4 b;
#pragma unroll
                for (int e = 0; e < 4; ++e) b[e] = (short)sW2[(32 * t + col) * DH + 8 * s + 4 * half + e];
                acc2[t] = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc2[t], 0, 0, 0);
            }
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < DH / 32; ++t)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                H[acc_row(r, lane) * kHStride + 32 * t + col] = to_bf16(gelu(acc2[t][r] + sB2[32 * t + col]));
        __syncthreads();
        // ---- layer 3: one 32 x 32 output tile (columns >= 16 are zero padding)
        f32x16 acc3 = {};
#pragma unroll
        for (int s = 0; s < DH / 8; ++s) {
            bf16x4 a, b;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                a[e] = (short)H[col * kHStride + 8 * s + 4 * half + e];
                b[e] = (short)sW3[col * DH + 8 * s + 4 * half + e];
            }
            acc3 = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, acc3, 0, 0, 0);
        }
        if (col < DO) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const long row = row0 + acc_row(r, lane);
                if (row < n) Y[row * DO + col] = (acc3[r] + sB3[col]) * sYs[col];
            }
        }
        __syncthreads();  // the next tile reuses H
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
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nb * DO) return;
    const int j = t % DO;
    float g = 0.0f;
    if (dY) {
        g = dY[t] * ys[j];
    } else if (j < n_used && ys[j] != 0.0f) {
        // loss in normalised output units: ((y - t) / y_scale)^2; an output
        // with y_scale 0 is held at zero and carries no loss
        const float d = (O[t] + b3[j]) - TB[t] / ys[j];
        g = 2.0f * d * inv_count;
        atomicAdd(loss, (double)d * (double)d * (double)inv_count);
    }
    dO[t] = g;
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
    const long tiles = (n + kRowsPerBlock - 1) / kRowsPerBlock;
    const unsigned grid = (unsigned)std::min<long>(tiles, 1024);
    hipLaunchKernelGGL(k_mlp_infer, dim3(grid), dim3(256), 0, st, X, n, params, w1t, w2t, w3t, Y);
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

hipError_t mlp_adam(float* p, const float* g, float* m, float* v, int n, float lr, float b1, float b2, float eps,
                    int step, hipStream_t st)
{
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(nb(n, 256)), dim3(256), 0, st, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace grim
