// Force-surrogate MLP kernels for gfx950 (paper Sec. 3.3: a neural proxy maps light direction and
// design parameters to force; trained with Adam on simulator samples).
//
// Numerics: BF16 operands (round to nearest even), FP32 accumulation on the matrix cores
// (v_mfma_f32_32x32x16_bf16), FP32 bias, SiLU and loss gradient, BF16 activations and BF16
// back-propagated gradients between layers, FP32 master weights and Adam state.
//
// k_gemm      C[M][N] = op(A)[M][K] . op(B)[K][N] on 64 x 64 tiles (4 wavefronts, one 32 x 32 MFMA
//             tile each), K staged through LDS 32 at a time, with the epilogue of the layer fused:
//             bias + SiLU (hidden forward), bias (output), x SiLU'(z) (back-propagation), += (weight
//             gradients over the batch).
// k_colsum_*  bias gradients (column sums over the batch, fixed order)
// k_adam      Adam with bias correction on the FP32 master weights
// k_pack      FP32 master -> BF16 weights (row-major, zero-padded input and output widths)
// k_mse       loss and dL/dy of the mean squared error
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mlp_internal.h"

namespace srp {
namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

constexpr int kTM = 64, kTN = 64, kTK = 32, kLdsK = kTK + 8;

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>((u >> 16) | 0x40u);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

__device__ __forceinline__ float silu_f(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float silu_grad_f(float z)
{
    const float s = 1.0f / (1.0f + expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

// 8 consecutive bf16 elements p[i], i < valid (zero beyond), vector load when aligned and whole
__device__ __forceinline__ void load8(const uint16_t* __restrict__ p, int valid, bool vec, uint16_t out[8])
{
    if (vec && valid >= 8) {
        const uint4 v = *reinterpret_cast<const uint4*>(p);
        const uint16_t* s = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
        for (int i = 0; i < 8; ++i) out[i] = s[i];
    } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) out[i] = i < valid ? p[i] : static_cast<uint16_t>(0);
    }
}

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[kTM][kLdsK];  // [m][k]
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kTN][kLdsK];  // [n][k]
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int m0 = blockIdx.y * kTM, n0 = blockIdx.x * kTN;
    const bool vecA = (g.lda % 8) == 0, vecB = (g.ldb % 8) == 0;
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;

    for (int k0 = 0; k0 < g.K; k0 += kTK) {
        uint16_t v[8];
        if (!TA) {  // A[m][k], contiguous in k
            const int row = tid >> 2, kc = (tid & 3) * 8;
            const int m = m0 + row, k = k0 + kc;
            const int valid = (m < g.M) ? min(8, g.K - k) : 0;
            load8(g.A + static_cast<int64_t>(m < g.M ? m : 0) * g.lda + (k < g.K ? k : 0), valid, vecA, v);
            *reinterpret_cast<uint4*>(&As[row][kc]) = *reinterpret_cast<const uint4*>(v);
        } else {  // A stored [k][m]: 8 consecutive m of one k, scattered into As
            const int kk = tid >> 3, mc = (tid & 7) * 8;
            const int k = k0 + kk, m = m0 + mc;
            const int valid = (k < g.K) ? min(8, g.M - m) : 0;
            load8(g.A + static_cast<int64_t>(k < g.K ? k : 0) * g.lda + (m < g.M ? m : 0), valid, vecA, v);
#pragma unroll
            for (int i = 0; i < 8; ++i) As[mc + i][kk] = v[i];
        }
        if (TB) {  // B stored [n][k], contiguous in k
            const int row = tid >> 2, kc = (tid & 3) * 8;
            const int n = n0 + row, k = k0 + kc;
            const int valid = (n < g.N) ? min(8, g.K - k) : 0;
            load8(g.B + static_cast<int64_t>(n < g.N ? n : 0) * g.ldb + (k < g.K ? k : 0), valid, vecB, v);
            *reinterpret_cast<uint4*>(&Bs[row][kc]) = *reinterpret_cast<const uint4*>(v);
        } else {  // B stored [k][n]: 8 consecutive n of one k
            const int kk = tid >> 3, nc = (tid & 7) * 8;
            const int k = k0 + kk, n = n0 + nc;
            const int valid = (k < g.K) ? min(8, g.N - n) : 0;
            load8(g.B + static_cast<int64_t>(k < g.K ? k : 0) * g.ldb + (n < g.N ? n : 0), valid, vecB, v);
#pragma unroll
            for (int i = 0; i < 8; ++i) Bs[nc + i][kk] = v[i];
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < kTK; ks += 16) {
            // operand layouts of v_mfma_f32_32x32x16_bf16: lane l holds A[l%32][8(l/32)+j] and
            // B[8(l/32)+j][l%32], j = 0..7
            const int kq = ks + 8 * (lane >> 5);
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[wm * 32 + (lane & 31)][kq]);
            const bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bs[wn * 32 + (lane & 31)][kq]);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }

    // D layout: lane l, register r -> row (r/4)*8 + (l/32)*4 + r%4, column l%32
    const int n = n0 + wn * 32 + (lane & 31);
    if (n >= g.N) return;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int m = m0 + wm * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
        if (m >= g.M) continue;
        float x = acc[r];
        switch (g.epi) {
            case kEpiStore:
                if (g.bias) x += g.bias[n];
                g.C[static_cast<int64_t>(m) * g.ldc + n] = x;
                break;
            case kEpiHidden: {
                const float z = x + g.bias[n];
                if (g.C) g.C[static_cast<int64_t>(m) * g.ldc + n] = z;
                g.Cb[static_cast<int64_t>(m) * g.ldcb + n] = f2bf(silu_f(z));
                break;
            }
            case kEpiBackprop: {
                const float gz = x * silu_grad_f(g.Z[static_cast<int64_t>(m) * g.ldz + n]);
                if (g.C) g.C[static_cast<int64_t>(m) * g.ldc + n] = gz;
                g.Cb[static_cast<int64_t>(m) * g.ldcb + n] = f2bf(gz);
                break;
            }
            default:  // kEpiAccumulate
                g.C[static_cast<int64_t>(m) * g.ldc + n] += x;
                break;
        }
    }
}

// bias gradients: out[c] += sum_r G[r][c] (FP32) in two fixed-order passes: chunk sums, then the
// sum of the chunk sums
constexpr int kColChunks = 64;
__global__ void k_colsum_part(const float* __restrict__ G, int64_t rows, int cols, int ldg, float* __restrict__ part)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    const int64_t per = (rows + kColChunks - 1) / kColChunks;
    const int64_t r0 = blockIdx.y * per, r1 = r0 + per < rows ? r0 + per : rows;
    float s = 0.0f;
    for (int64_t r = r0; r < r1; ++r) s += G[r * ldg + c];
    part[static_cast<int64_t>(blockIdx.y) * cols + c] = s;
}

__global__ void k_colsum_final(const float* __restrict__ part, int cols, float* __restrict__ out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float s = 0.0f;
    for (int q = 0; q < kColChunks; ++q) s += part[static_cast<int64_t>(q) * cols + c];
    out[c] += s;
}

// FP32 -> BF16 of a [rows][cols] matrix into a [rows][ld_out] matrix, zero-padding columns
__global__ void k_to_bf16(const float* __restrict__ in, int64_t rows, int cols, int ld_in, uint16_t* __restrict__ out,
                          int ld_out)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= rows * ld_out) return;
    const int64_t r = i / ld_out;
    const int c = static_cast<int>(i % ld_out);
    out[i] = c < cols ? f2bf(in[r * ld_in + c]) : static_cast<uint16_t>(0);
}

__global__ void k_fill_f32(float* __restrict__ p, int64_t n, float v)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ gr, float* __restrict__ m, float* __restrict__ v,
                       int64_t n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = gr[i];
    const float mi = b1 * m[i] + (1.0f - b1) * g;
    const float vi = b2 * v[i] + (1.0f - b2) * g * g;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// weight matrix of one layer: master FP32 [out][in] -> BF16 [out_pad][in_pad] (zeros outside)
__global__ void k_pack(const float* __restrict__ W, int out, int in, uint16_t* __restrict__ Wb, int out_pad, int in_pad)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= static_cast<int64_t>(out_pad) * in_pad) return;
    const int r = static_cast<int>(i / in_pad), c = static_cast<int>(i % in_pad);
    Wb[i] = (r < out && c < in) ? f2bf(W[static_cast<int64_t>(r) * in + c]) : static_cast<uint16_t>(0);
}

// mean squared error over rows x cols: per-block partial losses (FP64) and dL/dy = 2 (y - t) / count
__global__ void k_mse(const float* __restrict__ y, const float* __restrict__ t, int64_t count, float* __restrict__ gy,
                      double* __restrict__ partial)
{
    __shared__ double s[256];
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    double e = 0.0;
    if (i < count) {
        const float d = y[i] - t[i];
        gy[i] = 2.0f * d / static_cast<float>(count);
        e = static_cast<double>(d) * d;
    }
    s[threadIdx.x] = e;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = s[0];
}

__global__ void k_sum_partials(const double* __restrict__ partial, int n, int64_t count, double* __restrict__ out)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += partial[i];
        *out = s / static_cast<double>(count);
    }
}

}  // namespace

hipError_t launch_gemm(const GemmArgs& g, bool ta, bool tb, hipStream_t stream)
{
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    dim3 grid((g.N + kTN - 1) / kTN, (g.M + kTM - 1) / kTM);
    if (!ta && !tb)
        hipLaunchKernelGGL((k_gemm<false, false>), grid, dim3(256), 0, stream, g);
    else if (!ta && tb)
        hipLaunchKernelGGL((k_gemm<false, true>), grid, dim3(256), 0, stream, g);
    else if (ta && !tb)
        hipLaunchKernelGGL((k_gemm<true, false>), grid, dim3(256), 0, stream, g);
    else
        hipLaunchKernelGGL((k_gemm<true, true>), grid, dim3(256), 0, stream, g);
    return hipGetLastError();
}

hipError_t launch_colsum(const float* G, int64_t rows, int cols, int ldg, float* part, float* out, hipStream_t stream)
{
    hipLaunchKernelGGL(k_colsum_part, dim3((cols + 63) / 64, kColChunks), dim3(64), 0, stream, G, rows, cols, ldg, part);
    hipLaunchKernelGGL(k_colsum_final, dim3((cols + 63) / 64), dim3(64), 0, stream, part, cols, out);
    return hipGetLastError();
}

hipError_t launch_to_bf16(const float* in, int64_t rows, int cols, int ld_in, uint16_t* out, int ld_out,
                          hipStream_t stream)
{
    const int64_t n = rows * ld_out;
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_to_bf16, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, stream, in, rows, cols,
                       ld_in, out, ld_out);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, int64_t n, float v, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f32, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, stream, p, n, v);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                       float c1, float c2, hipStream_t stream)
{
    hipLaunchKernelGGL(k_adam, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, stream, p, g, m, v, n, lr,
                       b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_pack(const float* W, int out, int in, uint16_t* Wb, int out_pad, int in_pad, hipStream_t stream)
{
    const int64_t n = static_cast<int64_t>(out_pad) * in_pad;
    hipLaunchKernelGGL(k_pack, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, stream, W, out, in, Wb,
                       out_pad, in_pad);
    return hipGetLastError();
}

hipError_t launch_mse(const float* y, const float* t, int64_t count, float* gy, double* partial, double* loss,
                      hipStream_t stream)
{
    const int blocks = static_cast<int>((count + 255) / 256);
    hipLaunchKernelGGL(k_mse, dim3(blocks), dim3(256), 0, stream, y, t, count, gy, partial);
    hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(1), 0, stream, partial, blocks, count, loss);
    return hipGetLastError();
}

}  // namespace srp
