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
// k_wgrad     weight gradient of one layer split over the batch (64 x 64 tiles x batch chunks, each
//             chunk's tile stored on its own), with the bias partials (FP32 column sums) of the chunk
// k_wgrad_reduce  the chunks of every layer added to the gradient buffer in a fixed order
// k_adam_pack Adam with bias correction on the FP32 master weights, gradient cleared, BF16 copies
//             of the weights rewritten in the row-major padded packs
// k_pack      FP32 master -> BF16 weights (row-major, zero-padded input and output widths)
// k_mse       loss and dL/dy of the mean squared error
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mlp_internal.h"

namespace srp {
namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

// 64 x 64 output tiles; K staged through LDS 128 at a time (every load of a chunk issued before
// the one barrier that precedes its products, so a chunk costs one memory latency)
constexpr int kTM = 64, kTN = 64, kTK = 128, kLdsK = kTK + 8;

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

// Rows [r0, r0 + 64) x k in [k0, k1) of a BF16 operand, loaded into registers (zeros outside
// [0, rows) x [k0, k1)) and then stored to lds[row][k - k0]: the two halves are separate so that
// the next chunk's loads are in flight during this chunk's products.  KMAJOR = false: the operand
// is stored [row][ld] (k contiguous); KMAJOR = true: stored [k][ld] (rows contiguous), scattered
// into the k-contiguous LDS layout.
template <bool KMAJOR>
__device__ __forceinline__ void load_tile(const uint16_t* __restrict__ src, int ld, int rows, int r0, int k0, int k1,
                                          uint16_t (&v)[4][8])
{
    const int tid = threadIdx.x;
    const bool vec = (ld % 8) == 0;
    if (!KMAJOR) {
        // 16 threads per row, 8 k each: 16 rows per pass, 4 passes
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int row = p * 16 + (tid >> 4), kc = (tid & 15) * 8;
            const int r = r0 + row, k = k0 + kc;
            const int valid = (r < rows && k < k1) ? min(8, k1 - k) : 0;
            load8(src + static_cast<int64_t>(r < rows ? r : 0) * ld + (k < k1 ? k : k0), valid, vec, v[p]);
        }
    } else {
        // 8 threads per k, 8 rows each: 32 k per pass, 4 passes
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int kk = p * 32 + (tid >> 3), rc = (tid & 7) * 8;
            const int k = k0 + kk, r = r0 + rc;
            const int valid = (k < k1 && r < rows) ? min(8, rows - r) : 0;
            load8(src + static_cast<int64_t>(k < k1 ? k : k0) * ld + (r < rows ? r : 0), valid, vec, v[p]);
        }
    }
}

template <bool KMAJOR>
__device__ __forceinline__ void store_tile(const uint16_t (&v)[4][8], uint16_t (*lds)[kLdsK])
{
    const int tid = threadIdx.x;
    if (!KMAJOR) {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int row = p * 16 + (tid >> 4), kc = (tid & 15) * 8;
            *reinterpret_cast<uint4*>(&lds[row][kc]) = *reinterpret_cast<const uint4*>(v[p]);
        }
    } else {
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const int kk = p * 32 + (tid >> 3), rc = (tid & 7) * 8;
#pragma unroll
            for (int i = 0; i < 8; ++i) lds[rc + i][kk] = v[p][i];
        }
    }
}

// The products of one staged chunk: wave (wm, wn) accumulates its 32 x 32 block over the chunk.
__device__ __forceinline__ void mfma_chunk(const uint16_t (*As)[kLdsK], const uint16_t (*Bs)[kLdsK], int wm, int wn,
                                           int lane, f32x16& acc)
{
#pragma unroll
    for (int ks = 0; ks < kTK; ks += 16) {
        // operand layouts of v_mfma_f32_32x32x16_bf16: lane l holds A[l%32][8(l/32)+j] and
        // B[8(l/32)+j][l%32], j = 0..7
        const int kq = ks + 8 * (lane >> 5);
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[wm * 32 + (lane & 31)][kq]);
        const bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bs[wn * 32 + (lane & 31)][kq]);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
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
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;

    uint16_t va[4][8], vb[4][8];
    load_tile<TA>(g.A, g.lda, g.M, m0, 0, min(g.K, kTK), va);   // A [m][k], or stored [k][m] when transposed
    load_tile<!TB>(g.B, g.ldb, g.N, n0, 0, min(g.K, kTK), vb);  // B stored [n][k] when transposed, else [k][n]
    for (int k0 = 0; k0 < g.K; k0 += kTK) {
        store_tile<TA>(va, As);
        store_tile<!TB>(vb, Bs);
        __syncthreads();
        const int k2 = k0 + kTK;
        if (k2 < g.K) {
            load_tile<TA>(g.A, g.lda, g.M, m0, k2, min(g.K, k2 + kTK), va);
            load_tile<!TB>(g.B, g.ldb, g.N, n0, k2, min(g.K, k2 + kTK), vb);
        }
        mfma_chunk(As, Bs, wm, wn, lane, acc);
        __syncthreads();
    }

    // D layout: lane l, register r -> row (r/4)*8 + (l/32)*4 + r%4, column l%32.  Every load the
    // epilogue needs is issued before its first store (the stores could alias them otherwise, which
    // would serialise sixteen memory round trips).
    const int n = n0 + wn * 32 + (lane & 31);
    if (n >= g.N) return;
    const int mb = m0 + wm * 32 + (lane >> 5) * 4;
    const float bn = g.bias ? g.bias[n] : 0.0f;
    if (g.epi == kEpiBackprop) {
        float zv[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int m = mb + (r >> 2) * 8 + (r & 3);
            zv[r] = m < g.M ? g.Z[static_cast<int64_t>(m) * g.ldz + n] : 0.0f;
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int m = mb + (r >> 2) * 8 + (r & 3);
            if (m >= g.M) continue;
            const float gz = acc[r] * silu_grad_f(zv[r]);
            if (g.C) g.C[static_cast<int64_t>(m) * g.ldc + n] = gz;
            g.Cb[static_cast<int64_t>(m) * g.ldcb + n] = f2bf(gz);
        }
    } else if (g.epi == kEpiAccumulate) {
        float cv[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int m = mb + (r >> 2) * 8 + (r & 3);
            cv[r] = m < g.M ? g.C[static_cast<int64_t>(m) * g.ldc + n] : 0.0f;
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int m = mb + (r >> 2) * 8 + (r & 3);
            if (m < g.M) g.C[static_cast<int64_t>(m) * g.ldc + n] = cv[r] + acc[r];
        }
    } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int m = mb + (r >> 2) * 8 + (r & 3);
            if (m >= g.M) continue;
            const float z = g.bias ? acc[r] + bn : acc[r];
            if (g.epi == kEpiStore) {
                g.C[static_cast<int64_t>(m) * g.ldc + n] = z;
            } else {  // kEpiHidden
                if (g.C) g.C[static_cast<int64_t>(m) * g.ldc + n] = z;
                g.Cb[static_cast<int64_t>(m) * g.ldcb + n] = f2bf(silu_f(z));
            }
        }
    }
}

// Weight gradient of one layer, split over the batch: dW[m][n] = sum_k G[k][m] A[k][n] with G the
// BF16 back-propagated gradient [K][ldg] and A the layer's BF16 input [K][lda]; workgroup (x, y, z)
// computes the 64 x 64 tile (y, x) over batch rows [z kc, (z + 1) kc) and stores it to
// part[z][M][N] (no atomics: the chunks are added in a fixed order by k_wgrad_reduce).  Workgroups of
// tile column 0 also sum the FP32 gradient Gf [K][ldgf] over their rows: the bias partial
// bpart[z][M].
__global__ __launch_bounds__(256) void k_wgrad(WgradArgs g)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[kTM][kLdsK];  // [m][k]
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kTN][kLdsK];  // [n][k]
    __shared__ float bsum[4][kTM];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int m0 = blockIdx.y * kTM, n0 = blockIdx.x * kTN;
    const int kbeg = blockIdx.z * g.kc;
    const int kend = min(g.K, kbeg + g.kc);
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;

    uint16_t va[4][8], vb[4][8];
    if (kbeg < kend) {
        load_tile<true>(g.G, g.ldg, g.M, m0, kbeg, min(kend, kbeg + kTK), va);  // G stored [k][m]
        load_tile<true>(g.A, g.lda, g.N, n0, kbeg, min(kend, kbeg + kTK), vb);  // A stored [k][n]
    }
    for (int k0 = kbeg; k0 < kend; k0 += kTK) {
        store_tile<true>(va, As);
        store_tile<true>(vb, Bs);
        __syncthreads();
        const int k2 = k0 + kTK;
        if (k2 < kend) {
            load_tile<true>(g.G, g.ldg, g.M, m0, k2, min(kend, k2 + kTK), va);
            load_tile<true>(g.A, g.lda, g.N, n0, k2, min(kend, k2 + kTK), vb);
        }
        mfma_chunk(As, Bs, wm, wn, lane, acc);
        __syncthreads();
    }
    float* out = g.part + static_cast<int64_t>(blockIdx.z) * g.M * g.N;
    const int n = n0 + wn * 32 + (lane & 31);
    if (n < g.N) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int m = m0 + wm * 32 + (r >> 2) * 8 + (lane >> 5) * 4 + (r & 3);
            if (m < g.M) out[static_cast<int64_t>(m) * g.N + n] = acc[r];
        }
    }
    if (blockIdx.x == 0 && g.Gf) {
        // bias partial: column m of the FP32 gradient over this workgroup's rows, in 4 interleaved
        // row groups, then the 4 group sums in order
        const int mm = tid & 63, grp = tid >> 6;
        const int m = m0 + mm;
        float s = 0.0f;
        if (m < g.M)
#pragma unroll 8
            for (int k = kbeg + grp; k < kend; k += 4) s += g.Gf[static_cast<int64_t>(k) * g.ldgf + m];
        bsum[grp][mm] = s;
        __syncthreads();
        if (grp == 0 && m < g.M)
            g.bpart[static_cast<int64_t>(blockIdx.z) * g.M + m] = ((bsum[0][mm] + bsum[1][mm]) + bsum[2][mm]) + bsum[3][mm];
    }
}

// grad[w_off + i] += sum_z part[z][i] and grad[b_off + m] += sum_z bpart[z][m] for every layer, the
// chunks in order (deterministic)
__global__ void k_wgrad_reduce(ReduceArgs r)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= r.total) return;
    int l = 0;
    while (l + 1 < r.layers && i >= r.first[l + 1]) ++l;
    const int64_t j = i - r.first[l];
    const int64_t nw = static_cast<int64_t>(r.fout[l]) * r.fin[l];
    const int S = r.splits[l];
    if (j < nw) {
        const float* p = r.part + r.part_off[l] + j;
        float s = 0.0f;
#pragma unroll 8
        for (int z = 0; z < S; ++z) s += p[static_cast<int64_t>(z) * nw];
        r.grad[r.w_off[l] + j] += s;
    } else {
        const int64_t m = j - nw;
        const float* p = r.bpart + r.bpart_off[l] + m;
        float s = 0.0f;
#pragma unroll 8
        for (int z = 0; z < S; ++z) s += p[static_cast<int64_t>(z) * r.fout[l]];
        r.grad[r.b_off[l] + m] += s;
    }
}

// Adam on every parameter (FP32 masters), the gradient cleared, and each weight's BF16 copy
// written to its place in the row-major padded packs the GEMMs read (padding stays zero)
__global__ void k_adam_pack(AdamPackArgs a)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= a.P) return;
    const float g = a.g[i];
    const float mi = a.b1 * a.m[i] + (1.0f - a.b1) * g;
    const float vi = a.b2 * a.v[i] + (1.0f - a.b2) * g * g;
    a.m[i] = mi;
    a.v[i] = vi;
    const float p = a.p[i] - a.lr * (mi / a.c1) / (sqrtf(vi / a.c2) + a.eps);
    a.p[i] = p;
    a.g[i] = 0.0f;
    int l = 0;
    while (l + 1 < a.layers && i >= a.w_off[l + 1]) ++l;
    const int64_t j = i - a.w_off[l];
    const int64_t nw = static_cast<int64_t>(a.fout[l]) * a.fin[l];
    if (j < nw) {
        const int r = static_cast<int>(j / a.fin[l]), c = static_cast<int>(j % a.fin[l]);
        a.wb[a.wb_off[l] + static_cast<int64_t>(r) * a.fin_pad[l] + c] = f2bf(p);
    }
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

hipError_t launch_wgrad(const WgradArgs& g, int splits, hipStream_t stream)
{
    if (g.M <= 0 || g.N <= 0) return hipSuccess;
    dim3 grid((g.N + kTN - 1) / kTN, (g.M + kTM - 1) / kTM, splits);
    hipLaunchKernelGGL(k_wgrad, grid, dim3(256), 0, stream, g);
    return hipGetLastError();
}

hipError_t launch_wgrad_reduce(const ReduceArgs& r, hipStream_t stream)
{
    if (r.total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(static_cast<unsigned>((r.total + 255) / 256)), dim3(256), 0, stream, r);
    return hipGetLastError();
}

hipError_t launch_adam_pack(const AdamPackArgs& a, hipStream_t stream)
{
    hipLaunchKernelGGL(k_adam_pack, dim3(static_cast<unsigned>((a.P + 255) / 256)), dim3(256), 0, stream, a);
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
