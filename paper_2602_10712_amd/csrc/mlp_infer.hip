// Fused force-surrogate inference for gfx950: all layers of the MLP in one kernel.
//
// Layout trick.  Every layer is computed transposed, H^T = W . A^T, on v_mfma_f32_32x32x16_bf16
// with the batch as the MFMA N dimension.  Lane l of a wavefront then holds one query (column
// l % 32) in both the accumulator layout (rows (r/4)*8 + (l/32)*4 + r%4 of a 32-row block,
// r = 0..15) and the B-operand layout (8 consecutive K slots 8*(l/32) + j of a 16-wide K block),
// so a layer's output becomes the next layer's B operand without leaving registers: accumulator
// registers 8q..8q+7 of row block mb are K block 2*mb + q of the next layer, whose slot s stands
// for feature 16*kb + perm(s) with perm = [0 1 2 3 8 9 10 11 4 5 6 7 12 13 14 15].  The weights are
// stored in that permuted order, already split into the 64-lane A-operand pieces (16 bytes per
// lane per 32 x 16 block), so a wavefront reads its A operand from LDS with one ds_read_b128.
//
// Work split.  A workgroup of 4 wavefronts (one per SIMD) takes 256 queries, 64 per wavefront
// (two 32-query column blocks share every A operand).  Each layer's weights (at most 128 KB) are
// staged in LDS; activations (BF16) and accumulators (FP32) stay in registers.  Bias and SiLU are
// applied in FP32 in the epilogue, and activations are rounded to BF16 (nearest even).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mlp_internal.h"

namespace srp {
namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

constexpr int kW = 256;             // hidden width served by the fused kernel
constexpr int kMB = kW / 32;        // 32-row blocks of a hidden layer
constexpr int kKB = kW / 16;        // 16-wide K blocks of a hidden layer
constexpr int kQ = 64;              // queries per wavefront
constexpr int kLdsBytes = kMB * kKB * 64 * 16;  // one hidden layer: 128 KiB

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return static_cast<uint16_t>((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

__device__ __forceinline__ int kperm(int s)
{
    const int h = s >> 3, j = s & 7;
    return j < 4 ? 4 * h + j : 8 + 4 * h + (j - 4);
}

// Packs layer weights W (FP32 master [out][in]) into A-operand pieces:
// dst[((mb * KB + kb) * 64 + lane) * 8 + j] = W[mb*32 + lane%32][k], k = 16 kb + p(8 (lane/32) + j),
// p = identity for the network input layer, kperm for the others; zero outside [out] x [in].
__global__ void k_pack_mfma(const float* __restrict__ W, int out, int in, int MB, int KB, int identity,
                            uint16_t* __restrict__ dst)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= static_cast<int64_t>(MB) * KB * 512) return;
    const int j = static_cast<int>(i & 7);
    const int lane = static_cast<int>((i >> 3) & 63);
    const int blk = static_cast<int>(i >> 9);
    const int mb = blk / KB, kb = blk % KB;
    const int s = 8 * (lane >> 5) + j;
    const int m = mb * 32 + (lane & 31);
    const int k = 16 * kb + (identity ? s : kperm(s));
    dst[i] = (m < out && k < in) ? f2bf(W[static_cast<int64_t>(m) * in + k]) : static_cast<uint16_t>(0);
}

__device__ __forceinline__ void stage(uint4* __restrict__ lds, const uint4* __restrict__ src, int n16)
{
    for (int i = threadIdx.x; i < n16; i += 256) lds[i] = src[i];
}

__device__ __forceinline__ float silu_fast(float z) { return z * __frcp_rn(1.0f + __expf(-z)); }

// Bias + SiLU of the accumulators of row block mb into B-operand pieces 2*mb, 2*mb + 1.
__device__ __forceinline__ void epilogue(const f32x16& acc, const float* __restrict__ bias, int mb, int h,
                                         bf16x8& lo, bf16x8& hi)
{
    uint16_t v[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int feat = mb * 32 + (r >> 2) * 8 + h * 4 + (r & 3);
        v[r] = f2bf(silu_fast(acc[r] + bias[feat]));
    }
    lo = *reinterpret_cast<const bf16x8*>(&v[0]);
    hi = *reinterpret_cast<const bf16x8*>(&v[8]);
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_mlp_infer(
    const float* __restrict__ x, int32_t N, int32_t n_in, int32_t n_out, const uint16_t* __restrict__ wf,
    const int64_t* __restrict__ wf_off, const float* __restrict__ params, const int64_t* __restrict__ b_off,
    int32_t depth, float* __restrict__ y)
{
    __shared__ uint4 lds[kLdsBytes / 16];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int h = lane >> 5, c = lane & 31;
    const int64_t q0 = static_cast<int64_t>(blockIdx.x) * (4 * kQ) + wave * kQ;

    // ---- layer 0: input (n_in <= 16, one K block, identity order) -------------------------------
    bf16x8 xin[2];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        const int64_t q = q0 + cb * 32 + c;
        uint16_t v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int f = 8 * h + j;
            v[j] = (q < N && f < n_in) ? f2bf(x[q * n_in + f]) : static_cast<uint16_t>(0);
        }
        xin[cb] = *reinterpret_cast<const bf16x8*>(v);
    }
    stage(lds, reinterpret_cast<const uint4*>(wf + wf_off[0]), kMB * 1 * 64);
    __syncthreads();
    bf16x8 act[2][kKB];
    {
        const float* bias = params + b_off[0];
#pragma unroll
        for (int mb = 0; mb < kMB; ++mb) {
            const bf16x8 a = *reinterpret_cast<const bf16x8*>(&lds[mb * 64 + lane]);
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                f32x16 acc = {};
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, xin[cb], acc, 0, 0, 0);
                epilogue(acc, bias, mb, h, act[cb][2 * mb], act[cb][2 * mb + 1]);
            }
        }
    }
    __syncthreads();

    // ---- hidden layers 1 .. depth-1 ----------------------------------------------------------------
    for (int l = 1; l < depth; ++l) {
        stage(lds, reinterpret_cast<const uint4*>(wf + wf_off[l]), kMB * kKB * 64);
        __syncthreads();
        f32x16 acc[2][kMB];
#pragma unroll
        for (int mb = 0; mb < kMB; ++mb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[cb][mb][r] = 0.0f;
#pragma unroll
        for (int kb = 0; kb < kKB; ++kb) {
#pragma unroll
            for (int mb = 0; mb < kMB; ++mb) {
                const bf16x8 a = *reinterpret_cast<const bf16x8*>(&lds[(mb * kKB + kb) * 64 + lane]);
                acc[0][mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, act[0][kb], acc[0][mb], 0, 0, 0);
                acc[1][mb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, act[1][kb], acc[1][mb], 0, 0, 0);
            }
        }
        const float* bias = params + b_off[l];
#pragma unroll
        for (int mb = 0; mb < kMB; ++mb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) epilogue(acc[cb][mb], bias, mb, h, act[cb][2 * mb], act[cb][2 * mb + 1]);
        __syncthreads();
    }

    // ---- output layer (n_out <= 32: one row block) -----------------------------------------------
    stage(lds, reinterpret_cast<const uint4*>(wf + wf_off[depth]), kKB * 64);
    __syncthreads();
    f32x16 out[2] = {};
#pragma unroll
    for (int kb = 0; kb < kKB; ++kb) {
        const bf16x8 a = *reinterpret_cast<const bf16x8*>(&lds[kb * 64 + lane]);
        out[0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, act[0][kb], out[0], 0, 0, 0);
        out[1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, act[1][kb], out[1], 0, 0, 0);
    }
    const float* bias = params + b_off[depth];
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) {
        const int64_t q = q0 + cb * 32 + c;
        if (q >= N) continue;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int o = (r >> 2) * 8 + h * 4 + (r & 3);
            if (o < n_out) y[q * n_out + o] = out[cb][r] + bias[o];
        }
    }
}

}  // namespace

bool mlp_fused_supported(int n_in, int width, int depth, int n_out)
{
    return width == kW && n_in <= 16 && n_out <= 32 && depth >= 1;
}

int64_t mlp_fused_layer_elems(int layer, int depth)
{
    if (layer == 0) return static_cast<int64_t>(kMB) * 1 * 512;
    if (layer == depth) return static_cast<int64_t>(1) * kKB * 512;
    return static_cast<int64_t>(kMB) * kKB * 512;
}

hipError_t launch_pack_mfma(const float* W, int out, int in, int layer, int depth, uint16_t* dst, hipStream_t stream)
{
    const int MB = layer == depth ? 1 : kMB;
    const int KB = layer == 0 ? 1 : kKB;
    const int64_t n = static_cast<int64_t>(MB) * KB * 512;
    hipLaunchKernelGGL(k_pack_mfma, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, stream, W, out, in, MB,
                       KB, layer == 0 ? 1 : 0, dst);
    return hipGetLastError();
}

hipError_t launch_mlp_infer(const float* x, int32_t N, const uint16_t* wf, const int64_t* wf_off_dev,
                            const float* params, const int64_t* b_off_dev, int n_in, int depth, int n_out, float* y,
                            hipStream_t stream)
{
    if (N <= 0) return hipSuccess;
    const unsigned blocks = static_cast<unsigned>((static_cast<int64_t>(N) + 4 * kQ - 1) / (4 * kQ));
    hipLaunchKernelGGL(k_mlp_infer, dim3(blocks), dim3(256), 0, stream, x, N, n_in, n_out, wf, wf_off_dev, params,
                       b_off_dev, depth, y);
    return hipGetLastError();
}

}  // namespace srp
