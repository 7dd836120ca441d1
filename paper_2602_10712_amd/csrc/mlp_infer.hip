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
// Work split.  A persistent workgroup of 8 wavefronts (two per SIMD, up to 256 registers each)
// takes tiles of 256 queries, one 32-query column block per wavefront.  A hidden layer is computed
// one 32-row block at a time over all 16 K blocks, so one accumulator is live (plus the previous
// block's pre-activations) and the bias + SiLU epilogue of one row block runs between the MFMAs
// of the next, while the other wavefront of the SIMD keeps the matrix core busy; input and output
// activations of the layer (BF16) stay in registers.  (The kernel is written for NCB column blocks
// per wavefront; NCB = 2 with one wavefront per SIMD shares each A operand between two MFMAs but
// measured slower.)
//
// Weight pipeline.  The input layer, the output layer and all biases stay in LDS for the whole
// kernel.  A hidden layer (128 KiB) is streamed in two 64 KiB halves (row blocks 0-3 and 4-7)
// through two LDS buffers: while the wavefronts multiply with one half, every thread loads its
// 8 x 16 bytes of the next half into registers and writes them to the other buffer afterwards,
// so one barrier per half separates the buffer swaps and the L2 latency hides behind the MFMAs.
// Bias and SiLU are applied in FP32 in the epilogue, and activations are rounded to BF16 (nearest
// even, packed conversion).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdint.h>

#include "mlp_internal.h"

namespace srp {
namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(2))) __bf16 bf16x2;
typedef __attribute__((ext_vector_type(2))) float f32x2;
typedef __attribute__((ext_vector_type(16))) float f32x16;

constexpr int kW = 256;             // hidden width served by the fused kernel
constexpr int kMB = kW / 32;        // 32-row blocks of a hidden layer
constexpr int kKB = kW / 16;        // 16-wide K blocks of a hidden layer
constexpr int kTileQ = 256;         // queries per workgroup tile
constexpr int kHalfMB = kMB / 2;    // row blocks per streamed half layer
constexpr int kHalfU4 = kHalfMB * kKB * 64;     // one half layer: 64 KiB in 16-byte pieces
constexpr int kInU4 = kMB * 64;                 // input layer (one K block): 8 KiB
constexpr int kOutU4 = kKB * 64;                // output layer (one row block): 16 KiB
constexpr int kLdsU4Max = 10240;                // 160 KiB
constexpr int kMaxDepth = (kLdsU4Max - 2 * kHalfU4 - kInU4 - kOutU4) / 64 - 1;  // bias rows left

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

__device__ __forceinline__ float silu(float z) { return z * __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

__device__ __forceinline__ bf16x8 pack8(const float* v)
{
    const bf16x2 p0 = __builtin_convertvector((f32x2){v[0], v[1]}, bf16x2);
    const bf16x2 p1 = __builtin_convertvector((f32x2){v[2], v[3]}, bf16x2);
    const bf16x2 p2 = __builtin_convertvector((f32x2){v[4], v[5]}, bf16x2);
    const bf16x2 p3 = __builtin_convertvector((f32x2){v[6], v[7]}, bf16x2);
    return __builtin_shufflevector(__builtin_shufflevector(p0, p1, 0, 1, 2, 3),
                                   __builtin_shufflevector(p2, p3, 0, 1, 2, 3), 0, 1, 2, 3, 4, 5, 6, 7);
}

__device__ __forceinline__ f32x16 mfma(const bf16x8& a, const bf16x8& b, const f32x16& c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// Bias of row block mb in accumulator order (LDS): the MFMA chain of the block starts from it.
__device__ __forceinline__ f32x16 bias_acc(const float* __restrict__ bias, int mb, int h)
{
    f32x16 r;
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        const float4 b = *reinterpret_cast<const float4*>(&bias[mb * 32 + g * 8 + h * 4]);
        r[4 * g + 0] = b.x;
        r[4 * g + 1] = b.y;
        r[4 * g + 2] = b.z;
        r[4 * g + 3] = b.w;
    }
    return r;
}

// SiLU of pre-activations (bias included) into B-operand pieces 2*mb, 2*mb + 1, one stage at a time
// over the 16 values so that the transcendental latencies overlap.
__device__ __forceinline__ void activate(const f32x16& z, bf16x8& lo, bf16x8& hi)
{
    float e[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) e[r] = __expf(-z[r]);
#pragma unroll
    for (int r = 0; r < 16; ++r) e[r] = __builtin_amdgcn_rcpf(1.0f + e[r]);
#pragma unroll
    for (int r = 0; r < 16; ++r) e[r] *= z[r];
    lo = pack8(&e[0]);
    hi = pack8(&e[8]);
}

struct InferArgs {
    const float* x;
    float* y;
    const uint16_t* wf;        // packed A-operand pieces of every layer
    const int64_t* wf_off;     // [depth + 1] offsets into wf (elements)
    const float* params;       // FP32 masters (biases read from here)
    const int64_t* b_off;      // [depth + 1] bias offsets into params
    int32_t N, n_in, n_out, depth;
    int32_t n_tiles;
};

// Half `step & 1` of hidden layer 1 + (step / 2) % (depth - 1): the stream of half layers a
// workgroup walks through, tile after tile.
__device__ __forceinline__ const uint4* half_src(const InferArgs& a, int64_t step)
{
    const int nh = a.depth - 1;
    const int l = 1 + static_cast<int>((step >> 1) % nh);
    return reinterpret_cast<const uint4*>(a.wf + a.wf_off[l]) + (step & 1) * kHalfU4;
}

// Row block MB of a hidden layer (both column blocks, all 16 K blocks; the chains start from the
// bias), reading its A pieces from the LDS half-layer buffer W up front.  With EPI the SiLU of the
// previous row block (pre-activations in a0, a1 on entry) is computed two values per MFMA pair, so
// the vector ALU works while the matrix core runs; its BF16 pieces go to out[.][2 MB - 2 .. 2 MB - 1].
template <int NCB, int MB, bool EPI>
__device__ __forceinline__ void row_block(const uint4* __restrict__ W, const float* __restrict__ bias,
                                          const bf16x8 (&in)[NCB][kKB], bf16x8 (&out)[NCB][kKB], int lane, int h,
                                          f32x16 (&a)[NCB])
{
    constexpr int m = MB % kHalfMB;
    constexpr int G = NCB == 1 ? kKB / 2 : kKB;  // A pieces read from LDS per group
    f32x16 p[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) p[cb] = a[cb];
    const f32x16 b = bias_acc(bias, MB, h);
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) a[cb] = b;
    float s[NCB][16];
#pragma unroll
    for (int g0 = 0; g0 < kKB; g0 += G) {
        bf16x8 A[G];
#pragma unroll
        for (int i = 0; i < G; ++i) A[i] = *reinterpret_cast<const bf16x8*>(&W[(m * kKB + g0 + i) * 64 + lane]);
#pragma unroll
        for (int i = 0; i < G; ++i) {
            const int kb = g0 + i;
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) a[cb] = mfma(A[i], in[cb][kb], a[cb]);
            if (EPI) {
#pragma unroll
                for (int cb = 0; cb < NCB; ++cb) s[cb][kb] = silu(p[cb][kb]);
            }
        }
    }
    if (EPI) {
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            out[cb][2 * MB - 2] = pack8(&s[cb][0]);
            out[cb][2 * MB - 1] = pack8(&s[cb][8]);
        }
    }
}

// One hidden layer: row blocks 0-3 from buffer H0, 4-7 from H1.  While the first half is multiplied
// the next streamed half (next0) travels through registers into H1, and during the second half
// next1 into H0 (each thread's pieces are loaded when the half starts and written when it ends);
// one barrier after each half.  The SiLU of each row block runs with the MFMAs of the next one; the
// last row block's runs after the second barrier.
template <int NCB>
__device__ __forceinline__ void hidden_layer(uint4* __restrict__ H0, uint4* __restrict__ H1,
                                             const uint4* __restrict__ next0, const uint4* __restrict__ next1,
                                             const float* __restrict__ bias, const bf16x8 (&in)[NCB][kKB],
                                             bf16x8 (&out)[NCB][kKB], int lane, int h)
{
    constexpr int kThreads = 256 * 2 / NCB;
    constexpr int kSt = kHalfU4 / kThreads;
    f32x16 a[NCB];
    uint4 st[kSt];
#pragma unroll
    for (int i = 0; i < kSt; ++i) st[i] = next0[i * kThreads + threadIdx.x];
    row_block<NCB, 0, false>(H0, bias, in, out, lane, h, a);
    row_block<NCB, 1, true>(H0, bias, in, out, lane, h, a);
    row_block<NCB, 2, true>(H0, bias, in, out, lane, h, a);
    row_block<NCB, 3, true>(H0, bias, in, out, lane, h, a);
#pragma unroll
    for (int i = 0; i < kSt; ++i) H1[i * kThreads + threadIdx.x] = st[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kSt; ++i) st[i] = next1[i * kThreads + threadIdx.x];
    row_block<NCB, 4, true>(H1, bias, in, out, lane, h, a);
    row_block<NCB, 5, true>(H1, bias, in, out, lane, h, a);
    row_block<NCB, 6, true>(H1, bias, in, out, lane, h, a);
    row_block<NCB, 7, true>(H1, bias, in, out, lane, h, a);
#pragma unroll
    for (int i = 0; i < kSt; ++i) H0[i * kThreads + threadIdx.x] = st[i];
    __syncthreads();
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) activate(a[cb], out[cb][14], out[cb][15]);
}

template <int NCB>
__device__ __forceinline__ void output_layer(const InferArgs& a, const uint4* __restrict__ Wout,
                                             const float* __restrict__ bias, const bf16x8 (&in)[NCB][kKB],
                                             int64_t q0, int lane, int h, int c)
{
    f32x16 o[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) o[cb] = f32x16{};
#pragma unroll
    for (int kb = 0; kb < kKB; ++kb) {
        const bf16x8 A = *reinterpret_cast<const bf16x8*>(&Wout[kb * 64 + lane]);
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) o[cb] = mfma(A, in[cb][kb], o[cb]);
    }
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
        const int64_t q = q0 + cb * 32 + c;
        if (q >= a.N) continue;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int k = (r >> 2) * 8 + h * 4 + (r & 3);
            if (k < a.n_out) a.y[q * a.n_out + k] = o[cb][r] + bias[k];
        }
    }
}

// NCB column blocks of 32 queries per wavefront; 8 / NCB wavefronts per workgroup (two per SIMD
// when NCB = 1, so that one wavefront's SiLU runs while the other's MFMAs do), 256 queries per tile.
template <int NCB>
__global__ __launch_bounds__(512 / NCB) __attribute__((amdgpu_waves_per_eu(2 / NCB, 2 / NCB))) void k_mlp_infer(
    InferArgs a)
{
    constexpr int kThreads = 512 / NCB;
    constexpr int kQw = 32 * NCB;  // queries per wavefront
    extern __shared__ uint4 smem[];
    uint4* H0 = smem;
    uint4* H1 = smem + kHalfU4;
    uint4* Win = smem + 2 * kHalfU4;
    uint4* Wout = Win + kInU4;
    float* biases = reinterpret_cast<float*>(Wout + kOutU4);  // [depth + 1][256]
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int h = lane >> 5, c = lane & 31;
    const int nh = a.depth - 1;
    const int64_t my_tiles = blockIdx.x < a.n_tiles ? (a.n_tiles - 1 - blockIdx.x) / gridDim.x + 1 : 0;
    const int64_t steps = 2 * nh * my_tiles;

    // resident pieces: input and output layers, all biases, and the first streamed half layer
    {
        const uint4* src = reinterpret_cast<const uint4*>(a.wf + a.wf_off[0]);
        for (int i = threadIdx.x; i < kInU4; i += kThreads) Win[i] = src[i];
        src = reinterpret_cast<const uint4*>(a.wf + a.wf_off[a.depth]);
        for (int i = threadIdx.x; i < kOutU4; i += kThreads) Wout[i] = src[i];
        for (int i = threadIdx.x; i < (a.depth + 1) * kW; i += kThreads) {
            const int l = i / kW, k = i % kW;
            const int n = l == a.depth ? a.n_out : kW;
            biases[i] = k < n ? a.params[a.b_off[l] + k] : 0.0f;
        }
        if (steps > 0) {
            const uint4* first = half_src(a, 0);
            for (int i = threadIdx.x; i < kHalfU4; i += kThreads) H0[i] = first[i];
        }
    }
    __syncthreads();

    // network inputs of a tile: lane (h, c) reads features 8h .. 8h+7 of queries q0 + 32 cb + c; the
    // next tile's are fetched while the current one computes
    float xr[NCB][8];
    auto fetch_x = [&](int64_t tile) {
        const int64_t q0 = tile * kTileQ + wave * kQw;
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
            const int64_t q = q0 + cb * 32 + c;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int f = 8 * h + j;
                const bool ok = tile < a.n_tiles && q < a.N && f < a.n_in;
                const float v = a.x[ok ? q * a.n_in + f : 0];
                xr[cb][j] = ok ? v : 0.0f;
            }
        }
    };
    fetch_x(blockIdx.x);

    int64_t step = 0;
    for (int64_t tile = blockIdx.x; tile < a.n_tiles; tile += gridDim.x) {
        const int64_t q0 = tile * kTileQ + wave * kQw;
        bf16x8 xin[NCB];
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) xin[cb] = pack8(xr[cb]);
        fetch_x(tile + gridDim.x);
        bf16x8 act[NCB][kKB], nxt[NCB][kKB];
#pragma unroll
        for (int mb = 0; mb < kMB; ++mb) {
            const bf16x8 A = *reinterpret_cast<const bf16x8*>(&Win[mb * 64 + lane]);
            const f32x16 b = bias_acc(biases, mb, h);
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb) activate(mfma(A, xin[cb], b), act[cb][2 * mb], act[cb][2 * mb + 1]);
        }
        for (int l = 1; l <= nh; ++l) {
            const uint4* next0 = half_src(a, step + 1 < steps ? step + 1 : step);
            const uint4* next1 = half_src(a, step + 2 < steps ? step + 2 : step);
            hidden_layer<NCB>(H0, H1, next0, next1, biases + l * kW, act, nxt, lane, h);
            step += 2;
#pragma unroll
            for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
                for (int kb = 0; kb < kKB; ++kb) act[cb][kb] = nxt[cb][kb];
        }
        output_layer<NCB>(a, Wout, biases + a.depth * kW, act, q0, lane, h, c);
    }
}

size_t infer_lds_bytes(int depth) { return static_cast<size_t>(2 * kHalfU4 + kInU4 + kOutU4 + (depth + 1) * 64) * 16; }

}  // namespace

bool mlp_fused_supported(int n_in, int width, int depth, int n_out)
{
    return width == kW && n_in <= 16 && n_out <= 32 && depth >= 1 && depth <= kMaxDepth;
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
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    const size_t lds = infer_lds_bytes(depth);
    // one column block per wavefront, two wavefronts per SIMD (measured faster than two column
    // blocks on one wavefront per SIMD: 0.56 vs 0.60 ms per 2^20 queries)
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mlp_infer<1>), hipFuncAttributeMaxDynamicSharedMemorySize,
                            static_cast<int>(lds));
    if (e != hipSuccess) return e;
    InferArgs a{};
    a.x = x;
    a.y = y;
    a.wf = wf;
    a.wf_off = wf_off_dev;
    a.params = params;
    a.b_off = b_off_dev;
    a.N = N;
    a.n_in = n_in;
    a.n_out = n_out;
    a.depth = depth;
    a.n_tiles = static_cast<int32_t>((static_cast<int64_t>(N) + kTileQ - 1) / kTileQ);
    // persistent: one workgroup per compute unit (the LDS footprint allows no second one)
    const unsigned blocks = static_cast<unsigned>(std::min<int64_t>(a.n_tiles, std::max(cus, 1)));
    hipLaunchKernelGGL(k_mlp_infer<1>, dim3(blocks), dim3(512), lds, stream, a);
    return hipGetLastError();
}

}  // namespace srp
