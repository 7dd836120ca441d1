// Issue rates of the vector ALU on gfx950, per instruction class: the ceilings the ALU roofline of
// the ray walk is stated against.
//
// Each kernel runs one workgroup per compute unit (it claims the whole 160 KB LDS, so no second
// workgroup can join it) with W wavefronts per SIMD; every lane runs 16 independent dependency
// chains of one instruction kind, unrolled 64 instructions per loop trip.  The rate is the number
// of wave64 instructions each SIMD issued over the kernel's event-timed duration, in shader clock
// cycles; the clock is read inside the kernel (s_memtime against the 100 MHz s_memrealtime).  The
// MFMA rows time a dependent chain of v_mfma_f32_32x32x16_bf16 alone and with independent vector
// work beside it.
//
// Build: hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops
//        valu_rates.hip -o valu_rates          (build.py builds it beside libsrp.so)
#include <hip/hip_runtime.h>

#include <cstdio>

namespace {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

enum Kind : int {
    kFma = 0,     // v_fma_f32 / v_fmamk_f32
    kMul,         // v_mul_f32
    kAddF,        // v_add_f32
    kAddU,        // v_add_u32
    kMin,         // v_min_f32
    kMax3,        // v_max3_f32
    kSelect,      // v_cmp_gt_f32 + v_cndmask_b32
    kMulLo,       // v_mul_lo_u32
    kExp,         // v_exp_f32 (transcendental)
    kRcp,         // v_rcp_f32 (transcendental)
    kMov,         // v_mov_b32
    kXor,         // v_xor_b32
    kCnd,         // v_cndmask_b32 on a fixed lane mask
    kCmp,         // v_cmp_lt_f32 into a scalar register pair
    kNumKinds
};

const char* kind_name(int k)
{
    static const char* n[] = {"v_fma_f32", "v_mul_f32", "v_add_f32", "v_add_u32", "v_min_f32",
                              "v_max3_f32", "v_cmp+v_cndmask", "v_mul_lo_u32", "v_exp_f32", "v_rcp_f32",
                              "v_mov_b32", "v_xor_b32", "v_cndmask_b32", "v_cmp_lt_f32"};
    return n[k];
}

// One loop trip: NM chained MFMAs (0 or 16) and 16 x NV operations of kind K.  The instruction
// count of a trip is taken from this file's gfx950 assembly: 64 of the named instruction per trip,
// except v_min_f32 (64 + 16 v_max_f32 that quiet NaN inputs) and the select (64 v_cmp_gt_f32 +
// 64 v_cndmask_b32, with the s_nop wait states the compare-to-select dependency needs).  The last
// four kinds are single instructions written out (no memory access), as the compiler would
// otherwise fold them away.
template <int NM, int NV, int K>
__global__ void k_rate(float* out, unsigned long long* clk, int iters)
{
    extern __shared__ float lds_claim[];
    if (iters < 0) lds_claim[threadIdx.x] = 0.0f;  // never taken: keeps the LDS claim
    const int t = threadIdx.x + blockIdx.x * blockDim.x;
    unsigned long long c0 = 0, r0 = 0;
    if (t == 0) {
        c0 = clock64();
        r0 = wall_clock64();
    }
    bf16x8 a, b;
    for (int j = 0; j < 8; ++j) {
        a[j] = static_cast<__bf16>(0.001f * ((t + j) & 7));
        b[j] = static_cast<__bf16>(0.001f * ((t * 3 + j) & 7));
    }
    f32x16 acc = {};
    float v[16];
    unsigned u[16];
    for (int j = 0; j < 16; ++j) {
        v[j] = 0.5f + 0.01f * ((t + j) & 15);
        u[j] = t * 7 + j;
    }
    const unsigned long long lanes = 0x5555555555555555ull;
    unsigned long long cm[4] = {0, 0, 0, 0};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            if (m < NM) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                const int i = (m * NV + k) & 15;
                float& x = v[i];
                if (K == kFma) x = x * 0.999f + 0.0005f;
                else if (K == kMul) x = x * 0.999f;
                else if (K == kAddF) x = x + v[(i + 1) & 15];
                else if (K == kAddU) u[i] = u[i] + u[(i + 1) & 15];
                else if (K == kMin) x = fminf(x, v[(i + 1) & 15]);
                else if (K == kMax3) x = fmaxf(fmaxf(x, v[(i + 1) & 15]), v[(i + 2) & 15]);
                else if (K == kSelect) x = x > v[(i + 1) & 15] ? v[(i + 2) & 15] : x;
                else if (K == kMulLo) u[i] = u[i] * u[(i + 3) & 15];
                else if (K == kExp) x = __builtin_amdgcn_exp2f(-x);
                else if (K == kRcp) x = __builtin_amdgcn_rcpf(x);
                else if (K == kMov) asm volatile("v_mov_b32 %0, %1" : "=v"(u[i]) : "v"(u[(i + 1) & 15]));
                else if (K == kXor) asm volatile("v_xor_b32 %0, %1, %2" : "=v"(u[i]) : "v"(u[i]), "v"(u[(i + 5) & 15]));
                else if (K == kCnd)
                    asm volatile("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(u[i]) : "v"(u[i]), "v"(u[(i + 5) & 15]), "s"(lanes));
                else if (K == kCmp) asm volatile("v_cmp_lt_f32_e64 %0, %1, %2" : "=s"(cm[i & 3]) : "v"(x), "v"(v[(i + 5) & 15]));
            }
        }
    }
    float s = 0.0f;
    for (int j = 0; j < 16; ++j) s += acc[j];
    for (int j = 0; j < 16; ++j) s += v[j] + static_cast<float>(u[j] & 1);
    s += static_cast<float>((cm[0] ^ cm[1] ^ cm[2] ^ cm[3]) & 1);
    out[t] = s;
    if (t == 0) {
        clk[0] = clock64() - c0;
        clk[1] = wall_clock64() - r0;
    }
}

struct Ctx {
    float* out;
    unsigned long long* clk;
    int cus;
    int wall_khz;
};

template <int NM, int NV, int K>
bool run(const Ctx& c, int waves_per_simd, double instr_per_trip)
{
    const int block = 256 * waves_per_simd;
    const int iters = 4000;
    const size_t lds = 160 * 1024;
    auto fn = reinterpret_cast<const void*>(&k_rate<NM, NV, K>);
    if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)) != hipSuccess)
        return false;
    hipLaunchKernelGGL((k_rate<NM, NV, K>), dim3(c.cus), dim3(block), lds, 0, c.out, c.clk, 16);
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return false;
    (void)hipEventRecord(e0, 0);
    hipLaunchKernelGGL((k_rate<NM, NV, K>), dim3(c.cus), dim3(block), lds, 0, c.out, c.clk, iters);
    (void)hipEventRecord(e1, 0);
    if (hipEventSynchronize(e1) != hipSuccess) return false;
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    unsigned long long h[2] = {0, 0};
    if (hipMemcpy(h, c.clk, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) return false;
    const double ghz = h[1] ? static_cast<double>(h[0]) / (static_cast<double>(h[1]) / (c.wall_khz * 1e3)) * 1e-9 : 0.0;
    const double cycles = ms * 1e-3 * ghz * 1e9;
    const double trips = static_cast<double>(waves_per_simd) * iters;
    if (NM > 0) {
        printf("| MFMA 32x32x16 bf16 chain%s | %d | %.2f | %.3f | %.1f cycles per MFMA |\n",
               NV == 0 ? "" : (K == kExp ? " + 2 v_exp_f32 each" : " + 4 v_fma_f32 each"), waves_per_simd, ghz, ms,
               cycles / (trips * NM));
    } else {
        const double instr = trips * instr_per_trip;
        printf("| %s | %d | %.2f | %.3f | %.3f wave64 instructions per SIMD-cycle (%.1f lanes per cycle) |\n",
               kind_name(K), waves_per_simd, ghz, ms, instr / cycles, 64.0 * instr / cycles);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return true;
}

}  // namespace

int main()
{
    Ctx c{};
    if (hipDeviceGetAttribute(&c.cus, hipDeviceAttributeMultiprocessorCount, 0) != hipSuccess ||
        hipDeviceGetAttribute(&c.wall_khz, hipDeviceAttributeWallClockRate, 0) != hipSuccess) {
        fprintf(stderr, "no HIP device\n");
        return 1;
    }
    if (hipMalloc(&c.out, sizeof(float) * c.cus * 1024) != hipSuccess ||
        hipMalloc(&c.clk, 2 * sizeof(unsigned long long)) != hipSuccess) {
        fprintf(stderr, "allocation failed\n");
        return 1;
    }
    printf("%d compute units, one workgroup each; 100 MHz reference clock %d kHz\n\n", c.cus, c.wall_khz);
    printf("| Instruction | waves per SIMD | clock (GHz) | ms | rate |\n|---|---|---|---|---|\n");
    bool ok = true;
    for (int w : {2, 4}) {
        ok = ok && run<0, 4, kFma>(c, w, 64) && run<0, 4, kMul>(c, w, 64) && run<0, 4, kAddF>(c, w, 64) &&
             run<0, 4, kAddU>(c, w, 64) && run<0, 4, kMin>(c, w, 80) && run<0, 4, kMax3>(c, w, 64) &&
             run<0, 4, kSelect>(c, w, 128) && run<0, 4, kMulLo>(c, w, 64) && run<0, 4, kExp>(c, w, 64) &&
             run<0, 4, kRcp>(c, w, 64) && run<16, 0, kFma>(c, w, 0) && run<16, 4, kFma>(c, w, 0) &&
             run<16, 2, kExp>(c, w, 0) && run<0, 4, kMov>(c, w, 64) && run<0, 4, kXor>(c, w, 64) &&
             run<0, 4, kCnd>(c, w, 64) && run<0, 4, kCmp>(c, w, 64);
    }
    const hipError_t e = hipDeviceSynchronize();
    (void)hipFree(c.out);
    (void)hipFree(c.clk);
    if (!ok || e != hipSuccess) {
        fprintf(stderr, "failed: %s\n", hipGetErrorString(e));
        return 1;
    }
    return 0;
}
