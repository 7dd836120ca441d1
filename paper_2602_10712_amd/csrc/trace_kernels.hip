// HIP kernels of the ray-grid SRP tracer for gfx950 (CDNA4, wave64).
//
// k_frames     per sun direction: propagation d = -s, Duff et al. (JCGT 2017) basis (u, v),
//              rectangle bounding the projected mesh box, entry plane, ray-tube force
//              w = Phi du dv / c  (FP64, rounded to FP32 for the trace).
// k_pack_mat   per facet (BVH order): rho_s, rho_d and the frozen specular-sampling probability.
// k_trace      one wavefront traces an 8 x 8 pixel tile of parallel rays.  Traversal of the BVH is
//              wavefront-coherent: the whole wave walks one node sequence with a wave-uniform
//              stack in LDS, node and triangle records are fetched once per wave through the
//              scalar cache, and every lane tests its own ray against them.  Each lane then
//              deposits momentum at its closest hit (paper Sec. 3.2, l2f: incident minus reflected
//              momentum over c) and continues along a mirror or Lambertian direction for up to
//              `bounces` interactions; at the last one the expected reflected momentum
//              rho_s r + (2/3) rho_d n leaves the body (Lambertian factor 2/3, Sec. 5.9).
//              Force and torque (Sec. 3.2, torque integral about x_COM) are summed per lane in
//              FP32, per wave with cross-lane shuffles, per workgroup in FP64.
// k_reduce     fixed-order FP64 sum of the workgroup partials of each direction.
#include <float.h>

#include "srp_internal.h"
#include "srp_path.h"
#include "srp_traverse.h"

namespace srp {
namespace {

struct BoxArg {
    double lo[3], hi[3];
};

__global__ void k_frames(const double* __restrict__ sun, int64_t D, BoxArg box, double L, int32_t nu, int32_t nv,
                         double flux, const double* __restrict__ caller, double* __restrict__ f64,
                         DevFrame* __restrict__ f32)
{
    const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= D) return;
    const double s[3] = {sun[3 * j], sun[3 * j + 1], sun[3 * j + 2]};
    double f[12];
    if (caller) {
        for (int a = 0; a < 12; ++a) f[a] = caller[12 * j + a];
    } else {
        frame_from_box(s, box.lo, box.hi, L, nu, nv, f);
    }
    if (f64)
        for (int a = 0; a < 12; ++a) f64[12 * j + a] = f[a];
    if (f32) f32[j] = frame_to_device(s, f, flux);
}

// ---- materials ----------------------------------------------------------------------------------
__global__ void k_pack_mat(const float* __restrict__ rs, const float* __restrict__ rd, const float* __restrict__ ps,
                           const int32_t* __restrict__ perm, int64_t n, float4* __restrict__ mat,
                           int32_t* __restrict__ bad)
{
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int32_t f = perm[p];
    const float a = rs[f], b = rd[f];
    int flag = 0;
    if (!(a >= 0.0f) || !(b >= 0.0f) || !(a + b <= 1.0f)) flag |= 1;
    float q;
    if (ps) {
        q = ps[f];
        if (!(q >= 0.0f && q <= 1.0f)) flag |= 2;
    } else if (a > 0.0f && b > 0.0f) {
        q = a / (a + b);
        q = fminf(fmaxf(q, 0.01f), 0.99f);
    } else {
        q = a > 0.0f ? 1.0f : 0.0f;
    }
    if (flag) atomicOr(bad, flag);
    mat[p] = make_float4(a, b, q, 0.0f);
}

// BATCH: the launch covers n_scenes designs; hardware block b runs on XCD b % 8, so design s is
// handled entirely by XCD s % 8 (its BVH stays in that XCD's L2) in design-major order.
template <bool RECORDS, bool BATCH>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6))) void k_trace(TraceArgs a)
{
    __shared__ int s_stack[kWaves][kStackDepth];
    __shared__ int s_lane[kWaves][kLaneStack][64];
    __shared__ float s_red[kWaves][6];
    __shared__ float4 s_rect[kCullBoxes];
    __shared__ uint64_t s_live;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    int64_t unit;  // (scene *) D + direction
    int32_t blk;
    const BvhNode* __restrict__ nodes;
    const TriRec* __restrict__ tris;
    const float4* __restrict__ mat;
    float com[3], eps;
    uint32_t design = a.design_index;
    int64_t j;
    if (BATCH) {
        const int64_t per_design = a.D * a.blocks_per_dir;
        const int64_t b = blockIdx.x;
        const int64_t xcd = b & 7, k = b >> 3;
        const int64_t s = xcd + 8 * (k / per_design);
        if (s >= a.n_scenes) return;
        const int64_t r = k % per_design;
        j = r / a.blocks_per_dir;
        blk = static_cast<int32_t>(r % a.blocks_per_dir);
        unit = s * a.D + j;
        const SceneDesc sd = a.scenes[s];
        nodes = sd.nodes;
        tris = sd.tris;
        mat = sd.mat;
        com[0] = sd.com[0];
        com[1] = sd.com[1];
        com[2] = sd.com[2];
        eps = sd.eps;
        design += static_cast<uint32_t>(s);
    } else {
        if (!block_unit(a, blockIdx.x, j, blk)) return;  // whole workgroup: grid padding
        unit = j;
        nodes = a.nodes;
        tris = a.tris;
        mat = a.mat;
        com[0] = a.com[0];
        com[1] = a.com[1];
        com[2] = a.com[2];
        eps = a.eps;
    }
    const DevFrame fr = a.frames[unit];
    const uint32_t dir_global = static_cast<uint32_t>(a.dir_index_base + j);
    int* stack = s_stack[wave];
    int* lstack = &s_lane[wave][0][lane];

    // the workgroup's tiles that may contain a hit (grid mode; records mode traces every pixel)
    uint64_t live = ~0ull;
    if (!RECORDS && a.cull) {
        if (threadIdx.x < kCullBoxes) s_rect[threadIdx.x] = cull_rect(nodes, fr, threadIdx.x);
        __syncthreads();
        if (wave == 0) {
            const uint64_t m = live_tiles(a, s_rect, static_cast<int64_t>(blk) * a.tiles_per_wave * kWaves,
                                          a.tiles_per_wave * kWaves);
            if (lane == 0) s_live = m;
        }
        __syncthreads();
        live = s_live;
    }

    float acc[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    for (int m = 0; m < a.tiles_per_wave; ++m) {
        const int64_t tile = (static_cast<int64_t>(blk) * a.tiles_per_wave + m) * kWaves + wave;
        if (tile >= a.tiles_per_dir) break;
        if (((live >> (m * kWaves + wave)) & 1ull) == 0) continue;
        int64_t pixel, rec;
        const bool valid = tile_pixel<RECORDS>(a, tile, lane, pixel, rec);
        const int32_t pi = static_cast<int32_t>(pixel % a.nu);
        const int32_t pk = static_cast<int32_t>(pixel / a.nu);
        float o[3], d[3];
        primary_ray(fr, pi, pk, static_cast<uint32_t>(pixel), dir_global, design, a.seed_lo, a.seed_hi,
                    a.jitter != 0, o, d);
        float w = fr.w;
        bool alive = valid;
        int skip = -1;
        float ray[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        int b_done = 0;
        for (int b = 1; b <= a.bounces; ++b) {
            if (wave_ballot(alive) == 0) break;
            float t;
            int hit;
            // primary rays of a tile are coherent: one shared node sequence; secondary rays scatter
            if (b == 1)
                closest_hit_parallel(nodes, tris, o, d, alive, skip, t, hit, stack, fr.d);
            else if (!a.lane_walk)
                closest_hit(nodes, tris, o, d, alive, skip, t, hit, stack);
            else
                closest_hit_lane(nodes, tris, o, d, alive, skip, t, hit, lstack);
            if (!alive) continue;
            if (hit < 0) {
                alive = false;
                continue;
            }
            const TriRec tr = tris[hit];
            const float4 mt = mat[hit];
            if (RECORDS) a.rec_hit[(j * a.n_pix + rec) * a.bounces + (b - 1)] = __float_as_int(tr.f[0].w);
            b_done = b;
            const float n[3] = {tr.f[1].w, tr.f[2].w, tr.f[3].x};
            float x[3], g[3];
            alive = interact(o, d, w, t, n, mt.x, mt.y, mt.z, b, a.bounces, static_cast<uint32_t>(pixel), dir_global,
                             design, a.seed_lo, a.seed_hi, eps, x, g);
            const float lx = x[0] - com[0], ly = x[1] - com[1], lz = x[2] - com[2];
            ray[0] += g[0];
            ray[1] += g[1];
            ray[2] += g[2];
            ray[3] += ly * g[2] - lz * g[1];
            ray[4] += lz * g[0] - lx * g[2];
            ray[5] += lx * g[1] - ly * g[0];
            skip = hit;
        }
        if (RECORDS && valid) {
            for (int b = b_done + 1; b <= a.bounces; ++b) a.rec_hit[(j * a.n_pix + rec) * a.bounces + (b - 1)] = -1;
            if (a.rec_force) {
                float* rf = a.rec_force + (j * a.n_pix + rec) * 3;
                rf[0] = ray[0];
                rf[1] = ray[1];
                rf[2] = ray[2];
            }
        }
#pragma unroll
        for (int c = 0; c < 6; ++c) acc[c] += ray[c];
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[c] = wave_sum(acc[c]);
    if (lane == 0) {
#pragma unroll
        for (int c = 0; c < 6; ++c) s_red[wave][c] = acc[c];
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double s = 0.0;
        for (int q = 0; q < kWaves; ++q) s += static_cast<double>(s_red[q][threadIdx.x]);
        a.partials[(unit * a.blocks_per_dir + blk) * 6 + threadIdx.x] = s;
    }
}

__global__ void k_reduce(const double* __restrict__ partials, int64_t D, int32_t bpd, double* __restrict__ force,
                         double* __restrict__ torque)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= D * 6) return;
    const int64_t j = t / 6;
    const int c = static_cast<int>(t % 6);
    double s = 0.0;
    for (int32_t b = 0; b < bpd; ++b) s += partials[(j * bpd + b) * 6 + c];
    if (c < 3)
        force[3 * j + c] = s;
    else if (torque)
        torque[3 * j + c - 3] = s;
}

}  // namespace

hipError_t launch_frames(const double* sun_dirs, int64_t D, const double lo[3], const double hi[3], double L,
                         int32_t nu, int32_t nv, double flux, const double* caller_frames, double* frames64,
                         DevFrame* frames32, hipStream_t stream)
{
    if (D <= 0) return hipSuccess;
    BoxArg box;
    for (int a = 0; a < 3; ++a) {
        box.lo[a] = lo[a];
        box.hi[a] = hi[a];
    }
    const int threads = 64;
    const unsigned blocks = static_cast<unsigned>((D + threads - 1) / threads);
    hipLaunchKernelGGL(k_frames, dim3(blocks), dim3(threads), 0, stream, sun_dirs, D, box, L, nu, nv, flux,
                       caller_frames, frames64, frames32);
    return hipGetLastError();
}

hipError_t launch_pack_materials(const float* rho_s, const float* rho_d, const float* p_spec, const int32_t* perm,
                                 int64_t n, float4* mat, int32_t* bad_flag, hipStream_t stream)
{
    const int threads = 256;
    const unsigned blocks = static_cast<unsigned>((n + threads - 1) / threads);
    hipLaunchKernelGGL(k_pack_mat, dim3(blocks), dim3(threads), 0, stream, rho_s, rho_d, p_spec, perm, n, mat,
                       bad_flag);
    return hipGetLastError();
}

hipError_t launch_trace(const TraceArgs& a, bool records, hipStream_t stream)
{
    const int64_t blocks = single_scene_blocks(a);
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    if (records)
        hipLaunchKernelGGL((k_trace<true, false>), dim3(static_cast<unsigned>(blocks)), dim3(64 * kWaves), 0, stream,
                           a);
    else
        hipLaunchKernelGGL((k_trace<false, false>), dim3(static_cast<unsigned>(blocks)), dim3(64 * kWaves), 0, stream,
                           a);
    return hipGetLastError();
}

hipError_t launch_trace_batch(const TraceArgs& a, hipStream_t stream)
{
    const int64_t blocks = static_cast<int64_t>(a.scene_slots) * a.D * a.blocks_per_dir;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_trace<false, true>), dim3(static_cast<unsigned>(blocks)), dim3(64 * kWaves), 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_reduce(const double* partials, int64_t D, int32_t blocks_per_dir, double* force, double* torque,
                         hipStream_t stream)
{
    if (D <= 0) return hipSuccess;
    const int threads = 256;
    const unsigned blocks = static_cast<unsigned>((D * 6 + threads - 1) / threads);
    hipLaunchKernelGGL(k_reduce, dim3(blocks), dim3(threads), 0, stream, partials, D, blocks_per_dir, force, torque);
    return hipGetLastError();
}

}  // namespace srp
