// HIP kernels of the ray-grid SRP tracer for gfx950 (CDNA4, wave64).
//
// k_frames     per sun direction: propagation d = -s, Duff et al. (JCGT 2017) basis (u, v),
//              rectangle bounding the projected mesh box, entry plane, ray-tube force
//              w = Phi du dv / c  (FP64, rounded to FP32 for the trace).
// k_pack_mat   per facet (BVH order): rho_s, rho_d, the frozen specular-sampling probability and the
//              Phong exponent (+infinity: ideal mirror; only the surface-sampling estimator reads it).
// k_pack_phong the Phong exponents alone, validated (>= 1 or +infinity).
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
                           const float* __restrict__ phong, const int32_t* __restrict__ perm, int64_t n,
                           float4* __restrict__ mat, int32_t* __restrict__ bad)
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
        // a probability outside [0, 1], or one that can never choose an event whose reflectance
        // is not zero (that lobe's momentum would silently go missing from the estimate)
        if (!(q >= 0.0f && q <= 1.0f) || (q == 0.0f && a > 0.0f) || (q == 1.0f && b > 0.0f)) flag |= 2;
    } else if (a > 0.0f && b > 0.0f) {
        q = a / (a + b);
        q = fminf(fmaxf(q, 0.01f), 0.99f);
    } else {
        q = a > 0.0f ? 1.0f : 0.0f;
    }
    if (flag) atomicOr(bad, flag);
    mat[p] = make_float4(a, b, q, phong ? phong[f] : INFINITY);
}

__global__ void k_pack_phong(const float* __restrict__ phong, const int32_t* __restrict__ perm, int64_t n,
                             float4* __restrict__ mat, int32_t* __restrict__ flags)
{
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const float m = phong ? phong[perm[p]] : INFINITY;
    int flag = 0;
    if (!(m >= 1.0f)) flag |= 1;           // below 1, or NaN
    if (m >= 1.0f && m < INFINITY) flag |= 2;  // a finite lobe
    if (flag) atomicOr(flags, flag);
    if (mat) mat[p].w = m;
}

// LDS of one trace workgroup, with per-lane stacks of LS entries.
template <int LS>
struct TraceLds {
    int stack[kWaves][kStackDepth];    // wave-uniform stacks of the coherent walk
    int lane[kWaves][LS][64];          // per-lane stacks of the independent walk
    float red[kWaves][6];              // per-wave force and torque sums
    float4 rect[kCullBoxes];           // pixel rectangles of the culling boxes
    uint64_t live;                     // workgroup tiles that may contain a hit
};

// One workgroup's share of direction j: wave tiles blk * tiles_per_wave * kWaves onward of the
// direction's grid, traced against one scene and reduced into partials row `unit` (scene * D + j).
// Every thread of the workgroup calls it (it holds barriers).  RECORDS: per-pixel records for an
// explicit pixel list; PATHS: also write the triangle each traced path hits at each interaction
// into the path record (grid mode), for the adjoint.
template <bool RECORDS, bool PATHS, int LS>
__device__ __forceinline__ void trace_workgroup(const TraceArgs& a, const BvhNode* __restrict__ nodes,
                                                const TriRec* __restrict__ tris, const float4* __restrict__ mat,
                                                const float com[3], float eps, uint32_t design, int64_t j,
                                                int64_t unit, int32_t blk, TraceLds<LS>& L,
                                                int32_t* __restrict__ paths = nullptr)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const DevFrame fr = a.frames[unit];
    const uint32_t dir_global = static_cast<uint32_t>(a.dir_index_base + j);
    int* stack = L.stack[wave];
    int* lstack = &L.lane[wave][0][lane];

    // the workgroup's tiles that may contain a hit (grid mode; records mode traces every pixel)
    uint64_t live = ~0ull;
    if (!RECORDS && a.cull) {
        if (threadIdx.x < kCullBoxes) L.rect[threadIdx.x] = cull_rect(nodes, fr, threadIdx.x);
        __syncthreads();
        if (wave == 0) {
            const uint64_t m = live_tiles(a, L.rect, static_cast<int64_t>(blk) * a.tiles_per_wave * kWaves,
                                          a.tiles_per_wave * kWaves);
            if (lane == 0) L.live = m;
        }
        __syncthreads();
        live = L.live;
    }

    float acc[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    for (int m = 0; m < a.tiles_per_wave; ++m) {
        const int64_t tile = (static_cast<int64_t>(blk) * a.tiles_per_wave + m) * kWaves + wave;
        if (tile >= a.tiles_per_dir) break;
        if (((live >> (m * kWaves + wave)) & 1ull) == 0) continue;
        int64_t pixel, rec;
        int32_t pi, pk;
        const bool valid = tile_pixel<RECORDS>(a, tile, lane, pixel, rec, pi, pk);
        float o[3], d[3];
        primary_ray(fr, pi, pk, static_cast<uint32_t>(pixel), dir_global, design, a.seed_lo, a.seed_hi,
                    a.jitter != 0, o, d);
        float w = fr.w;
        bool alive = valid;
        if (a.ray_mask && valid && ray_masked(a, j, pixel)) alive = false;
        int skip = -1;
        float ray[6] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
        int b_done = 0;
        // path record (at most kRecordBounces interactions): the triangles are held in registers
        // and stored after the path ends -- vector loads and stores share one wait counter, so a
        // store inside the walk would make the walk's load waits conservative
        int h0 = -1, h1 = -1, h2 = -1, n_rec = 0;
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
            if (PATHS) {
                n_rec = b;
                if (b == 1)
                    h0 = hit;
                else if (b == 2)
                    h1 = hit;
                else
                    h2 = hit;
            }
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
            if (RECORDS && a.rec_point) {
                float* rp = a.rec_point + ((j * a.n_pix + rec) * a.bounces + (b - 1)) * 3;
                rp[0] = x[0];
                rp[1] = x[1];
                rp[2] = x[2];
            }
            const float lx = x[0] - com[0], ly = x[1] - com[1], lz = x[2] - com[2];
            ray[0] += g[0];
            ray[1] += g[1];
            ray[2] += g[2];
            ray[3] += ly * g[2] - lz * g[1];
            ray[4] += lz * g[0] - lx * g[2];
            ray[5] += lx * g[1] - ly * g[0];
            skip = hit;
        }
        if (PATHS) {
            if (n_rec >= 1) paths[path_slot(a, j, 1, tile, lane)] = h0;
            if (n_rec >= 2) paths[path_slot(a, j, 2, tile, lane)] = h1;
            if (n_rec >= 3) paths[path_slot(a, j, 3, tile, lane)] = h2;
        }
        if (RECORDS && valid) {
            for (int b = b_done + 1; b <= a.bounces; ++b) {
                a.rec_hit[(j * a.n_pix + rec) * a.bounces + (b - 1)] = -1;
                if (a.rec_point) {
                    float* rp = a.rec_point + ((j * a.n_pix + rec) * a.bounces + (b - 1)) * 3;
                    rp[0] = rp[1] = rp[2] = __builtin_nanf("");
                }
            }
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
        for (int c = 0; c < 6; ++c) L.red[wave][c] = acc[c];
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double s = 0.0;
        for (int q = 0; q < kWaves; ++q) s += static_cast<double>(L.red[q][threadIdx.x]);
        a.partials[(unit * a.blocks_per_dir + blk) * 6 + threadIdx.x] = s;
    }
}

// Single scene: one workgroup per (direction, blk), placed by block_unit.  LS = kLaneStackShort
// for trees that fit it: the smaller LDS footprint (and at most 72 VGPRs) lets 7 workgroups share
// a CU instead of 6.
template <bool RECORDS, int LS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(LS == kLaneStackShort ? 7 : 6))) void k_trace(
    TraceArgs a)
{
    __shared__ TraceLds<LS> L;
    int64_t j;
    int32_t blk;
    if (!block_unit(a, a.D, blockIdx.x, j, blk)) return;  // whole workgroup: grid padding
    trace_workgroup<RECORDS, false, LS>(a, a.nodes, a.tris, a.mat, a.com, a.eps, a.design_index, j, j, blk, L);
}

// k_trace that also writes the path record.  The record and the scene arrays come as separate
// __restrict__ parameters: the record stores then provably leave the scene untouched, and node
// and triangle records can still be fetched through the scalar cache.
template <int LS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(LS == kLaneStackShort ? 7 : 6))) void k_trace_paths(
    TraceArgs a, const BvhNode* __restrict__ nodes, const TriRec* __restrict__ tris, const float4* __restrict__ mat,
    int32_t* __restrict__ paths)
{
    __shared__ TraceLds<LS> L;
    int64_t j;
    int32_t blk;
    if (!block_unit(a, a.D, blockIdx.x, j, blk)) return;  // whole workgroup: grid padding
    trace_workgroup<false, true, LS>(a, nodes, tris, mat, a.com, a.eps, a.design_index, j, j, blk, L, paths);
}

// Batched designs: the n_scenes x D (design, direction) units in design-major order, placed like
// the directions of a single scene (unit u on XCD u % 8), so all XCDs work through the designs
// together and a design's directions are spread evenly over them.
template <int LS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(LS == kLaneStackShort ? 7 : 6))) void k_trace_batch(
    TraceArgs a)
{
    __shared__ TraceLds<LS> L;
    int64_t u;
    int32_t blk;
    if (!block_unit(a, a.n_scenes * a.D, blockIdx.x, u, blk)) return;  // whole workgroup: grid padding
    const int64_t s = u / a.D, j = u % a.D;
    const SceneDesc sd = a.scenes[s];
    trace_workgroup<false, false, LS>(a, (const BvhNode*)sd.nodes, (const TriRec*)sd.tris, (const float4*)sd.mat, sd.com,
                                  sd.eps, a.design_index + static_cast<uint32_t>(s), j, u, blk, L);
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

hipError_t launch_pack_materials(const float* rho_s, const float* rho_d, const float* p_spec, const float* phong,
                                 const int32_t* perm, int64_t n, float4* mat, int32_t* bad_flag, hipStream_t stream)
{
    const int threads = 256;
    const unsigned blocks = static_cast<unsigned>((n + threads - 1) / threads);
    hipLaunchKernelGGL(k_pack_mat, dim3(blocks), dim3(threads), 0, stream, rho_s, rho_d, p_spec, phong, perm, n, mat,
                       bad_flag);
    return hipGetLastError();
}

hipError_t launch_pack_phong(const float* phong, const int32_t* perm, int64_t n, float4* mat, int32_t* flags,
                             hipStream_t stream)
{
    const int threads = 256;
    const unsigned blocks = static_cast<unsigned>((n + threads - 1) / threads);
    hipLaunchKernelGGL(k_pack_phong, dim3(blocks), dim3(threads), 0, stream, phong, perm, n, mat, flags);
    return hipGetLastError();
}

hipError_t launch_trace(const TraceArgs& a, bool records, hipStream_t stream)
{
    const int64_t blocks = grid_blocks(a, a.D);
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    const dim3 grid(static_cast<unsigned>(blocks)), block(64 * kWaves);
    const bool short_stack = a.lane_walk == 2;
    if (records)
        hipLaunchKernelGGL((k_trace<true, kLaneStack>), grid, block, 0, stream, a);
    else if (a.path_hit && short_stack)
        hipLaunchKernelGGL((k_trace_paths<kLaneStackShort>), grid, block, 0, stream, a, a.nodes, a.tris, a.mat,
                           a.path_hit);
    else if (a.path_hit)
        hipLaunchKernelGGL((k_trace_paths<kLaneStack>), grid, block, 0, stream, a, a.nodes, a.tris, a.mat, a.path_hit);
    else if (short_stack)
        hipLaunchKernelGGL((k_trace<false, kLaneStackShort>), grid, block, 0, stream, a);
    else
        hipLaunchKernelGGL((k_trace<false, kLaneStack>), grid, block, 0, stream, a);
    return hipGetLastError();
}

hipError_t launch_trace_batch(const TraceArgs& a, hipStream_t stream)
{
    const int64_t blocks = grid_blocks(a, static_cast<int64_t>(a.n_scenes) * a.D);
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    if (a.lane_walk == 2)
        hipLaunchKernelGGL((k_trace_batch<kLaneStackShort>), dim3(static_cast<unsigned>(blocks)), dim3(64 * kWaves), 0,
                           stream, a);
    else
        hipLaunchKernelGGL((k_trace_batch<kLaneStack>), dim3(static_cast<unsigned>(blocks)), dim3(64 * kWaves), 0,
                           stream, a);
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
