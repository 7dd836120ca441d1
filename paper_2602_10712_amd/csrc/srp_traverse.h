// Device-side BVH traversal and wavefront helpers shared by the forward and adjoint kernels.
#pragma once

#include <float.h>

#include "srp_internal.h"
#include "srp_path.h"

namespace srp {

__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Closest front-facing hit of each lane's ray (o, d) among all triangles except `skip` (the
// triangle the ray leaves); an exact tie in t goes to the lower original triangle index.  Lanes
// with alive == false never hit.  The traversal is wavefront-coherent: one node sequence for the
// whole wave (so node and triangle records arrive through scalar loads), a child is entered when
// any lane's ray overlaps its box, the nearer child first by majority over the lanes that overlap
// both, and the stack of deferred children is wave-uniform in LDS.
//
// SGN >= 0: every lane's direction has the sign pattern SGN (bit a set <=> axis a negative), as for
// the parallel primary rays of one grid.  The near and far slab of each axis are then fixed at
// compile time, so a box test needs no per-lane min/max of the slab distances.  Rounding is
// monotonic, so the chosen slab equals the min/max of the general test and the hits are identical.
template <int SGN = -1>
__device__ __forceinline__ void closest_hit(const BvhNode* __restrict__ nodes, const TriRec* __restrict__ tris,
                                            const float o[3], const float d[3], bool alive, int skip, float& t_out,
                                            int& hit_out, int* __restrict__ stack)
{
    constexpr bool PARALLEL = SGN >= 0;
    // safe_rcp keeps the sign (also of -0): a non-negative reciprocal makes the lower slab nearer
    constexpr bool px = (SGN & 1) == 0, py = (SGN & 2) == 0, pz = (SGN & 4) == 0;
    const float ix = safe_rcp(d[0]), iy = safe_rcp(d[1]), iz = safe_rcp(d[2]);
    const float nx = -o[0] * ix, ny = -o[1] * iy, nz = -o[2] * iz;
    float tbest = alive ? FLT_MAX : -1.0f;
    int hit = -1;
    int hit_id = 0x7fffffff;
    int sp = 0;
    int cur = 0;
    for (;;) {
        if (cur >= 0) {
            const BvhNode* N = nodes + cur;
            const float4 f0 = N->f[0];
            const float4 f1 = N->f[1];
            const float4 f2 = N->f[2];
            const float4 f3 = N->f[3];
            const int c0 = __float_as_int(f3.x);
            const int c1 = __float_as_int(f3.y);
            float tn0, tf0, tn1, tf1;
            if (PARALLEL) {
                // near / far planes chosen per wave (scalar selects of the node's fields)
                const float ax0 = fmaf(px ? f0.x : f0.y, ix, nx), ax1 = fmaf(px ? f0.y : f0.x, ix, nx);
                const float ay0 = fmaf(py ? f0.z : f0.w, iy, ny), ay1 = fmaf(py ? f0.w : f0.z, iy, ny);
                const float az0 = fmaf(pz ? f2.x : f2.y, iz, nz), az1 = fmaf(pz ? f2.y : f2.x, iz, nz);
                const float bx0 = fmaf(px ? f1.x : f1.y, ix, nx), bx1 = fmaf(px ? f1.y : f1.x, ix, nx);
                const float by0 = fmaf(py ? f1.z : f1.w, iy, ny), by1 = fmaf(py ? f1.w : f1.z, iy, ny);
                const float bz0 = fmaf(pz ? f2.z : f2.w, iz, nz), bz1 = fmaf(pz ? f2.w : f2.z, iz, nz);
                tn0 = fmaxf(fmaxf(ax0, ay0), fmaxf(az0, 0.0f));
                tf0 = fminf(fminf(ax1, ay1), fminf(az1, tbest));
                tn1 = fmaxf(fmaxf(bx0, by0), fmaxf(bz0, 0.0f));
                tf1 = fminf(fminf(bx1, by1), fminf(bz1, tbest));
            } else {
                const float ax0 = fmaf(f0.x, ix, nx), ax1 = fmaf(f0.y, ix, nx);
                const float ay0 = fmaf(f0.z, iy, ny), ay1 = fmaf(f0.w, iy, ny);
                const float az0 = fmaf(f2.x, iz, nz), az1 = fmaf(f2.y, iz, nz);
                const float bx0 = fmaf(f1.x, ix, nx), bx1 = fmaf(f1.y, ix, nx);
                const float by0 = fmaf(f1.z, iy, ny), by1 = fmaf(f1.w, iy, ny);
                const float bz0 = fmaf(f2.z, iz, nz), bz1 = fmaf(f2.w, iz, nz);
                tn0 = fmaxf(fmaxf(fminf(ax0, ax1), fminf(ay0, ay1)), fmaxf(fminf(az0, az1), 0.0f));
                tf0 = fminf(fminf(fmaxf(ax0, ax1), fmaxf(ay0, ay1)), fminf(fmaxf(az0, az1), tbest));
                tn1 = fmaxf(fmaxf(fminf(bx0, bx1), fminf(by0, by1)), fmaxf(fminf(bz0, bz1), 0.0f));
                tf1 = fminf(fminf(fmaxf(bx0, bx1), fmaxf(by0, by1)), fminf(fmaxf(bz0, bz1), tbest));
            }
            const bool h0 = tn0 <= tf0;
            const bool h1 = tn1 <= tf1;
            const uint64_t m0 = wave_ballot(h0);
            const uint64_t m1 = wave_ballot(h1);
            if (m0 && m1) {
                const uint64_t first1 = wave_ballot(h0 && h1 && tn1 < tn0);
                const bool swap = 2 * __popcll(first1) > __popcll(m0 & m1);
                stack[sp] = swap ? c0 : c1;
                ++sp;
                cur = swap ? c1 : c0;
            } else if (m0) {
                cur = c0;
            } else if (m1) {
                cur = c1;
            } else {
                if (sp == 0) break;
                --sp;
                cur = __builtin_amdgcn_readfirstlane(stack[sp]);
            }
        } else {
            const int code = ~cur;
            const int first = code >> 3;
            const int cnt = code & 7;
            for (int q = 0; q < cnt; ++q) {
                const int tri = first + q;
                const TriRec* T = tris + tri;
                const float4 g0 = T->f[0];
                const float4 g1 = T->f[1];
                const float4 g2 = T->f[2];
                const float t = tri_hit(o, d, g0, g1, g2);
                const int id = __float_as_int(g0.w);
                if (t > 0.0f && tri != skip && (t < tbest || (t == tbest && id < hit_id))) {
                    tbest = t;
                    hit = tri;
                    hit_id = id;
                }
            }
            if (sp == 0) break;
            --sp;
            cur = __builtin_amdgcn_readfirstlane(stack[sp]);
        }
    }
    t_out = tbest;
    hit_out = hit;
}

// closest_hit for rays that all travel along the wave-uniform direction `dir` (the primary rays of
// one grid frame): dispatches on the sign pattern of dir.
__device__ __forceinline__ void closest_hit_parallel(const BvhNode* __restrict__ nodes,
                                                     const TriRec* __restrict__ tris, const float o[3],
                                                     const float d[3], bool alive, int skip, float& t_out,
                                                     int& hit_out, int* __restrict__ stack, const float dir[3])
{
    const uint32_t sgn = __builtin_amdgcn_readfirstlane((__float_as_uint(dir[0]) >> 31) |
                                                        ((__float_as_uint(dir[1]) >> 31) << 1) |
                                                        ((__float_as_uint(dir[2]) >> 31) << 2));
    switch (sgn) {
    case 0: closest_hit<0>(nodes, tris, o, d, alive, skip, t_out, hit_out, stack); break;
    case 1: closest_hit<1>(nodes, tris, o, d, alive, skip, t_out, hit_out, stack); break;
    case 2: closest_hit<2>(nodes, tris, o, d, alive, skip, t_out, hit_out, stack); break;
    case 3: closest_hit<3>(nodes, tris, o, d, alive, skip, t_out, hit_out, stack); break;
    case 4: closest_hit<4>(nodes, tris, o, d, alive, skip, t_out, hit_out, stack); break;
    case 5: closest_hit<5>(nodes, tris, o, d, alive, skip, t_out, hit_out, stack); break;
    case 6: closest_hit<6>(nodes, tris, o, d, alive, skip, t_out, hit_out, stack); break;
    default: closest_hit<7>(nodes, tris, o, d, alive, skip, t_out, hit_out, stack); break;
    }
}

// Closest hit with an independent walk per lane (same result as closest_hit): each lane follows
// its own node sequence, nearer child first, with its own stack of deferred children in LDS
// (lstack points at the lane's column; entry k sits at lstack[64 k], so the 64 lanes of a wave
// touch 64 consecutive words).  Node and triangle records arrive through vector loads.  Used for
// secondary segments, whose rays scatter over the scene: the lanes' node sets then barely
// overlap, and a shared sequence would visit their union.  The tree depth must not exceed
// kLaneStack (every push is matched by a descent, so the stack never holds more entries than
// the depth of the current node).
__device__ __forceinline__ void closest_hit_lane(const BvhNode* __restrict__ nodes, const TriRec* __restrict__ tris,
                                                 const float o[3], const float d[3], bool alive, int skip,
                                                 float& t_out, int& hit_out, int* __restrict__ lstack)
{
    const float ix = safe_rcp(d[0]), iy = safe_rcp(d[1]), iz = safe_rcp(d[2]);
    const float nx = -o[0] * ix, ny = -o[1] * iy, nz = -o[2] * iz;
    float tbest = alive ? FLT_MAX : -1.0f;
    int hit = -1;
    int hit_id = 0x7fffffff;
    int sp = 0;
    int cur = alive ? 0 : kWalkDone;
    while (cur != kWalkDone) {
        if (cur >= 0) {
            const BvhNode* N = nodes + cur;
            const float4 f0 = N->f[0];
            const float4 f1 = N->f[1];
            const float4 f2 = N->f[2];
            const float4 f3 = N->f[3];
            const int c0 = __float_as_int(f3.x);
            const int c1 = __float_as_int(f3.y);
            const float ax0 = fmaf(f0.x, ix, nx), ax1 = fmaf(f0.y, ix, nx);
            const float ay0 = fmaf(f0.z, iy, ny), ay1 = fmaf(f0.w, iy, ny);
            const float az0 = fmaf(f2.x, iz, nz), az1 = fmaf(f2.y, iz, nz);
            const float bx0 = fmaf(f1.x, ix, nx), bx1 = fmaf(f1.y, ix, nx);
            const float by0 = fmaf(f1.z, iy, ny), by1 = fmaf(f1.w, iy, ny);
            const float bz0 = fmaf(f2.z, iz, nz), bz1 = fmaf(f2.w, iz, nz);
            const float tn0 = fmaxf(fmaxf(fminf(ax0, ax1), fminf(ay0, ay1)), fmaxf(fminf(az0, az1), 0.0f));
            const float tf0 = fminf(fminf(fmaxf(ax0, ax1), fmaxf(ay0, ay1)), fminf(fmaxf(az0, az1), tbest));
            const float tn1 = fmaxf(fmaxf(fminf(bx0, bx1), fminf(by0, by1)), fmaxf(fminf(bz0, bz1), 0.0f));
            const float tf1 = fminf(fminf(fmaxf(bx0, bx1), fmaxf(by0, by1)), fminf(fmaxf(bz0, bz1), tbest));
            const bool h0 = tn0 <= tf0;
            const bool h1 = tn1 <= tf1;
            if (h0 && h1) {
                const bool swap = tn1 < tn0;
                lstack[sp * 64] = swap ? c0 : c1;
                ++sp;
                cur = swap ? c1 : c0;
            } else if (h0) {
                cur = c0;
            } else if (h1) {
                cur = c1;
            } else if (sp > 0) {
                --sp;
                cur = lstack[sp * 64];
            } else {
                cur = kWalkDone;
            }
        } else {
            const int code = ~cur;
            const int first = code >> 3;
            const int cnt = code & 7;
            for (int q = 0; q < cnt; ++q) {
                const int tri = first + q;
                const TriRec* T = tris + tri;
                const float4 g0 = T->f[0];
                const float4 g1 = T->f[1];
                const float4 g2 = T->f[2];
                const float t = tri_hit(o, d, g0, g1, g2);
                const int id = __float_as_int(g0.w);
                if (t > 0.0f && tri != skip && (t < tbest || (t == tbest && id < hit_id))) {
                    tbest = t;
                    hit = tri;
                    hit_id = id;
                }
            }
            if (sp > 0) {
                --sp;
                cur = lstack[sp * 64];
            } else {
                cur = kWalkDone;
            }
        }
    }
    t_out = tbest;
    hit_out = hit;
}

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Empty-tile culling (library frames only: the caller's frames need not be perpendicular to the
// rays).  All rays of a grid travel along d, perpendicular to the frame axes U, V, so
// the pixel coordinate (p - o0).U / |U|^2 of any point p a ray meets equals the ray's own, which for
// tile (tx, ty) lies in [8 tx, 8 tx + 8) (same for V).  A tile whose pixel rectangle misses the
// projected pixel rectangles of a set of boxes that together hold every triangle has no hit.
// kCullBoxes boxes at depth kCullDepth of the BVH (or shallower leaves) are used, widened by one
// pixel.
constexpr int kCullDepth = 3;
constexpr int kCullBoxes = 1 << kCullDepth;

// Pixel rectangle (lo_i, hi_i, lo_k, hi_k) of top box t: the child reached by the bits of t from the
// root (stopping at a leaf); an empty leaf gives a rectangle no tile overlaps.
__device__ __forceinline__ float4 cull_rect(const BvhNode* __restrict__ nodes, const DevFrame& fr, int t)
{
    int node = 0;
    float lo[3] = {0.0f, 0.0f, 0.0f}, hi[3] = {0.0f, 0.0f, 0.0f};
    for (int lev = 0; lev < kCullDepth; ++lev) {
        const BvhNode N = nodes[node];
        const int side = (t >> (kCullDepth - 1 - lev)) & 1;
        const float4 xy = side ? N.f[1] : N.f[0];
        lo[0] = xy.x;
        hi[0] = xy.y;
        lo[1] = xy.z;
        hi[1] = xy.w;
        lo[2] = side ? N.f[2].z : N.f[2].x;
        hi[2] = side ? N.f[2].w : N.f[2].y;
        const int code = __float_as_int(side ? N.f[3].y : N.f[3].x);
        if (code < 0) {
            if ((~code & 7) == 0) return make_float4(1e30f, -1e30f, 1e30f, -1e30f);
            break;
        }
        node = code;
    }
    float cu = 0.0f, cv = 0.0f, eu = 0.0f, ev = 0.0f, uu = 0.0f, vv = 0.0f;
    for (int a = 0; a < 3; ++a) {
        const float c = 0.5f * (lo[a] + hi[a]) - fr.o0[a], e = 0.5f * (hi[a] - lo[a]);
        cu += c * fr.U[a];
        cv += c * fr.V[a];
        eu += e * fabsf(fr.U[a]);
        ev += e * fabsf(fr.V[a]);
        uu += fr.U[a] * fr.U[a];
        vv += fr.V[a] * fr.V[a];
    }
    if (!(uu > 0.0f) || !(vv > 0.0f)) return make_float4(-1e30f, 1e30f, -1e30f, 1e30f);  // degenerate frame
    return make_float4((cu - eu) / uu - 1.0f, (cu + eu) / uu + 1.0f, (cv - ev) / vv - 1.0f, (cv + ev) / vv + 1.0f);
}

// Bit i of the result: wave tile first_tile + i (i < n) may contain a hit.  Called by one whole
// wavefront; rects are the kCullBoxes rectangles of cull_rect.  A tile is dropped only when it is
// provably disjoint from every rectangle (a NaN bound keeps it).
__device__ __forceinline__ uint64_t live_tiles(const TraceArgs& a, const float4* rects, int64_t first_tile, int n)
{
    const int lane = threadIdx.x & 63;
    const int64_t tile = first_tile + lane;
    bool live = false;
    if (lane < n && tile < a.tiles_per_dir) {
        const float tx = static_cast<float>((tile % a.tiles_x) * kTileW);
        const float ty = static_cast<float>((tile / a.tiles_x) * kTileH);
#pragma unroll
        for (int r = 0; r < kCullBoxes; ++r) {
            const float4 R = rects[r];
            live = live || !(tx >= R.y || tx + kTileW <= R.x || ty >= R.w || ty + kTileH <= R.z);
        }
    }
    return wave_ballot(live);
}

// Unit u (a direction, or a (design, direction) pair of a batched trace) and workgroup index blk
// (within the unit) of hardware workgroup b, for n_units units.  Direction-major:
// b = u * blocks_per_dir + blk.  XCD-major: the hardware places workgroup b on accelerator
// complex (XCD) b % 8, and unit u is traced by XCD u % 8 alone, its workgroups consecutive in that
// XCD's share of the grid; the grid is padded to whole groups of 8 units and a padding workgroup
// gets false.
__device__ __forceinline__ bool block_unit(const TraceArgs& a, int64_t n_units, int64_t b, int64_t& u, int32_t& blk)
{
    if (!a.xcd_major) {
        u = b / a.blocks_per_dir;
        blk = static_cast<int32_t>(b % a.blocks_per_dir);
        return true;
    }
    const int64_t k = b / kXcds;
    u = b % kXcds + kXcds * (k / a.blocks_per_dir);
    blk = static_cast<int32_t>(k % a.blocks_per_dir);
    return u < n_units;
}

// Pixel of lane `lane` in wave tile `tile`: 8 x 8 pixel tiles in row-major order (trace mode) or
// 64 consecutive entries of an explicit pixel list (records mode).
template <bool RECORDS>
__device__ __forceinline__ bool tile_pixel(const TraceArgs& a, int64_t tile, int lane, int64_t& pixel, int64_t& rec,
                                           int32_t& pi, int32_t& pk)
{
    if (RECORDS) {
        rec = tile * 64 + lane;
        const bool valid = rec < a.n_pix;
        pixel = valid ? (a.pix ? a.pix[rec] : rec) : 0;
        pi = static_cast<int32_t>(pixel % a.nu);
        pk = static_cast<int32_t>(pixel / a.nu);
        return valid;
    }
    // a grid holds at most 2^31 pixels, so tile and pixel indices fit 32 bits; the tile index is
    // wave-uniform, so its division runs once per wave
    rec = 0;
    const uint32_t t = static_cast<uint32_t>(tile), tiles_x = static_cast<uint32_t>(a.tiles_x);
    const uint32_t tx = t % tiles_x, ty = t / tiles_x;
    pi = static_cast<int32_t>(tx * kTileW + (lane & 7));
    pk = static_cast<int32_t>(ty * kTileH + (lane >> 3));
    pixel = static_cast<int64_t>(pi) + static_cast<int64_t>(pk) * a.nu;
    return pi < a.nu && pk < a.nv;
}

}  // namespace srp
