// Visibility-edge terms of the hinge-angle gradient by edge sampling, gfx950.
//
// Per sun direction the ray grid estimates F = (Phi/c) int g(y) dy over the grid plane, g(y) the
// momentum a unit-weight path started at image point y deposits.  Turning a hinge moves the
// images of the edges of the facets it carries, across which g jumps (silhouettes, edges between
// facets, occlusion of one part by another).  Besides the pathwise part that k_adjoint computes
// (every path at its image position with its facet sequence held), the derivative has, for every
// moving edge, (Phi/c) int_edge (g(y - delta n) - g(y + delta n)) v_n dl: n the edge's unit
// normal in the grid plane, v_n the normal image velocity of the edge point under the rotation.
//
// Across an edge where the moving surface continues in one plane with the same material on both
// sides, g is continuous (the two side paths meet the same plane and material and leave with the
// same draws; their deposits differ by O(delta)), so such edges carry no term and are left out:
// k_edge_keep marks them from facet pairs found on the host, and only the other edges are launched.
//
// k_edge_keep  one thread per moving edge: compares the packed materials of its facet pairs.
// k_edge_term  one lane per (edge, sample): sample s = (m + xi)/M along moving edge e (e its index
//              among all moving edges), the two side points y -+ delta n (delta = the
//              secondary-ray offset, 1e-5 L) each start a full path with the same Philox draws
//              (key seed ^ kEdgeKey, counter (e M + m, direction, bounce, design)), and the lane
//              adds (Phi/c)(len/M) v_n (deposit(y-) - deposit(y+)) contracted with the direction's
//              cotangents to its hinge.  Paths are walked per lane: a wave holds the samples of
//              a few edges that can each span the whole panel, so the union of the nodes its side
//              paths need is large (the wave-coherent walk, tried for the parallel first segments,
//              took twice as long).  The lane's two side paths run 2 delta apart, mostly through
//              the same nodes and, after equal interactions, in the same directions, so both are
//              walked in one traversal (closest_hit_pair) that fetches each node once.
// k_add_edges  per-direction sums of the workgroup partials, added in a fixed order to the
//              per-direction hinge sums of the adjoint.
#include <float.h>

#include "srp_internal.h"
#include "srp_path.h"
#include "srp_traverse.h"

namespace srp {
namespace {

constexpr uint64_t kEdgeKey = 0x9E3779B97F4A7C15ull;

__device__ __forceinline__ void cross3e(const float a[3], const float b[3], float r[3])
{
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}

// One unit-weight path from o along d; its force and torque about com.
template <bool LANE>
__device__ __forceinline__ void edge_path(const BvhNode* __restrict__ nodes, const TriRec* __restrict__ tris,
                                          const float4* __restrict__ mat, float o[3], float d[3], bool alive,
                                          int bounces, uint32_t ctr0, uint32_t dir, uint32_t design, uint32_t key_lo,
                                          uint32_t key_hi, float eps, const float com[3], int* stack, int* lstack,
                                          float F[3], float T[3])
{
    float w = 1.0f;
    int skip = -1;
    for (int c = 0; c < 3; ++c) F[c] = T[c] = 0.0f;
    for (int b = 1; b <= bounces; ++b) {
        if (wave_ballot(alive) == 0) break;
        float t;
        int hit;
        if (LANE)
            closest_hit_lane(nodes, tris, o, d, alive, skip, t, hit, lstack);
        else
            closest_hit(nodes, tris, o, d, alive, skip, t, hit, stack);
        if (!alive) continue;
        if (hit < 0) {
            alive = false;
            continue;
        }
        const TriRec tr = tris[hit];
        const float4 mt = mat[hit];
        const float n[3] = {tr.f[1].w, tr.f[2].w, tr.f[3].x};
        float x[3], g[3];
        alive = interact(o, d, w, t, n, mt.x, mt.y, mt.z, b, bounces, ctr0, dir, design, key_lo, key_hi, eps, x, g);
        const float l[3] = {x[0] - com[0], x[1] - com[1], x[2] - com[2]};
        float tq[3];
        cross3e(l, g, tq);
        for (int c = 0; c < 3; ++c) {
            F[c] += g[c];
            T[c] += tq[c];
        }
        skip = hit;
    }
}

// Closest hits of a lane's two side rays in one per-lane walk: a node is entered when either ray
// meets its box before that ray's best hit, the nearer child first by the smaller of the two rays'
// entry distances, and a leaf's triangles are tested against both rays.  Every node a ray meets is
// visited and a ray's closest hit (with its index tie-break) does not depend on the visiting
// order, so each ray gets the hit of its own walk (closest_hit_lane); the two rays start 2 delta
// apart along one direction and mostly visit the same nodes, whose records are fetched once.
__device__ __forceinline__ void closest_hit_pair(const BvhNode* __restrict__ nodes, const TriRec* __restrict__ tris,
                                                 const float (&o)[2][3], const float (&d)[2][3],
                                                 const bool (&alive)[2], const int (&skip)[2], float (&t_out)[2],
                                                 int (&hit_out)[2], int* __restrict__ lstack)
{
    float ix[2], iy[2], iz[2], nx[2], ny[2], nz[2], tbest[2];
    int hit_id[2];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        ix[r] = safe_rcp(d[r][0]);
        iy[r] = safe_rcp(d[r][1]);
        iz[r] = safe_rcp(d[r][2]);
        nx[r] = -o[r][0] * ix[r];
        ny[r] = -o[r][1] * iy[r];
        nz[r] = -o[r][2] * iz[r];
        tbest[r] = alive[r] ? FLT_MAX : -1.0f;
        hit_out[r] = -1;
        hit_id[r] = 0x7fffffff;
    }
    int sp = 0;
    int cur = alive[0] || alive[1] ? 0 : kWalkDone;
    while (cur != kWalkDone) {
        if (cur >= 0) {
            const BvhNode* N = nodes + cur;
            const float4 f0 = N->f[0];
            const float4 f1 = N->f[1];
            const float4 f2 = N->f[2];
            const float4 f3 = N->f[3];
            const int c0 = __float_as_int(f3.x);
            const int c1 = __float_as_int(f3.y);
            bool h0 = false, h1 = false;
            float n0 = FLT_MAX, n1 = FLT_MAX;
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const float ax0 = fmaf(f0.x, ix[r], nx[r]), ax1 = fmaf(f0.y, ix[r], nx[r]);
                const float ay0 = fmaf(f0.z, iy[r], ny[r]), ay1 = fmaf(f0.w, iy[r], ny[r]);
                const float az0 = fmaf(f2.x, iz[r], nz[r]), az1 = fmaf(f2.y, iz[r], nz[r]);
                const float bx0 = fmaf(f1.x, ix[r], nx[r]), bx1 = fmaf(f1.y, ix[r], nx[r]);
                const float by0 = fmaf(f1.z, iy[r], ny[r]), by1 = fmaf(f1.w, iy[r], ny[r]);
                const float bz0 = fmaf(f2.z, iz[r], nz[r]), bz1 = fmaf(f2.w, iz[r], nz[r]);
                const float tn0 = fmaxf(fmaxf(fminf(ax0, ax1), fminf(ay0, ay1)), fmaxf(fminf(az0, az1), 0.0f));
                const float tf0 = fminf(fminf(fmaxf(ax0, ax1), fmaxf(ay0, ay1)), fminf(fmaxf(az0, az1), tbest[r]));
                const float tn1 = fmaxf(fmaxf(fminf(bx0, bx1), fminf(by0, by1)), fmaxf(fminf(bz0, bz1), 0.0f));
                const float tf1 = fminf(fminf(fmaxf(bx0, bx1), fmaxf(by0, by1)), fminf(fmaxf(bz0, bz1), tbest[r]));
                if (tn0 <= tf0) {
                    h0 = true;
                    n0 = fminf(n0, tn0);
                }
                if (tn1 <= tf1) {
                    h1 = true;
                    n1 = fminf(n1, tn1);
                }
            }
            if (h0 && h1) {
                const bool swap = n1 < n0;
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
                const int id = __float_as_int(g0.w);
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const float t = tri_hit(o[r], d[r], g0, g1, g2);
                    if (t > 0.0f && tri != skip[r] && (t < tbest[r] || (t == tbest[r] && id < hit_id[r]))) {
                        tbest[r] = t;
                        hit_out[r] = tri;
                        hit_id[r] = id;
                    }
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
    t_out[0] = tbest[0];
    t_out[1] = tbest[1];
}

// edge_path<true> for both side paths of a lane at once, every segment walked by closest_hit_pair;
// each path takes exactly the steps it takes alone.
__device__ __forceinline__ void edge_paths_pair(const BvhNode* __restrict__ nodes, const TriRec* __restrict__ tris,
                                                const float4* __restrict__ mat, float (&o)[2][3], float (&d)[2][3],
                                                bool live, int bounces, uint32_t ctr0, uint32_t dir, uint32_t design,
                                                uint32_t key_lo, uint32_t key_hi, float eps, const float com[3],
                                                int* lstack, float (&F)[2][3], float (&T)[2][3])
{
    float w[2] = {1.0f, 1.0f};
    int skip[2] = {-1, -1};
    bool alive[2] = {live, live};
#pragma unroll
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) F[r][c] = T[r][c] = 0.0f;
    for (int b = 1; b <= bounces; ++b) {
        if (wave_ballot(alive[0] || alive[1]) == 0) break;
        float t[2];
        int hit[2];
        closest_hit_pair(nodes, tris, o, d, alive, skip, t, hit, lstack);
#pragma unroll
        for (int r = 0; r < 2; ++r) {
            if (!alive[r]) continue;
            if (hit[r] < 0) {
                alive[r] = false;
                continue;
            }
            const TriRec tr = tris[hit[r]];
            const float4 mt = mat[hit[r]];
            const float n[3] = {tr.f[1].w, tr.f[2].w, tr.f[3].x};
            float x[3], g[3];
            alive[r] = interact(o[r], d[r], w[r], t[r], n, mt.x, mt.y, mt.z, b, bounces, ctr0, dir, design, key_lo,
                                key_hi, eps, x, g);
            const float l[3] = {x[0] - com[0], x[1] - com[1], x[2] - com[2]};
            float tq[3];
            cross3e(l, g, tq);
            for (int c = 0; c < 3; ++c) {
                F[r][c] += g[c];
                T[r][c] += tq[c];
            }
            skip[r] = hit[r];
        }
    }
}

// Five waves per SIMD (96 VGPRs, a few spilled around the walk) beat four without spills (124
// VGPRs): the divergent per-lane walks wait on fetches, and a fifth wave hides more of that.
template <bool LANE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_edge_term(EdgeArgs E, const BvhNode* __restrict__ nodes,
                                                   const TriRec* __restrict__ tris, const float4* __restrict__ mat,
                                                   const DevFrame* __restrict__ frames,
                                                   const double* __restrict__ g_force,
                                                   const double* __restrict__ g_torque,
                                                   double* __restrict__ partials)
{
    __shared__ int s_stack[kWaves][kStackDepth];
    __shared__ int s_lane[kWaves][kLaneStack][64];
    __shared__ float s_red[kWaves][kMaxHinges];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t j = blockIdx.y;
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t n_samp = static_cast<int64_t>(E.n_edges) * E.samples;
    const bool valid = idx < n_samp;
    const int e = valid ? static_cast<int>(idx / E.samples) : 0;
    const int m = valid ? static_cast<int>(idx % E.samples) : 0;
    const DevFrame fr = frames[j];
    const uint32_t dir = static_cast<uint32_t>(E.dir_index_base + j);
    const int4 ed = E.edges[e];
    const float4 p0v = E.verts[ed.x], p1v = E.verts[ed.y];
    const float p0[3] = {p0v.x, p0v.y, p0v.z}, p1[3] = {p1v.x, p1v.y, p1v.z};
    const int h = ed.z;
    // grid-plane axes and pixel sizes of the frame
    const float du = sqrtf(fr.U[0] * fr.U[0] + fr.U[1] * fr.U[1] + fr.U[2] * fr.U[2]);
    const float dv = sqrtf(fr.V[0] * fr.V[0] + fr.V[1] * fr.V[1] + fr.V[2] * fr.V[2]);
    const float u[3] = {fr.U[0] / du, fr.U[1] / du, fr.U[2] / du};
    const float v[3] = {fr.V[0] / dv, fr.V[1] / dv, fr.V[2] / dv};
    const float r0[3] = {p0[0] - fr.o0[0], p0[1] - fr.o0[1], p0[2] - fr.o0[2]};
    const float r1[3] = {p1[0] - fr.o0[0], p1[1] - fr.o0[1], p1[2] - fr.o0[2]};
    const float y0u = r0[0] * u[0] + r0[1] * u[1] + r0[2] * u[2];
    const float y0v = r0[0] * v[0] + r0[1] * v[1] + r0[2] * v[2];
    const float tu = (r1[0] * u[0] + r1[1] * u[1] + r1[2] * u[2]) - y0u;
    const float tv = (r1[0] * v[0] + r1[1] * v[1] + r1[2] * v[2]) - y0v;
    const float len = sqrtf(tu * tu + tv * tv);
    const bool live = valid && len > 0.0f;  // an edge seen end-on sweeps no area
    const float nu_ = live ? tv / len : 0.0f, nv_ = live ? -tu / len : 0.0f;
    const uint32_t key_lo = E.seed_lo ^ static_cast<uint32_t>(kEdgeKey);
    const uint32_t key_hi = E.seed_hi ^ static_cast<uint32_t>(kEdgeKey >> 32);
    const uint32_t ctr0 = static_cast<uint32_t>(static_cast<int64_t>(ed.w) * E.samples + m);
    uint32_t c0 = ctr0, c1 = dir, c2 = 0u, c3 = E.design_index;
    philox4x32_10(c0, c1, c2, c3, key_lo, key_hi);
    const float sp = (static_cast<float>(m) + unit24(c0)) / static_cast<float>(E.samples);
    // the edge point, its image, and its image velocity under the rotation about hinge h
    float x[3], rx[3], xd[3];
    for (int c = 0; c < 3; ++c) x[c] = p0[c] + sp * (p1[c] - p0[c]);
    for (int c = 0; c < 3; ++c) rx[c] = x[c] - E.hinge_origin[h & 3][c];
    cross3e(E.hinge_axis[h & 3], rx, xd);
    const float vn = (xd[0] * u[0] + xd[1] * u[1] + xd[2] * u[2]) * nu_ +
                     (xd[0] * v[0] + xd[1] * v[1] + xd[2] * v[2]) * nv_;
    const float yu = y0u + sp * tu, yv = y0v + sp * tv;
    float Fs[2][3], Ts[2][3];
    int* stack = s_stack[wave];
    int* lstack = &s_lane[wave][0][lane];
    if (LANE) {
        float o[2][3], d[2][3];
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const float sg = side == 0 ? -E.delta : E.delta;
            const float au = yu + sg * nu_, av = yv + sg * nv_;
            for (int c = 0; c < 3; ++c) {
                o[side][c] = fr.o0[c] + au * u[c] + av * v[c];
                d[side][c] = fr.d[c];
            }
        }
        edge_paths_pair(nodes, tris, mat, o, d, live, E.bounces, ctr0, dir, E.design_index, key_lo, key_hi, E.eps,
                        E.com, lstack, Fs, Ts);
    } else {
        for (int side = 0; side < 2; ++side) {
            const float sg = side == 0 ? -E.delta : E.delta;
            const float au = yu + sg * nu_, av = yv + sg * nv_;
            float o[3], d[3];
            for (int c = 0; c < 3; ++c) {
                o[c] = fr.o0[c] + au * u[c] + av * v[c];
                d[c] = fr.d[c];
            }
            edge_path<false>(nodes, tris, mat, o, d, live, E.bounces, ctr0, dir, E.design_index, key_lo, key_hi,
                             E.eps, E.com, stack, lstack, Fs[side], Ts[side]);
        }
    }
    // contribution to dL/d theta_h, L = gF . F + gT . tau
    const float flux_c = fr.w / (du * dv);
    const float scale = live ? flux_c * len / static_cast<float>(E.samples) * vn : 0.0f;
    float gF[3], gT[3] = {0.0f, 0.0f, 0.0f};
    for (int c = 0; c < 3; ++c) gF[c] = static_cast<float>(g_force[3 * j + c]);
    if (g_torque)
        for (int c = 0; c < 3; ++c) gT[c] = static_cast<float>(g_torque[3 * j + c]);
    float Lc = 0.0f;
    for (int c = 0; c < 3; ++c) Lc += gF[c] * (Fs[0][c] - Fs[1][c]) + gT[c] * (Ts[0][c] - Ts[1][c]);
    Lc *= scale;
    float acc[kMaxHinges];
#pragma unroll
    for (int k = 0; k < kMaxHinges; ++k) acc[k] = wave_sum(h == k ? Lc : 0.0f);
    if (lane == 0)
        for (int k = 0; k < kMaxHinges; ++k) s_red[wave][k] = acc[k];
    __syncthreads();
    if (threadIdx.x < kMaxHinges) {
        double s = 0.0;
        for (int q = 0; q < kWaves; ++q) s += static_cast<double>(s_red[q][threadIdx.x]);
        partials[(j * gridDim.x + blockIdx.x) * kMaxHinges + threadIdx.x] = s;
    }
}

__device__ __forceinline__ bool same_material(float4 a, float4 b)
{
    return a.x == b.x && a.y == b.y && a.z == b.z;
}

__global__ void k_edge_keep(const int4* __restrict__ pairs, int32_t n, const int32_t* __restrict__ bvh_pos,
                            const float4* __restrict__ mat, int32_t* __restrict__ keep)
{
    const int32_t i = static_cast<int32_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int4 p = pairs[i];
    bool flat = p.x >= 0 && same_material(mat[bvh_pos[p.x]], mat[bvh_pos[p.y]]);
    if (flat && p.z >= 0) flat = same_material(mat[bvh_pos[p.z]], mat[bvh_pos[p.w]]);
    keep[i] = flat ? 0 : 1;
}

__global__ void k_add_edges(const double* __restrict__ partials, int64_t D, int32_t blocks,
                            double* __restrict__ per_dir)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= D * kMaxHinges) return;
    const int64_t j = t / kMaxHinges;
    const int k = static_cast<int>(t % kMaxHinges);
    double s = 0.0;
    for (int32_t b = 0; b < blocks; ++b) s += partials[(j * blocks + b) * kMaxHinges + k];
    per_dir[t] += s;
}

}  // namespace

int32_t edge_blocks(const EdgeArgs& E)
{
    const int64_t n = static_cast<int64_t>(E.n_edges) * E.samples;
    return static_cast<int32_t>((n + 255) / 256);
}

hipError_t launch_edge_keep(const int4* pairs, int32_t n, const int32_t* bvh_pos, const float4* mat, int32_t* keep,
                            hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_edge_keep, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, stream, pairs, n,
                       bvh_pos, mat, keep);
    return hipGetLastError();
}

hipError_t launch_edge_term(const EdgeArgs& E, const BvhNode* nodes, const TriRec* tris, const float4* mat,
                            const DevFrame* frames, const double* g_force, const double* g_torque, int lane_walk,
                            double* partials, double* per_dir, hipStream_t stream)
{
    const int32_t nb = edge_blocks(E);
    if (E.D <= 0 || nb <= 0) return hipSuccess;
    if (E.D > 65535) return hipErrorInvalidValue;
    dim3 grid(static_cast<unsigned>(nb), static_cast<unsigned>(E.D));
    if (lane_walk)
        hipLaunchKernelGGL((k_edge_term<true>), grid, dim3(64 * kWaves), 0, stream, E, nodes, tris, mat, frames, g_force,
                           g_torque, partials);
    else
        hipLaunchKernelGGL((k_edge_term<false>), grid, dim3(64 * kWaves), 0, stream, E, nodes, tris, mat, frames,
                           g_force, g_torque, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nt = E.D * kMaxHinges;
    hipLaunchKernelGGL(k_add_edges, dim3(static_cast<unsigned>((nt + 255) / 256)), dim3(256), 0, stream, partials, E.D,
                       nb, per_dir);
    return hipGetLastError();
}

}  // namespace srp
