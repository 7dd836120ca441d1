// Surface-sampling SRP estimator (paper Sec. 3.2, "Estimation", and its equation for F) on gfx950.
//
// One lane evaluates one sample: a facet drawn by area (FP64 search of the cumulative areas in
// original facet order) and a uniform point x on it (square-root barycentric mapping); the light
// reaching x is gathered by path tracing with next-event estimation toward the Sun at every path
// vertex (one cosine-distributed gathering direction at x, then mirror or cosine continuations
// with weights rho_s/p_s and rho_d/(1 - p_s), up to bounces - 1 vertices); one sampled outgoing
// event at x (mirror with weight rho_s/p_s, else a cosine direction with rho_d/(1 - p_s)) turns
// every arriving contribution of power W and propagation p into the deposit W (p - reflected).
// The sample's force is the total area times that force density.
//
// Shadow rays: sunlight reaching a point along -s is blocked by a facet whose outward side faces
// the Sun (n.s > 0) and that the ray toward the Sun crosses; gathering rays take the closest facet
// whose outward side faces the ray (as the light rays of the ray-grid estimator do).
//
// Two ways to find intersections, selected at compile time:
//   BRUTE  every ray is tested against every triangle of its scene (the paper's massively
//          parallel test, usable when every sample belongs to a different design): the loop index
//          is wave-uniform, so triangle records arrive through scalar loads, once per wavefront;
//   BVH    the scene's BVH with an independent walk per lane (the samples of a wavefront are
//          scattered over the surface), any-hit for shadow rays.
//
// Random numbers: Philox4x32-10 with counter (sample, global direction, stage, design); stage 0:
// facet, two barycentric uniforms, the outgoing event; stage 1: the outgoing direction (2) and the
// first gathering direction (2); stage k + 1: the event at gathered vertex k and its direction.
#include <float.h>

#include "srp_internal.h"
#include "srp_path.h"
#include "srp_traverse.h"

namespace srp {
namespace {

constexpr int kSurfThreads = 256;  // samples per workgroup

// Moller-Trumbore test of the side facing AWAY from the ray (the outward side of a facet whose
// normal points along d): t of the crossing, or a negative value.
__device__ __forceinline__ float tri_hit_back(const float o[3], const float d[3], const float4& g0, const float4& g1,
                                              const float4& g2)
{
    const float px = d[1] * g2.z - d[2] * g2.y;
    const float py = d[2] * g2.x - d[0] * g2.z;
    const float pz = d[0] * g2.y - d[1] * g2.x;
    const float det = -(g1.x * px + g1.y * py + g1.z * pz);
    const float tx = o[0] - g0.x, ty = o[1] - g0.y, tz = o[2] - g0.z;
    const float uu = -(tx * px + ty * py + tz * pz);
    const float qx = ty * g1.z - tz * g1.y;
    const float qy = tz * g1.x - tx * g1.z;
    const float qz = tx * g1.y - ty * g1.x;
    const float vv = -(d[0] * qx + d[1] * qy + d[2] * qz);
    const float tnum = -(g2.x * qx + g2.y * qy + g2.z * qz);
    const float t = fast_div(tnum, det);
    const bool ok = det > 0.0f && uu >= 0.0f && uu <= det && vv >= 0.0f && uu + vv <= det && t > 0.0f;
    return ok ? t : -1.0f;
}

// Closest facet whose outward side faces the ray (o, d), other than `skip`; exact ties go to the
// lower original index.  BVH positions in, BVH position out (-1: none).
template <bool BRUTE>
__device__ __forceinline__ int gather_hit(const SurfaceScene& sc, const float o[3], const float d[3], int skip,
                                          float& t_out, int* __restrict__ lstack)
{
    if (!BRUTE) {
        int hit;
        closest_hit_lane((const BvhNode*)sc.nodes, (const TriRec*)sc.tris, o, d, true, skip, t_out, hit, lstack);
        return hit;
    }
    float tbest = FLT_MAX;
    int hit = -1, hit_id = 0x7fffffff;
    const TriRec* __restrict__ tris = (const TriRec*)sc.tris;
    for (int tri = 0; tri < sc.n_tris; ++tri) {
        const TriRec* T = tris + tri;
        const float4 g0 = T->f[0], g1 = T->f[1], g2 = T->f[2];
        const float t = tri_hit(o, d, g0, g1, g2);
        const int id = __float_as_int(g0.w);
        if (t > 0.0f && tri != skip && (t < tbest || (t == tbest && id < hit_id))) {
            tbest = t;
            hit = tri;
            hit_id = id;
        }
    }
    t_out = tbest;
    return hit;
}

// Is sunlight toward o (from direction s) blocked?  Any facet other than `skip` whose outward side
// faces the Sun and that the ray o + t s, t > 0, crosses.
template <bool BRUTE>
__device__ __forceinline__ bool sun_blocked(const SurfaceScene& sc, const float o[3], const float s[3], int skip,
                                            int* __restrict__ lstack)
{
    const TriRec* __restrict__ tris = (const TriRec*)sc.tris;
    if (BRUTE) {
        bool blocked = false;
        for (int tri = 0; tri < sc.n_tris; ++tri) {
            const TriRec* T = tris + tri;
            const float t = tri_hit_back(o, s, T->f[0], T->f[1], T->f[2]);
            blocked = blocked || (t > 0.0f && tri != skip);
        }
        return blocked;
    }
    // any-hit walk per lane: the first crossing ends it
    const BvhNode* __restrict__ nodes = (const BvhNode*)sc.nodes;
    const float ix = safe_rcp(s[0]), iy = safe_rcp(s[1]), iz = safe_rcp(s[2]);
    const float nx = -o[0] * ix, ny = -o[1] * iy, nz = -o[2] * iz;
    int sp = 0;
    int cur = 0;
    while (cur != kWalkDone) {
        if (cur >= 0) {
            const BvhNode* N = nodes + cur;
            const float4 f0 = N->f[0], f1 = N->f[1], f2 = N->f[2], f3 = N->f[3];
            const int c0 = __float_as_int(f3.x), c1 = __float_as_int(f3.y);
            const float ax0 = fmaf(f0.x, ix, nx), ax1 = fmaf(f0.y, ix, nx);
            const float ay0 = fmaf(f0.z, iy, ny), ay1 = fmaf(f0.w, iy, ny);
            const float az0 = fmaf(f2.x, iz, nz), az1 = fmaf(f2.y, iz, nz);
            const float bx0 = fmaf(f1.x, ix, nx), bx1 = fmaf(f1.y, ix, nx);
            const float by0 = fmaf(f1.z, iy, ny), by1 = fmaf(f1.w, iy, ny);
            const float bz0 = fmaf(f2.z, iz, nz), bz1 = fmaf(f2.w, iz, nz);
            const float tn0 = fmaxf(fmaxf(fminf(ax0, ax1), fminf(ay0, ay1)), fmaxf(fminf(az0, az1), 0.0f));
            const float tf0 = fminf(fminf(fmaxf(ax0, ax1), fmaxf(ay0, ay1)), fmaxf(az0, az1));
            const float tn1 = fmaxf(fmaxf(fminf(bx0, bx1), fminf(by0, by1)), fmaxf(fminf(bz0, bz1), 0.0f));
            const float tf1 = fminf(fminf(fmaxf(bx0, bx1), fmaxf(by0, by1)), fmaxf(bz0, bz1));
            const bool h0 = tn0 <= tf0;
            const bool h1 = tn1 <= tf1;
            if (h0 && h1) {
                lstack[sp * 64] = c1;
                ++sp;
                cur = c0;
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
            bool found = false;
            for (int q = 0; q < cnt; ++q) {
                const int tri = first + q;
                const TriRec* T = tris + tri;
                const float t = tri_hit_back(o, s, T->f[0], T->f[1], T->f[2]);
                found = found || (t > 0.0f && tri != skip);
            }
            if (found) return true;
            if (sp > 0) {
                --sp;
                cur = lstack[sp * 64];
            } else {
                cur = kWalkDone;
            }
        }
    }
    return false;
}

__device__ __forceinline__ void cosine_dir(const float n[3], float u1, float u2, float out[3])
{
    const float rad = sqrtf(u1);
    float sphi, cphi;
    sincosf(6.283185307179586f * u2, &sphi, &cphi);
    const float px = rad * cphi, py = rad * sphi, pz = sqrtf(fmaxf(0.0f, 1.0f - u1));
    float t1[3], t2[3];
    duff_basis<float>(n, t1, t2);
    for (int a = 0; a < 3; ++a) out[a] = px * t1[a] + py * t2[a] + pz * n[a];
}

// A direction on the hemisphere of n and its weight relative to cosine sampling: cosine-distributed
// (the Lambertian BRDF's importance sampling, weight 1) or, with `uniform`, uniform over solid angle
// (cos theta = u1, weight 2 cos theta).
__device__ __forceinline__ float hemi_dir(const float n[3], float u1, float u2, bool uniform, float out[3])
{
    if (!uniform) {
        cosine_dir(n, u1, u2, out);
        return 1.0f;
    }
    const float rad = sqrtf(fmaxf(0.0f, 1.0f - u1 * u1));
    float sphi, cphi;
    sincosf(6.283185307179586f * u2, &sphi, &cphi);
    const float px = rad * cphi, py = rad * sphi, pz = u1;
    float t1[3], t2[3];
    duff_basis<float>(n, t1, t2);
    for (int a = 0; a < 3; ++a) out[a] = px * t1[a] + py * t2[a] + pz * n[a];
    return 2.0f * u1;
}

__device__ __forceinline__ void philox_at(uint32_t sample, uint32_t dir, uint32_t stage, uint32_t design,
                                          const SurfaceArgs& a, float u[4])
{
    uint32_t c0 = sample, c1 = dir, c2 = stage, c3 = design;
    philox4x32_10(c0, c1, c2, c3, a.seed_lo, a.seed_hi);
    u[0] = unit24(c0);
    u[1] = unit24(c1);
    u[2] = unit24(c2);
    u[3] = unit24(c3);
}

// One sample: force and torque (area applied) and its record.
template <bool BRUTE>
__device__ __forceinline__ void surface_sample(const SurfaceArgs& a, const SurfaceScene& sc, const float s[3],
                                               uint32_t sample, uint32_t dir, uint32_t design, float F[3], float T[3],
                                               int32_t& rec_facet, int32_t* rec_hits, int32_t& rec_lit,
                                               int* __restrict__ lstack)
{
    float u0[4], u1[4];
    uint32_t c0 = sample, c1 = dir, c2 = 0u, c3 = design;
    philox4x32_10(c0, c1, c2, c3, a.seed_lo, a.seed_hi);
    philox_at(sample, dir, 1u, design, a, u1);
    // facet by area (FP64, original facet order): the first f with u A < cum[f]
    const double* __restrict__ cum = (const double*)sc.cum_area;
    // stratified: sample i of N takes the area coordinate (i + u) / N
    const double uf = (a.sampling & 1)
                          ? (static_cast<double>(sample) + static_cast<double>(unit24(c0))) / static_cast<double>(a.n_samples)
                          : static_cast<double>(unit24(c0));
    const double target = uf * sc.area;
    int lo = 0, hi = sc.n_tris - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (target < cum[mid])
            hi = mid;
        else
            lo = mid + 1;
    }
    rec_facet = lo;
    const int p = ((const int32_t*)sc.bvh_pos)[lo];
    const TriRec tr = ((const TriRec*)sc.tris)[p];
    const float4 mt = ((const float4*)sc.mat)[p];
    u0[1] = unit24(c1);
    u0[2] = unit24(c2);
    u0[3] = unit24(c3);
    const float sq = sqrtf(u0[1]);
    const float b1 = sq * (1.0f - u0[2]), b2 = sq * u0[2];
    float x[3], n[3], o[3];
    const float v0[3] = {tr.f[0].x, tr.f[0].y, tr.f[0].z};
    const float e1[3] = {tr.f[1].x, tr.f[1].y, tr.f[1].z};
    const float e2[3] = {tr.f[2].x, tr.f[2].y, tr.f[2].z};
    n[0] = tr.f[1].w;
    n[1] = tr.f[2].w;
    n[2] = tr.f[3].x;
    for (int c = 0; c < 3; ++c) {
        x[c] = v0[c] + b1 * e1[c] + b2 * e2[c];
        o[c] = x[c] + sc.eps * n[c];
    }
    const float rs = mt.x, rd = mt.y, ps = mt.z;
    const bool uniform = (a.sampling & 2) != 0;
    const bool mirror = u0[3] < ps;
    float odir[3], w[3];
    const float wo = hemi_dir(n, u1[0], u1[1], uniform, odir);
    const float wg = hemi_dir(n, u1[2], u1[3], uniform, w);
    const float kout = mirror ? rs / ps : (rd > 0.0f ? rd / (1.0f - ps) * wo : 0.0f);
    float dep[3] = {0.0f, 0.0f, 0.0f};
    int32_t lit = 0;
    const float cs = n[0] * s[0] + n[1] * s[1] + n[2] * s[2];
    if (cs > 0.0f && !sun_blocked<BRUTE>(sc, o, s, p, lstack)) {
        lit |= 1;
        const float W = a.flux_c * cs;
        const float pv[3] = {-s[0], -s[1], -s[2]};
        const float pn = pv[0] * n[0] + pv[1] * n[1] + pv[2] * n[2];
        for (int c = 0; c < 3; ++c) {
            const float r = pv[c] - 2.0f * pn * n[c];
            dep[c] += W * (pv[c] - kout * (mirror ? r : odir[c]));
        }
    }
    if (a.bounces >= 2) {
        float ro[3] = {o[0], o[1], o[2]}, rdir[3] = {w[0], w[1], w[2]};
        int skip = p;
        float beta = 1.0f, radiance = 0.0f;
        for (int k = 1; k <= a.bounces - 1; ++k) {
            float t;
            const int g = gather_hit<BRUTE>(sc, ro, rdir, skip, t, lstack);
            if (g < 0) break;
            const TriRec tg = ((const TriRec*)sc.tris)[g];
            if (rec_hits) rec_hits[k - 1] = __float_as_int(tg.f[0].w);
            const float4 mg = ((const float4*)sc.mat)[g];
            const float ng[3] = {tg.f[1].w, tg.f[2].w, tg.f[3].x};
            float oy[3];
            for (int c = 0; c < 3; ++c) oy[c] = ro[c] + t * rdir[c] + sc.eps * ng[c];
            const float cg = ng[0] * s[0] + ng[1] * s[1] + ng[2] * s[2];
            if (mg.y > 0.0f && cg > 0.0f && !sun_blocked<BRUTE>(sc, oy, s, g, lstack)) {
                lit |= 1 << k;
                radiance += beta * mg.y * cg;
            }
            if (k == a.bounces - 1) break;
            float ev[4];
            philox_at(sample, dir, static_cast<uint32_t>(k + 1), design, a, ev);
            float nd[3];
            if (ev[0] < mg.z) {
                const float dn = rdir[0] * ng[0] + rdir[1] * ng[1] + rdir[2] * ng[2];
                for (int c = 0; c < 3; ++c) nd[c] = rdir[c] - 2.0f * dn * ng[c];
                beta *= mg.x / mg.z;
            } else {
                const float wv = hemi_dir(ng, ev[1], ev[2], uniform, nd);
                beta *= mg.y > 0.0f ? mg.y / (1.0f - mg.z) * wv : 0.0f;
            }
            if (beta == 0.0f) break;
            for (int c = 0; c < 3; ++c) {
                ro[c] = oy[c];
                rdir[c] = nd[c];
            }
            skip = g;
        }
        if (radiance > 0.0f) {
            const float W = a.flux_c * radiance * wg;
            const float pv[3] = {-w[0], -w[1], -w[2]};
            const float pn = pv[0] * n[0] + pv[1] * n[1] + pv[2] * n[2];
            for (int c = 0; c < 3; ++c) {
                const float r = pv[c] - 2.0f * pn * n[c];
                dep[c] += W * (pv[c] - kout * (mirror ? r : odir[c]));
            }
        }
    }
    const float A = static_cast<float>(sc.area);
    for (int c = 0; c < 3; ++c) F[c] = A * dep[c];
    const float lx = x[0] - sc.com[0], ly = x[1] - sc.com[1], lz = x[2] - sc.com[2];
    T[0] = ly * F[2] - lz * F[1];
    T[1] = lz * F[0] - lx * F[2];
    T[2] = lx * F[1] - ly * F[0];
    rec_lit = lit;
}

// Workgroup = kSurfThreads consecutive samples of one unit (scene, direction).
template <bool BRUTE>
__global__ __launch_bounds__(kSurfThreads) void k_surface(SurfaceArgs a)
{
    __shared__ int s_lane[kSurfThreads / 64][kLaneStack][64];
    __shared__ float s_red[kSurfThreads / 64][6];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t u = blockIdx.x / a.chunks;
    const int64_t chunk = blockIdx.x % a.chunks;
    const int64_t scene = u / a.D, j = u % a.D;
    const int64_t i = chunk * kSurfThreads + threadIdx.x;
    const bool valid = i < a.n_samples;
    const SurfaceScene sc = a.scenes[scene];
    const float s[3] = {static_cast<float>(a.sun[3 * j]), static_cast<float>(a.sun[3 * j + 1]),
                        static_cast<float>(a.sun[3 * j + 2])};
    float F[3] = {0.0f, 0.0f, 0.0f}, T[3] = {0.0f, 0.0f, 0.0f};
    int32_t hits[kMaxBounces];
    for (int k = 0; k < kMaxBounces; ++k) hits[k] = -1;
    int32_t facet = -1, lit = 0;
    // brute force keeps every lane in the wave-uniform triangle loops; the walk skips invalid lanes
    if (BRUTE || valid)
        surface_sample<BRUTE>(a, sc, s, static_cast<uint32_t>(valid ? i : 0), static_cast<uint32_t>(a.dir_index_base + j),
                              a.design_index + static_cast<uint32_t>(scene), F, T, facet,
                              a.rec_hits ? hits : nullptr, lit, &s_lane[wave][0][lane]);
    if (!valid)
        for (int c = 0; c < 3; ++c) F[c] = T[c] = 0.0f;
    if (valid && a.rec_facet) {
        const int64_t r = u * a.n_samples + i;
        a.rec_facet[r] = facet;
        a.rec_lit[r] = lit;
        if (a.rec_hits)
            for (int k = 0; k < a.bounces - 1; ++k) a.rec_hits[r * (a.bounces - 1) + k] = hits[k];
    }
    float acc[6] = {F[0], F[1], F[2], T[0], T[1], T[2]};
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[c] = wave_sum(acc[c]);
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < 6; ++c) s_red[wave][c] = acc[c];
    __syncthreads();
    if (threadIdx.x < 6) {
        double sum = 0.0;
        for (int q = 0; q < kSurfThreads / 64; ++q) sum += static_cast<double>(s_red[q][threadIdx.x]);
        a.partials[(u * a.chunks + chunk) * 6 + threadIdx.x] = sum;
    }
}

// Fixed-order mean over the workgroups of each unit.
__global__ void k_surface_mean(const double* __restrict__ partials, int64_t units, int32_t chunks, double inv_n,
                               double* __restrict__ force, double* __restrict__ torque)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= units * 6) return;
    const int64_t u = t / 6;
    const int c = static_cast<int>(t % 6);
    double sum = 0.0;
    for (int32_t k = 0; k < chunks; ++k) sum += partials[(u * chunks + k) * 6 + c];
    if (c < 3)
        force[3 * u + c] = sum * inv_n;
    else if (torque)
        torque[3 * u + c - 3] = sum * inv_n;
}

}  // namespace

hipError_t launch_surface(const SurfaceArgs& a, bool brute, double* force, double* torque, hipStream_t stream)
{
    const int64_t units = static_cast<int64_t>(a.n_scenes) * a.D;
    const int64_t blocks = units * a.chunks;
    if (blocks == 0) return hipSuccess;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    if (brute)
        hipLaunchKernelGGL(k_surface<true>, dim3(static_cast<unsigned>(blocks)), dim3(kSurfThreads), 0, stream, a);
    else
        hipLaunchKernelGGL(k_surface<false>, dim3(static_cast<unsigned>(blocks)), dim3(kSurfThreads), 0, stream, a);
    const int threads = 256;
    hipLaunchKernelGGL(k_surface_mean, dim3(static_cast<unsigned>((units * 6 + threads - 1) / threads)), dim3(threads),
                       0, stream, a.partials, units, a.chunks, 1.0 / static_cast<double>(a.n_samples), force, torque);
    return hipGetLastError();
}

}  // namespace srp
