// Surface-sampling SRP estimator (paper Sec. 3.2, "Estimation", and its equation for F) on gfx950.
//
// One lane evaluates one sample: a facet drawn by area (FP64 search of the cumulative areas in
// original facet order) and a uniform point x on it (square-root barycentric mapping); the light
// reaching x is gathered by path tracing with next-event estimation toward the Sun at every path
// vertex (one cosine-distributed gathering direction at x, then specular or cosine continuations
// with weights rho_s/p_s (times the lobe weight) and rho_d/(1 - p_s), up to bounces - 1
// vertices); one sampled outgoing event at x (specular with weight rho_s/p_s, else a cosine
// direction with rho_d/(1 - p_s)) turns every arriving contribution of power W and propagation p
// into the deposit W (p - reflected).  The sample's force is the total area times that force
// density.
//
// Materials: the modified Phong BRDF rho_d/pi + rho_s (m + 2)/(2 pi) ((r.o)+)^m (Lafortune and
// Willems 1994), r the mirror direction of the arriving light, exponent m per facet (mat.w;
// +infinity is the ideal mirror).  A specular event draws o about r with cos(alpha) =
// u^(1/(m+1)) (the lobe's importance sampling), weight (m + 2)/(m + 1) (n.o)+ per unit rho_s, or
// under the plain-MC option uniformly over the hemisphere, weight (m + 2) ((r.o)+)^m (n.o).
// Sunlight that a gathered vertex reflects into its lobe toward the previous vertex is added by
// next-event estimation like its Lambertian share.
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

// The specular event for light of propagation p at a point with normal n: the outgoing direction
// and its weight per unit rho_s (see the header comment); m = +infinity is the ideal mirror.
__device__ __forceinline__ float specular_dir(const float p[3], const float n[3], float m, float u1, float u2,
                                              bool uniform, float out[3])
{
    const float pn = p[0] * n[0] + p[1] * n[1] + p[2] * n[2];
    float r[3];
    for (int c = 0; c < 3; ++c) r[c] = p[c] - 2.0f * pn * n[c];
    if (!(m < INFINITY)) {
        for (int c = 0; c < 3; ++c) out[c] = r[c];
        return 1.0f;
    }
    if (uniform) {
        hemi_dir(n, u1, u2, true, out);
        const float ro = fmaxf(0.0f, r[0] * out[0] + r[1] * out[1] + r[2] * out[2]);
        return (m + 2.0f) * powf(ro, m) * (n[0] * out[0] + n[1] * out[1] + n[2] * out[2]);
    }
    const float ca = powf(u1, 1.0f / (m + 1.0f));
    const float sa = sqrtf(fmaxf(0.0f, 1.0f - ca * ca));
    float sphi, cphi;
    sincosf(6.283185307179586f * u2, &sphi, &cphi);
    float t1[3], t2[3];
    duff_basis<float>(r, t1, t2);
    for (int c = 0; c < 3; ++c) out[c] = sa * cphi * t1[c] + sa * sphi * t2[c] + ca * r[c];
    return (m + 2.0f) / (m + 1.0f) * fmaxf(0.0f, n[0] * out[0] + n[1] * out[1] + n[2] * out[2]);
}

// Whether the specular weight of direction o is nonzero by the model (not by rounding): always for
// the ideal mirror; for a lobe, o above the horizon and, when drawn uniformly, with r.o > 0.
__device__ __forceinline__ bool lobe_open(const float p[3], const float n[3], float m, bool uniform, const float o[3])
{
    if (!(m < INFINITY)) return true;
    const float pn = p[0] * n[0] + p[1] * n[1] + p[2] * n[2];
    float ro = 0.0f;
    for (int c = 0; c < 3; ++c) ro += (p[c] - 2.0f * pn * n[c]) * o[c];
    return n[0] * o[0] + n[1] * o[1] + n[2] * o[2] > 0.0f && (!uniform || ro > 0.0f);
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

// The geometry a sample sees, for one scene in its current pose: facet records in BVH order, the
// BVH walk or brute force for its rays.
template <bool BRUTE>
struct SceneGeo {
    const SurfaceScene& sc;
    int* __restrict__ lstack;
    __device__ __forceinline__ double area() const { return sc.area; }
    __device__ __forceinline__ int n_tris() const { return sc.n_tris; }
    __device__ __forceinline__ const double* cum() const { return (const double*)sc.cum_area; }
    __device__ __forceinline__ float eps() const { return sc.eps; }
    __device__ __forceinline__ const float* com() const { return sc.com; }
    // record of original facet f
    __device__ __forceinline__ int position(int f) const { return ((const int32_t*)sc.bvh_pos)[f]; }
    // point at barycentric (b1, b2) of record p, its outward normal and its material
    __device__ __forceinline__ void point(int p, float b1, float b2, float x[3], float n[3], float4& mt) const
    {
        const TriRec tr = ((const TriRec*)sc.tris)[p];
        mt = ((const float4*)sc.mat)[p];
        n[0] = tr.f[1].w;
        n[1] = tr.f[2].w;
        n[2] = tr.f[3].x;
        x[0] = tr.f[0].x + b1 * tr.f[1].x + b2 * tr.f[2].x;
        x[1] = tr.f[0].y + b1 * tr.f[1].y + b2 * tr.f[2].y;
        x[2] = tr.f[0].z + b1 * tr.f[1].z + b2 * tr.f[2].z;
    }
    // normal, original index and material of record g
    __device__ __forceinline__ void facet(int g, float ng[3], int& id, float4& mt) const
    {
        const TriRec tg = ((const TriRec*)sc.tris)[g];
        mt = ((const float4*)sc.mat)[g];
        ng[0] = tg.f[1].w;
        ng[1] = tg.f[2].w;
        ng[2] = tg.f[3].x;
        id = __float_as_int(tg.f[0].w);
    }
    __device__ __forceinline__ bool blocked(const float o[3], const float s[3], int skip) const
    {
        return sun_blocked<BRUTE>(sc, o, s, skip, lstack);
    }
    __device__ __forceinline__ int closest(const float o[3], const float d[3], int skip, float& t) const
    {
        return gather_hit<BRUTE>(sc, o, d, skip, t, lstack);
    }
};

// The geometry of one pair of the multi-world estimator: the rest-pose records of every rigid part,
// this lane's hinge angles turning them.  Instead of moving the part, a ray is turned into the part's
// rest frame (by the inverse rotation about its hinge), so all lanes test the same records -- a
// wave-uniform loop over every triangle with scalar loads, each lane in its own world.  Points and
// normals of the part are turned back into the world frame.
struct MwGeo {
    const MwScene& sc;
    float cs[kMaxHinges], sn[kMaxHinges];  // cos and sin of this lane's hinge angles
    const float* mat;                       // this lane's group materials [3 G]
    __device__ __forceinline__ double area() const { return sc.area; }
    __device__ __forceinline__ int n_tris() const { return sc.n_tris; }
    __device__ __forceinline__ const double* cum() const { return (const double*)sc.cum_area; }
    __device__ __forceinline__ float eps() const { return sc.eps; }
    __device__ __forceinline__ const float* com() const { return sc.com; }
    __device__ __forceinline__ int position(int f) const { return ((const int32_t*)sc.pos)[f]; }
    // hinge h's rotation (selected without indexing registers by a lane-varying h)
    struct Turn {
        float c, s, k[3], o[3];
    };
    __device__ __forceinline__ Turn hinge(int h, float sgn) const
    {
        Turn r{1.0f, 0.0f, {0.0f, 0.0f, 1.0f}, {0.0f, 0.0f, 0.0f}};
#pragma unroll
        for (int q = 0; q < kMaxHinges; ++q)
            if (h == q) {
                r.c = cs[q];
                r.s = sgn * sn[q];
                for (int a = 0; a < 3; ++a) {
                    r.k[a] = sc.hinge_axis[q][a];
                    r.o[a] = sc.hinge_origin[q][a];
                }
            }
        return r;
    }
    // v turned by the rotation (Rodrigues' formula), or the point v turned about the hinge line
    __device__ __forceinline__ static void turn(const Turn& r, const float v[3], float out[3])
    {
        const float kv = r.k[0] * v[0] + r.k[1] * v[1] + r.k[2] * v[2];
        const float kx[3] = {r.k[1] * v[2] - r.k[2] * v[1], r.k[2] * v[0] - r.k[0] * v[2],
                             r.k[0] * v[1] - r.k[1] * v[0]};
        for (int a = 0; a < 3; ++a) out[a] = v[a] * r.c + kx[a] * r.s + r.k[a] * kv * (1.0f - r.c);
    }
    __device__ __forceinline__ static void turn_point(const Turn& r, const float v[3], float out[3])
    {
        const float d[3] = {v[0] - r.o[0], v[1] - r.o[1], v[2] - r.o[2]};
        turn(r, d, out);
        for (int a = 0; a < 3; ++a) out[a] += r.o[a];
    }
    __device__ __forceinline__ float4 material(const TriRec& tr) const
    {
        const float* m = mat + 3 * __float_as_int(tr.f[3].z);
        const float a = m[0], b = m[1];
        float q;
        if (a > 0.0f && b > 0.0f) {
            q = a / (a + b);
            q = fminf(fmaxf(q, 0.01f), 0.99f);
        } else {
            q = a > 0.0f ? 1.0f : 0.0f;
        }
        return make_float4(a, b, q, m[2]);
    }
    __device__ __forceinline__ void point(int p, float b1, float b2, float x[3], float n[3], float4& mt) const
    {
        const TriRec tr = ((const TriRec*)sc.tris)[p];
        mt = material(tr);
        const float xr[3] = {tr.f[0].x + b1 * tr.f[1].x + b2 * tr.f[2].x, tr.f[0].y + b1 * tr.f[1].y + b2 * tr.f[2].y,
                             tr.f[0].z + b1 * tr.f[1].z + b2 * tr.f[2].z};
        const float nr[3] = {tr.f[1].w, tr.f[2].w, tr.f[3].x};
        const int h = __float_as_int(tr.f[3].y);
        if (h < 0) {
            for (int a = 0; a < 3; ++a) {
                x[a] = xr[a];
                n[a] = nr[a];
            }
        } else {
            const Turn r = hinge(h, 1.0f);
            turn_point(r, xr, x);
            turn(r, nr, n);
        }
    }
    __device__ __forceinline__ void facet(int g, float ng[3], int& id, float4& mt) const
    {
        const TriRec tg = ((const TriRec*)sc.tris)[g];
        mt = material(tg);
        const float nr[3] = {tg.f[1].w, tg.f[2].w, tg.f[3].x};
        const int h = __float_as_int(tg.f[3].y);
        if (h < 0) {
            for (int a = 0; a < 3; ++a) ng[a] = nr[a];
        } else {
            turn(hinge(h, 1.0f), nr, ng);
        }
        id = __float_as_int(tg.f[0].w);
    }
    // the ray in the rest frame of part q
    __device__ __forceinline__ void to_part(int q, const float o[3], const float d[3], float o2[3], float d2[3]) const
    {
        const int h = sc.part_hinge[q];
        if (h < 0) {
            for (int a = 0; a < 3; ++a) {
                o2[a] = o[a];
                d2[a] = d[a];
            }
        } else {
            const Turn r = hinge(h, -1.0f);
            turn_point(r, o, o2);
            turn(r, d, d2);
        }
    }
    __device__ __forceinline__ bool blocked(const float o[3], const float s[3], int skip) const
    {
        const TriRec* __restrict__ tris = (const TriRec*)sc.tris;
        bool blk = false;
        int begin = 0;
        for (int q = 0; q < sc.n_parts; ++q) {
            float o2[3], s2[3];
            to_part(q, o, s, o2, s2);
            for (int tri = begin; tri < sc.part_end[q]; ++tri) {
                const TriRec* T = tris + tri;
                const float t = tri_hit_back(o2, s2, T->f[0], T->f[1], T->f[2]);
                blk = blk || (t > 0.0f && tri != skip);
            }
            begin = sc.part_end[q];
        }
        return blk;
    }
    __device__ __forceinline__ int closest(const float o[3], const float d[3], int skip, float& t_out) const
    {
        const TriRec* __restrict__ tris = (const TriRec*)sc.tris;
        float tbest = FLT_MAX;
        int hit = -1, hit_id = 0x7fffffff;
        int begin = 0;
        for (int q = 0; q < sc.n_parts; ++q) {
            float o2[3], d2[3];
            to_part(q, o, d, o2, d2);
            for (int tri = begin; tri < sc.part_end[q]; ++tri) {
                const TriRec* T = tris + tri;
                const float4 g0 = T->f[0], g1 = T->f[1], g2 = T->f[2];
                const float t = tri_hit(o2, d2, g0, g1, g2);
                const int id = __float_as_int(g0.w);
                if (t > 0.0f && tri != skip && (t < tbest || (t == tbest && id < hit_id))) {
                    tbest = t;
                    hit = tri;
                    hit_id = id;
                }
            }
            begin = sc.part_end[q];
        }
        t_out = tbest;
        return hit;
    }
};

// One sample: force and torque (area applied) and its record.  `n_samples` scales the stratified
// area coordinate.
template <class Geo>
__device__ __forceinline__ void surface_sample(const SurfaceArgs& a, const Geo& geo, int64_t n_samples, const float s[3],
                                               uint32_t sample, uint32_t dir, uint32_t design, float F[3], float T[3],
                                               int32_t& rec_facet, int32_t* rec_hits, int32_t& rec_lit)
{
    float u0[4], u1[4];
    uint32_t c0 = sample, c1 = dir, c2 = 0u, c3 = design;
    philox4x32_10(c0, c1, c2, c3, a.seed_lo, a.seed_hi);
    philox_at(sample, dir, 1u, design, a, u1);
    // facet by area (FP64, original facet order): the first f with u A < cum[f]
    const double* __restrict__ cum = geo.cum();
    // stratified: sample i of N takes the area coordinate (i + u) / N
    const double uf = (a.sampling & 1)
                          ? (static_cast<double>(sample) + static_cast<double>(unit24(c0))) / static_cast<double>(n_samples)
                          : static_cast<double>(unit24(c0));
    const double target = uf * geo.area();
    int lo = 0, hi = geo.n_tris() - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (target < cum[mid])
            hi = mid;
        else
            lo = mid + 1;
    }
    rec_facet = lo;
    const int p = geo.position(lo);
    u0[1] = unit24(c1);
    u0[2] = unit24(c2);
    u0[3] = unit24(c3);
    const float sq = sqrtf(u0[1]);
    const float b1 = sq * (1.0f - u0[2]), b2 = sq * u0[2];
    float x[3], n[3], o[3];
    float4 mt;
    geo.point(p, b1, b2, x, n, mt);
    for (int c = 0; c < 3; ++c) o[c] = x[c] + geo.eps() * n[c];
    const float rs = mt.x, rd = mt.y, ps = mt.z, mx = mt.w;
    const bool uniform = (a.sampling & 2) != 0;
    // the outgoing event at x: specular (about each arriving contribution's mirror direction,
    // drawn from the same two uniforms) or one cosine direction for all contributions
    const bool spec = u0[3] < ps;
    float odir[3], w[3];
    const float wo = hemi_dir(n, u1[0], u1[1], uniform, odir);
    const float wg = hemi_dir(n, u1[2], u1[3], uniform, w);
    const float kdif = rd > 0.0f ? rd / (1.0f - ps) * wo : 0.0f;
    float dep[3] = {0.0f, 0.0f, 0.0f};
    int32_t lit = 0;
    const float cs = n[0] * s[0] + n[1] * s[1] + n[2] * s[2];
    if (cs > 0.0f && !geo.blocked(o, s, p)) {
        lit |= 1;
        const float W = a.flux_c * cs;
        const float pv[3] = {-s[0], -s[1], -s[2]};
        float od[3];
        float k = kdif;
        if (spec) k = rs / ps * specular_dir(pv, n, mx, u1[0], u1[1], uniform, od);
        for (int c = 0; c < 3; ++c) dep[c] += W * (pv[c] - k * (spec ? od[c] : odir[c]));
    }
    if (a.bounces >= 2) {
        float ro[3] = {o[0], o[1], o[2]}, rdir[3] = {w[0], w[1], w[2]};
        int skip = p;
        float beta = 1.0f, radiance = 0.0f;
        for (int k = 1; k <= a.bounces - 1; ++k) {
            float t;
            const int g = geo.closest(ro, rdir, skip, t);
            if (g < 0) break;
            float ng[3];
            float4 mg;
            int gid;
            geo.facet(g, ng, gid, mg);
            if (rec_hits) rec_hits[k - 1] = gid;
            float oy[3];
            for (int c = 0; c < 3; ++c) oy[c] = ro[c] + t * rdir[c] + geo.eps() * ng[c];
            const float cg = ng[0] * s[0] + ng[1] * s[1] + ng[2] * s[2];
            const bool lobe = mg.x > 0.0f && mg.w < INFINITY;
            if ((mg.y > 0.0f || lobe) && cg > 0.0f && !geo.blocked(oy, s, g)) {
                lit |= 1 << k;
                float add = mg.y * cg;
                if (lobe) {
                    // pi times the lobe's radiance toward the previous vertex (along -rdir) for
                    // sunlight of propagation -s
                    const float sn = s[0] * ng[0] + s[1] * ng[1] + s[2] * ng[2];
                    float rr = 0.0f;
                    for (int c = 0; c < 3; ++c) rr -= (-s[c] + 2.0f * sn * ng[c]) * rdir[c];
                    add += mg.x * (mg.w + 2.0f) * 0.5f * powf(fmaxf(0.0f, rr), mg.w) * cg;
                }
                radiance += beta * add;
            }
            if (k == a.bounces - 1) break;
            float ev[4];
            philox_at(sample, dir, static_cast<uint32_t>(k + 1), design, a, ev);
            float nd[3];
            bool live;
            if (ev[0] < mg.z) {
                // light leaving the vertex along -rdir comes from about the reflection of rdir
                beta *= mg.x / mg.z * specular_dir(rdir, ng, mg.w, ev[1], ev[2], uniform, nd);
                live = mg.x > 0.0f && lobe_open(rdir, ng, mg.w, uniform, nd);
            } else {
                const float wv = hemi_dir(ng, ev[1], ev[2], uniform, nd);
                beta *= mg.y > 0.0f ? mg.y / (1.0f - mg.z) * wv : 0.0f;
                live = mg.y > 0.0f && wv > 0.0f;
            }
            // the path ends where its weight is zero by the model, not where the product underflows
            if (!live) break;
            for (int c = 0; c < 3; ++c) {
                ro[c] = oy[c];
                rdir[c] = nd[c];
            }
            skip = g;
        }
        if (radiance > 0.0f) {
            const float W = a.flux_c * radiance * wg;
            const float pv[3] = {-w[0], -w[1], -w[2]};
            float od[3];
            float k = kdif;
            if (spec) k = rs / ps * specular_dir(pv, n, mx, u1[0], u1[1], uniform, od);
            for (int c = 0; c < 3; ++c) dep[c] += W * (pv[c] - k * (spec ? od[c] : odir[c]));
        }
    }
    const float A = static_cast<float>(geo.area());
    for (int c = 0; c < 3; ++c) F[c] = A * dep[c];
    const float* com = geo.com();
    const float lx = x[0] - com[0], ly = x[1] - com[1], lz = x[2] - com[2];
    T[0] = ly * F[2] - lz * F[1];
    T[1] = lz * F[0] - lx * F[2];
    T[2] = lx * F[1] - ly * F[0];
    rec_lit = lit;
}

// Workgroup = kSurfThreads consecutive samples of one unit (scene, direction).  Five waves per
// SIMD: the BVH mode (99 VGPRs at its natural allocation, four waves) then keeps 96 with 2
// spilled, and its divergent per-lane walks hide more fetch latency (about 8 % faster).
template <bool BRUTE>
__global__ __launch_bounds__(kSurfThreads) __attribute__((amdgpu_waves_per_eu(5))) void k_surface(SurfaceArgs a)
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
    if (BRUTE || valid) {
        const SceneGeo<BRUTE> geo{sc, &s_lane[wave][0][lane]};
        surface_sample(a, geo, a.n_samples, s, static_cast<uint32_t>(valid ? i : 0),
                       static_cast<uint32_t>(a.dir_index_base + j), a.design_index + static_cast<uint32_t>(scene), F, T,
                       facet, a.rec_hits ? hits : nullptr, lit);
    }
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

// Multi-world: lane = (pair, sample); pair i's design turns the parts, its sun direction lights
// them.  Every lane runs the wave-uniform triangle loops (invalid lanes too, with pair 0).
__global__ __launch_bounds__(kSurfThreads) void k_surface_designs(MwArgs A)
{
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * kSurfThreads + threadIdx.x;
    const bool valid = idx < A.n_pairs * A.samples;
    const int64_t i = valid ? idx / A.samples : 0;
    const int32_t k = valid ? static_cast<int32_t>(idx % A.samples) : 0;
    const float* row = A.designs + i * A.stride;
    MwGeo geo{A.sc, {}, {}, row + A.n_hinges};
    for (int h = 0; h < kMaxHinges; ++h) {
        const float ang = h < A.n_hinges ? row[h] : 0.0f;
        sincosf(ang, &geo.sn[h], &geo.cs[h]);
    }
    const float s[3] = {static_cast<float>(A.sun[3 * i]), static_cast<float>(A.sun[3 * i + 1]),
                        static_cast<float>(A.sun[3 * i + 2])};
    float F[3], T[3];
    int32_t hits[kMaxBounces];
    for (int q = 0; q < kMaxBounces; ++q) hits[q] = -1;
    int32_t facet = -1, lit = 0;
    surface_sample(A.base, geo, A.samples, s, static_cast<uint32_t>(k), static_cast<uint32_t>(A.base.dir_index_base + i),
                   A.base.design_index, F, T, facet, A.rec_hits ? hits : nullptr, lit);
    if (!valid) return;
    float* out = A.sample_out + idx * 6;
    for (int c = 0; c < 3; ++c) {
        out[c] = F[c];
        out[3 + c] = T[c];
    }
    if (A.rec_facet) {
        A.rec_facet[idx] = facet;
        A.rec_lit[idx] = lit;
        if (A.rec_hits)
            for (int q = 0; q < A.base.bounces - 1; ++q) A.rec_hits[idx * (A.base.bounces - 1) + q] = hits[q];
    }
}

// Mean of each pair's samples, in sample order (FP64).
__global__ void k_pair_mean(const float* __restrict__ sample_out, int64_t n_pairs, int32_t samples,
                            double* __restrict__ force, double* __restrict__ torque)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n_pairs * 6) return;
    const int64_t i = t / 6;
    const int c = static_cast<int>(t % 6);
    double sum = 0.0;
    for (int32_t k = 0; k < samples; ++k) sum += static_cast<double>(sample_out[(i * samples + k) * 6 + c]);
    sum /= static_cast<double>(samples);
    if (c < 3)
        force[3 * i + c] = sum;
    else if (torque)
        torque[3 * i + c - 3] = sum;
}

__global__ void k_check_designs(const float* __restrict__ designs, int64_t n_pairs, int32_t n_hinges, int32_t n_groups,
                                int32_t* __restrict__ flags)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= n_pairs * n_groups) return;
    const int64_t i = t / n_groups;
    const int g = static_cast<int>(t % n_groups);
    const float* row = designs + i * (n_hinges + 3 * n_groups);
    const float* m = row + n_hinges + 3 * g;
    bool bad = !(m[0] >= 0.0f) || !(m[1] >= 0.0f) || !(m[0] + m[1] <= 1.0f) || !(m[2] >= 1.0f);
    if (g == 0)
        for (int h = 0; h < n_hinges; ++h) bad = bad || !(fabsf(row[h]) < INFINITY);
    if (bad) atomicOr(flags, 1);
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

hipError_t launch_check_designs(const float* designs, int64_t n_pairs, int32_t n_hinges, int32_t n_groups,
                                int32_t* flags, hipStream_t stream)
{
    const int64_t n = n_pairs * n_groups;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_check_designs, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, stream, designs,
                       n_pairs, n_hinges, n_groups, flags);
    return hipGetLastError();
}

hipError_t launch_surface_designs(const MwArgs& a, double* force, double* torque, hipStream_t stream)
{
    const int64_t total = a.n_pairs * a.samples;
    if (total == 0) return hipSuccess;
    const int64_t blocks = (total + kSurfThreads - 1) / kSurfThreads;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_surface_designs, dim3(static_cast<unsigned>(blocks)), dim3(kSurfThreads), 0, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n = a.n_pairs * 6;
    hipLaunchKernelGGL(k_pair_mean, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, stream, a.sample_out,
                       a.n_pairs, a.samples, force, torque);
    return hipGetLastError();
}

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
