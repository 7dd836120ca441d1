// Per-path arithmetic of the ray-grid SRP estimator, shared by the HIP kernels and the host-side
// instrumented traversal (ray statistics for the bandwidth model).  FP32 except the frames.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "srp_internal.h"

namespace srp {

#define SRP_HD __host__ __device__ __forceinline__

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the 4x32 S-box with the
// published multipliers 0xD2511F53, 0xCD9E8D57 and key increments 0x9E3779B9, 0xBB67AE85.
SRP_HD void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32 x 32 -> 64-bit product gives both halves of each S-box multiplication
        const uint64_t pa = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t pb = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        const uint32_t n0 = static_cast<uint32_t>(pb >> 32) ^ c1 ^ k0;
        const uint32_t n2 = static_cast<uint32_t>(pa >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = static_cast<uint32_t>(pb);
        c2 = n2;
        c3 = static_cast<uint32_t>(pa);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// top 24 bits -> [0, 1), exact in float
SRP_HD float unit24(uint32_t x) { return static_cast<float>(x >> 8) * (1.0f / 16777216.0f); }

// Orthonormal (b1, b2) with b1 x b2 = n: Duff et al., "Building an Orthonormal Basis, Revisited",
// JCGT 2017; sign(0) = +1.
template <class R>
SRP_HD void duff_basis(const R n[3], R b1[3], R b2[3])
{
    const R s = n[2] >= R(0) ? R(1) : R(-1);
    const R a = R(-1) / (s + n[2]);
    const R b = n[0] * n[1] * a;
    b1[0] = R(1) + s * n[0] * n[0] * a;
    b1[1] = s * b;
    b1[2] = -s * n[0];
    b2[0] = b;
    b2[1] = s + n[1] * n[1] * a;
    b2[2] = -n[1];
}

// Grid frame of one sun direction (FP64): basis of the propagation d = -s, rectangle bounding
// the projected corners of the box [lo, hi], entry plane 0.01 L in front of the nearest corner.
// Writes the 12-double layout u, v, o0, du, dv, 0.
SRP_HD void frame_from_box(const double sun[3], const double lo[3], const double hi[3], double L, int32_t nu,
                           int32_t nv, double out[12])
{
    const double len = sqrt(sun[0] * sun[0] + sun[1] * sun[1] + sun[2] * sun[2]);
    const double d[3] = {-sun[0] / len, -sun[1] / len, -sun[2] / len};
    double u[3], v[3];
    duff_basis<double>(d, u, v);
    double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY, smin = INFINITY;
    for (int c = 0; c < 8; ++c) {
        const double p[3] = {(c & 1) ? hi[0] : lo[0], (c & 2) ? hi[1] : lo[1], (c & 4) ? hi[2] : lo[2]};
        const double pu = p[0] * u[0] + p[1] * u[1] + p[2] * u[2];
        const double pv = p[0] * v[0] + p[1] * v[1] + p[2] * v[2];
        const double ps = p[0] * d[0] + p[1] * d[1] + p[2] * d[2];
        umin = fmin(umin, pu);
        umax = fmax(umax, pu);
        vmin = fmin(vmin, pv);
        vmax = fmax(vmax, pv);
        smin = fmin(smin, ps);
    }
    const double s0 = smin - 0.01 * L;
    for (int a = 0; a < 3; ++a) {
        out[a] = u[a];
        out[3 + a] = v[a];
        out[6 + a] = s0 * d[a] + umin * u[a] + vmin * v[a];
    }
    out[9] = (umax - umin) / nu;
    out[10] = (vmax - vmin) / nv;
    out[11] = 0.0;
}

// FP32 frame the trace consumes; w = Phi du dv / c is the force carried by one ray tube.
SRP_HD DevFrame frame_to_device(const double sun[3], const double f[12], double flux)
{
    const double len = sqrt(sun[0] * sun[0] + sun[1] * sun[1] + sun[2] * sun[2]);
    DevFrame fr;
    for (int a = 0; a < 3; ++a) {
        fr.o0[a] = static_cast<float>(f[6 + a]);
        fr.U[a] = static_cast<float>(f[9] * f[a]);
        fr.V[a] = static_cast<float>(f[10] * f[3 + a]);
        fr.d[a] = static_cast<float>(-sun[a] / len);
    }
    fr.w = static_cast<float>(flux * f[9] * f[10] / kSpeedOfLight);
    fr.pad[0] = fr.pad[1] = fr.pad[2] = 0.0f;
    return fr;
}

// Primary ray of pixel (pi, pk): one Philox point in the pixel (counter (pixel, dir, 0, design))
// or the pixel centre.
SRP_HD void primary_ray(const DevFrame& fr, int32_t pi, int32_t pk, uint32_t pixel, uint32_t dir, uint32_t design,
                        uint32_t seed_lo, uint32_t seed_hi, bool jitter, float o[3], float d[3])
{
    float ja = 0.5f, jb = 0.5f;
    if (jitter) {
        uint32_t c0 = pixel, c1 = dir, c2 = 0u, c3 = design;
        philox4x32_10(c0, c1, c2, c3, seed_lo, seed_hi);
        ja = unit24(c0);
        jb = unit24(c1);
    }
    const float fi = static_cast<float>(pi) + ja, fk = static_cast<float>(pk) + jb;
    for (int a = 0; a < 3; ++a) {
        o[a] = fr.o0[a] + fi * fr.U[a] + fk * fr.V[a];
        d[a] = fr.d[a];
    }
}

// Internals of one interaction that the adjoint needs.
struct InteractInfo {
    float r[3];          // mirror direction
    float cth;           // cos(theta) = -d . n
    float w_in, w_out;   // weights before and after (w_out = 0 at the last interaction)
    float k;             // w_out / w_in as rho_s / p_spec or rho_d / (1 - p_spec)
    float lam[3];        // Lambertian draw in the (t1, t2, n) basis
    bool last, mirror;
};

// One surface interaction (paper Sec. 3.2, l2f): at hit point x = o + t d on a facet with outward
// normal n and material (rho_s, rho_d, p_spec), the deposit is the incident momentum w d minus the
// momentum that leaves.  At the last interaction (b == bounces, or a black facet) the expected
// outgoing momentum w (rho_s r + (2/3) rho_d n) leaves (mirror direction r; Lambertian mean 2/3 n,
// Sec. 5.9) and the path ends.  Otherwise Philox counter (pixel, dir, b, design) draws the event:
// u_e < p_spec selects the mirror direction with weight w rho_s / p_spec, else a cosine-weighted
// direction (Malley's method in the Duff basis of n) with weight w rho_d / (1 - p_spec); that
// sampled momentum leaves and the path continues from x + eps n.
// Returns the force deposit in g[3]; updates o, d, w; returns false when the path ends.
// `info` (may be null) receives the internals the adjoint needs.
template <class Info>
SRP_HD bool interact_ex(float o[3], float d[3], float& w, float t, const float n[3], float rs, float rd, float ps, int b,
                        int bounces, uint32_t pixel, uint32_t dir, uint32_t design, uint32_t seed_lo, uint32_t seed_hi,
                        float eps, float x[3], float g[3], Info* info)
{
    for (int a = 0; a < 3; ++a) x[a] = o[a] + t * d[a];
    const float cth = -(d[0] * n[0] + d[1] * n[1] + d[2] * n[2]);
    float r[3];
    for (int a = 0; a < 3; ++a) r[a] = d[a] + 2.0f * cth * n[a];
    for (int a = 0; a < 3; ++a) g[a] = w * d[a];
    if (info) {
        for (int a = 0; a < 3; ++a) info->r[a] = r[a];
        info->cth = cth;
        info->w_in = w;
        info->w_out = 0.0f;
        info->k = 0.0f;
        info->last = false;
        info->mirror = false;
    }
    if (b == bounces || (rs == 0.0f && rd == 0.0f)) {
        const float kd = (2.0f / 3.0f) * rd;
        for (int a = 0; a < 3; ++a) g[a] -= w * (rs * r[a] + kd * n[a]);
        if (info) info->last = true;
        return false;
    }
    uint32_t c0 = pixel, c1 = dir, c2 = static_cast<uint32_t>(b), c3 = design;
    philox4x32_10(c0, c1, c2, c3, seed_lo, seed_hi);
    const float ue = unit24(c0), u1 = unit24(c1), u2 = unit24(c2);
    float od[3], w2;
    if (ue < ps) {
        for (int a = 0; a < 3; ++a) od[a] = r[a];
        w2 = w * rs / ps;
        if (info) {
            info->mirror = true;
            info->k = rs / ps;
        }
    } else {
        const float rad = sqrtf(u1);
        float sphi, cphi;
        sincosf(6.283185307179586f * u2, &sphi, &cphi);
        const float px = rad * cphi, py = rad * sphi, pz = sqrtf(fmaxf(0.0f, 1.0f - u1));
        float t1[3], t2[3];
        duff_basis<float>(n, t1, t2);
        for (int a = 0; a < 3; ++a) od[a] = px * t1[a] + py * t2[a] + pz * n[a];
        w2 = w * rd / (1.0f - ps);
        if (info) {
            info->k = rd / (1.0f - ps);
            info->lam[0] = px;
            info->lam[1] = py;
            info->lam[2] = pz;
        }
    }
    if (info) info->w_out = w2;
    for (int a = 0; a < 3; ++a) {
        g[a] -= w2 * od[a];
        o[a] = x[a] + eps * n[a];
        d[a] = od[a];
    }
    w = w2;
    return true;
}

SRP_HD bool interact(float o[3], float d[3], float& w, float t, const float n[3], float rs, float rd, float ps, int b,
                     int bounces, uint32_t pixel, uint32_t dir, uint32_t design, uint32_t seed_lo, uint32_t seed_hi,
                     float eps, float x[3], float g[3])
{
    return interact_ex<InteractInfo>(o, d, w, t, n, rs, rd, ps, b, bounces, pixel, dir, design, seed_lo, seed_hi, eps, x,
                                     g, nullptr);
}

// Quotient and reciprocal: on the GPU the hardware reciprocal (1 ulp) replaces the IEEE division
// sequence; these values only place hits along a ray and order them, where 1 ulp is far below
// the geometric tolerances.  The host uses the correctly rounded operations.
SRP_HD float fast_rcp(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}

SRP_HD float fast_div(float a, float b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return a * __builtin_amdgcn_rcpf(b);
#else
    return a / b;
#endif
}

// Moller-Trumbore (1997), one-sided (det > 0 <=> the ray meets the outward side), inclusive
// barycentric bounds, returns t (or a negative value when there is no hit).
SRP_HD float tri_hit(const float o[3], const float d[3], const float4& g0, const float4& g1, const float4& g2)
{
    const float px = d[1] * g2.z - d[2] * g2.y;
    const float py = d[2] * g2.x - d[0] * g2.z;
    const float pz = d[0] * g2.y - d[1] * g2.x;
    const float det = g1.x * px + g1.y * py + g1.z * pz;
    const float tx = o[0] - g0.x, ty = o[1] - g0.y, tz = o[2] - g0.z;
    const float uu = tx * px + ty * py + tz * pz;
    const float qx = ty * g1.z - tz * g1.y;
    const float qy = tz * g1.x - tx * g1.z;
    const float qz = tx * g1.y - ty * g1.x;
    const float vv = d[0] * qx + d[1] * qy + d[2] * qz;
    const float tnum = g2.x * qx + g2.y * qy + g2.z * qz;
    const float t = fast_div(tnum, det);
    const bool ok = det > 0.0f && uu >= 0.0f && uu <= det && vv >= 0.0f && uu + vv <= det && t > 0.0f;
    return ok ? t : -1.0f;
}

SRP_HD float safe_rcp(float x)
{
    const float m = 1e-20f;
    return fast_rcp(fabsf(x) < m ? copysignf(m, x) : x);
}

}  // namespace srp
