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

namespace srp {
namespace {

// ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) ------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t& c0, uint32_t& c1, uint32_t& c2, uint32_t& c3, uint32_t k0,
                                              uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo_a = 0xD2511F53u * c0;
        const uint32_t hi_a = __umulhi(0xD2511F53u, c0);
        const uint32_t lo_b = 0xCD9E8D57u * c2;
        const uint32_t hi_b = __umulhi(0xCD9E8D57u, c2);
        const uint32_t n0 = hi_b ^ c1 ^ k0;
        const uint32_t n2 = hi_a ^ c3 ^ k1;
        c0 = n0;
        c1 = lo_b;
        c2 = n2;
        c3 = lo_a;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

__device__ __forceinline__ float unit24(uint32_t x) { return static_cast<float>(x >> 8) * (1.0f / 16777216.0f); }

// ---- frames (FP64) ----------------------------------------------------------------------------
__device__ void duff_basis(const double n[3], double b1[3], double b2[3])
{
    const double s = n[2] >= 0.0 ? 1.0 : -1.0;
    const double a = -1.0 / (s + n[2]);
    const double b = n[0] * n[1] * a;
    b1[0] = 1.0 + s * n[0] * n[0] * a;
    b1[1] = s * b;
    b1[2] = -s * n[0];
    b2[0] = b;
    b2[1] = s + n[1] * n[1] * a;
    b2[2] = -n[1];
}

struct BoxArg {
    double lo[3], hi[3];
};

__global__ void k_frames(const double* __restrict__ sun, int64_t D, BoxArg box, double L, int32_t nu, int32_t nv,
                         double flux, const double* __restrict__ caller, double* __restrict__ f64,
                         DevFrame* __restrict__ f32)
{
    const int64_t j = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= D) return;
    const double sx = sun[3 * j], sy = sun[3 * j + 1], sz = sun[3 * j + 2];
    const double len = sqrt(sx * sx + sy * sy + sz * sz);
    const double d[3] = {-sx / len, -sy / len, -sz / len};
    double u[3], v[3], o0[3], du, dv;
    if (caller) {
        const double* c = caller + 12 * j;
        for (int a = 0; a < 3; ++a) {
            u[a] = c[a];
            v[a] = c[3 + a];
            o0[a] = c[6 + a];
        }
        du = c[9];
        dv = c[10];
    } else {
        duff_basis(d, u, v);
        double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY, smin = INFINITY;
        for (int c = 0; c < 8; ++c) {
            const double p[3] = {(c & 1) ? box.hi[0] : box.lo[0], (c & 2) ? box.hi[1] : box.lo[1],
                                 (c & 4) ? box.hi[2] : box.lo[2]};
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
        for (int a = 0; a < 3; ++a) o0[a] = s0 * d[a] + umin * u[a] + vmin * v[a];
        du = (umax - umin) / nu;
        dv = (vmax - vmin) / nv;
    }
    if (f64) {
        double* o = f64 + 12 * j;
        for (int a = 0; a < 3; ++a) {
            o[a] = u[a];
            o[3 + a] = v[a];
            o[6 + a] = o0[a];
        }
        o[9] = du;
        o[10] = dv;
        o[11] = 0.0;
    }
    if (f32) {
        DevFrame fr;
        for (int a = 0; a < 3; ++a) {
            fr.o0[a] = static_cast<float>(o0[a]);
            fr.U[a] = static_cast<float>(du * u[a]);
            fr.V[a] = static_cast<float>(dv * v[a]);
            fr.d[a] = static_cast<float>(d[a]);
        }
        fr.w = static_cast<float>(flux * du * dv / kSpeedOfLight);
        fr.pad[0] = fr.pad[1] = fr.pad[2] = 0.0f;
        f32[j] = fr;
    }
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

// ---- traversal -------------------------------------------------------------------------------------
__device__ __forceinline__ float safe_rcp(float x)
{
    const float m = 1e-20f;
    return 1.0f / (fabsf(x) < m ? copysignf(m, x) : x);
}

__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Closest front-facing hit of each lane's ray (o, d) among all triangles except `skip` (the
// triangle the ray leaves).  Lanes with alive == false never hit.  The traversal is
// wavefront-coherent: one node sequence for the whole wave, a child is entered when any lane's
// ray overlaps it, and the nearer child (by majority over the lanes that overlap both) first.
__device__ __forceinline__ void closest_hit(const BvhNode* __restrict__ nodes, const TriRec* __restrict__ tris,
                                            float ox, float oy, float oz, float dx, float dy, float dz, bool alive,
                                            int skip, float& t_out, int& hit_out, int* __restrict__ stack)
{
    const float ix = safe_rcp(dx), iy = safe_rcp(dy), iz = safe_rcp(dz);
    const float nx = -ox * ix, ny = -oy * iy, nz = -oz * iz;
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
            const uint64_t m0 = wave_ballot(h0);
            const uint64_t m1 = wave_ballot(h1);
            if (m0 && m1) {
                const uint64_t first1 = wave_ballot(h0 && h1 && tn1 < tn0);
                const bool swap = 2 * __popcll(first1) > __popcll(m0 & m1);
                const int nearc = swap ? c1 : c0;
                const int farc = swap ? c0 : c1;
                stack[sp] = farc;
                ++sp;
                cur = nearc;
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
                // Moller-Trumbore (1997), one-sided: det > 0 <=> d . n < 0
                const float px = dy * g2.z - dz * g2.y;
                const float py = dz * g2.x - dx * g2.z;
                const float pz = dx * g2.y - dy * g2.x;
                const float det = g1.x * px + g1.y * py + g1.z * pz;
                const float tx = ox - g0.x, ty = oy - g0.y, tz = oz - g0.z;
                const float uu = tx * px + ty * py + tz * pz;
                const float qx = ty * g1.z - tz * g1.y;
                const float qy = tz * g1.x - tx * g1.z;
                const float qz = tx * g1.y - ty * g1.x;
                const float vv = dx * qx + dy * qy + dz * qz;
                const float tnum = g2.x * qx + g2.y * qy + g2.z * qz;
                const float t = tnum / det;
                const int id = __float_as_int(g0.w);
                const bool ok = det > 0.0f && uu >= 0.0f && uu <= det && vv >= 0.0f && uu + vv <= det && t > 0.0f &&
                                tri != skip && (t < tbest || (t == tbest && id < hit_id));
                if (ok) {
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

__device__ __forceinline__ float wave_sum(float v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <bool RECORDS>
__global__ __launch_bounds__(256) void k_trace(TraceArgs a)
{
    __shared__ int s_stack[kWaves][kStackDepth];
    __shared__ float s_red[kWaves][6];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t j = blockIdx.x / a.blocks_per_dir;
    const int32_t blk = blockIdx.x % a.blocks_per_dir;
    const DevFrame fr = a.frames[j];
    const uint32_t dir_global = static_cast<uint32_t>(a.dir_index_base + j);
    const BvhNode* __restrict__ nodes = a.nodes;
    const TriRec* __restrict__ tris = a.tris;
    int* stack = s_stack[wave];

    float aF0 = 0.0f, aF1 = 0.0f, aF2 = 0.0f, aT0 = 0.0f, aT1 = 0.0f, aT2 = 0.0f;
    for (int m = 0; m < a.tiles_per_wave; ++m) {
        const int64_t tile = (static_cast<int64_t>(blk) * a.tiles_per_wave + m) * kWaves + wave;
        if (tile >= a.tiles_per_dir) break;
        int64_t pixel = 0, rec = 0;
        bool valid;
        if (RECORDS) {
            rec = tile * 64 + lane;
            valid = rec < a.n_pix;
            if (valid) pixel = a.pix ? a.pix[rec] : rec;
        } else {
            const int64_t tx = tile % a.tiles_x, ty = tile / a.tiles_x;
            const int64_t pi = tx * kTileW + (lane & 7), pk = ty * kTileH + (lane >> 3);
            valid = pi < a.nu && pk < a.nv;
            pixel = pi + pk * a.nu;
        }
        const int32_t pi = static_cast<int32_t>(pixel % a.nu);
        const int32_t pk = static_cast<int32_t>(pixel / a.nu);
        float ja = 0.5f, jb = 0.5f;
        if (a.jitter) {
            uint32_t c0 = static_cast<uint32_t>(pixel), c1 = dir_global, c2 = 0u, c3 = a.design_index;
            philox4x32_10(c0, c1, c2, c3, a.seed_lo, a.seed_hi);
            ja = unit24(c0);
            jb = unit24(c1);
        }
        const float fi = static_cast<float>(pi) + ja, fk = static_cast<float>(pk) + jb;
        float ox = fr.o0[0] + fi * fr.U[0] + fk * fr.V[0];
        float oy = fr.o0[1] + fi * fr.U[1] + fk * fr.V[1];
        float oz = fr.o0[2] + fi * fr.U[2] + fk * fr.V[2];
        float dx = fr.d[0], dy = fr.d[1], dz = fr.d[2];
        float w = fr.w;
        bool alive = valid;
        int skip = -1;
        float rF0 = 0.0f, rF1 = 0.0f, rF2 = 0.0f, rT0 = 0.0f, rT1 = 0.0f, rT2 = 0.0f;
        int b_done = 0;
        for (int b = 1; b <= a.bounces; ++b) {
            if (wave_ballot(alive) == 0) break;
            float t;
            int hit;
            closest_hit(nodes, tris, ox, oy, oz, dx, dy, dz, alive, skip, t, hit, stack);
            if (!alive) continue;
            if (hit < 0) {
                alive = false;
                continue;
            }
            const TriRec tr = tris[hit];
            const float4 mt = a.mat[hit];
            if (RECORDS) a.rec_hit[(j * a.n_pix + rec) * a.bounces + (b - 1)] = __float_as_int(tr.f[0].w);
            b_done = b;
            const float nx = tr.f[1].w, ny = tr.f[2].w, nz = tr.f[3].x;
            const float xx = ox + t * dx, xy = oy + t * dy, xz = oz + t * dz;
            const float lx = xx - a.com[0], ly = xy - a.com[1], lz = xz - a.com[2];
            const float cth = -(dx * nx + dy * ny + dz * nz);
            const float rx = dx + 2.0f * cth * nx, ry = dy + 2.0f * cth * ny, rz = dz + 2.0f * cth * nz;
            // incident momentum, minus what leaves
            float ex, ey, ez;  // outgoing momentum (force units)
            float gx = w * dx, gy = w * dy, gz = w * dz;
            const float rs = mt.x, rd = mt.y, ps = mt.z;
            bool last = (b == a.bounces) || (rs == 0.0f && rd == 0.0f);
            float odx = 0.0f, ody = 0.0f, odz = 0.0f, w2 = 0.0f;
            if (last) {
                const float kd = (2.0f / 3.0f) * rd;
                ex = w * (rs * rx + kd * nx);
                ey = w * (rs * ry + kd * ny);
                ez = w * (rs * rz + kd * nz);
            } else {
                uint32_t c0 = static_cast<uint32_t>(pixel), c1 = dir_global, c2 = static_cast<uint32_t>(b),
                         c3 = a.design_index;
                philox4x32_10(c0, c1, c2, c3, a.seed_lo, a.seed_hi);
                const float ue = unit24(c0), u1 = unit24(c1), u2 = unit24(c2);
                if (ue < ps) {
                    odx = rx;
                    ody = ry;
                    odz = rz;
                    w2 = w * rs / ps;
                } else {
                    // cosine-weighted direction about n (Malley's method) in the Duff basis of n
                    const float rad = sqrtf(u1);
                    float sphi, cphi;
                    __sincosf(6.283185307179586f * u2, &sphi, &cphi);
                    const float px = rad * cphi, py = rad * sphi, pz = sqrtf(fmaxf(0.0f, 1.0f - u1));
                    const float sg = nz >= 0.0f ? 1.0f : -1.0f;
                    const float aa = -1.0f / (sg + nz);
                    const float bb = nx * ny * aa;
                    const float t1x = 1.0f + sg * nx * nx * aa, t1y = sg * bb, t1z = -sg * nx;
                    const float t2x = bb, t2y = sg + ny * ny * aa, t2z = -ny;
                    odx = px * t1x + py * t2x + pz * nx;
                    ody = px * t1y + py * t2y + pz * ny;
                    odz = px * t1z + py * t2z + pz * nz;
                    w2 = w * rd / (1.0f - ps);
                }
                ex = w2 * odx;
                ey = w2 * ody;
                ez = w2 * odz;
            }
            gx -= ex;
            gy -= ey;
            gz -= ez;
            rF0 += gx;
            rF1 += gy;
            rF2 += gz;
            rT0 += ly * gz - lz * gy;
            rT1 += lz * gx - lx * gz;
            rT2 += lx * gy - ly * gx;
            if (last) {
                alive = false;
            } else {
                ox = xx + a.eps * nx;
                oy = xy + a.eps * ny;
                oz = xz + a.eps * nz;
                dx = odx;
                dy = ody;
                dz = odz;
                w = w2;
                skip = hit;
            }
        }
        if (RECORDS && valid) {
            for (int b = b_done + 1; b <= a.bounces; ++b) a.rec_hit[(j * a.n_pix + rec) * a.bounces + (b - 1)] = -1;
            if (a.rec_force) {
                float* rf = a.rec_force + (j * a.n_pix + rec) * 3;
                rf[0] = rF0;
                rf[1] = rF1;
                rf[2] = rF2;
            }
        }
        aF0 += rF0;
        aF1 += rF1;
        aF2 += rF2;
        aT0 += rT0;
        aT1 += rT1;
        aT2 += rT2;
    }
    aF0 = wave_sum(aF0);
    aF1 = wave_sum(aF1);
    aF2 = wave_sum(aF2);
    aT0 = wave_sum(aT0);
    aT1 = wave_sum(aT1);
    aT2 = wave_sum(aT2);
    if (lane == 0) {
        s_red[wave][0] = aF0;
        s_red[wave][1] = aF1;
        s_red[wave][2] = aF2;
        s_red[wave][3] = aT0;
        s_red[wave][4] = aT1;
        s_red[wave][5] = aT2;
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        double s = 0.0;
        for (int q = 0; q < kWaves; ++q) s += static_cast<double>(s_red[q][threadIdx.x]);
        a.partials[(j * a.blocks_per_dir + blk) * 6 + threadIdx.x] = s;
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
    const unsigned blocks = static_cast<unsigned>(a.D * a.blocks_per_dir);
    if (blocks == 0) return hipSuccess;
    if (records)
        hipLaunchKernelGGL(k_trace<true>, dim3(blocks), dim3(64 * kWaves), 0, stream, a);
    else
        hipLaunchKernelGGL(k_trace<false>, dim3(blocks), dim3(64 * kWaves), 0, stream, a);
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
