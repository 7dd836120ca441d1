// Host-side instrumented single-ray traversal of the scene's BVH on the same rays the GPU traces.
// It counts, per primary ray, the BVH nodes fetched, the triangles tested and the hits of a
// classic one-ray depth-first closest-hit traversal (nearer child first).  These counts define the
// algorithmic bytes a ray must touch (no credit for sharing between rays), which is the bandwidth
// model the benchmark's roofline uses.
#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstring>
#include <algorithm>
#include <thread>
#include <vector>

#include "../../include/srp.h"
#include "scene.h"
#include "srp_path.h"

namespace {

struct Counts {
    double rays = 0, segments = 0, nodes = 0, tris = 0, hits = 0, hit_rays = 0;
};

int closest_hit_counted(const std::vector<srp::BvhNode>& nodes, const std::vector<srp::TriRec>& tris, const float o[3],
                        const float d[3], int skip, float& tbest, Counts& c)
{
    const float ix = srp::safe_rcp(d[0]), iy = srp::safe_rcp(d[1]), iz = srp::safe_rcp(d[2]);
    const float nx = -o[0] * ix, ny = -o[1] * iy, nz = -o[2] * iz;
    tbest = FLT_MAX;
    int hit = -1, hit_id = 0x7fffffff;
    int stack[srp::kStackDepth];
    int sp = 0;
    int cur = 0;
    auto slab = [&](float lx, float hx, float ly, float hy, float lz, float hz, float& tn) {
        const float x0 = std::fma(lx, ix, nx), x1 = std::fma(hx, ix, nx);
        const float y0 = std::fma(ly, iy, ny), y1 = std::fma(hy, iy, ny);
        const float z0 = std::fma(lz, iz, nz), z1 = std::fma(hz, iz, nz);
        tn = std::fmax(std::fmax(std::fmin(x0, x1), std::fmin(y0, y1)), std::fmax(std::fmin(z0, z1), 0.0f));
        const float tf = std::fmin(std::fmin(std::fmax(x0, x1), std::fmax(y0, y1)), std::fmin(std::fmax(z0, z1), tbest));
        return tn <= tf;
    };
    for (;;) {
        if (cur >= 0) {
            c.nodes += 1;
            const srp::BvhNode& N = nodes[cur];
            float tn0, tn1;
            const bool h0 = slab(N.f[0].x, N.f[0].y, N.f[0].z, N.f[0].w, N.f[2].x, N.f[2].y, tn0);
            const bool h1 = slab(N.f[1].x, N.f[1].y, N.f[1].z, N.f[1].w, N.f[2].z, N.f[2].w, tn1);
            int c0, c1;
            std::memcpy(&c0, &N.f[3].x, 4);
            std::memcpy(&c1, &N.f[3].y, 4);
            if (h0 && h1) {
                const bool swap = tn1 < tn0;
                stack[sp++] = swap ? c0 : c1;
                cur = swap ? c1 : c0;
                continue;
            }
            if (h0) { cur = c0; continue; }
            if (h1) { cur = c1; continue; }
        } else {
            const int code = ~cur;
            const int first = code >> 3, cnt = code & 7;
            for (int q = 0; q < cnt; ++q) {
                const int tri = first + q;
                c.tris += 1;
                const float t = srp::tri_hit(o, d, tris[tri].f[0], tris[tri].f[1], tris[tri].f[2]);
                int id;
                std::memcpy(&id, &tris[tri].f[0].w, 4);
                if (t > 0.0f && tri != skip && (t < tbest || (t == tbest && id < hit_id))) {
                    tbest = t;
                    hit = tri;
                    hit_id = id;
                }
            }
        }
        if (sp == 0) break;
        cur = stack[--sp];
    }
    return hit;
}

}  // namespace

extern "C" srp_status srp_scene_ray_stats(srp_scene s, const double* sun_dirs, int64_t D, const srp_trace_params* p,
                                          const double* frames, int64_t pixel_stride, double* out)
{
    if (!s || !p || !out || (D > 0 && !sun_dirs) || pixel_stride < 1) return srp_fail(SRP_EINVAL, "bad argument");
    if (p->nu < 1 || p->nv < 1 || p->bounces < 1 || p->bounces > srp::kMaxBounces)
        return srp_fail(SRP_EINVAL, "bad trace parameters");
    if (p->frame_mode == 1 && !frames) return srp_fail(SRP_EINVAL, "frame_mode 1 needs frames");
    if (p->ray_mask) return srp_fail(SRP_EUNSUPPORTED, "ray_mask is not supported by the statistics");
    if (s->phong_finite) return srp_fail(SRP_EUNSUPPORTED, "Phong lobes are served by srp_surface_estimate only");
    std::vector<float4> mat(s->n_tris);
    if (hipSetDevice(s->device) != hipSuccess || hipMemcpy(mat.data(), s->d_mat, sizeof(float4) * s->n_tris,
                                                           hipMemcpyDeviceToHost) != hipSuccess)
        return srp_fail(SRP_EDEVICE, "copying the materials to the host failed");
    const srp_status pulled = srp_pull_host_tree(s);
    if (pulled != SRP_OK) return pulled;
    const int64_t n_pix = static_cast<int64_t>(p->nu) * p->nv;
    const unsigned n_thr = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<Counts> part(n_thr);
    std::vector<std::thread> th;
    for (unsigned tid = 0; tid < n_thr; ++tid) {
        th.emplace_back([&, tid]() {
            Counts& c = part[tid];
            for (int64_t j = 0; j < D; ++j) {
                double f[12];
                if (p->frame_mode == 1)
                    for (int a = 0; a < 12; ++a) f[a] = frames[12 * j + a];
                else
                    srp::frame_from_box(sun_dirs + 3 * j, s->lo, s->hi, s->L, p->nu, p->nv, f);
                const srp::DevFrame fr = srp::frame_to_device(sun_dirs + 3 * j, f, p->flux);
                const uint32_t dir = static_cast<uint32_t>(p->dir_index_base + j);
                for (int64_t pix = static_cast<int64_t>(tid) * pixel_stride; pix < n_pix;
                     pix += static_cast<int64_t>(n_thr) * pixel_stride) {
                    float o[3], d[3];
                    srp::primary_ray(fr, static_cast<int32_t>(pix % p->nu), static_cast<int32_t>(pix / p->nu),
                                     static_cast<uint32_t>(pix), dir, static_cast<uint32_t>(p->design_index),
                                     static_cast<uint32_t>(p->seed), static_cast<uint32_t>(p->seed >> 32),
                                     p->jitter != 0, o, d);
                    float w = fr.w;
                    int skip = -1;
                    c.rays += 1;
                    for (int b = 1; b <= p->bounces; ++b) {
                        c.segments += 1;
                        float t;
                        const int hit = closest_hit_counted(s->h_nodes, s->h_tris, o, d, skip, t, c);
                        if (hit < 0) break;
                        c.hits += 1;
                        if (b == 1) c.hit_rays += 1;
                        const srp::TriRec& tr = s->h_tris[hit];
                        const float n[3] = {tr.f[1].w, tr.f[2].w, tr.f[3].x};
                        float x[3], g[3];
                        const float4 m = mat[hit];
                        const bool more = srp::interact(o, d, w, t, n, m.x, m.y, m.z, b, p->bounces,
                                                        static_cast<uint32_t>(pix), dir,
                                                        static_cast<uint32_t>(p->design_index),
                                                        static_cast<uint32_t>(p->seed),
                                                        static_cast<uint32_t>(p->seed >> 32),
                                                        static_cast<float>(1e-5 * s->L), x, g);
                        if (!more) break;
                        skip = hit;
                    }
                }
            }
        });
    }
    for (auto& t : th) t.join();
    Counts tot;
    for (const Counts& c : part) {
        tot.rays += c.rays;
        tot.segments += c.segments;
        tot.nodes += c.nodes;
        tot.tris += c.tris;
        tot.hits += c.hits;
        tot.hit_rays += c.hit_rays;
    }
    out[0] = tot.rays;
    out[1] = tot.segments;
    out[2] = tot.nodes;
    out[3] = tot.tris;
    out[4] = tot.hits;
    out[5] = tot.hit_rays;
    return SRP_OK;
}
