// libsrp host side: C ABI (include/srp.h), scene lifecycle, design application (hinge rotation
// in FP64; host BVH build at creation, refit of its boxes when hinge angles change), workspace
// management and kernel launches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/srp.h"
#include "bvh_build.h"
#include "scene.h"
#include "srp_internal.h"

namespace {

thread_local std::string g_error;

srp_status fail(srp_status st, const std::string& msg)
{
    g_error = msg;
    return st;
}

#define SRP_HIP(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(SRP_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <class T>
hipError_t ensure(T*& ptr, size_t& cap, size_t n)
{
    if (n <= cap && ptr) return hipSuccess;
    if (ptr) {
        hipError_t e = hipFree(ptr);
        ptr = nullptr;
        cap = 0;
        if (e != hipSuccess) return e;
    }
    size_t bytes = std::max<size_t>(n, 1) * sizeof(T);
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&ptr), bytes);
    if (e != hipSuccess) {
        ptr = nullptr;
        return e;
    }
    cap = std::max<size_t>(n, 1);
    return hipSuccess;
}

}  // namespace

srp_status srp_pull_host_tree(srp_scene_s* s)
{
    if (!s->h_tree_stale && !s->h_tris_stale) return SRP_OK;
    if (hipSetDevice(s->device) != hipSuccess) return srp_fail(SRP_EDEVICE, "hipSetDevice failed");
    if (s->h_tree_stale) {
        s->h_nodes.resize(static_cast<size_t>(s->n_nodes));
        s->perm.resize(static_cast<size_t>(s->n_tris));
        if (hipMemcpy(s->h_nodes.data(), s->d_nodes, sizeof(srp::BvhNode) * s->n_nodes, hipMemcpyDeviceToHost) !=
                hipSuccess ||
            hipMemcpy(s->perm.data(), s->d_perm, sizeof(int32_t) * s->n_tris, hipMemcpyDeviceToHost) != hipSuccess)
            return srp_fail(SRP_EDEVICE, "copying the tree to the host failed");
        s->h_tree_stale = false;
        s->h_perm_stale = false;
    }
    if (s->h_tris_stale) {
        s->h_tris.resize(static_cast<size_t>(s->n_tris));
        if (hipMemcpy(s->h_tris.data(), s->d_tris, sizeof(srp::TriRec) * s->n_tris, hipMemcpyDeviceToHost) !=
            hipSuccess)
            return srp_fail(SRP_EDEVICE, "copying the triangle records to the host failed");
        s->h_tris_stale = false;
    }
    return SRP_OK;
}

srp_status srp_fail(srp_status st, const std::string& msg) { return fail(st, msg); }

namespace {
// tiles_per_wave candidates of the autotuner
constexpr int32_t kTuneFirst = 8;
constexpr int32_t kTuneLast = srp::kMaxTilesPerWave;
}  // namespace

namespace {

void rotate_hinges(srp_scene_s* s)
{
    s->cur = s->rest;
    for (int32_t k = 0; k < s->n_hinges; ++k) {
        const double ang = s->angles[k];
        if (ang == 0.0) continue;
        const double* o = s->hinges[k].origin;
        const double* ax = s->hinges[k].axis;
        const double c = std::cos(ang), sn = std::sin(ang);
        for (int64_t i = 0; i < s->n_verts; ++i) {
            if (s->vhinge[i] != k) continue;
            double p[3] = {s->rest[3 * i] - o[0], s->rest[3 * i + 1] - o[1], s->rest[3 * i + 2] - o[2]};
            const double kd = ax[0] * p[0] + ax[1] * p[1] + ax[2] * p[2];
            const double kx[3] = {ax[1] * p[2] - ax[2] * p[1], ax[2] * p[0] - ax[0] * p[2], ax[0] * p[1] - ax[1] * p[0]};
            for (int a = 0; a < 3; ++a) s->cur[3 * i + a] = o[a] + p[a] * c + kx[a] * sn + ax[a] * kd * (1.0 - c);
        }
    }
}

// Scene size L: twice the largest distance of a vertex from the vertex mean (rotation-invariant).
double scene_size(const std::vector<double>& v, int64_t n)
{
    double m[3] = {0, 0, 0};
    for (int64_t i = 0; i < n; ++i)
        for (int a = 0; a < 3; ++a) m[a] += v[3 * i + a];
    for (int a = 0; a < 3; ++a) m[a] /= static_cast<double>(n);
    double r2 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double q[3] = {v[3 * i] - m[0], v[3 * i + 1] - m[1], v[3 * i + 2] - m[2]};
        r2 = std::max(r2, q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    }
    return 2.0 * std::sqrt(r2);
}

// The hinge carrying all three vertices of facet f, else -1.
int32_t facet_hinge(const srp_scene_s* s, int64_t f)
{
    const int32_t* t = &s->tris[3 * f];
    const int32_t k = s->vhinge[t[0]];
    return k >= 0 && s->vhinge[t[1]] == k && s->vhinge[t[2]] == k ? k : -1;
}

std::array<double, 6> edge_key(const srp_scene_s* s, int32_t a, int32_t b)
{
    const double* pa = &s->rest[3 * static_cast<int64_t>(a)];
    const double* pb = &s->rest[3 * static_cast<int64_t>(b)];
    const bool swap = std::lexicographical_compare(pb, pb + 3, pa, pa + 3);
    const double* lo = swap ? pb : pa;
    const double* hi = swap ? pa : pb;
    return {lo[0], lo[1], lo[2], hi[0], hi[1], hi[2]};
}

// Where the surface continues across moving edge `ed` in one plane: every facet containing the
// edge rides the edge's hinge, their unit normals (rest pose) fall into at most two groups with
// opposite normals (the layers of a two-sided sheet), and each group holds two facets whose
// third vertices lie on opposite sides of the edge.  Returns the two facet pairs (a0, b0, a1, b1;
// a1 = b1 = -1 for one layer), or all -1 when the edge is not such a continuation.
int4 flat_continuation(const srp_scene_s* s, const int4& ed, const std::vector<int2>& incident)
{
    const int4 none = make_int4(-1, -1, -1, -1);
    constexpr double kTol = 1e-9;
    struct Group {
        double n[3];
        int32_t f[2], c[2];
        int count;
    } g[2];
    int ng = 0;
    for (const int2& fc : incident) {
        if (facet_hinge(s, fc.x) != ed.z) return none;
        const double* p0 = &s->rest[3 * static_cast<int64_t>(s->tris[3 * static_cast<int64_t>(fc.x)])];
        const double* p1 = &s->rest[3 * static_cast<int64_t>(s->tris[3 * static_cast<int64_t>(fc.x) + 1])];
        const double* p2 = &s->rest[3 * static_cast<int64_t>(s->tris[3 * static_cast<int64_t>(fc.x) + 2])];
        const double e1[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
        const double e2[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
        double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        const double len = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        for (double& x : n) x /= len;
        int gi = -1;
        for (int q = 0; q < ng && gi < 0; ++q)
            if (std::max({std::fabs(g[q].n[0] - n[0]), std::fabs(g[q].n[1] - n[1]), std::fabs(g[q].n[2] - n[2])}) <= kTol)
                gi = q;
        if (gi < 0) {
            if (ng == 2) return none;
            gi = ng++;
            std::copy(n, n + 3, g[gi].n);
            g[gi].count = 0;
        }
        if (g[gi].count == 2) return none;
        g[gi].f[g[gi].count] = fc.x;
        g[gi].c[g[gi].count] = fc.y;
        ++g[gi].count;
    }
    if (ng == 0) return none;
    if (ng == 2 && std::max({std::fabs(g[0].n[0] + g[1].n[0]), std::fabs(g[0].n[1] + g[1].n[1]),
                             std::fabs(g[0].n[2] + g[1].n[2])}) > kTol)
        return none;
    const double* pa = &s->rest[3 * static_cast<int64_t>(ed.x)];
    const double* pb = &s->rest[3 * static_cast<int64_t>(ed.y)];
    const double ab[3] = {pb[0] - pa[0], pb[1] - pa[1], pb[2] - pa[2]};
    for (int q = 0; q < ng; ++q) {
        if (g[q].count != 2) return none;
        double side[2];
        for (int i = 0; i < 2; ++i) {
            const double* pc = &s->rest[3 * static_cast<int64_t>(g[q].c[i])];
            const double ac[3] = {pc[0] - pa[0], pc[1] - pa[1], pc[2] - pa[2]};
            const double cr[3] = {ab[1] * ac[2] - ab[2] * ac[1], ab[2] * ac[0] - ab[0] * ac[2],
                                  ab[0] * ac[1] - ab[1] * ac[0]};
            side[i] = cr[0] * g[q].n[0] + cr[1] * g[q].n[1] + cr[2] * g[q].n[2];
        }
        if (!(side[0] * side[1] < 0.0)) return none;
    }
    return make_int4(g[0].f[0], g[0].f[1], ng == 2 ? g[1].f[0] : -1, ng == 2 ? g[1].f[1] : -1);
}

// The distinct edges of hinge-carried facets (all three vertices on one hinge), in order of first
// appearance over the facets and their edge slots; edges at the same pair of rest positions (the
// two layers of a two-sided sheet, the edge two facets share) are one edge.  Also the facet pairs
// across which each of them continues the surface in one plane (flat_continuation).
void build_moving_edges(srp_scene_s* s)
{
    s->h_edges.clear();
    s->h_edge_pairs.clear();
    std::map<std::array<double, 6>, int32_t> seen;
    for (int64_t f = 0; f < s->n_tris; ++f) {
        const int32_t k = facet_hinge(s, f);
        if (k < 0) continue;
        const int32_t* t = &s->tris[3 * f];
        for (int e = 0; e < 3; ++e) {
            const int32_t a = t[e], b = t[(e + 1) % 3];
            if (seen.emplace(edge_key(s, a, b), static_cast<int32_t>(s->h_edges.size())).second)
                s->h_edges.push_back(make_int4(a, b, k, 0));
        }
    }
    if (s->h_edges.empty()) return;
    std::vector<std::vector<int2>> incident(s->h_edges.size());  // (facet, opposite vertex)
    for (int64_t f = 0; f < s->n_tris; ++f) {
        const int32_t* t = &s->tris[3 * f];
        for (int e = 0; e < 3; ++e) {
            const auto it = seen.find(edge_key(s, t[e], t[(e + 1) % 3]));
            if (it != seen.end()) incident[it->second].push_back(make_int2(static_cast<int32_t>(f), t[(e + 2) % 3]));
        }
    }
    for (size_t i = 0; i < s->h_edges.size(); ++i)
        s->h_edge_pairs.push_back(flat_continuation(s, s->h_edges[i], incident[i]));
}

// The edges the edge term takes under the current materials: an edge is left out where the
// surface continues across it in one plane with the same (rho_s, rho_d, p_spec) on both sides of
// every layer, since the momentum a path deposits is continuous there (the two side paths differ
// by O(delta) only).  Synchronises `stream`.
hipError_t classify_edges(srp_scene_s* s, hipStream_t stream)
{
    const size_t n = s->h_edges.size();
    hipError_t e = ensure(s->d_edge_keep, s->edge_keep_cap, n);
    if (e == hipSuccess)
        e = srp::launch_edge_keep(s->d_edge_pairs, static_cast<int32_t>(n), s->d_bvh_pos, s->d_mat, s->d_edge_keep,
                                  stream);
    std::vector<int32_t> keep(n);
    if (e == hipSuccess)
        e = hipMemcpyAsync(keep.data(), s->d_edge_keep, sizeof(int32_t) * n, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return e;
    s->h_live_edges.clear();
    for (size_t i = 0; i < n; ++i)
        if (keep[i])
            s->h_live_edges.push_back(
                make_int4(s->h_edges[i].x, s->h_edges[i].y, s->h_edges[i].z, static_cast<int32_t>(i)));
    if (!s->h_live_edges.empty()) {
        e = ensure(s->d_live_edges, s->live_edges_cap, s->h_live_edges.size());
        if (e == hipSuccess)
            e = hipMemcpyAsync(s->d_live_edges, s->h_live_edges.data(), sizeof(int4) * s->h_live_edges.size(),
                               hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return e;
    }
    s->edge_class_gen = s->geom_gen;
    return hipSuccess;
}

// Current vertex positions (FP32) for the edge terms; synchronous with `stream`.
hipError_t upload_vertices(srp_scene_s* s, hipStream_t stream)
{
    if (s->h_edges.empty()) return hipSuccess;
    hipError_t e0 = ensure(s->d_vpos, s->vpos_cap, static_cast<size_t>(s->n_verts));
    if (e0 != hipSuccess) return e0;
    std::vector<float4> v(static_cast<size_t>(s->n_verts));
    for (int64_t i = 0; i < s->n_verts; ++i)
        v[i] = make_float4(static_cast<float>(s->cur[3 * i]), static_cast<float>(s->cur[3 * i + 1]),
                           static_cast<float>(s->cur[3 * i + 2]), 0.0f);
    hipError_t e = hipMemcpyAsync(s->d_vpos, v.data(), v.size() * sizeof(float4), hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    return e;
}

// The moving edges of the rest pose and the current vertex positions, on the device; synchronous.
hipError_t upload_edges(srp_scene_s* s, hipStream_t stream)
{
    build_moving_edges(s);
    s->edge_class_gen = ~0ull;
    if (s->h_edges.empty()) return hipSuccess;
    hipError_t e = ensure(s->d_edges, s->edges_cap, s->h_edges.size());
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->d_edges, s->h_edges.data(), sizeof(int4) * s->h_edges.size(), hipMemcpyHostToDevice,
                           stream);
    if (e == hipSuccess) e = ensure(s->d_edge_pairs, s->edge_pairs_cap, s->h_edge_pairs.size());
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->d_edge_pairs, s->h_edge_pairs.data(), sizeof(int4) * s->h_edge_pairs.size(),
                           hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = upload_vertices(s, stream);
    return e;
}

// Record ranges of every node's two child slots (first0, last0, first1, last1; last < first for
// an empty leaf) of a pre-order tree whose leaves hold consecutive records.
std::vector<int4> child_ranges(const std::vector<srp::BvhNode>& nodes)
{
    const int32_t n = static_cast<int32_t>(nodes.size());
    std::vector<int4> r(n);
    std::vector<int2> own(n);
    for (int32_t i = n - 1; i >= 0; --i) {
        int32_t codes[2];
        std::memcpy(codes, &nodes[i].f[3], 8);
        int2 sl[2];
        for (int slot = 0; slot < 2; ++slot) {
            const int32_t c = codes[slot];
            if (c >= 0) {
                sl[slot] = own[c];
            } else {
                const int32_t first = (~c) >> 3, cnt = (~c) & 7;
                sl[slot] = make_int2(first, first + cnt - 1);
            }
        }
        r[i] = make_int4(sl[0].x, sl[0].y, sl[1].x, sl[1].y);
        const bool e0 = sl[0].y < sl[0].x, e1 = sl[1].y < sl[1].x;
        own[i] = e0 ? sl[1] : e1 ? sl[0] : make_int2(std::min(sl[0].x, sl[1].x), std::max(sl[0].y, sl[1].y));
    }
    return r;
}

// Bounds and scene size of the current vertices.
void update_bounds(srp_scene_s* s)
{
    const auto& V = s->cur;
    for (int a = 0; a < 3; ++a) {
        s->lo[a] = INFINITY;
        s->hi[a] = -INFINITY;
    }
    for (int64_t i = 0; i < s->n_verts; ++i)
        for (int a = 0; a < 3; ++a) {
            s->lo[a] = std::min(s->lo[a], V[3 * i + a]);
            s->hi[a] = std::max(s->hi[a], V[3 * i + a]);
        }
    s->L = scene_size(V, s->n_verts);
}

// Bounds, scene size, triangle records and cumulative areas for the current vertices; the tree
// is built on the host, or (refit) kept and its boxes refitted on the device.  Fails before any
// change to the tree or the records when the new tree is deeper than the traversal stack.
srp_status rebuild(srp_scene_s* s, hipStream_t stream, bool refit = false)
{
    const auto& V = s->cur;
    update_bounds(s);
    const bool device_refit = refit && s->d_nodes && s->ranges_nodes == s->n_nodes;
    if (!device_refit) {
        srp::BvhBuildResult bvh = srp::build_bvh(V.data(), s->tris.data(), s->n_tris, 1e-6 * s->L);
        if (bvh.depth >= srp::kStackDepth - 1) return fail(SRP_EUNSUPPORTED, "BVH deeper than the traversal stack");
        s->n_nodes = static_cast<int32_t>(bvh.nodes.size());
        s->depth = bvh.depth;
        s->perm = std::move(bvh.perm);
        s->h_nodes = std::move(bvh.nodes);
        s->h_tree_stale = false;
    } else {
        // the records are formed on the host in tree order: bring the order back after a GPU build
        if (s->h_perm_stale) {
            const srp_status st = srp_pull_host_tree(s);
            if (st != SRP_OK) return st;
        }
        s->h_tree_stale = true;  // the refit changes the device boxes only; the host order stays valid
    }
    std::vector<srp::TriRec> recs(s->n_tris);
    for (int64_t p = 0; p < s->n_tris; ++p) {
        const int32_t f = s->perm[p];
        const double* a = &V[3 * static_cast<int64_t>(s->tris[3 * f])];
        const double* b = &V[3 * static_cast<int64_t>(s->tris[3 * f + 1])];
        const double* c = &V[3 * static_cast<int64_t>(s->tris[3 * f + 2])];
        double e1[3], e2[3];
        for (int k = 0; k < 3; ++k) {
            e1[k] = b[k] - a[k];
            e2[k] = c[k] - a[k];
        }
        double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        const double len = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        if (!(len > 0.0) || !std::isfinite(len)) return fail(SRP_EDEGENERATE, "zero-area or non-finite facet");
        for (int k = 0; k < 3; ++k) n[k] /= len;
        srp::TriRec& r = recs[p];
        int32_t fid = f;
        float fid_bits;
        std::memcpy(&fid_bits, &fid, 4);
        r.f[0] = make_float4(static_cast<float>(a[0]), static_cast<float>(a[1]), static_cast<float>(a[2]), fid_bits);
        r.f[1] = make_float4(static_cast<float>(e1[0]), static_cast<float>(e1[1]), static_cast<float>(e1[2]),
                             static_cast<float>(n[0]));
        r.f[2] = make_float4(static_cast<float>(e2[0]), static_cast<float>(e2[1]), static_cast<float>(e2[2]),
                             static_cast<float>(n[1]));
        // hinge carrying the facet (-1: rigid); a facet is carried by hinge k when all three
        // vertices are
        int32_t h0 = s->vhinge[s->tris[3 * f]], h1 = s->vhinge[s->tris[3 * f + 1]], h2 = s->vhinge[s->tris[3 * f + 2]];
        int32_t hid = (h0 == h1 && h1 == h2) ? h0 : -1;
        float hid_bits;
        std::memcpy(&hid_bits, &hid, 4);
        r.f[3] = make_float4(static_cast<float>(n[2]), hid_bits, 0.0f, 0.0f);
    }
    // cumulative facet areas in original order (FP64) and the BVH position of each facet
    std::vector<double> cum(s->n_tris);
    std::vector<int32_t> pos(s->n_tris);
    double acc = 0.0;
    for (int64_t f = 0; f < s->n_tris; ++f) {
        const double* a = &V[3 * static_cast<int64_t>(s->tris[3 * f])];
        const double* b = &V[3 * static_cast<int64_t>(s->tris[3 * f + 1])];
        const double* c = &V[3 * static_cast<int64_t>(s->tris[3 * f + 2])];
        const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        const double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                              e1[0] * e2[1] - e1[1] * e2[0]};
        acc += 0.5 * std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        cum[f] = acc;
    }
    for (int64_t p = 0; p < s->n_tris; ++p) pos[s->perm[p]] = static_cast<int32_t>(p);
    s->area = acc;
    SRP_HIP(ensure(s->d_cum_area, s->cum_cap, static_cast<size_t>(s->n_tris)));
    SRP_HIP(ensure(s->d_bvh_pos, s->bvh_pos_cap, static_cast<size_t>(s->n_tris)));
    SRP_HIP(hipMemcpyAsync(s->d_cum_area, cum.data(), cum.size() * sizeof(double), hipMemcpyHostToDevice, stream));
    SRP_HIP(hipMemcpyAsync(s->d_bvh_pos, pos.data(), pos.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream));
    SRP_HIP(ensure(s->d_tris, s->tris_cap, static_cast<size_t>(s->n_tris)));
    SRP_HIP(hipMemcpyAsync(s->d_tris, recs.data(), recs.size() * sizeof(srp::TriRec), hipMemcpyHostToDevice, stream));
    if (!device_refit) {
        SRP_HIP(ensure(s->d_nodes, s->nodes_cap, s->h_nodes.size()));
        SRP_HIP(ensure(s->d_perm, s->perm_cap, static_cast<size_t>(s->n_tris)));
        SRP_HIP(hipMemcpyAsync(s->d_nodes, s->h_nodes.data(), s->h_nodes.size() * sizeof(srp::BvhNode),
                               hipMemcpyHostToDevice, stream));
        SRP_HIP(hipMemcpyAsync(s->d_perm, s->perm.data(), s->perm.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                               stream));
        const std::vector<int4> ranges = child_ranges(s->h_nodes);
        SRP_HIP(ensure(s->d_ranges, s->ranges_cap, ranges.size()));
        SRP_HIP(hipMemcpyAsync(s->d_ranges, ranges.data(), ranges.size() * sizeof(int4), hipMemcpyHostToDevice,
                               stream));
        s->ranges_nodes = s->n_nodes;
    } else {
        const int32_t n = static_cast<int32_t>(s->n_tris);
        int32_t levels = 1;
        while ((int64_t(1) << levels) <= n) ++levels;
        SRP_HIP(ensure(s->d_win, s->win_cap, static_cast<size_t>(6) * n * levels));
        SRP_HIP(srp::launch_refit(s->d_tris, n, s->d_nodes, s->d_ranges, s->n_nodes, s->d_win, levels,
                                  static_cast<float>(1e-6 * s->L), stream));
    }
    SRP_HIP(hipStreamSynchronize(stream));
    s->h_tris = std::move(recs);
    s->h_tris_stale = false;
    return SRP_OK;
}

// Wave tiles per wave (and so per workgroup: kWaves times as many) of a trace of total_tiles
// tiles: the caller's choice, else enough workgroups to fill 256 CUs many times over with few
// partials per direction, at most kTilesPerWaveLarge.
int64_t tiles_per_wave_for(const srp_trace_params* p, int64_t total_tiles)
{
    if (p->tiles_per_wave > 0) return p->tiles_per_wave;
    const int64_t tpw = total_tiles / (int64_t(srp::kWaves) * 8192);
    return std::max<int64_t>(1, std::min<int64_t>(srp::kTilesPerWaveLarge, tpw));
}

// Secondary segments take the per-lane walk when the tree fits its stack, unless the environment
// sets SRP_SECONDARY_WALK=wave (every segment then takes the wave-coherent walk).  Both walks give
// identical hits; the switch exists for performance comparisons.
int32_t lane_walk_for(int32_t depth)
{
    static const bool wave_only = [] {
        const char* e = std::getenv("SRP_SECONDARY_WALK");
        return e != nullptr && std::strcmp(e, "wave") == 0;
    }();
    if (wave_only || depth > srp::kLaneStack) return 0;
    return depth <= srp::kLaneStackShort ? 2 : 1;
}

srp_status check_params(const srp_trace_params* p)
{
    if (!p) return fail(SRP_EINVAL, "params is NULL");
    if (p->nu < 1 || p->nv < 1) return fail(SRP_EINVAL, "nu and nv must be >= 1");
    if (static_cast<int64_t>(p->nu) * p->nv > (int64_t(1) << 31)) return fail(SRP_EINVAL, "nu * nv exceeds 2^31");
    if (p->bounces < 1 || p->bounces > srp::kMaxBounces) return fail(SRP_EINVAL, "bounces must be in 1..8");
    if (!(p->flux >= 0.0) || !std::isfinite(p->flux)) return fail(SRP_EINVAL, "flux must be finite and >= 0");
    if (p->frame_mode != 0 && p->frame_mode != 1) return fail(SRP_EINVAL, "frame_mode must be 0 or 1");
    if (p->dir_index_base < 0) return fail(SRP_EINVAL, "dir_index_base must be >= 0");
    if (p->tiles_per_wave < 0 || p->tiles_per_wave > srp::kMaxTilesPerWave)
        return fail(SRP_EINVAL, "tiles_per_wave must be in 0..16");
    if (p->sampling < 0 || p->sampling > 3) return fail(SRP_EINVAL, "sampling must be in 0..3");
    if (p->edge_samples < 0 || p->edge_samples > 4096) return fail(SRP_EINVAL, "edge_samples must be in 0..4096");
    return SRP_OK;
}

srp_status bind_device(const srp_scene_s* s)
{
    int cur = -1;
    SRP_HIP(hipGetDevice(&cur));
    if (cur != s->device) SRP_HIP(hipSetDevice(s->device));
    return SRP_OK;
}

// Frames launch + trace arguments shared by srp_trace, srp_trace_records and srp_trace_adjoint.
// The grid frames and per-workgroup partial sums live in the scene's workspace, or in `ws` when it
// is given (forward traces only): then nothing is allocated and a trace that needs more than
// ws->bytes is rejected before anything is enqueued.
srp_status prepare_trace(srp_scene_s* s, const double* sun_dirs, int64_t D, const srp_trace_params* p,
                         const double* frames, bool records, const int64_t* pix, int64_t n_pix, int32_t* rec_hit,
                         float* rec_force, hipStream_t stream, srp::TraceArgs& a,
                         const srp::TraceWorkspace* ws = nullptr, float* rec_point = nullptr)
{
    if (s->phong_finite)
        return fail(SRP_EUNSUPPORTED, "Phong lobes are served by srp_surface_estimate only (the ray grid has mirrors)");
    a = srp::TraceArgs{};
    a.ray_mask = p->ray_mask;
    a.mask_words = (static_cast<int64_t>(p->nu) * p->nv + 31) / 32;
    a.rec_point = rec_point;
    a.nodes = s->d_nodes;
    a.tris = s->d_tris;
    a.mat = s->d_mat;
    a.D = D;
    a.nu = p->nu;
    a.nv = p->nv;
    a.bounces = p->bounces;
    a.jitter = p->jitter ? 1 : 0;
    a.seed_lo = static_cast<uint32_t>(p->seed);
    a.seed_hi = static_cast<uint32_t>(p->seed >> 32);
    a.dir_index_base = p->dir_index_base;
    a.design_index = static_cast<uint32_t>(p->design_index);
    for (int k = 0; k < 3; ++k) a.com[k] = static_cast<float>(s->com[k]);
    a.eps = static_cast<float>(1e-5 * s->L);
    a.tiles_x = (p->nu + srp::kTileW - 1) / srp::kTileW;
    a.tiles_y = (p->nv + srp::kTileH - 1) / srp::kTileH;
    a.lane_walk = lane_walk_for(s->depth);
    a.cull = p->frame_mode == 0 ? 1 : 0;
    if (records) {
        a.pix = pix;
        a.n_pix = pix ? n_pix : static_cast<int64_t>(p->nu) * p->nv;
        a.tiles_per_dir = (a.n_pix + 63) / 64;
        a.rec_hit = rec_hit;
        a.rec_force = rec_force;
    } else {
        a.tiles_per_dir = static_cast<int64_t>(a.tiles_x) * a.tiles_y;
    }
    const int64_t tpw = tiles_per_wave_for(p, a.tiles_per_dir * D);
    a.tiles_per_wave = static_cast<int32_t>(tpw);
    const int64_t per_block = tpw * srp::kWaves;
    const int64_t bpd = std::max<int64_t>(1, (a.tiles_per_dir + per_block - 1) / per_block);
    if (bpd * D > 0x7fffffffLL) return fail(SRP_EINVAL, "trace too large for one launch");
    a.blocks_per_dir = static_cast<int32_t>(bpd);
    // with at least one direction per XCD, each direction stays on one XCD (no image row is tied to
    // an XCD); fewer directions are spread over all of them
    a.xcd_major = D >= srp::kXcds ? 1 : 0;
    if (srp::grid_blocks(a, D) > 0x7fffffffLL) return fail(SRP_EINVAL, "trace too large for one launch");
    const size_t n_partials = static_cast<size_t>(bpd * D * std::max(6, srp::kMaxHinges));
    if (ws) {
        const size_t frame_bytes = (static_cast<size_t>(D) * sizeof(srp::DevFrame) + 255) / 256 * 256;
        const size_t need = frame_bytes + n_partials * sizeof(double);
        if (need > ws->bytes)
            return fail(SRP_EINVAL, "this trace needs " + std::to_string(need) + " bytes of workspace (" +
                                        std::to_string(D) + " directions x " + std::to_string(bpd) +
                                        " workgroups each); the fixed workspace holds " + std::to_string(ws->bytes));
        a.frames = reinterpret_cast<srp::DevFrame*>(ws->base);
        a.partials = reinterpret_cast<double*>(static_cast<char*>(ws->base) + frame_bytes);
    } else {
        SRP_HIP(ensure(s->d_frames, s->frames_cap, static_cast<size_t>(D)));
        SRP_HIP(ensure(s->d_partials, s->partials_cap, n_partials));
        a.frames = s->d_frames;
        a.partials = s->d_partials;
    }
    SRP_HIP(srp::launch_frames(sun_dirs, D, s->lo, s->hi, s->L, p->nu, p->nv, p->flux,
                               p->frame_mode == 1 ? frames : nullptr, nullptr,
                               const_cast<srp::DevFrame*>(a.frames), stream));
    return SRP_OK;
}

srp_status enqueue_trace(srp_scene_s* s, const double* sun_dirs, int64_t D, const srp_trace_params* p,
                         const double* frames, bool records, const int64_t* pix, int64_t n_pix, int32_t* rec_hit,
                         float* rec_force, float* rec_point, hipStream_t stream, int32_t* bpd_out)
{
    srp::TraceArgs a;
    srp_status st = prepare_trace(s, sun_dirs, D, p, frames, records, pix, n_pix, rec_hit, rec_force, stream, a,
                                  nullptr, rec_point);
    if (st != SRP_OK) return st;
    SRP_HIP(srp::launch_trace(a, records, stream));
    *bpd_out = a.blocks_per_dir;
    return SRP_OK;
}

}  // namespace

namespace srp {

int64_t path_record_bytes(const srp_trace_params* p, int64_t D)
{
    const int64_t tiles = static_cast<int64_t>((p->nu + kTileW - 1) / kTileW) * ((p->nv + kTileH - 1) / kTileH);
    return D * p->bounces * tiles * 64 * static_cast<int64_t>(sizeof(int32_t));
}

srp_status trace_into(srp_scene_s* s, const double* sun_dirs, int64_t D, const srp_trace_params* p,
                      const double* frames, double* force, double* torque, hipStream_t stream,
                      const TraceWorkspace* ws, int32_t* paths)
{
    if (!s) return fail(SRP_EINVAL, "scene is NULL");
    srp_status st = check_params(p);
    if (st != SRP_OK) return st;
    if (D < 0) return fail(SRP_EINVAL, "D must be >= 0");
    if (D == 0) return SRP_OK;
    if (!sun_dirs || !force) return fail(SRP_EINVAL, "sun_dirs and force are required");
    if (p->frame_mode == 1 && !frames) return fail(SRP_EINVAL, "frame_mode 1 needs frames");
    if (p->dir_index_base + D > (int64_t(1) << 32)) return fail(SRP_EINVAL, "direction index exceeds 32 bits");
    st = bind_device(s);
    if (st != SRP_OK) return st;
    TraceArgs a;
    st = prepare_trace(s, sun_dirs, D, p, frames, false, nullptr, 0, nullptr, nullptr, stream, a, ws);
    if (st != SRP_OK) return st;
    a.path_hit = paths;
    SRP_HIP(launch_trace(a, false, stream));
    SRP_HIP(launch_reduce(a.partials, D, a.blocks_per_dir, force, torque, stream));
    return SRP_OK;
}

}  // namespace srp

extern "C" {

const char* srp_last_error(void) { return g_error.c_str(); }

srp_status srp_sync(void* stream)
{
    SRP_HIP(hipStreamSynchronize(static_cast<hipStream_t>(stream)));
    SRP_HIP(hipGetLastError());
    return SRP_OK;
}

srp_status srp_scene_create(const double* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                            const int32_t* vert_hinge, const srp_hinge* hinges, int32_t n_hinges, const double* com,
                            srp_scene* out)
{
    if (!out) return fail(SRP_EINVAL, "out is NULL");
    *out = nullptr;
    if (!verts || n_verts < 3 || !tris || n_tris < 1) return fail(SRP_EINVAL, "empty mesh");
    if (n_tris > (int64_t(1) << 26)) return fail(SRP_EINVAL, "more than 2^26 triangles");
    if (n_hinges < 0 || (n_hinges > 0 && !hinges)) return fail(SRP_EINVAL, "bad hinges");
    for (int64_t i = 0; i < 3 * n_verts; ++i)
        if (!std::isfinite(verts[i])) return fail(SRP_EDEGENERATE, "non-finite vertex");
    for (int64_t i = 0; i < 3 * n_tris; ++i)
        if (tris[i] < 0 || tris[i] >= n_verts) return fail(SRP_EINVAL, "triangle index out of range");
    if (vert_hinge)
        for (int64_t i = 0; i < n_verts; ++i)
            if (vert_hinge[i] < -1 || vert_hinge[i] >= n_hinges) return fail(SRP_EINVAL, "vert_hinge out of range");
    srp_scene_s* s = new (std::nothrow) srp_scene_s();
    if (!s) return fail(SRP_ENOMEM, "host allocation failed");
    hipError_t e = hipGetDevice(&s->device);
    if (e != hipSuccess) {
        delete s;
        return fail(SRP_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
    }
    s->n_verts = n_verts;
    s->n_tris = n_tris;
    s->n_hinges = n_hinges;
    s->rest.assign(verts, verts + 3 * n_verts);
    s->tris.assign(tris, tris + 3 * n_tris);
    s->vhinge.assign(n_verts, -1);
    if (vert_hinge) s->vhinge.assign(vert_hinge, vert_hinge + n_verts);
    for (int32_t k = 0; k < n_hinges; ++k) {
        srp_hinge h = hinges[k];
        const double len = std::sqrt(h.axis[0] * h.axis[0] + h.axis[1] * h.axis[1] + h.axis[2] * h.axis[2]);
        if (!(len > 0.0) || !std::isfinite(len)) {
            delete s;
            return fail(SRP_EINVAL, "hinge axis must be non-zero");
        }
        for (int a = 0; a < 3; ++a) h.axis[a] /= len;
        s->hinges.push_back(h);
    }
    s->angles.assign(n_hinges, 0.0);
    if (com)
        for (int a = 0; a < 3; ++a) s->com[a] = com[a];
    rotate_hinges(s);
    srp_status st = rebuild(s, nullptr);
    if (st != SRP_OK) {
        srp_scene_destroy(s);
        return st;
    }
    e = ensure(s->d_mat, s->mat_cap, static_cast<size_t>(n_tris));
    if (e == hipSuccess) e = hipMemset(s->d_mat, 0, sizeof(float4) * n_tris);
    if (e == hipSuccess) e = ensure(s->d_flag, s->flag_cap, 1);
    if (e == hipSuccess) e = srp::launch_pack_phong(nullptr, s->d_perm, n_tris, s->d_mat, s->d_flag, nullptr);
    if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
    if (e == hipSuccess) e = upload_edges(s, nullptr);
    if (e != hipSuccess) {
        srp_scene_destroy(s);
        return fail(SRP_EDEVICE, std::string("scene buffers: ") + hipGetErrorString(e));
    }
    *out = s;
    return SRP_OK;
}

srp_status srp_scene_set_design(srp_scene s, const double* hinge_angles, const float* rho_s, const float* rho_d,
                                const float* p_spec, void* stream_)
{
    if (!s) return fail(SRP_EINVAL, "scene is NULL");
    if (!rho_s || !rho_d) return fail(SRP_EINVAL, "rho_s and rho_d are required");
    srp_status st = bind_device(s);
    if (st != SRP_OK) return st;
    ++s->geom_gen;  // path records of earlier calls no longer describe the scene
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    if (hinge_angles) {
        bool changed = false;
        for (int32_t k = 0; k < s->n_hinges; ++k) {
            if (!std::isfinite(hinge_angles[k])) return fail(SRP_EINVAL, "non-finite hinge angle");
            if (hinge_angles[k] != s->angles[k]) changed = true;
        }
        if (changed) {
            SRP_HIP(hipStreamSynchronize(stream));  // kernels in flight may still read the old BVH
            s->angles.assign(hinge_angles, hinge_angles + s->n_hinges);
            rotate_hinges(s);
            st = rebuild(s, stream, s->refit_on_hinge);
            if (st != SRP_OK) return st;
            SRP_HIP(upload_vertices(s, stream));
        }
    }
    SRP_HIP(hipMemsetAsync(s->d_flag, 0, sizeof(int32_t), stream));
    SRP_HIP(srp::launch_pack_materials(rho_s, rho_d, p_spec, s->d_phong, s->d_perm, s->n_tris, s->d_mat, s->d_flag,
                                       stream));
    int32_t flag = 0;
    SRP_HIP(hipMemcpyAsync(&flag, s->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    SRP_HIP(hipStreamSynchronize(stream));
    if (flag & 1) return fail(SRP_EINVAL, "reflectances must satisfy rho_s >= 0, rho_d >= 0, rho_s + rho_d <= 1");
    if (flag & 2)
        return fail(SRP_EINVAL, "p_spec must lie in [0, 1], and may be 0 only where rho_s = 0 and 1 only where rho_d = 0");
    return SRP_OK;
}

srp_status srp_scene_set_phong(srp_scene s, const float* exponents, void* stream_)
{
    if (!s) return fail(SRP_EINVAL, "scene is NULL");
    srp_status st = bind_device(s);
    if (st != SRP_OK) return st;
    ++s->geom_gen;  // path records of earlier calls no longer describe the scene
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    SRP_HIP(hipStreamSynchronize(stream));  // kernels in flight may still read the materials
    // a private copy, checked before anything of the scene changes
    float* staged = nullptr;
    if (exponents) {
        SRP_HIP(hipMalloc(reinterpret_cast<void**>(&staged), sizeof(float) * s->n_tris));
        hipError_t e = hipMemcpyAsync(staged, exponents, sizeof(float) * s->n_tris, hipMemcpyDeviceToDevice, stream);
        if (e != hipSuccess) {
            (void)hipFree(staged);
            return fail(SRP_EDEVICE, std::string("copying the exponents: ") + hipGetErrorString(e));
        }
    }
    int32_t flag = 0;
    hipError_t e = hipMemsetAsync(s->d_flag, 0, sizeof(int32_t), stream);
    if (e == hipSuccess) e = srp::launch_pack_phong(staged, s->d_perm, s->n_tris, nullptr, s->d_flag, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, s->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess || (flag & 1)) {
        (void)hipFree(staged);
        if (e != hipSuccess) return fail(SRP_EDEVICE, std::string("checking the exponents: ") + hipGetErrorString(e));
        return fail(SRP_EINVAL, "Phong exponents must be >= 1 (or +infinity for an ideal mirror)");
    }
    (void)hipFree(s->d_phong);
    s->d_phong = staged;
    s->phong_finite = (flag & 2) != 0;
    SRP_HIP(srp::launch_pack_phong(s->d_phong, s->d_perm, s->n_tris, s->d_mat, s->d_flag, stream));
    SRP_HIP(hipStreamSynchronize(stream));
    return SRP_OK;
}

srp_status srp_scene_set_vertices(srp_scene s, const double* verts, int64_t n_verts, int32_t mode, void* stream_)
{
    if (!s || !verts) return fail(SRP_EINVAL, "NULL argument");
    if (n_verts != s->n_verts) return fail(SRP_EINVAL, "n_verts does not match the scene");
    if (mode != 0 && mode != 1) return fail(SRP_EINVAL, "mode must be 0 (refit the tree) or 1 (rebuild it)");
    for (int64_t i = 0; i < 3 * n_verts; ++i)
        if (!std::isfinite(verts[i])) return fail(SRP_EDEGENERATE, "non-finite vertex");
    srp_status st = bind_device(s);
    if (st != SRP_OK) return st;
    ++s->geom_gen;  // path records of earlier calls no longer describe the scene
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    // every facet of the new pose must keep a positive area before anything changes
    std::vector<double> old_rest;
    old_rest.swap(s->rest);
    s->rest.assign(verts, verts + 3 * n_verts);
    rotate_hinges(s);
    for (int64_t f = 0; f < s->n_tris; ++f) {
        const double* a = &s->cur[3 * static_cast<int64_t>(s->tris[3 * f])];
        const double* b = &s->cur[3 * static_cast<int64_t>(s->tris[3 * f + 1])];
        const double* c = &s->cur[3 * static_cast<int64_t>(s->tris[3 * f + 2])];
        const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
        const double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
        const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                              e1[0] * e2[1] - e1[1] * e2[0]};
        const double len = std::sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
        if (!(len > 0.0) || !std::isfinite(len)) {
            s->rest.swap(old_rest);
            rotate_hinges(s);
            return fail(SRP_EDEGENERATE, "zero-area or non-finite facet");
        }
    }
    SRP_HIP(hipStreamSynchronize(stream));  // kernels in flight may still read the old tree
    // a rebuild reorders the records: the packed materials follow their facets
    std::vector<int32_t> old_pos;
    if (mode == 1) {
        if (s->h_perm_stale) {
            st = srp_pull_host_tree(s);
            if (st != SRP_OK) return st;
        }
        old_pos.resize(static_cast<size_t>(s->n_tris));
        for (int64_t q = 0; q < s->n_tris; ++q) old_pos[s->perm[q]] = static_cast<int32_t>(q);
    }
    st = rebuild(s, stream, mode == 0);
    if (st == SRP_EUNSUPPORTED) {
        // a tree deeper than the stack: nothing changed but the bounds
        s->rest.swap(old_rest);
        rotate_hinges(s);
        update_bounds(s);
        return st;
    }
    if (st != SRP_OK) return st;
    if (mode == 1) {
        std::vector<float4> m_old(static_cast<size_t>(s->n_tris)), m_new(static_cast<size_t>(s->n_tris));
        SRP_HIP(hipMemcpyAsync(m_old.data(), s->d_mat, sizeof(float4) * s->n_tris, hipMemcpyDeviceToHost, stream));
        SRP_HIP(hipStreamSynchronize(stream));
        for (int64_t q = 0; q < s->n_tris; ++q) m_new[q] = m_old[old_pos[s->perm[q]]];
        SRP_HIP(hipMemcpyAsync(s->d_mat, m_new.data(), sizeof(float4) * s->n_tris, hipMemcpyHostToDevice, stream));
        SRP_HIP(hipStreamSynchronize(stream));
    }
    SRP_HIP(upload_edges(s, stream));
    s->mw_groups.clear();  // the multi-world records hold the old rest pose
    return SRP_OK;
}

srp_status srp_scene_get_vertices(srp_scene s, double* out, int64_t n_verts)
{
    if (!s || !out) return fail(SRP_EINVAL, "NULL argument");
    if (n_verts != s->n_verts) return fail(SRP_EINVAL, "n_verts does not match the scene");
    std::memcpy(out, s->cur.data(), sizeof(double) * 3 * n_verts);
    return SRP_OK;
}

srp_status srp_scene_info(srp_scene s, int32_t* n_nodes, int32_t* depth, int32_t* n_tris)
{
    if (!s) return fail(SRP_EINVAL, "scene is NULL");
    if (n_nodes) *n_nodes = s->n_nodes;
    if (depth) *depth = s->depth;
    if (n_tris) *n_tris = static_cast<int32_t>(s->n_tris);
    return SRP_OK;
}

srp_status srp_frames(srp_scene s, const double* sun_dirs, int64_t D, int32_t nu, int32_t nv, double* frames,
                      void* stream)
{
    if (!s || (D > 0 && (!sun_dirs || !frames))) return fail(SRP_EINVAL, "NULL argument");
    if (D < 0 || nu < 1 || nv < 1) return fail(SRP_EINVAL, "bad sizes");
    srp_status st = bind_device(s);
    if (st != SRP_OK) return st;
    SRP_HIP(srp::launch_frames(sun_dirs, D, s->lo, s->hi, s->L, nu, nv, 0.0, nullptr, frames, nullptr,
                               static_cast<hipStream_t>(stream)));
    return SRP_OK;
}

srp_status srp_trace(srp_scene s, const double* sun_dirs, int64_t D, const srp_trace_params* p, const double* frames,
                     double* force, double* torque, void* stream_)
{
    return srp::trace_into(s, sun_dirs, D, p, frames, force, torque, static_cast<hipStream_t>(stream_), nullptr);
}

srp_status srp_trace_records(srp_scene s, const double* sun_dirs, int64_t D, const srp_trace_params* p,
                             const double* frames, const int64_t* pix, int64_t n_pix, int32_t* hit_prim,
                             float* ray_force, float* hit_point, void* stream_)
{
    if (!s) return fail(SRP_EINVAL, "scene is NULL");
    srp_status st = check_params(p);
    if (st != SRP_OK) return st;
    if (D < 0 || (pix && n_pix < 0)) return fail(SRP_EINVAL, "bad sizes");
    if (D == 0 || (pix && n_pix == 0)) return SRP_OK;
    if (!sun_dirs || !hit_prim) return fail(SRP_EINVAL, "sun_dirs and hit_prim are required");
    if (p->frame_mode == 1 && !frames) return fail(SRP_EINVAL, "frame_mode 1 needs frames");
    if (p->dir_index_base + D > (int64_t(1) << 32)) return fail(SRP_EINVAL, "direction index exceeds 32 bits");
    st = bind_device(s);
    if (st != SRP_OK) return st;
    int32_t bpd = 0;
    return enqueue_trace(s, sun_dirs, D, p, frames, true, pix, n_pix, hit_prim, ray_force, hit_point,
                         static_cast<hipStream_t>(stream_), &bpd);
}

static srp_status adjoint_into(srp_scene s, const double* sun_dirs, int64_t D, const srp_trace_params* p,
                               const double* frames, const double* g_force, const double* g_torque, float* g_rho_s,
                               float* g_rho_d, double* g_hinge, void* stream_, const int32_t* paths)
{
    if (!s) return fail(SRP_EINVAL, "scene is NULL");
    srp_status st = check_params(p);
    if (st != SRP_OK) return st;
    if (D < 0) return fail(SRP_EINVAL, "D must be >= 0");
    if (D == 0) return SRP_OK;
    if (!sun_dirs || !g_force) return fail(SRP_EINVAL, "sun_dirs and g_force are required");
    if (p->frame_mode == 1 && !frames) return fail(SRP_EINVAL, "frame_mode 1 needs frames");
    if (p->dir_index_base + D > (int64_t(1) << 32)) return fail(SRP_EINVAL, "direction index exceeds 32 bits");
    if (g_hinge && s->n_hinges > srp::kMaxHinges)
        return fail(SRP_EUNSUPPORTED, "hinge gradients support at most 4 hinges");
    if (g_hinge && p->edge_samples > 0 && D > 65535)
        return fail(SRP_EUNSUPPORTED, "visibility-edge terms support at most 65535 directions per call");
    st = bind_device(s);
    if (st != SRP_OK) return st;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    const bool edges = g_hinge && p->edge_samples > 0 && !s->h_edges.empty();
    if (edges && s->edge_class_gen != s->geom_gen) SRP_HIP(classify_edges(s, stream));
    srp::AdjointArgs A{};
    st = prepare_trace(s, sun_dirs, D, p, frames, false, nullptr, 0, nullptr, nullptr, stream, A.t);
    if (st != SRP_OK) return st;
    A.t.path_hit = const_cast<int32_t*>(paths);
    SRP_HIP(ensure(s->d_grho, s->grho_cap, static_cast<size_t>(2 * s->n_tris)));
    SRP_HIP(ensure(s->d_hdir, s->hdir_cap, static_cast<size_t>(D * srp::kMaxHinges)));
    SRP_HIP(srp::launch_fill_f64(s->d_grho, 2 * s->n_tris, 0.0, stream));
    A.g_force = g_force;
    A.g_torque = g_torque;
    A.g_rho = s->d_grho;
    A.n_tris = static_cast<int32_t>(s->n_tris);
    A.n_hinges = g_hinge ? s->n_hinges : 0;
    for (int k = 0; k < A.n_hinges; ++k)
        for (int c = 0; c < 3; ++c) {
            A.hinge_axis[k][c] = static_cast<float>(s->hinges[k].axis[c]);
            A.hinge_origin[k][c] = static_cast<float>(s->hinges[k].origin[c]);
        }
    A.hinge_partials = s->d_partials;  // sized for kMaxHinges per workgroup
    SRP_HIP(srp::launch_adjoint(A, stream));
    if (A.n_hinges > 0) {
        SRP_HIP(srp::launch_reduce_hinges(s->d_partials, D, A.t.blocks_per_dir, s->d_hdir, stream));
        if (edges && !s->h_live_edges.empty()) {
            srp::EdgeArgs E{};
            E.edges = s->d_live_edges;
            E.verts = s->d_vpos;
            E.n_edges = static_cast<int32_t>(s->h_live_edges.size());
            E.samples = p->edge_samples;
            E.D = D;
            E.bounces = p->bounces;
            E.seed_lo = A.t.seed_lo;
            E.seed_hi = A.t.seed_hi;
            E.dir_index_base = p->dir_index_base;
            E.design_index = A.t.design_index;
            E.eps = A.t.eps;
            E.delta = A.t.eps;
            for (int c = 0; c < 3; ++c) E.com[c] = A.t.com[c];
            for (int k = 0; k < A.n_hinges; ++k)
                for (int c = 0; c < 3; ++c) {
                    E.hinge_axis[k][c] = A.hinge_axis[k][c];
                    E.hinge_origin[k][c] = A.hinge_origin[k][c];
                }
            const int64_t nb = srp::edge_blocks(E);
            SRP_HIP(ensure(s->d_edge_part, s->edge_part_cap, static_cast<size_t>(D * nb * srp::kMaxHinges)));
            SRP_HIP(srp::launch_edge_term(E, s->d_nodes, s->d_tris, s->d_mat, A.t.frames, g_force, g_torque,
                                          A.t.lane_walk, s->d_edge_part, s->d_hdir, stream));
        }
    }
    SRP_HIP(srp::launch_finish_adjoint(s->d_grho, A.n_tris, g_rho_s, g_rho_d, D, A.n_hinges, s->d_hdir, g_hinge,
                                       stream));
    return SRP_OK;
}

srp_status srp_trace_adjoint(srp_scene s, const double* sun_dirs, int64_t D, const srp_trace_params* p,
                             const double* frames, const double* g_force, const double* g_torque, float* g_rho_s,
                             float* g_rho_d, double* g_hinge, void* stream_)
{
    return adjoint_into(s, sun_dirs, D, p, frames, g_force, g_torque, g_rho_s, g_rho_d, g_hinge, stream_, nullptr);
}

static bool same_params(const srp_trace_params& a, const srp_trace_params& b)
{
    return a.nu == b.nu && a.nv == b.nv && a.bounces == b.bounces && a.jitter == b.jitter && a.flux == b.flux &&
           a.seed == b.seed && a.dir_index_base == b.dir_index_base && a.design_index == b.design_index &&
           a.frame_mode == b.frame_mode && a.tiles_per_wave == b.tiles_per_wave && a.sampling == b.sampling &&
           a.ray_mask == b.ray_mask;
}

srp_status srp_path_record_bytes(srp_scene s, int64_t D, const srp_trace_params* p, int64_t* bytes)
{
    if (!s) return fail(SRP_EINVAL, "scene is NULL");
    srp_status st = check_params(p);
    if (st != SRP_OK) return st;
    if (D < 0 || !bytes) return fail(SRP_EINVAL, "D must be >= 0 and bytes non-NULL");
    *bytes = srp::path_record_bytes(p, D);
    return SRP_OK;
}

srp_status srp_trace_recorded(srp_scene s, const double* sun_dirs, int64_t D, const srp_trace_params* p,
                              const double* frames, double* force, double* torque, int32_t* paths,
                              int64_t paths_bytes, void* stream_)
{
    if (!s) return fail(SRP_EINVAL, "scene is NULL");
    srp_status st = check_params(p);
    if (st != SRP_OK) return st;
    if (D < 0) return fail(SRP_EINVAL, "D must be >= 0");
    if (!paths) return fail(SRP_EINVAL, "paths is required");
    if (p->bounces > srp::kRecordBounces)
        return fail(SRP_EUNSUPPORTED, "path records hold at most 3 interactions per path");
    const int64_t need = srp::path_record_bytes(p, D);
    if (paths_bytes < need)
        return fail(SRP_EINVAL, "the path record needs " + std::to_string(need) + " bytes, got " +
                                    std::to_string(paths_bytes));
    s->path_stamp = srp_scene_s::PathStamp{};
    st = srp::trace_into(s, sun_dirs, D, p, frames, force, torque, static_cast<hipStream_t>(stream_), nullptr, paths);
    if (st != SRP_OK) return st;
    s->path_stamp.paths = paths;
    s->path_stamp.gen = s->geom_gen;
    s->path_stamp.sun = sun_dirs;
    s->path_stamp.frames = p->frame_mode == 1 ? frames : nullptr;
    s->path_stamp.D = D;
    s->path_stamp.p = *p;
    return SRP_OK;
}

srp_status srp_trace_adjoint_recorded(srp_scene s, const double* sun_dirs, int64_t D, const srp_trace_params* p,
                                      const double* frames, const double* g_force, const double* g_torque,
                                      const int32_t* paths, int64_t paths_bytes, float* g_rho_s, float* g_rho_d,
                                      double* g_hinge, void* stream_)
{
    if (!s) return fail(SRP_EINVAL, "scene is NULL");
    srp_status st = check_params(p);
    if (st != SRP_OK) return st;
    if (!paths) return fail(SRP_EINVAL, "paths is required");
    if (p->bounces > srp::kRecordBounces)
        return fail(SRP_EUNSUPPORTED, "path records hold at most 3 interactions per path");
    if (D < 0 || paths_bytes < srp::path_record_bytes(p, D)) return fail(SRP_EINVAL, "path record too small");
    const srp_scene_s::PathStamp& k = s->path_stamp;
    if (k.paths != paths || k.gen != s->geom_gen || k.sun != sun_dirs || k.D != D || !same_params(k.p, *p) ||
        (p->frame_mode == 1 && k.frames != frames))
        return fail(SRP_EINVAL, "paths was not written by the last srp_trace_recorded on this scene with the current "
                                "design and these arguments");
    return adjoint_into(s, sun_dirs, D, p, frames, g_force, g_torque, g_rho_s, g_rho_d, g_hinge, stream_, paths);
}

srp_status srp_batch_trace(const srp_scene* scenes, int32_t S, const double* sun_dirs, int64_t D,
                           const srp_trace_params* p, double* force, double* torque, void* stream_)
{
    if (!scenes || S < 1) return fail(SRP_EINVAL, "need at least one scene");
    srp_status st = check_params(p);
    if (st == SRP_OK && p->ray_mask) return fail(SRP_EUNSUPPORTED, "ray_mask is supported by single-scene traces only");
    if (st != SRP_OK) return st;
    if (p->frame_mode != 0) return fail(SRP_EUNSUPPORTED, "batched traces derive their frames from each mesh");
    if (D < 0) return fail(SRP_EINVAL, "D must be >= 0");
    if (D == 0) return SRP_OK;
    if (!sun_dirs || !force) return fail(SRP_EINVAL, "sun_dirs and force are required");
    if (p->dir_index_base + D > (int64_t(1) << 32)) return fail(SRP_EINVAL, "direction index exceeds 32 bits");
    srp_scene_s* lead = scenes[0];
    for (int32_t s = 0; s < S; ++s) {
        if (!scenes[s]) return fail(SRP_EINVAL, "NULL scene in the batch");
        if (scenes[s]->device != lead->device) return fail(SRP_EINVAL, "all scenes must live on one device");
        if (scenes[s]->phong_finite)
            return fail(SRP_EUNSUPPORTED, "Phong lobes are served by srp_surface_estimate only (the ray grid has mirrors)");
    }
    st = bind_device(lead);
    if (st != SRP_OK) return st;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    const int64_t units = static_cast<int64_t>(S) * D;
    SRP_HIP(ensure(lead->d_frames, lead->frames_cap, static_cast<size_t>(units)));
    for (int32_t s = 0; s < S; ++s)
        SRP_HIP(srp::launch_frames(sun_dirs, D, scenes[s]->lo, scenes[s]->hi, scenes[s]->L, p->nu, p->nv, p->flux,
                                   nullptr, nullptr, lead->d_frames + static_cast<int64_t>(s) * D, stream));
    // the staging table is rewritten only after the previous upload from it has run
    if (lead->batch_ev) SRP_HIP(hipEventSynchronize(lead->batch_ev));
    if (lead->h_batch_desc_cap < static_cast<size_t>(S)) {
        if (lead->h_batch_desc) SRP_HIP(hipHostFree(lead->h_batch_desc));
        lead->h_batch_desc = nullptr;
        lead->h_batch_desc_cap = 0;
        SRP_HIP(hipHostMalloc(reinterpret_cast<void**>(&lead->h_batch_desc), sizeof(srp::SceneDesc) * S));
        lead->h_batch_desc_cap = static_cast<size_t>(S);
    }
    for (int32_t s = 0; s < S; ++s) {
        srp::SceneDesc& d = lead->h_batch_desc[s];
        d.nodes = (decltype(d.nodes))scenes[s]->d_nodes;  // device passes see global-qualified members
        d.tris = (decltype(d.tris))scenes[s]->d_tris;
        d.mat = (decltype(d.mat))scenes[s]->d_mat;
        for (int k = 0; k < 3; ++k) d.com[k] = static_cast<float>(scenes[s]->com[k]);
        d.eps = static_cast<float>(1e-5 * scenes[s]->L);
    }
    SRP_HIP(ensure(lead->d_batch_desc, lead->batch_desc_cap, static_cast<size_t>(S)));
    SRP_HIP(hipMemcpyAsync(lead->d_batch_desc, lead->h_batch_desc, sizeof(srp::SceneDesc) * S,
                           hipMemcpyHostToDevice, stream));
    if (!lead->batch_ev) SRP_HIP(hipEventCreateWithFlags(&lead->batch_ev, hipEventDisableTiming));
    SRP_HIP(hipEventRecord(lead->batch_ev, stream));
    srp::TraceArgs a{};
    a.scenes = lead->d_batch_desc;
    a.n_scenes = S;
    a.frames = lead->d_frames;
    a.D = D;
    a.nu = p->nu;
    a.nv = p->nv;
    a.bounces = p->bounces;
    a.jitter = p->jitter ? 1 : 0;
    a.seed_lo = static_cast<uint32_t>(p->seed);
    a.seed_hi = static_cast<uint32_t>(p->seed >> 32);
    a.dir_index_base = p->dir_index_base;
    a.design_index = static_cast<uint32_t>(p->design_index);
    a.tiles_x = (p->nu + srp::kTileW - 1) / srp::kTileW;
    a.tiles_y = (p->nv + srp::kTileH - 1) / srp::kTileH;
    a.tiles_per_dir = static_cast<int64_t>(a.tiles_x) * a.tiles_y;
    int32_t max_depth = 0;
    for (int32_t s = 0; s < S; ++s) max_depth = std::max(max_depth, scenes[s]->depth);
    a.lane_walk = lane_walk_for(max_depth);
    a.cull = 1;
    const int64_t tpw = tiles_per_wave_for(p, a.tiles_per_dir * units);
    a.tiles_per_wave = static_cast<int32_t>(tpw);
    const int64_t bpd = std::max<int64_t>(1, (a.tiles_per_dir + tpw * srp::kWaves - 1) / (tpw * srp::kWaves));
    a.blocks_per_dir = static_cast<int32_t>(bpd);
    a.xcd_major = units >= srp::kXcds ? 1 : 0;
    if (srp::grid_blocks(a, units) > 0x7fffffffLL) return fail(SRP_EINVAL, "batched trace too large for one launch");
    SRP_HIP(ensure(lead->d_partials, lead->partials_cap, static_cast<size_t>(bpd * units * 6)));
    a.partials = lead->d_partials;
    SRP_HIP(srp::launch_trace_batch(a, stream));
    SRP_HIP(srp::launch_reduce(lead->d_partials, units, a.blocks_per_dir, force, torque, stream));
    return SRP_OK;
}

srp_status srp_scene_build_gpu(srp_scene s, int32_t* n_nodes_out, int32_t* depth_out, void* stream_)
{
    if (!s) return fail(SRP_EINVAL, "scene is NULL");
    if (s->n_tris < 8) return fail(SRP_EUNSUPPORTED, "GPU build needs at least 8 triangles");
    if (s->n_tris > 0x3fffffff) return fail(SRP_EUNSUPPORTED, "too many triangles for the GPU build");
    srp_status st = bind_device(s);
    if (st != SRP_OK) return st;
    ++s->geom_gen;  // path records of earlier calls no longer describe the scene
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    SRP_HIP(hipStreamSynchronize(stream));  // kernels in flight may still read the current tree
    const int32_t n = static_cast<int32_t>(s->n_tris);
    srp::LbvhArgs a{};
    a.n = n;
    // cubic Morton cells (one scale for all axes): per-axis scaling stretches the cells of long,
    // flat parts such as solar arrays and roughly doubles the tree's surface-area cost
    const double ext = std::max({s->hi[0] - s->lo[0], s->hi[1] - s->lo[1], s->hi[2] - s->lo[2], 1e-30});
    const float sc = static_cast<float>(1024.0 / ext);
    a.lo = make_float3(static_cast<float>(s->lo[0]), static_cast<float>(s->lo[1]), static_cast<float>(s->lo[2]));
    a.scale = make_float3(sc, sc, sc);
    a.pad = static_cast<float>(1e-6 * s->L);
    a.tris_in = s->d_tris;
    a.mat_in = s->d_mat;
    a.perm_in = s->d_perm;
    int32_t levels = 1;
    while ((int64_t(1) << levels) <= n) ++levels;
    a.levels = levels;
    // workspace: one block kept by the scene, carved in 256-byte-aligned pieces
    a.tmp_bytes = srp::lbvh_tmp_bytes(n);
    const size_t nn = static_cast<size_t>(n);
    const size_t sizes[] = {4 * nn, 4 * nn, 4 * nn, 4 * nn, a.tmp_bytes, 64 * nn, 16 * nn, 4 * nn, 4 * nn,
                            8 * nn, 8 * nn, 4 * nn, 4 * nn, 4 * nn, 4 * (nn + 1), 24 * nn * levels, 64 * nn, 16 * nn, 4};
    size_t total = 0;
    for (size_t z : sizes) total += (z + 255) / 256 * 256;
    SRP_HIP(ensure(s->d_lbvh_ws, s->lbvh_ws_cap, total));
    char* ws = s->d_lbvh_ws;
    size_t off = 0, piece = 0;
    auto take = [&]() {
        char* p = ws + off;
        off += (sizes[piece++] + 255) / 256 * 256;
        return p;
    };
    a.keys = reinterpret_cast<uint32_t*>(take());
    a.keys_sorted = reinterpret_cast<uint32_t*>(take());
    a.pos = reinterpret_cast<int32_t*>(take());
    a.order = reinterpret_cast<int32_t*>(take());
    a.tmp = take();
    a.tris_out = reinterpret_cast<srp::TriRec*>(take());
    a.mat_out = reinterpret_cast<float4*>(take());
    a.perm_out = reinterpret_cast<int32_t*>(take());
    a.bvh_pos_out = reinterpret_cast<int32_t*>(take());
    a.child = reinterpret_cast<int2*>(take());
    a.range = reinterpret_cast<int2*>(take());
    a.parent = reinterpret_cast<int32_t*>(take());
    a.leaf_parent = reinterpret_cast<int32_t*>(take());
    a.start = reinterpret_cast<int32_t*>(take());
    a.scan = reinterpret_cast<int32_t*>(take());
    a.win = reinterpret_cast<float*>(take());
    a.nodes_out = reinterpret_cast<srp::BvhNode*>(take());
    a.ranges_out = reinterpret_cast<int4*>(take());
    a.depth_out = reinterpret_cast<int32_t*>(take());
    hipError_t e = srp::launch_lbvh(a, stream);
    int32_t records = 0, depth = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&records, a.scan + n, 4, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&depth, a.depth_out, 4, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    const int32_t count = records - 1;  // a full binary tree over its leaf records
    if (e != hipSuccess) return fail(SRP_EDEVICE, std::string("GPU BVH build: ") + hipGetErrorString(e));
    if (count < 1 || count > n - 1) return fail(SRP_EDEVICE, "GPU BVH build: inconsistent node count");
    if (depth >= srp::kMaxTreeDepth) return fail(SRP_EUNSUPPORTED, "GPU-built tree deeper than the traversal stack");
    // adopt the new tree and record order; the host copies are read back only when host code needs
    // them (refit, statistics)
    e = ensure(s->d_nodes, s->nodes_cap, static_cast<size_t>(count));
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->d_nodes, a.nodes_out, sizeof(srp::BvhNode) * count, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->d_tris, a.tris_out, sizeof(srp::TriRec) * nn, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(s->d_mat, a.mat_out, 16 * nn, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(s->d_perm, a.perm_out, 4 * nn, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) e = hipMemcpyAsync(s->d_bvh_pos, a.bvh_pos_out, 4 * nn, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) e = ensure(s->d_ranges, s->ranges_cap, static_cast<size_t>(count));
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->d_ranges, a.ranges_out, sizeof(int4) * count, hipMemcpyDeviceToDevice, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return fail(SRP_EDEVICE, std::string("GPU BVH build: ") + hipGetErrorString(e));
    s->h_tree_stale = true;
    s->h_tris_stale = true;
    s->h_perm_stale = true;
    s->ranges_nodes = count;
    s->n_nodes = count;
    s->depth = depth;
    if (n_nodes_out) *n_nodes_out = count;
    if (depth_out) *depth_out = depth;
    return SRP_OK;
}

srp_status srp_surface_estimate(const srp_scene* scenes, int32_t S, const double* sun_dirs, int64_t D,
                                int64_t n_samples, const srp_trace_params* p, int32_t brute_force, double* force,
                                double* torque, int32_t* rec_facet, int32_t* rec_hits, int32_t* rec_lit,
                                void* stream_)
{
    if (!scenes || S < 1) return fail(SRP_EINVAL, "need at least one scene");
    srp_status st = check_params(p);
    if (st == SRP_OK && p->ray_mask) return fail(SRP_EUNSUPPORTED, "ray_mask is supported by single-scene traces only");
    if (st != SRP_OK) return st;
    if (D < 0 || n_samples < 1) return fail(SRP_EINVAL, "D must be >= 0 and n_samples >= 1");
    if (D == 0) return SRP_OK;
    if (!sun_dirs || !force) return fail(SRP_EINVAL, "sun_dirs and force are required");
    if ((rec_hits || rec_lit) && !rec_facet) return fail(SRP_EINVAL, "records need rec_facet");
    if (rec_facet && !rec_lit) return fail(SRP_EINVAL, "rec_facet needs rec_lit");
    if (p->dir_index_base + D > (int64_t(1) << 32)) return fail(SRP_EINVAL, "direction index exceeds 32 bits");
    if (n_samples > (int64_t(1) << 32)) return fail(SRP_EINVAL, "sample index exceeds 32 bits");
    srp_scene_s* lead = scenes[0];
    for (int32_t s = 0; s < S; ++s) {
        if (!scenes[s]) return fail(SRP_EINVAL, "NULL scene");
        if (scenes[s]->device != lead->device) return fail(SRP_EINVAL, "all scenes must live on one device");
        if (!brute_force && scenes[s]->depth > srp::kLaneStack)
            return fail(SRP_EUNSUPPORTED, "BVH deeper than the per-lane stack: use brute force");
    }
    st = bind_device(lead);
    if (st != SRP_OK) return st;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    if (lead->surf_ev) SRP_HIP(hipEventSynchronize(lead->surf_ev));
    if (lead->h_surf_desc_cap < static_cast<size_t>(S)) {
        if (lead->h_surf_desc) SRP_HIP(hipHostFree(lead->h_surf_desc));
        lead->h_surf_desc = nullptr;
        lead->h_surf_desc_cap = 0;
        SRP_HIP(hipHostMalloc(reinterpret_cast<void**>(&lead->h_surf_desc), sizeof(srp::SurfaceScene) * S));
        lead->h_surf_desc_cap = static_cast<size_t>(S);
    }
    for (int32_t s = 0; s < S; ++s) {
        srp::SurfaceScene& d = lead->h_surf_desc[s];
        d.nodes = (decltype(d.nodes))scenes[s]->d_nodes;  // device passes see global-qualified members
        d.tris = (decltype(d.tris))scenes[s]->d_tris;
        d.mat = (decltype(d.mat))scenes[s]->d_mat;
        d.cum_area = (decltype(d.cum_area))scenes[s]->d_cum_area;
        d.bvh_pos = (decltype(d.bvh_pos))scenes[s]->d_bvh_pos;
        d.area = scenes[s]->area;
        for (int k = 0; k < 3; ++k) d.com[k] = static_cast<float>(scenes[s]->com[k]);
        d.eps = static_cast<float>(1e-5 * scenes[s]->L);
        d.n_tris = static_cast<int32_t>(scenes[s]->n_tris);
        d.pad = 0;
    }
    SRP_HIP(ensure(lead->d_surf_desc, lead->surf_desc_cap, static_cast<size_t>(S)));
    SRP_HIP(hipMemcpyAsync(lead->d_surf_desc, lead->h_surf_desc, sizeof(srp::SurfaceScene) * S,
                           hipMemcpyHostToDevice, stream));
    if (!lead->surf_ev) SRP_HIP(hipEventCreateWithFlags(&lead->surf_ev, hipEventDisableTiming));
    SRP_HIP(hipEventRecord(lead->surf_ev, stream));
    srp::SurfaceArgs a{};
    a.scenes = lead->d_surf_desc;
    a.n_scenes = S;
    a.bounces = p->bounces;
    a.sun = sun_dirs;
    a.D = D;
    a.n_samples = n_samples;
    const int64_t chunks = (n_samples + 255) / 256;
    const int64_t units = static_cast<int64_t>(S) * D;
    if (chunks > 0x7fffffffLL || units * chunks > 0x7fffffffLL) return fail(SRP_EINVAL, "estimate too large");
    a.chunks = static_cast<int32_t>(chunks);
    a.flux_c = static_cast<float>(p->flux / srp::kSpeedOfLight);
    a.seed_lo = static_cast<uint32_t>(p->seed);
    a.seed_hi = static_cast<uint32_t>(p->seed >> 32);
    a.dir_index_base = p->dir_index_base;
    a.design_index = static_cast<uint32_t>(p->design_index);
    a.sampling = p->sampling;
    SRP_HIP(ensure(lead->d_partials, lead->partials_cap, static_cast<size_t>(units * chunks * 6)));
    a.partials = lead->d_partials;
    a.rec_facet = rec_facet;
    a.rec_hits = p->bounces > 1 ? rec_hits : nullptr;
    a.rec_lit = rec_lit;
    SRP_HIP(srp::launch_surface(a, brute_force != 0, force, torque, stream));
    return SRP_OK;
}

namespace {

// Rest-pose facet records grouped by rigid part (the body, then each hinge) for the multi-world
// estimator; a facet spanning a hinge and the body (it would stretch, not turn) is refused.
srp_status build_multiworld(srp_scene_s* s, const int32_t* group)
{
    if (!s->mw_groups.empty() && std::equal(s->mw_groups.begin(), s->mw_groups.end(), group)) return SRP_OK;
    const int64_t T = s->n_tris;
    std::vector<int32_t> part(static_cast<size_t>(T));
    for (int64_t f = 0; f < T; ++f) {
        const int32_t h0 = s->vhinge[s->tris[3 * f]], h1 = s->vhinge[s->tris[3 * f + 1]], h2 = s->vhinge[s->tris[3 * f + 2]];
        if (h0 != h1 || h1 != h2)
            return fail(SRP_EUNSUPPORTED, "a facet spans a hinge and the body: its design would stretch it");
        part[f] = h0 + 1;
    }
    const int32_t n_parts = s->n_hinges + 1;
    std::vector<int32_t> order(static_cast<size_t>(T));
    for (int64_t f = 0; f < T; ++f) order[f] = static_cast<int32_t>(f);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return part[a] < part[b]; });
    std::vector<srp::TriRec> recs(static_cast<size_t>(T));
    std::vector<int32_t> pos(static_cast<size_t>(T));
    const auto& V = s->rest;
    for (int64_t q = 0; q < T; ++q) {
        const int32_t f = order[q];
        pos[f] = static_cast<int32_t>(q);
        const double* a = &V[3 * static_cast<int64_t>(s->tris[3 * f])];
        const double* b = &V[3 * static_cast<int64_t>(s->tris[3 * f + 1])];
        const double* c = &V[3 * static_cast<int64_t>(s->tris[3 * f + 2])];
        double e1[3], e2[3];
        for (int k = 0; k < 3; ++k) {
            e1[k] = b[k] - a[k];
            e2[k] = c[k] - a[k];
        }
        double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        const double len = std::sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        for (int k = 0; k < 3; ++k) n[k] /= len;
        int32_t fid = f, hid = part[f] - 1, gid = group[f];
        float fb, hb, gb;
        std::memcpy(&fb, &fid, 4);
        std::memcpy(&hb, &hid, 4);
        std::memcpy(&gb, &gid, 4);
        srp::TriRec& r = recs[q];
        r.f[0] = make_float4(static_cast<float>(a[0]), static_cast<float>(a[1]), static_cast<float>(a[2]), fb);
        r.f[1] = make_float4(static_cast<float>(e1[0]), static_cast<float>(e1[1]), static_cast<float>(e1[2]),
                             static_cast<float>(n[0]));
        r.f[2] = make_float4(static_cast<float>(e2[0]), static_cast<float>(e2[1]), static_cast<float>(e2[2]),
                             static_cast<float>(n[1]));
        r.f[3] = make_float4(static_cast<float>(n[2]), hb, gb, 0.0f);
    }
    if (!s->d_mw_tris) {
        SRP_HIP(hipMalloc(reinterpret_cast<void**>(&s->d_mw_tris), sizeof(srp::TriRec) * T));
        SRP_HIP(hipMalloc(reinterpret_cast<void**>(&s->d_mw_pos), sizeof(int32_t) * T));
    }
    SRP_HIP(hipMemcpy(s->d_mw_tris, recs.data(), sizeof(srp::TriRec) * T, hipMemcpyHostToDevice));
    SRP_HIP(hipMemcpy(s->d_mw_pos, pos.data(), sizeof(int32_t) * T, hipMemcpyHostToDevice));
    s->mw_n_parts = n_parts;
    for (int32_t q = 0; q < n_parts; ++q) {
        int32_t end = 0;
        for (int64_t f = 0; f < T; ++f) end += part[f] <= q ? 1 : 0;
        s->mw_part_end[q] = end;
        s->mw_part_hinge[q] = q - 1;
    }
    s->mw_groups.assign(group, group + T);
    return SRP_OK;
}

}  // namespace

srp_status srp_surface_designs(srp_scene s, const int32_t* facet_group, int32_t n_groups, const double* sun_dirs,
                               const float* designs, int64_t n_pairs, int32_t samples, const srp_trace_params* p,
                               double* force, double* torque, int32_t* rec_facet, int32_t* rec_hits, int32_t* rec_lit,
                               void* stream_)
{
    if (!s || !facet_group) return fail(SRP_EINVAL, "scene and facet_group are required");
    srp_status st = check_params(p);
    if (st == SRP_OK && p->ray_mask) return fail(SRP_EUNSUPPORTED, "ray_mask is supported by single-scene traces only");
    if (st != SRP_OK) return st;
    if (n_groups < 1 || n_groups > 64) return fail(SRP_EINVAL, "n_groups must be in 1..64");
    if (s->n_hinges > srp::kMaxHinges) return fail(SRP_EUNSUPPORTED, "at most 4 hinges");
    if (n_pairs < 0 || samples < 1) return fail(SRP_EINVAL, "n_pairs must be >= 0 and samples >= 1");
    if (n_pairs == 0) return SRP_OK;
    if (!sun_dirs || !designs || !force) return fail(SRP_EINVAL, "sun_dirs, designs and force are required");
    if ((rec_hits || rec_lit) && !rec_facet) return fail(SRP_EINVAL, "records need rec_facet");
    if (rec_facet && !rec_lit) return fail(SRP_EINVAL, "rec_facet needs rec_lit");
    if (p->dir_index_base + n_pairs > (int64_t(1) << 32)) return fail(SRP_EINVAL, "direction index exceeds 32 bits");
    if (n_pairs * samples > (int64_t(1) << 40)) return fail(SRP_EINVAL, "too many samples in one call");
    for (int64_t f = 0; f < s->n_tris; ++f)
        if (facet_group[f] < 0 || facet_group[f] >= n_groups) return fail(SRP_EINVAL, "facet group out of range");
    st = bind_device(s);
    if (st != SRP_OK) return st;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    SRP_HIP(hipStreamSynchronize(stream));  // the records and the sample buffer may be in use
    st = build_multiworld(s, facet_group);
    if (st != SRP_OK) return st;
    // materials of every pair in range
    int32_t flag = 0;
    SRP_HIP(hipMemsetAsync(s->d_flag, 0, sizeof(int32_t), stream));
    SRP_HIP(srp::launch_check_designs(designs, n_pairs, s->n_hinges, n_groups, s->d_flag, stream));
    SRP_HIP(hipMemcpyAsync(&flag, s->d_flag, sizeof(int32_t), hipMemcpyDeviceToHost, stream));
    SRP_HIP(hipStreamSynchronize(stream));
    if (flag) return fail(SRP_EINVAL, "a design's materials are out of range (rho >= 0, rho_s + rho_d <= 1, exponent >= 1)"
                                      " or a hinge angle is not finite");
    SRP_HIP(ensure(s->d_mw_samples, s->mw_samples_cap, static_cast<size_t>(n_pairs * samples * 6)));
    srp::MwArgs a{};
    a.base.bounces = p->bounces;
    a.base.flux_c = static_cast<float>(p->flux / srp::kSpeedOfLight);
    a.base.seed_lo = static_cast<uint32_t>(p->seed);
    a.base.seed_hi = static_cast<uint32_t>(p->seed >> 32);
    a.base.dir_index_base = p->dir_index_base;
    a.base.design_index = static_cast<uint32_t>(p->design_index);
    a.base.sampling = p->sampling;
    a.sc.tris = (decltype(a.sc.tris))s->d_mw_tris;
    a.sc.pos = (decltype(a.sc.pos))s->d_mw_pos;
    a.sc.cum_area = (decltype(a.sc.cum_area))s->d_cum_area;
    a.sc.area = s->area;
    for (int k = 0; k < 3; ++k) a.sc.com[k] = static_cast<float>(s->com[k]);
    a.sc.eps = static_cast<float>(1e-5 * s->L);
    a.sc.n_tris = static_cast<int32_t>(s->n_tris);
    a.sc.n_parts = s->mw_n_parts;
    for (int32_t q = 0; q <= srp::kMaxHinges; ++q) {
        a.sc.part_end[q] = q < s->mw_n_parts ? s->mw_part_end[q] : 0;
        a.sc.part_hinge[q] = q < s->mw_n_parts ? s->mw_part_hinge[q] : -1;
    }
    for (int32_t h = 0; h < srp::kMaxHinges; ++h)
        for (int k = 0; k < 3; ++k) {
            a.sc.hinge_origin[h][k] = h < s->n_hinges ? static_cast<float>(s->hinges[h].origin[k]) : 0.0f;
            a.sc.hinge_axis[h][k] = h < s->n_hinges ? static_cast<float>(s->hinges[h].axis[k]) : 0.0f;
        }
    a.sun = sun_dirs;
    a.designs = designs;
    a.n_pairs = n_pairs;
    a.samples = samples;
    a.n_hinges = s->n_hinges;
    a.n_groups = n_groups;
    a.stride = s->n_hinges + 3 * n_groups;
    a.sample_out = s->d_mw_samples;
    a.rec_facet = rec_facet;
    a.rec_hits = p->bounces > 1 ? rec_hits : nullptr;
    a.rec_lit = rec_lit;
    SRP_HIP(srp::launch_surface_designs(a, force, torque, stream));
    return SRP_OK;
}

srp_status srp_autotune_tiles_per_wave(const srp_scene* scenes, int32_t S, const double* sun_dirs, int64_t D,
                                       const srp_trace_params* p, int32_t* best, double* ms_out, void* stream_)
{
    if (!scenes || S < 1 || !best) return fail(SRP_EINVAL, "need scenes and an output");
    srp_status st = check_params(p);
    if (st == SRP_OK && p->ray_mask) return fail(SRP_EUNSUPPORTED, "ray_mask is supported by single-scene traces only");
    if (st != SRP_OK) return st;
    if (D < 1 || !sun_dirs) return fail(SRP_EINVAL, "need at least one sun direction");
    for (int32_t s = 0; s < S; ++s)
        if (!scenes[s]) return fail(SRP_EINVAL, "NULL scene");
    st = bind_device(scenes[0]);
    if (st != SRP_OK) return st;
    hipStream_t stream = static_cast<hipStream_t>(stream_);
    double* F = nullptr;
    const size_t bytes = sizeof(double) * 3 * static_cast<size_t>(S) * static_cast<size_t>(D);
    SRP_HIP(hipMalloc(reinterpret_cast<void**>(&F), bytes));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    double best_ms = 0.0;
    int32_t best_tpw = 0;
    st = SRP_OK;
    for (int32_t c = kTuneFirst; c <= kTuneLast && he == hipSuccess && st == SRP_OK; ++c) {
        srp_trace_params q = *p;
        q.tiles_per_wave = c;
        float ms = 0.0f;
        for (int rep = 0; rep < 2 && st == SRP_OK; ++rep) {  // the first run warms caches and clocks
            if (rep == 1 && (he = hipEventRecord(e0, stream)) != hipSuccess) break;
            st = S == 1 ? srp_trace(scenes[0], sun_dirs, D, &q, nullptr, F, nullptr, stream_)
                        : srp_batch_trace(scenes, S, sun_dirs, D, &q, F, nullptr, stream_);
        }
        if (st != SRP_OK) break;
        if (he == hipSuccess) he = hipEventRecord(e1, stream);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (he != hipSuccess) break;
        if (ms_out) ms_out[c - kTuneFirst] = ms;
        if (best_tpw == 0 || ms < best_ms) {
            best_ms = ms;
            best_tpw = c;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(F);  // waits for the device
    if (st != SRP_OK) return st;
    if (he != hipSuccess) return fail(SRP_EDEVICE, std::string("autotune timing: ") + hipGetErrorString(he));
    *best = best_tpw;
    return SRP_OK;
}

srp_status srp_scene_destroy(srp_scene s)
{
    if (!s) return SRP_OK;
    int prev = -1;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(s->device);
    (void)hipFree(s->d_nodes);
    (void)hipFree(s->d_tris);
    (void)hipFree(s->d_mat);
    (void)hipFree(s->d_perm);
    (void)hipFree(s->d_flag);
    (void)hipFree(s->d_frames);
    (void)hipFree(s->d_partials);
    (void)hipFree(s->d_grho);
    (void)hipFree(s->d_hdir);
    (void)hipFree(s->d_batch_desc);
    (void)hipFree(s->d_cum_area);
    (void)hipFree(s->d_bvh_pos);
    (void)hipFree(s->d_surf_desc);
    (void)hipFree(s->d_lbvh_ws);
    (void)hipFree(s->d_edges);
    (void)hipFree(s->d_edge_pairs);
    (void)hipFree(s->d_live_edges);
    (void)hipFree(s->d_edge_keep);
    (void)hipFree(s->d_phong);
    (void)hipFree(s->d_mw_tris);
    (void)hipFree(s->d_mw_pos);
    (void)hipFree(s->d_mw_samples);
    (void)hipFree(s->d_vpos);
    (void)hipFree(s->d_edge_part);
    if (s->surf_ev) {
        (void)hipEventSynchronize(s->surf_ev);
        (void)hipEventDestroy(s->surf_ev);
    }
    (void)hipHostFree(s->h_surf_desc);
    if (s->batch_ev) {
        (void)hipEventSynchronize(s->batch_ev);
        (void)hipEventDestroy(s->batch_ev);
    }
    (void)hipHostFree(s->h_batch_desc);
    if (prev >= 0) (void)hipSetDevice(prev);
    delete s;
    return SRP_OK;
}

}  // extern "C"
