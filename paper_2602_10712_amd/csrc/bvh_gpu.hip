// BVH build on the GPU: linear BVH after Karras, "Maximizing Parallelism in the Construction of
// BVHs, Octrees, and k-d Trees" (HPG 2012), with subtrees of at most kLbvhLeaf triangles collapsed
// into leaves and the kept inner nodes written in pre-order (the layout of the host-built tree:
// node 0 the root, every child after its parent).
//
//   1. 30-bit Morton code of every triangle centroid (10 bits per axis, cubic cells over the scene
//      box);
//   2. radix sort of (code, position) pairs (rocPRIM);
//   3. triangle, material and permutation records gathered into the sorted order, with the box
//      of every triangle;
//   4. the binary radix tree over the sorted codes (one thread per inner node; equal codes are
//      ordered by position), parents and leaf ranges;
//   5. the leaf records of the final tree: every maximal subtree of at most kLbvhLeaf triangles,
//      and every single triangle outside them; a scan over the leaves that open one counts the
//      kept inner nodes of any subtree (a full binary tree over its leaf records);
//   6. a window table (box of leaves [i, i + 2^k) for every k; the first eight levels in one pass
//      through LDS), from which the box of any node, a contiguous leaf range, is the union of two
//      windows;
//   7. pre-order positions (each kept node walks to the root) and the node records.
// The same window table refits a kept tree after the vertices move (launch_refit): every child
// slot's subtree covers a contiguous range of records, so its box is the union of two windows.
// Every node covers a contiguous range of sorted leaves, so no step waits on another thread: there
// is no bottom-up pass with device-scope counters and fences, whose cost grows with the tree height.
#include <float.h>

#include <algorithm>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "srp_internal.h"

namespace srp {
namespace {

__device__ __forceinline__ uint32_t spread10(uint32_t x)
{
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

__global__ void k_morton(const TriRec* __restrict__ tris, int32_t n, float3 lo, float3 scale, uint32_t* __restrict__ keys,
                         int32_t* __restrict__ pos)
{
    const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    const TriRec t = tris[i];
    const float third = 1.0f / 3.0f;
    const float cx = t.f[0].x + (t.f[1].x + t.f[2].x) * third;
    const float cy = t.f[0].y + (t.f[1].y + t.f[2].y) * third;
    const float cz = t.f[0].z + (t.f[1].z + t.f[2].z) * third;
    auto q = [](float c, float l, float s) {
        const float u = fminf(fmaxf((c - l) * s, 0.0f), 1023.0f);
        return static_cast<uint32_t>(u);
    };
    keys[i] = (spread10(q(cx, lo.x, scale.x)) << 2) | (spread10(q(cy, lo.y, scale.y)) << 1) |
              spread10(q(cz, lo.z, scale.z));
    pos[i] = i;
}

struct Box6 {
    float lo[3], hi[3];
};

__device__ __forceinline__ Box6 tri_box(const TriRec& t)
{
    Box6 b;
    const float v0[3] = {t.f[0].x, t.f[0].y, t.f[0].z};
    const float e1[3] = {t.f[1].x, t.f[1].y, t.f[1].z};
    const float e2[3] = {t.f[2].x, t.f[2].y, t.f[2].z};
    for (int a = 0; a < 3; ++a) {
        const float p1 = v0[a] + e1[a], p2 = v0[a] + e2[a];
        b.lo[a] = fminf(v0[a], fminf(p1, p2));
        b.hi[a] = fmaxf(v0[a], fmaxf(p1, p2));
    }
    return b;
}

// window-table entries: (lo.x, hi.x), (lo.y, hi.y), (lo.z, hi.z)
__device__ __forceinline__ Box6 load_box(const float* __restrict__ w, int64_t i)
{
    const float2* q = reinterpret_cast<const float2*>(w + 6 * i);
    Box6 r;
    for (int a = 0; a < 3; ++a) {
        const float2 v = q[a];
        r.lo[a] = v.x;
        r.hi[a] = v.y;
    }
    return r;
}

__device__ __forceinline__ void store_box(float* __restrict__ w, int64_t i, const Box6& b)
{
    float2* q = reinterpret_cast<float2*>(w + 6 * i);
    for (int a = 0; a < 3; ++a) q[a] = make_float2(b.lo[a], b.hi[a]);
}

__device__ __forceinline__ Box6 join(const Box6& a, const Box6& b)
{
    Box6 r;
    for (int k = 0; k < 3; ++k) {
        r.lo[k] = fminf(a.lo[k], b.lo[k]);
        r.hi[k] = fmaxf(a.hi[k], b.hi[k]);
    }
    return r;
}

// records at their sorted positions; perm maps positions to original facets, bvh_pos the inverse;
// level 0 of the window table holds the triangle boxes
__global__ void k_gather(const TriRec* __restrict__ tris_in, const float4* __restrict__ mat_in,
                         const int32_t* __restrict__ perm_in, const int32_t* __restrict__ order, int32_t n,
                         TriRec* __restrict__ tris_out, float4* __restrict__ mat_out, int32_t* __restrict__ perm_out,
                         int32_t* __restrict__ bvh_pos_out, float* __restrict__ win)
{
    const int32_t k = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    if (k >= n) return;
    const int32_t q = order[k];
    const TriRec t = tris_in[q];
    const int32_t f = perm_in[q];
    tris_out[k] = t;
    mat_out[k] = mat_in[q];
    perm_out[k] = f;
    bvh_pos_out[f] = k;
    store_box(win, k, tri_box(t));
}

// level k of the window table from level k - 1: box of leaves [i, i + 2 half)
__global__ void k_window(const float* __restrict__ prev, float* __restrict__ cur, int32_t count, int32_t half)
{
    const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= count) return;
    store_box(cur, i, join(load_box(prev, i), load_box(prev, static_cast<int64_t>(i) + half)));
}

// Levels 1 .. n_levels (at most kWinFused) of the window table in one pass: a workgroup stages the
// level-0 boxes of its 256 entries and of the 255 leaves after them in LDS and builds each level
// there (min and max are exact, so the result equals level-by-level construction).
constexpr int kWinFused = 8;
constexpr int kWinSpan = 512;  // 256 entries + 2^kWinFused - 1 following leaves, rounded up

__global__ __launch_bounds__(256) void k_window_fused(float* __restrict__ win, int32_t n, int32_t n_levels)
{
    __shared__ float2 sb[2][kWinSpan][3];
    const int64_t i0 = static_cast<int64_t>(blockIdx.x) * 256;
    for (int j = threadIdx.x; j < kWinSpan; j += 256) {
        const int64_t g = i0 + j;
        const Box6 b = g < n ? load_box(win, g) : Box6{{FLT_MAX, FLT_MAX, FLT_MAX}, {-FLT_MAX, -FLT_MAX, -FLT_MAX}};
        for (int a = 0; a < 3; ++a) sb[0][j][a] = make_float2(b.lo[a], b.hi[a]);
    }
    __syncthreads();
    int cur = 0;
    for (int k = 1; k <= n_levels; ++k) {
        const int half = 1 << (k - 1);
        for (int j = threadIdx.x; j < kWinSpan - (1 << k) + 1; j += 256)
            for (int a = 0; a < 3; ++a) {
                const float2 u = sb[cur][j][a], v = sb[cur][j + half][a];
                sb[cur ^ 1][j][a] = make_float2(fminf(u.x, v.x), fmaxf(u.y, v.y));
            }
        __syncthreads();
        cur ^= 1;
        const int64_t g = i0 + threadIdx.x;
        if (g < static_cast<int64_t>(n) - (1 << k) + 1) {
            Box6 b;
            for (int a = 0; a < 3; ++a) {
                b.lo[a] = sb[cur][threadIdx.x][a].x;
                b.hi[a] = sb[cur][threadIdx.x][a].y;
            }
            store_box(win + static_cast<int64_t>(k) * n * 6, g, b);
        }
    }
}

// box of sorted leaves [a, b]: the union of the two windows of the largest power of two not above
// its length that start at a and end at b
__device__ __forceinline__ Box6 range_box(const float* __restrict__ win, int32_t n, int32_t a, int32_t b)
{
    const uint32_t len = static_cast<uint32_t>(b - a + 1);
    const int k = 31 - __clz(len);
    const float* level = win + static_cast<int64_t>(k) * n * 6;
    return join(load_box(level, a), load_box(level, b - (1 << k) + 1));
}

// common-prefix length of sorted keys i and j (ties broken by position); -1 outside [0, n)
__device__ __forceinline__ int prefix(const uint32_t* __restrict__ keys, int32_t n, int32_t i, int32_t j)
{
    if (j < 0 || j >= n) return -1;
    const uint32_t a = keys[i], b = keys[j];
    if (a != b) return __clz(a ^ b);
    return 32 + __clz(static_cast<uint32_t>(i ^ j));
}

// Inner node i of the radix tree over n sorted keys (n >= 2): its range [first, last], its two
// children (inner index, or ~leaf) and their parents.
__global__ void k_karras(const uint32_t* __restrict__ keys, int32_t n, int2* __restrict__ child,
                         int2* __restrict__ range, int32_t* __restrict__ parent, int32_t* __restrict__ leaf_parent)
{
    const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n - 1) return;
    const int d = prefix(keys, n, i, i + 1) - prefix(keys, n, i, i - 1) >= 0 ? 1 : -1;
    const int dmin = prefix(keys, n, i, i - d);
    int32_t lmax = 2;
    while (prefix(keys, n, i, i + lmax * d) > dmin) lmax *= 2;
    int32_t l = 0;
    for (int32_t t = lmax / 2; t >= 1; t /= 2)
        if (prefix(keys, n, i, i + (l + t) * d) > dmin) l += t;
    const int32_t j = i + l * d;
    const int dnode = prefix(keys, n, i, j);
    int32_t s = 0;
    for (int32_t div = 2;; div *= 2) {
        const int32_t t = (l + div - 1) / div;
        if (prefix(keys, n, i, i + (s + t) * d) > dnode) s += t;
        if (t <= 1) break;
    }
    const int32_t split = i + s * d + (d < 0 ? -1 : 0);
    const int32_t first = min(i, j), last = max(i, j);
    const int32_t left = first == split ? ~split : split;
    const int32_t right = last == split + 1 ? ~(split + 1) : split + 1;
    child[i] = make_int2(left, right);
    range[i] = make_int2(first, last);
    if (left >= 0) parent[left] = i; else leaf_parent[~left] = i;
    if (right >= 0) parent[right] = i; else leaf_parent[~right] = i;
    if (i == 0) parent[0] = -1;
}

// Marks the leaves that open a leaf record of the final tree: the record of leaf p is the largest
// subtree of at most kLbvhLeaf triangles that holds it (p alone when its parent holds more).
__global__ void k_frontier(const int2* __restrict__ range, const int32_t* __restrict__ parent,
                           const int32_t* __restrict__ leaf_parent, int32_t n, int32_t* __restrict__ start)
{
    const int32_t p = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    if (p >= n) return;
    int32_t first = p;
    int32_t y = leaf_parent[p];
    while (y >= 0) {  // the root holds n >= 8 triangles, so the walk stops below it
        const int2 r = range[y];
        if (r.y - r.x + 1 > kLbvhLeaf) break;
        first = r.x;
        y = parent[y];
    }
    start[p] = first == p ? 1 : 0;
}

// kept inner nodes in the subtree of inner node x: its leaf records minus one; 0 when x is collapsed
__device__ __forceinline__ int32_t kept_nodes(const int2* __restrict__ range, const int32_t* __restrict__ scan,
                                              int32_t x)
{
    const int2 r = range[x];
    if (r.y - r.x + 1 <= kLbvhLeaf) return 0;
    return scan[r.y + 1] - scan[r.x] - 1;
}

// Pre-order node records of the kept inner nodes (those holding more than kLbvhLeaf triangles;
// their ancestors hold more still).
__global__ void k_emit(int32_t n, const int2* __restrict__ child, const int2* __restrict__ range,
                       const int32_t* __restrict__ parent, const int32_t* __restrict__ scan,
                       const float* __restrict__ win, float pad, BvhNode* __restrict__ out,
                       int4* __restrict__ ranges_out, int32_t* __restrict__ depth_out)
{
    const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n - 1) return;
    const int2 ri = range[i];
    if (ri.y - ri.x + 1 <= kLbvhLeaf) return;
    // position: the root is 0; a left child follows its parent, a right child follows the parent's
    // left subtree
    int32_t pre = 0, depth = 0, node = i;
    while (node != 0) {
        const int32_t p = parent[node];
        const int2 c = child[p];
        pre += 1;
        if (c.y == node && c.x >= 0) pre += kept_nodes(range, scan, c.x);
        node = p;
        ++depth;
    }
    const int2 c = child[i];
    BvhNode rec;
    int32_t codes[2];
    int2 cover[2];
    const int32_t kids[2] = {c.x, c.y};
    int32_t next = pre + 1;
    for (int slot = 0; slot < 2; ++slot) {
        const int32_t ch = kids[slot];
        Box6 b;
        if (ch < 0) {
            b = load_box(win, ~ch);
            codes[slot] = ~((~ch << 3) | 1);
            cover[slot] = make_int2(~ch, ~ch);
        } else {
            const int2 r = range[ch];
            cover[slot] = r;
            b = range_box(win, n, r.x, r.y);
            const int32_t k = kept_nodes(range, scan, ch);
            if (k == 0) {
                codes[slot] = ~((r.x << 3) | (r.y - r.x + 1));
            } else {
                codes[slot] = next;
                next += k;
            }
        }
        const float lx = b.lo[0] - pad, hx = b.hi[0] + pad;
        const float ly = b.lo[1] - pad, hy = b.hi[1] + pad;
        const float lz = b.lo[2] - pad, hz = b.hi[2] + pad;
        if (slot == 0) {
            rec.f[0] = make_float4(lx, hx, ly, hy);
            rec.f[2].x = lz;
            rec.f[2].y = hz;
        } else {
            rec.f[1] = make_float4(lx, hx, ly, hy);
            rec.f[2].z = lz;
            rec.f[2].w = hz;
        }
    }
    rec.f[3] = make_float4(__int_as_float(codes[0]), __int_as_float(codes[1]), 0.0f, 0.0f);
    out[pre] = rec;
    ranges_out[pre] = make_int4(cover[0].x, cover[0].y, cover[1].x, cover[1].y);
    atomicMax(depth_out, depth + 1);  // the children of this node sit one level below it
}

// Refit of a kept tree: level 0 of the window table from the current records (in tree order).
__global__ void k_tri_boxes(const TriRec* __restrict__ tris, int32_t n, float* __restrict__ win)
{
    const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    store_box(win, i, tri_box(tris[i]));
}

// Refit of a kept tree: the two child boxes of node i from the record ranges their subtrees cover
// (ranges[i] = first0, last0, first1, last1; last < first for an empty leaf, whose unreachable box
// stays), widened by pad and rounded outward.
__global__ void k_refit_nodes(BvhNode* __restrict__ nodes, const int4* __restrict__ ranges, int32_t n_nodes,
                              const float* __restrict__ win, int32_t n, float pad)
{
    const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n_nodes) return;
    const int4 r = ranges[i];
    BvhNode rec = nodes[i];
    for (int slot = 0; slot < 2; ++slot) {
        const int32_t a = slot == 0 ? r.x : r.z, b = slot == 0 ? r.y : r.w;
        if (b < a) continue;
        const Box6 bx = range_box(win, n, a, b);
        // widened, then one more ulp outward: the rounded sums can never cut into the box
        const float lx = nextafterf(bx.lo[0] - pad, -FLT_MAX), hx = nextafterf(bx.hi[0] + pad, FLT_MAX);
        const float ly = nextafterf(bx.lo[1] - pad, -FLT_MAX), hy = nextafterf(bx.hi[1] + pad, FLT_MAX);
        const float lz = nextafterf(bx.lo[2] - pad, -FLT_MAX), hz = nextafterf(bx.hi[2] + pad, FLT_MAX);
        if (slot == 0) {
            rec.f[0] = make_float4(lx, hx, ly, hy);
            rec.f[2].x = lz;
            rec.f[2].y = hz;
        } else {
            rec.f[1] = make_float4(lx, hx, ly, hy);
            rec.f[2].z = lz;
            rec.f[2].w = hz;
        }
    }
    nodes[i] = rec;
}

__global__ void k_fill_words(uint32_t* __restrict__ p, int64_t n, uint32_t v)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

size_t lbvh_tmp_bytes(int32_t n)
{
    size_t sort = 0, scan = 0;
    (void)rocprim::radix_sort_pairs(nullptr, sort, static_cast<const uint32_t*>(nullptr),
                                    static_cast<uint32_t*>(nullptr), static_cast<const int32_t*>(nullptr),
                                    static_cast<int32_t*>(nullptr), n, 0, 30);
    (void)rocprim::inclusive_scan(nullptr, scan, static_cast<const int32_t*>(nullptr), static_cast<int32_t*>(nullptr),
                                  static_cast<size_t>(n), rocprim::plus<int32_t>());
    return std::max(sort, scan);
}

// Levels 1 .. levels - 1 of the window table over n boxes (level 0 filled).
void launch_windows(float* win, int32_t n, int32_t levels, hipStream_t stream)
{
    const int threads = 256;
    const unsigned bl = static_cast<unsigned>((n + threads - 1) / threads);
    const int32_t fused = std::min<int32_t>(levels - 1, kWinFused);
    if (fused > 0) hipLaunchKernelGGL(k_window_fused, dim3(bl), dim3(threads), 0, stream, win, n, fused);
    for (int32_t k = fused + 1; k < levels; ++k) {
        const int32_t half = 1 << (k - 1);
        const int32_t count = n - (1 << k) + 1;
        hipLaunchKernelGGL(k_window, dim3(static_cast<unsigned>((count + threads - 1) / threads)), dim3(threads), 0,
                           stream, win + static_cast<int64_t>(k - 1) * n * 6, win + static_cast<int64_t>(k) * n * 6,
                           count, half);
    }
}

hipError_t launch_refit(const TriRec* tris, int32_t n, BvhNode* nodes, const int4* ranges, int32_t n_nodes, float* win,
                        int32_t levels, float pad, hipStream_t stream)
{
    const int threads = 256;
    hipLaunchKernelGGL(k_tri_boxes, dim3(static_cast<unsigned>((n + threads - 1) / threads)), dim3(threads), 0, stream,
                       tris, n, win);
    launch_windows(win, n, levels, stream);
    hipLaunchKernelGGL(k_refit_nodes, dim3(static_cast<unsigned>((n_nodes + threads - 1) / threads)), dim3(threads), 0,
                       stream, nodes, ranges, n_nodes, win, n, pad);
    return hipGetLastError();
}

hipError_t launch_lbvh(const LbvhArgs& a, hipStream_t stream)
{
    const int32_t n = a.n;
    const int threads = 256;
    const unsigned bl = static_cast<unsigned>((n + threads - 1) / threads);
    hipLaunchKernelGGL(k_morton, dim3(bl), dim3(threads), 0, stream, a.tris_in, n, a.lo, a.scale, a.keys,
                       a.pos);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    size_t bytes = a.tmp_bytes;
    e = rocprim::radix_sort_pairs(a.tmp, bytes, a.keys, a.keys_sorted, a.pos, a.order, n, 0u, 30u, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gather, dim3(bl), dim3(threads), 0, stream, a.tris_in, a.mat_in, a.perm_in, a.order, n,
                       a.tris_out, a.mat_out, a.perm_out, a.bvh_pos_out, a.win);
    launch_windows(a.win, n, a.levels, stream);
    hipLaunchKernelGGL(k_karras, dim3(bl), dim3(threads), 0, stream, a.keys_sorted, n, a.child, a.range, a.parent,
                       a.leaf_parent);
    hipLaunchKernelGGL(k_frontier, dim3(bl), dim3(threads), 0, stream, a.range, a.parent, a.leaf_parent, n, a.start);
    hipLaunchKernelGGL(k_fill_words, dim3(1), dim3(threads), 0, stream, reinterpret_cast<uint32_t*>(a.scan),
                       int64_t(1), 0u);
    bytes = a.tmp_bytes;
    e = rocprim::inclusive_scan(a.tmp, bytes, a.start, a.scan + 1, static_cast<size_t>(n), rocprim::plus<int32_t>(),
                                stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_fill_words, dim3(1), dim3(threads), 0, stream, reinterpret_cast<uint32_t*>(a.depth_out),
                       int64_t(1), 0u);
    hipLaunchKernelGGL(k_emit, dim3(bl), dim3(threads), 0, stream, n, a.child, a.range, a.parent, a.scan, a.win,
                       a.pad, a.nodes_out, a.ranges_out, a.depth_out);
    return hipGetLastError();
}

}  // namespace srp
