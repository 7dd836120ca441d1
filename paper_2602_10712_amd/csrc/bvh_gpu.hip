// BVH build on the GPU: linear BVH after Karras, "Maximizing Parallelism in the Construction of
// BVHs, Octrees, and k-d Trees" (HPG 2012), with subtrees of at most kLbvhLeaf triangles collapsed
// into leaves and the kept inner nodes written in pre-order (the layout of the host-built tree:
// node 0 the root, every child after its parent).
//
//   1. 30-bit Morton code of every triangle centroid (10 bits per axis over the scene box);
//   2. radix sort of (code, position) pairs (rocPRIM);
//   3. triangle, material and permutation records gathered into the sorted order;
//   4. the binary radix tree over the sorted codes (one thread per inner node; equal codes are
//      ordered by position), parents and leaf ranges;
//   5. bottom-up boxes and kept-node counts: one thread per triangle climbs toward the root, the
//      second thread to reach a node finishes it (device-scope counter per node);
//   6. pre-order positions from the counts (each kept node walks to the root) and the node records.
#include <float.h>

#include <rocprim/device/device_radix_sort.hpp>

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

// records at their sorted positions; perm maps positions to original facets
__global__ void k_gather(const TriRec* __restrict__ tris_in, const float4* __restrict__ mat_in,
                         const int32_t* __restrict__ perm_in, const int32_t* __restrict__ order, int32_t n,
                         TriRec* __restrict__ tris_out, float4* __restrict__ mat_out, int32_t* __restrict__ perm_out)
{
    const int32_t k = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    if (k >= n) return;
    const int32_t q = order[k];
    tris_out[k] = tris_in[q];
    mat_out[k] = mat_in[q];
    perm_out[k] = perm_in[q];
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

__device__ __forceinline__ Box6 load_box(const float* b, int32_t i)
{
    Box6 r;
    for (int a = 0; a < 3; ++a) {
        r.lo[a] = b[6 * i + a];
        r.hi[a] = b[6 * i + 3 + a];
    }
    return r;
}

// Bottom-up: boxes of inner nodes and, per inner node, the number of kept inner nodes in its
// subtree (0 when its subtree holds at most kLbvhLeaf triangles and becomes a leaf).
__global__ void k_bottom_up(const TriRec* __restrict__ tris, int32_t n, const int2* __restrict__ child,
                            const int2* __restrict__ range, const int32_t* __restrict__ parent,
                            const int32_t* __restrict__ leaf_parent, uint32_t* visits, float* leaf_box,
                            float* node_box, int32_t* kept)
{
    const int32_t k = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    if (k >= n) return;
    const Box6 lb = tri_box(tris[k]);
    for (int a = 0; a < 3; ++a) {
        leaf_box[6 * k + a] = lb.lo[a];
        leaf_box[6 * k + 3 + a] = lb.hi[a];
    }
    int32_t node = leaf_parent[k];
    while (node >= 0) {
        __threadfence();  // this thread's boxes are visible before its arrival is counted
        const uint32_t seen = atomicAdd(&visits[node], 1u);
        if (seen == 0) return;  // the sibling subtree is not done; its thread finishes this node
        __threadfence();  // see the sibling's boxes
        const int2 c = child[node];
        const Box6 b0 = c.x >= 0 ? load_box(node_box, c.x) : load_box(leaf_box, ~c.x);
        const Box6 b1 = c.y >= 0 ? load_box(node_box, c.y) : load_box(leaf_box, ~c.y);
        for (int a = 0; a < 3; ++a) {
            node_box[6 * node + a] = fminf(b0.lo[a], b1.lo[a]);
            node_box[6 * node + 3 + a] = fmaxf(b0.hi[a], b1.hi[a]);
        }
        const int2 r = range[node];
        const int32_t k0 = c.x >= 0 ? kept[c.x] : 0;
        const int32_t k1 = c.y >= 0 ? kept[c.y] : 0;
        kept[node] = (r.y - r.x + 1 <= kLbvhLeaf && node != 0) ? 0 : 1 + k0 + k1;
        node = parent[node];
    }
}

// Pre-order node records of the kept inner nodes.  A node is kept when neither it nor an ancestor
// holds at most kLbvhLeaf triangles (the root always is).
__global__ void k_emit(int32_t n, const int2* __restrict__ child, const int2* __restrict__ range,
                       const int32_t* __restrict__ parent, const int32_t* __restrict__ kept,
                       const float* __restrict__ leaf_box, const float* __restrict__ node_box, float pad,
                       BvhNode* __restrict__ out, int32_t* __restrict__ depth_out)
{
    const int32_t i = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n - 1) return;
    if (kept[i] == 0) return;
    // position: the root is 0; a left child follows its parent, a right child follows the parent's
    // left subtree
    int32_t pre = 0, depth = 0, node = i;
    while (node != 0) {
        const int32_t p = parent[node];
        if (kept[p] == 0) return;  // inside a collapsed subtree
        const int2 c = child[p];
        pre += 1;
        if (c.y == node && c.x >= 0) pre += kept[c.x];
        node = p;
        ++depth;
    }
    const int2 c = child[i];
    BvhNode rec;
    int32_t codes[2];
    const int32_t kids[2] = {c.x, c.y};
    int32_t next = pre + 1;
    for (int slot = 0; slot < 2; ++slot) {
        const int32_t ch = kids[slot];
        Box6 b;
        if (ch < 0) {
            b = load_box(leaf_box, ~ch);
            codes[slot] = ~((~ch << 3) | 1);
        } else {
            b = load_box(node_box, ch);
            const int2 r = range[ch];
            if (kept[ch] == 0) {
                codes[slot] = ~((r.x << 3) | (r.y - r.x + 1));
            } else {
                codes[slot] = next;
                next += kept[ch];
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
    atomicMax(depth_out, depth + 1);  // the children of this node sit one level below it
}

__global__ void k_fill_words(uint32_t* __restrict__ p, int64_t n, uint32_t v)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace

size_t lbvh_sort_bytes(int32_t n)
{
    size_t bytes = 0;
    (void)rocprim::radix_sort_pairs(nullptr, bytes, static_cast<const uint32_t*>(nullptr), static_cast<uint32_t*>(nullptr),
                              static_cast<const int32_t*>(nullptr), static_cast<int32_t*>(nullptr), n, 0, 30);
    return bytes;
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
    size_t bytes = a.sort_bytes;
    e = rocprim::radix_sort_pairs(a.sort_tmp, bytes, a.keys, a.keys_sorted, a.pos, a.order, n, 0u, 30u, stream);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gather, dim3(bl), dim3(threads), 0, stream, a.tris_in, a.mat_in, a.perm_in, a.order, n,
                       a.tris_out, a.mat_out, a.perm_out);
    hipLaunchKernelGGL(k_fill_words, dim3(bl), dim3(threads), 0, stream, a.visits, static_cast<int64_t>(n), 0u);
    hipLaunchKernelGGL(k_fill_words, dim3(1), dim3(threads), 0, stream, reinterpret_cast<uint32_t*>(a.depth_out),
                       int64_t(1), 0u);
    hipLaunchKernelGGL(k_karras, dim3(bl), dim3(threads), 0, stream, a.keys_sorted, n, a.child, a.range, a.parent,
                       a.leaf_parent);
    hipLaunchKernelGGL(k_bottom_up, dim3(bl), dim3(threads), 0, stream, a.tris_out, n, a.child, a.range, a.parent,
                       a.leaf_parent, a.visits, a.leaf_box, a.node_box, a.kept);
    hipLaunchKernelGGL(k_emit, dim3(bl), dim3(threads), 0, stream, n, a.child, a.range, a.parent, a.kept,
                       a.leaf_box, a.node_box, a.pad, a.nodes_out, a.depth_out);
    return hipGetLastError();
}

}  // namespace srp
