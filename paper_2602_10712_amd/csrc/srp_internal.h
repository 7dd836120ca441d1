// Internal data layouts of libsrp, shared by the host code and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace srp {

constexpr double kSpeedOfLight = 299792458.0;  // m/s, exact
constexpr int kMaxBounces = 8;
constexpr int kRecordBounces = 3;  // interactions a path record holds (srp_trace_recorded)
constexpr int kStackDepth = 64;    // wave-uniform traversal stack (tree depth is capped below it)
constexpr int kMaxTreeDepth = 56;
constexpr int kLeafMax = 7;        // triangles per leaf (3-bit count in the child code)
constexpr int kWaves = 4;          // wavefronts per trace workgroup
constexpr int kTileW = 8;          // a wavefront traces an 8 x 8 pixel tile
constexpr int kTileH = 8;
constexpr int kMaxTilesPerWave = 16;  // a workgroup covers at most 64 wave tiles (one 64-bit mask)
static_assert(kMaxTilesPerWave * kWaves <= 64, "the live-tile mask holds one bit per workgroup tile");
// Tiles per wave of large traces.  A workgroup then spans 60 tiles, which does not divide the
// power-of-two tile rows of the usual grids: spans drift across rows from one workgroup to the next,
// so the round-robin placement of consecutive workgroups on shader engines does not hand the same
// rows (panels seen edge-on, the bus) to the same engines in every direction.
constexpr int kTilesPerWaveLarge = 15;
static_assert(kTilesPerWaveLarge <= kMaxTilesPerWave, "within the live-tile mask");
constexpr int kXcds = 8;           // MI355X: hardware workgroup b runs on accelerator complex b % 8
constexpr int kMaxHinges = 4;     // hinge-angle gradients (adjoint) and multi-world hinges supported
constexpr int kLaneStack = 24;     // per-lane stack of the independent walk (trees up to this depth)
constexpr int kLaneStackShort = 20;  // the trace kernels' shorter per-lane stack for trees up to this
                                     // depth: 21.7 KB of LDS per workgroup, so 7 workgroups share a CU
constexpr int kWalkDone = INT32_MIN;  // per-lane walk finished (never a node index or leaf code)

// BVH2 node, 64 bytes, both child boxes stored in the parent:
//   f[0] = (c0.lo.x, c0.hi.x, c0.lo.y, c0.hi.y)
//   f[1] = (c1.lo.x, c1.hi.x, c1.lo.y, c1.hi.y)
//   f[2] = (c0.lo.z, c0.hi.z, c1.lo.z, c1.hi.z)
//   f[3] = (child0, child1, -, -) as int bits; child >= 0: inner node index;
//          child < 0: leaf, ~child = first_triangle << 3 | count (count 0..7)
struct BvhNode {
    float4 f[4];
};

// Triangle record in BVH order, 64 bytes:
//   (v0.x, v0.y, v0.z, original index as int bits), (e1.xyz, n.x), (e2.xyz, n.y),
//   (n.z, hinge index as int bits (-1 rigid), 0, 0)
struct TriRec {
    float4 f[4];
};

// Per-direction grid frame as the trace kernel consumes it (FP32, rounded from FP64):
// origin of pixel (i, k) with offsets (a, b): o0 + (i + a) U + (k + b) V; propagation d;
// w = Phi du dv / c is the force carried by one ray tube.
struct DevFrame {
    float o0[3];
    float U[3];
    float V[3];
    float d[3];
    float w;
    float pad[3];
};

// One design of a batched trace (device array, one entry per scene).
// Pointers that kernels read from memory rather than receive as arguments carry the global address
// space in device code, so loads through them are global (and scalar where the address is
// wave-uniform) rather than generic; the host sees plain pointers of the same size.
#if defined(__HIP_DEVICE_COMPILE__)
#define SRP_GLOBAL __attribute__((address_space(1)))
#else
#define SRP_GLOBAL
#endif

// One design of a batched trace.
struct SceneDesc {
    const SRP_GLOBAL BvhNode* nodes;
    const SRP_GLOBAL TriRec* tris;
    const SRP_GLOBAL float4* mat;
    float com[3];
    float eps;
};

struct TraceArgs {
    const SceneDesc* scenes;  // batched trace: [n_scenes] (null for a single scene)
    int32_t n_scenes;
    const BvhNode* nodes;
    const TriRec* tris;
    const float4* mat;        // BVH order: (rho_s, rho_d, p_spec, 0)
    const DevFrame* frames;   // [D], or [n_scenes][D] for a batched trace
    int64_t D;
    int32_t nu, nv;
    int32_t bounces;
    int32_t jitter;
    uint32_t seed_lo, seed_hi;
    int64_t dir_index_base;
    uint32_t design_index;
    float com[3];
    float eps;                // secondary-ray offset along the normal
    int32_t tiles_x, tiles_y; // wave tiles per direction (grid mode)
    int64_t tiles_per_dir;
    int32_t tiles_per_wave;
    int32_t blocks_per_dir;
    int32_t lane_walk;        // nonzero: secondary segments use the per-lane walk (tree depth <= kLaneStack);
                              // 2: the tree also fits kLaneStackShort
    int32_t cull;             // 1: skip wave tiles that provably miss the scene (library frames)
    int32_t xcd_major;        // 1: unit u (direction, or design x direction) is traced by XCD u % 8
    const int64_t* pix;       // records mode: explicit pixel list, or null = all pixels
    int64_t n_pix;
    double* partials;         // [(scene *) D][blocks_per_dir][6]
    int32_t* rec_hit;         // [D][n_pix][bounces]
    float* rec_force;         // [D][n_pix][3]
    float* rec_point;         // [D][n_pix][bounces][3] hit points (NaN after the path ended), or null
    const uint32_t* ray_mask; // single scene: [D][mask_words] bitmap of primary pixels left out, or null
    int64_t mask_words;       // words per direction: ceil(nu * nv / 32)
    int32_t* path_hit;        // grid mode, single scene: [D][bounces][tiles_per_dir][64] triangle (BVH
                              // order) each traced path hit at each interaction, -1 for none; written
                              // by the forward, read by the adjoint instead of walking the BVH; or null
};

// Slot of (direction j, interaction b >= 1, wave tile, lane) in TraceArgs::path_hit.
__host__ __device__ inline int64_t path_slot(const TraceArgs& a, int64_t j, int b, int64_t tile, int lane)
{
    return ((j * a.bounces + (b - 1)) * a.tiles_per_dir + tile) * 64 + lane;
}

// Primary pixel `pixel` of direction j (of a single-scene call) is left out by the caller's mask.
__device__ __forceinline__ bool ray_masked(const TraceArgs& a, int64_t j, int64_t pixel)
{
    return ((a.ray_mask[j * a.mask_words + (pixel >> 5)] >> (pixel & 31)) & 1u) != 0u;
}

// Workgroups of a trace or adjoint launch over n_units units (directions, or (design, direction)
// pairs).  Direction-major order needs n_units x blocks_per_dir; XCD-major order pads n_units to
// whole groups of kXcds.
inline int64_t grid_blocks(const TraceArgs& a, int64_t n_units)
{
    const int64_t units = a.xcd_major ? (n_units + kXcds - 1) / kXcds * kXcds : n_units;
    return units * a.blocks_per_dir;
}

// One scene of the surface-sampling estimator: BVH-order records plus the cumulative facet areas
// (FP64, original facet order) and the BVH position of every original facet.
struct SurfaceScene {
    const SRP_GLOBAL BvhNode* nodes;
    const SRP_GLOBAL TriRec* tris;
    const SRP_GLOBAL float4* mat;
    const SRP_GLOBAL double* cum_area;
    const SRP_GLOBAL int32_t* bvh_pos;
    double area;              // total area
    float com[3];
    float eps;                // ray offset along the normal
    int32_t n_tris;
    int32_t pad;
};

struct SurfaceArgs {
    const SurfaceScene* scenes;  // [n_scenes]
    int32_t n_scenes;
    int32_t bounces;
    const double* sun;           // [D][3]
    int64_t D;
    int64_t n_samples;           // per (scene, direction) unit
    int32_t chunks;              // workgroups per unit
    float flux_c;                // Phi / c
    uint32_t seed_lo, seed_hi;
    int64_t dir_index_base;
    uint32_t design_index;
    int32_t sampling;            // bit 0: stratified surface; bit 1: uniform hemisphere directions
    double* partials;            // [units][chunks][6]
    int32_t* rec_facet;          // [units][n_samples] or null
    int32_t* rec_hits;           // [units][n_samples][bounces - 1] or null
    int32_t* rec_lit;            // [units][n_samples] (with rec_facet)
};

// Multi-world surface sampling: the rest-pose mesh with its facet records grouped by rigid part
// (part 0 the body, part q a hinge), each pair's design applied by turning its rays into the
// parts' rest frames.
struct MwScene {
    const SRP_GLOBAL TriRec* tris;     // rest-pose records, grouped by part; f[3].y hinge, f[3].z group
    const SRP_GLOBAL int32_t* pos;     // original facet -> record
    const SRP_GLOBAL double* cum_area; // cumulative facet areas, original order
    double area;
    float com[3];
    float eps;
    int32_t n_tris;
    int32_t n_parts;
    int32_t part_end[kMaxHinges + 1];    // exclusive record ends
    int32_t part_hinge[kMaxHinges + 1];  // -1: the body
    float hinge_origin[kMaxHinges][3];
    float hinge_axis[kMaxHinges][3];
};

struct MwArgs {
    SurfaceArgs base;      // sampling, bounces, flux_c, seed_lo/hi (per-unit fields unused)
    MwScene sc;
    const double* sun;     // [N][3]
    const float* designs;  // [N][stride]: hinge angles, then per group rho_s, rho_d, Phong exponent
    int64_t n_pairs;
    int32_t samples;       // per pair
    int32_t n_hinges;
    int32_t n_groups;
    int32_t stride;
    float* sample_out;     // [N * samples][6] force and torque of each sample
    int32_t* rec_facet;    // [N][samples] or null
    int32_t* rec_hits;     // [N][samples][bounces - 1] or null
    int32_t* rec_lit;      // [N][samples] (with rec_facet)
};
// flags |= 1 for a pair whose materials are out of range (rho < 0, rho_s + rho_d > 1, exponent < 1)
hipError_t launch_check_designs(const float* designs, int64_t n_pairs, int32_t n_hinges, int32_t n_groups,
                                int32_t* flags, hipStream_t stream);
hipError_t launch_surface_designs(const MwArgs& a, double* force, double* torque, hipStream_t stream);

// GPU BVH build (linear BVH): buffers of one build over n >= 2 triangles.
constexpr int kLbvhLeaf = 4;    // subtrees of at most this many triangles become one leaf
struct LbvhArgs {
    int32_t n;
    int32_t levels;                 // window-table levels: floor(log2 n) + 1
    float3 lo, scale;               // Morton grid: (centroid - lo) * scale in [0, 1024)
    float pad;                      // box widening, metres
    const TriRec* tris_in;          // current order
    const float4* mat_in;
    const int32_t* perm_in;         // current position -> original facet
    uint32_t* keys;                 // [n]
    uint32_t* keys_sorted;          // [n]
    int32_t* pos;                   // [n]
    int32_t* order;                 // [n] new position -> current position
    void* tmp;                      // sort and scan scratch
    size_t tmp_bytes;
    TriRec* tris_out;               // [n] new order
    float4* mat_out;
    int32_t* perm_out;              // [n] new position -> original facet
    int32_t* bvh_pos_out;           // [n] original facet -> new position
    int2* child;                    // [n - 1] inner index, or ~leaf
    int2* range;                    // [n - 1] first, last leaf
    int32_t* parent;                // [n - 1]
    int32_t* leaf_parent;           // [n]
    int32_t* start;                 // [n] 1 where a leaf opens a leaf record of the final tree
    int32_t* scan;                  // [n + 1] leaf records opened before each leaf; scan[n] - 1 nodes
    float* win;                     // [levels][n][6] box of leaves [i, i + 2^level)
    BvhNode* nodes_out;             // [n - 1], pre-order, scan[n] - 1 of them written
    int4* ranges_out;               // [n - 1] record ranges of each written node's child slots
    int32_t* depth_out;             // deepest level (root = 0)
};


struct AdjointArgs {
    TraceArgs t;                 // geometry, frames and grid of the replayed forward trace
    const double* g_force;       // [D][3] seed dL/dF
    const double* g_torque;      // [D][3] seed dL/dtau, or null
    double* g_rho;               // [2][n_tris] FP64 accumulators, original facet order
    int32_t n_tris;
    int32_t n_hinges;
    float hinge_axis[kMaxHinges][3];
    float hinge_origin[kMaxHinges][3];
    double* hinge_partials;      // [D][blocks_per_dir][kMaxHinges]
};

// Host-side launchers (defined in trace_kernels.hip and adjoint_kernels.hip).
hipError_t launch_frames(const double* sun_dirs, int64_t D, const double lo[3], const double hi[3], double L,
                         int32_t nu, int32_t nv, double flux, const double* caller_frames, double* frames64,
                         DevFrame* frames32, hipStream_t stream);
hipError_t launch_pack_materials(const float* rho_s, const float* rho_d, const float* p_spec, const float* phong,
                                 const int32_t* perm, int64_t n, float4* mat, int32_t* bad_flag, hipStream_t stream);
// Phong exponents (original facet order, NULL: +infinity) into mat[].w (mat NULL: check only);
// flags |= 1 for an exponent below 1 or NaN, |= 2 when any is finite.
hipError_t launch_pack_phong(const float* phong, const int32_t* perm, int64_t n, float4* mat, int32_t* flags,
                             hipStream_t stream);
hipError_t launch_trace(const TraceArgs& a, bool records, hipStream_t stream);
hipError_t launch_trace_batch(const TraceArgs& a, hipStream_t stream);
hipError_t launch_reduce(const double* partials, int64_t D, int32_t blocks_per_dir, double* force, double* torque,
                         hipStream_t stream);
hipError_t launch_adjoint(const AdjointArgs& a, hipStream_t stream);

// Visibility-edge terms of the hinge-angle gradient (edge_kernels.hip).
struct EdgeArgs {
    const int4* edges;      // [n_edges]: vertex a, vertex b, hinge, index among all moving edges
    const float4* verts;    // [n_verts] current vertex positions
    int32_t n_edges;
    int32_t samples;        // points per edge
    int64_t D;
    int32_t bounces;
    uint32_t seed_lo, seed_hi;
    int64_t dir_index_base;
    uint32_t design_index;
    float eps;              // secondary-ray offset along the normal
    float delta;            // offset of the two side points from the edge
    float com[3];
    float hinge_origin[kMaxHinges][3];
    float hinge_axis[kMaxHinges][3];
};
int32_t edge_blocks(const EdgeArgs& E);
// keep[i] = 0 where pairs[i] (facet pairs, original indices; x < 0: none) have equal packed
// materials (rho_s, rho_d, p_spec) on both sides of every layer, else 1.
hipError_t launch_edge_keep(const int4* pairs, int32_t n, const int32_t* bvh_pos, const float4* mat, int32_t* keep,
                            hipStream_t stream);
hipError_t launch_edge_term(const EdgeArgs& E, const BvhNode* nodes, const TriRec* tris, const float4* mat,
                            const DevFrame* frames, const double* g_force, const double* g_torque, int lane_walk,
                            double* partials, double* per_dir, hipStream_t stream);
hipError_t launch_reduce_hinges(const double* hinge_partials, int64_t D, int32_t blocks_per_dir, double* per_dir,
                                hipStream_t stream);
size_t lbvh_tmp_bytes(int32_t n);
hipError_t launch_lbvh(const LbvhArgs& a, hipStream_t stream);
// Device refit of a kept tree over n records: win holds [levels][n][6] floats of workspace,
// ranges[i] the record ranges (first0, last0, first1, last1) of node i's two child slots.
hipError_t launch_refit(const TriRec* tris, int32_t n, BvhNode* nodes, const int4* ranges, int32_t n_nodes, float* win,
                        int32_t levels, float pad, hipStream_t stream);
hipError_t launch_surface(const SurfaceArgs& a, bool brute, double* force, double* torque, hipStream_t stream);
hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t stream);
hipError_t launch_finish_adjoint(const double* g_rho, int32_t n_tris, float* g_rho_s, float* g_rho_d, int64_t D,
                                 int32_t n_hinges, const double* per_dir, double* g_hinge, hipStream_t stream);

}  // namespace srp
