// Scene object of libsrp (host view), shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/srp.h"
#include "srp_internal.h"

struct srp_scene_s {
    int device = 0;
    int64_t n_verts = 0, n_tris = 0;
    int32_t n_hinges = 0;
    std::vector<double> rest, cur;       // rest-pose and current (hinge-rotated) vertices
    std::vector<int32_t> tris, vhinge;
    std::vector<srp_hinge> hinges;       // axes normalised
    std::vector<double> angles;
    // Bumped by every change of geometry or materials; a path record is valid for one value of it.
    uint64_t geom_gen = 0;
    // The last srp_trace_recorded call: its record buffer, the scene state and the arguments it ran
    // with (pointers compared by address).
    struct PathStamp {
        const void* paths = nullptr;
        uint64_t gen = 0;
        const double* sun = nullptr;
        const double* frames = nullptr;
        int64_t D = 0;
        srp_trace_params p{};
    } path_stamp;
    bool refit_on_hinge = true;          // hinge changes refit the rest-pose tree instead of rebuilding
    double com[3] = {0, 0, 0};
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};  // current vertex bounding box
    double L = 0;                        // scene size: twice the largest vertex distance from the mean
    int32_t n_nodes = 0, depth = 0;
    std::vector<int32_t> perm;           // BVH triangle position -> original index
    std::vector<srp::BvhNode> h_nodes;   // host copies for the instrumented traversal
    std::vector<srp::TriRec> h_tris;
    bool h_tris_stale = false;           // the device records changed (GPU build); read back on use
    bool h_tree_stale = false;           // the device nodes (and order) changed; read back on use
    bool h_perm_stale = false;           // the device record order changed (GPU build); read back on use
    srp::BvhNode* d_nodes = nullptr;
    size_t nodes_cap = 0;
    srp::TriRec* d_tris = nullptr;
    size_t tris_cap = 0;
    float4* d_mat = nullptr;             // BVH order: rho_s, rho_d, p_spec, 0
    size_t mat_cap = 0;
    int32_t* d_perm = nullptr;
    size_t perm_cap = 0;
    int32_t* d_flag = nullptr;
    size_t flag_cap = 0;
    srp::DevFrame* d_frames = nullptr;
    size_t frames_cap = 0;
    double* d_partials = nullptr;        // per-workgroup FP64 partials (force/torque or hinge terms)
    size_t partials_cap = 0;
    double* d_grho = nullptr;            // adjoint: FP64 reflectance-gradient accumulators [2][n_tris]
    size_t grho_cap = 0;
    double* d_hdir = nullptr;            // adjoint: per-direction hinge sums [D][kMaxHinges]
    size_t hdir_cap = 0;
    // batched traces led by this scene: design table, staged in pinned host memory and uploaded
    // on the caller's stream; batch_ev marks the end of the last upload (staging reuse waits on it)
    srp::SceneDesc* h_batch_desc = nullptr;
    size_t h_batch_desc_cap = 0;
    hipEvent_t batch_ev = nullptr;
    srp::SceneDesc* d_batch_desc = nullptr;
    size_t batch_desc_cap = 0;
    // surface-sampling estimator: cumulative facet areas (FP64, original order), the BVH position
    // of each original facet, and the scene table of calls led by this scene (pinned staging)
    double area = 0;
    double* d_cum_area = nullptr;
    size_t cum_cap = 0;
    int32_t* d_bvh_pos = nullptr;
    size_t bvh_pos_cap = 0;
    srp::SurfaceScene* h_surf_desc = nullptr;
    size_t h_surf_desc_cap = 0;
    hipEvent_t surf_ev = nullptr;
    srp::SurfaceScene* d_surf_desc = nullptr;
    size_t surf_desc_cap = 0;
    // GPU BVH build: one workspace block, kept for later rebuilds
    char* d_lbvh_ws = nullptr;
    size_t lbvh_ws_cap = 0;
    // visibility-edge terms of the hinge gradient: the distinct edges of hinge-carried facets
    // (vertex a, vertex b, hinge), numbered by first appearance in facet order, and the current
    // vertex positions on the device
    std::vector<int4> h_edges;
    int4* d_edges = nullptr;
    size_t edges_cap = 0;
    // per moving edge, the facets on its two sides where the surface continues in one plane on
    // the edge's hinge (original indices a0, b0 and, for the back layer of a two-sided sheet,
    // a1, b1; a1 = -1: one layer; a0 = -1: no such continuation, the edge is always taken), from
    // the rest pose
    std::vector<int4> h_edge_pairs;
    int4* d_edge_pairs = nullptr;
    size_t edge_pairs_cap = 0;
    // the edges the edge term takes under the current materials (vertex a, vertex b, hinge, index
    // among all moving edges, which keys its draws), classified by the first edge-sampled adjoint
    // after a change of the scene
    std::vector<int4> h_live_edges;
    int4* d_live_edges = nullptr;
    size_t live_edges_cap = 0;
    int32_t* d_edge_keep = nullptr;
    size_t edge_keep_cap = 0;
    uint64_t edge_class_gen = ~0ull;
    // multi-world surface sampling: rest-pose records grouped by part (kept while the rest pose and
    // the facet groups stay the same) and the per-sample output of the last call
    srp::TriRec* d_mw_tris = nullptr;
    int32_t* d_mw_pos = nullptr;
    std::vector<int32_t> mw_groups;      // groups the records were built with (empty: not built)
    int32_t mw_part_end[srp::kMaxHinges + 1] = {};
    int32_t mw_part_hinge[srp::kMaxHinges + 1] = {};
    int32_t mw_n_parts = 0;
    float* d_mw_samples = nullptr;
    size_t mw_samples_cap = 0;
    // Phong exponents of the surface-sampling estimator (original facet order; NULL: ideal mirrors)
    float* d_phong = nullptr;
    bool phong_finite = false;  // some facet has a finite lobe (the ray-grid calls refuse the scene)
    float4* d_vpos = nullptr;
    size_t vpos_cap = 0;
    double* d_edge_part = nullptr;       // [D][edge workgroups][kMaxHinges]
    size_t edge_part_cap = 0;
    // device refit of the current tree: record ranges of every node's two child slots (valid for
    // ranges_nodes == n_nodes) and the window-table workspace
    int4* d_ranges = nullptr;
    size_t ranges_cap = 0;
    int32_t ranges_nodes = -1;
    float* d_win = nullptr;
    size_t win_cap = 0;
};

// Records `msg` as the thread's last error and returns `st`.
srp_status srp_fail(srp_status st, const std::string& msg);

// Brings the host copies of the tree (nodes, order, triangle records) up to date after a build on
// the device; host code that reads them (refit, statistics) calls this first.  Synchronous.
srp_status srp_pull_host_tree(srp_scene_s* s);

namespace srp {

// Device memory a forward trace takes its workspace from instead of the scene's own buffers:
// the grid frames first (rounded up to 256 bytes), then the per-workgroup partial sums.
struct TraceWorkspace {
    void* base;
    size_t bytes;
};

// srp_trace with its argument checks; `ws` NULL uses (and grows) the scene's workspace, else the
// trace runs in ws and fails with SRP_EINVAL, enqueueing nothing, when ws is too small.
// `paths` (non-null only without ws): the path record to write, sized by path_record_bytes.
srp_status trace_into(srp_scene_s* s, const double* sun_dirs, int64_t D, const srp_trace_params* p,
                      const double* frames, double* force, double* torque, hipStream_t stream,
                      const TraceWorkspace* ws, int32_t* paths = nullptr);

// Bytes of the path record of a grid trace: D x bounces x wave tiles x 64 int32.
int64_t path_record_bytes(const srp_trace_params* p, int64_t D);

}  // namespace srp
