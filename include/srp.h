/*
 * srp.h -- C ABI of libsrp: ray-grid Monte Carlo solar radiation pressure (SRP) on MI355X.
 *
 * The problem (paper Sec. 3.2, "Radiation Pressure Simulation"): light arrives from a single,
 * infinitely distant direction; a spacecraft is a triangle mesh with per-face materials whose
 * geometry depends on design parameters; the outputs are the body-frame force F(w, theta) and
 * torque tau(w, theta) about the centre of mass (Sec. 3.2, force and torque integrals; Sec.
 * 3.4.1 uses them in the body frame).  The estimator is a parallel ray grid per sun direction:
 * every grid ray carries the flux through its pixel, is traced through a BVH to its closest
 * front-facing hit, deposits photon momentum there through the light-to-force map l2f
 * (Sec. 3.2: incident momentum minus reflected momentum, over c) with an ideal-mirror part
 * rho_s, a Lambertian part rho_d and an absorbed part 1 - rho_s - rho_d, and is followed over
 * up to `bounces` surface interactions.  Deposits are reduced to one FP64 force and torque per
 * direction.
 *
 * Conventions
 *   - Body frame, metres, newtons.  Triangles are counter-clockwise seen from outside; the
 *     outward normal is normalize((v1 - v0) x (v2 - v0)); only the outward side is hit.
 *   - Sun directions are unit vectors pointing TOWARD the Sun; light travels along -s.
 *   - Every call returns an srp_status; 0 is success.  On failure nothing is enqueued and
 *     srp_last_error() returns a message (thread-local, valid until the next call on the thread).
 *   - "device" pointers are HIP device memory (e.g. torch.Tensor.data_ptr() of a cuda tensor);
 *     they stay owned by the caller and must stay alive until the enqueued work completes.
 *     "host" pointers are read during the call only (copied where kept).
 *   - stream: a hipStream_t passed as void* (NULL = the null stream).  Launches are enqueued
 *     on it without synchronising, except where a call says otherwise.  Device faults surface
 *     as SRP_EDEVICE from a later call or from srp_sync().
 *   - A scene owns workspace (frames, partial sums, gradient accumulators) that every call on it
 *     reuses: calls on one scene must be ordered, i.e. issued on one stream or synchronised by
 *     the caller.  Calls on different scenes are independent.
 *   - Random draws: Philox4x32-10 (Salmon et al., SC'11) with key = seed and counter =
 *     (pixel, global direction index, bounce, design index); uniforms are the top 24 bits
 *     times 2^-24.  Identical arguments give bit-identical ray sets on every call.
 */
#ifndef SRP_H
#define SRP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t srp_status;
#define SRP_OK 0
#define SRP_EINVAL (-1)         /* bad argument */
#define SRP_ENOMEM (-2)         /* host or device allocation failed */
#define SRP_EDEVICE (-3)        /* a HIP runtime error */
#define SRP_EDEGENERATE (-4)    /* unusable mesh: zero-area facet or non-finite vertex */
#define SRP_EUNSUPPORTED (-5)   /* valid request this build cannot serve */

typedef struct srp_scene_s* srp_scene;

/* A hinge line in the body frame: panel vertices assigned to it rotate about (origin, axis) by
 * the hinge angle, right-hand rule.  axis need not be normalised (it is normalised on copy). */
typedef struct {
    double origin[3];
    double axis[3];
} srp_hinge;

/* Parameters of one trace.
 *   nu, nv        grid resolution per direction (pixels along the frame's u and v axes), >= 1
 *   bounces       surface interactions followed per path, 1..8; at the last one the expected
 *                 reflected momentum leaves the body
 *   jitter        1: one Philox-drawn point per pixel; 0: pixel centres
 *   flux          solar flux Phi in W/m^2 (e.g. 1361)
 *   seed          Philox key
 *   dir_index_base  global index of direction 0 of this call (Philox counter word 1)
 *   design_index  Philox counter word 3
 *   frame_mode    0: the grid frame of each direction is derived from the mesh (Duff et al. 2017
 *                 basis of the propagation direction, rectangle bounding the projected box,
 *                 entry plane 0.01 L in front, L = twice the largest vertex distance from the
 *                 vertex mean); 1: the caller passes frames (see srp_frames for the layout)
 *   tiles_per_wave  launch shape only: 8 x 8-pixel tiles per wavefront and workgroup, 1..16, or 0
 *                 for the library's rule (srp_autotune_tiles_per_wave measures the choices).  Results
 *                 are the same up to the FP32 summation order of the per-wave partial sums.
 *   sampling      surface-sampling estimator only (srp_surface_estimate; ignored elsewhere): the variance-
 *                 reduction options of the paper's convergence study, bit 0 stratified surface
 *                 sampling (sample i of N takes the area coordinate (i + u)/N), bit 1 plain Monte
 *                 Carlo directions (uniform over the hemisphere, weight 2 cos theta) instead of the
 *                 Lambertian BRDF's cosine importance sampling; 0..3.
 *   edge_samples  srp_trace_adjoint only: points per moving edge for the visibility-edge part of the
 *                 hinge-angle gradient (0: that part is left out), 0..4096; see srp_trace_adjoint.
 *   ray_mask      device uint32 bitmap [D][ceil(nu * nv / 32)] or NULL: a set bit (p & 31) in word
 *                 p >> 5 of direction j leaves primary pixel p of that direction out, its whole path
 *                 included (no deposit, no gradient; in records its hits are -1 and its force 0).
 *                 srp_trace, srp_trace_noalloc, srp_trace_records and srp_trace_adjoint only (other
 *                 calls reject it with SRP_EUNSUPPORTED).  For restricting a trace to a region of the
 *                 image and for parity checks on a chosen set of rays. */
typedef struct {
    int32_t nu, nv;
    int32_t bounces;
    int32_t jitter;
    double flux;
    uint64_t seed;
    int64_t dir_index_base;
    int32_t design_index;
    int32_t frame_mode;
    int32_t tiles_per_wave;
    int32_t sampling;
    int32_t edge_samples;
    const uint32_t* ray_mask;
} srp_trace_params;

/* Creates a scene from a rest-pose mesh.  Host arrays, copied:
 *   verts [n_verts][3], tris [n_tris][3] (vertex indices), vert_hinge [n_verts] (-1 rigid, k: carried
 *   by hinge k; NULL = all rigid), hinges [n_hinges], com [3] (NULL = origin).
 * The scene is bound to the current HIP device.  Until srp_scene_set_design is called every
 * facet is black (rho_s = rho_d = 0) and all hinge angles are 0.
 * Errors: SRP_EINVAL (bad index, sizes, n_tris > 2^26), SRP_EDEGENERATE (zero-area facet, NaN). */
srp_status srp_scene_create(const double* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                            const int32_t* vert_hinge, const srp_hinge* hinges, int32_t n_hinges,
                            const double* com, srp_scene* out);

/* Applies a design (paper Sec. 3.1: the design maps to a mesh with per-face materials):
 *   hinge_angles host [n_hinges] radians (NULL = keep the current angles); the panel vertices
 *   are rotated in FP64 and, when the angles change, the triangle records are rebuilt on the host
 *   and uploaded and the boxes of the current BVH are refitted on the device (same topology and
 *   triangle order; each box the union of its records' boxes, widened by 1e-6 L and rounded
 *   outward);
 *   rho_s, rho_d device float [n_tris] (original facet order), 0 <= rho, rho_s + rho_d <= 1;
 *   p_spec device float [n_tris] or NULL: frozen probability of sampling the specular event at
 *   each facet, in [0, 1], 0 only where rho_s = 0 and 1 only where rho_d = 0 (else an event with
 *   nonzero reflectance could never be sampled: SRP_EINVAL).  NULL selects rho_s/(rho_s + rho_d)
 *   clamped to [0.01, 0.99] when both are positive, else 1 (mirror only) or 0.
 * Synchronises `stream` once to validate the materials (SRP_EINVAL if out of range). */
srp_status srp_scene_set_design(srp_scene scene, const double* hinge_angles, const float* rho_s,
                                const float* rho_d, const float* p_spec, void* stream);

/* Per-face Phong exponents (paper Sec. 3.2, "Estimation": the design maps to a mesh with per-face
 * Phong material parameters) for the surface-sampling estimator: facet f reflects with the
 * modified Phong BRDF rho_d/pi + rho_s (m + 2)/(2 pi) ((r.o)+)^m (Lafortune and Willems 1994), r
 * the mirror direction of the arriving light, m = exponents[f].
 *   exponents device float [n_tris] (original facet order), each >= 1 or +infinity (the ideal
 *   mirror), copied; NULL restores ideal mirrors everywhere.
 * Kept across srp_scene_set_design, GPU rebuilds and srp_scene_set_vertices.  The ray-grid calls
 * (srp_trace*, srp_trace_adjoint, srp_batch_trace, srp_scene_ray_stats) model ideal mirrors only
 * and refuse a scene with any finite exponent (SRP_EUNSUPPORTED).  Synchronises `stream`.
 * Errors: SRP_EINVAL (an exponent below 1 or NaN; the scene keeps its exponents). */
srp_status srp_scene_set_phong(srp_scene scene, const float* exponents, void* stream);

/* Replaces the rest-pose vertices (paper Sec. 3.1: any design that maps to a mesh of fixed
 * connectivity, e.g. a parametric bus or panel size), keeping the triangles, the hinge
 * assignment, the hinge angles (applied on top of the new rest pose) and the materials.
 *   verts host double [n_verts][3], copied; n_verts must equal the scene's;
 *   mode 0: keep the tree and refit its boxes on the device (fast; traversal slows down as the
 *           geometry drifts from the pose the tree was built for), 1: build a new SAH tree on the
 *           host (the packed materials are reordered with the records).
 * The moving edges of the hinge gradient are re-derived from the new rest pose.  Synchronises
 * `stream`.  Errors: SRP_EINVAL (NULL, size, mode), SRP_EDEGENERATE (non-finite vertex or a
 * zero-area facet in the new pose; the scene keeps its old geometry), SRP_EUNSUPPORTED (mode 1:
 * tree deeper than the traversal stack; the scene keeps its old geometry), SRP_EDEVICE (the scene
 * is left undefined and must be destroyed). */
srp_status srp_scene_set_vertices(srp_scene scene, const double* verts, int64_t n_verts, int32_t mode,
                                  void* stream);

/* Host copy of the current (hinge-rotated) vertices, [n_verts][3]. */
srp_status srp_scene_get_vertices(srp_scene scene, double* verts_out, int64_t n_verts);

/* BVH statistics: number of BVH nodes, tree depth, triangles (host ints, any may be NULL). */
srp_status srp_scene_info(srp_scene scene, int32_t* n_nodes, int32_t* depth, int32_t* n_tris);

/* Grid frames for D directions, device double [D][12]: u[3], v[3], o0[3], du, dv, 0; the ray of
 * pixel (i, k) with in-pixel offsets (a, b) starts at o0 + (i+a) du u + (k+b) dv v and travels
 * along -s.  sun_dirs device double [D][3]. */
srp_status srp_frames(srp_scene scene, const double* sun_dirs, int64_t D, int32_t nu, int32_t nv, double* frames,
                      void* stream);

/* Forward trace.  sun_dirs device double [D][3] (unit, toward the Sun), frames device double
 * [D][12] when params->frame_mode == 1 (else ignored, may be NULL); force device double [D][3]
 * and torque device double [D][3] (torque may be NULL) are overwritten with the per-direction
 * sums.  The sum is deterministic for given arguments: FP32 per ray and per wavefront, FP64 per
 * workgroup and a fixed-order FP64 sum per direction. */
srp_status srp_trace(srp_scene scene, const double* sun_dirs, int64_t D, const srp_trace_params* params,
                     const double* frames, double* force, double* torque, void* stream);

/* srp_trace for callers that cannot allocate device memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  Same arguments, kernels and results as
 * srp_trace (bit-identical), but the per-direction grid frames and FP64 per-workgroup partial
 * sums live in one fixed array of SRP_NOALLOC_WORKSPACE_BYTES (16 MiB) that the library holds
 * on each device it runs on until the process ends; the call allocates nothing (the scene itself
 * must already exist).  A trace needs 64 D bytes (rounded up to 256) plus 48 bytes per direction
 * and workgroup: about 13.2 KB per direction at 1024 x 1024 pixels with the library's launch
 * shape, so up to ~1,260 directions per call there.  Larger requests fail with SRP_EINVAL and
 * enqueue nothing.  Every call on a device shares that device's array, which keeps the last
 * call's contents (every partial sum is rewritten before it is read): calls that overlap on one
 * device, on different streams or threads, race and must be ordered by the caller. */
#define SRP_NOALLOC_WORKSPACE_BYTES (16u << 20)
srp_status srp_trace_noalloc(srp_scene scene, const double* sun_dirs, int64_t D, const srp_trace_params* params,
                             const double* frames, double* force, double* torque, void* stream);

/* Per-ray records of the same estimator for an explicit pixel list (parity and debugging).
 *   pix device int64 [n_pix] pixel ids (i + k*nu), or NULL for all nu*nv pixels in order;
 *   hit_prim device int32 [D][n_pix][bounces]: ORIGINAL index of the facet hit at each
 *   interaction, -1 after the path ended; ray_force device float [D][n_pix][3] or NULL;
 *   hit_point device float [D][n_pix][bounces][3] or NULL: the FP32 hit point of each interaction
 *   (body frame, m), NaN after the path ended.  A ray_mask in params is indexed by pixel id. */
srp_status srp_trace_records(srp_scene scene, const double* sun_dirs, int64_t D, const srp_trace_params* params,
                             const double* frames, const int64_t* pix, int64_t n_pix, int32_t* hit_prim,
                             float* ray_force, float* hit_point, void* stream);

/* Reverse-mode gradient of the forward estimator (paper Sec. 3.4, differentiable radiation
 * pressure: gradients of force and torque with respect to the design), for the same rays as
 * srp_trace with the same arguments.  Given cotangents g_force and g_torque (device double [D][3];
 * g_torque may be NULL = 0) of L = sum_j g_force[j].F_j + g_torque[j].tau_j, the call ADDS
 *   dL/d rho_s, dL/d rho_d  to g_rho_s, g_rho_d (device float [n_tris], original facet order, may be
 *                           NULL): exact derivatives of the estimator with the sampled event
 *                           sequences held fixed (the specular-sampling probabilities are
 *                           frozen, so each path's weight is a polynomial in the reflectances);
 *   dL/d hinge angle        to g_hinge (device double [n_hinges], may be NULL; at most 4 hinges,
 *                           else SRP_EUNSUPPORTED), in two parts: the pathwise part -- every path
 *                           keeps its image position and the facet hit at every interaction, and
 *                           its hit points, normals and secondary rays follow the rotation; and,
 *                           with params->edge_samples = M > 0, the visibility-edge part by edge
 *                           sampling -- for every distinct edge of a hinge-carried facet, M
 *                           stratified points along its image, each starting full paths just on
 *                           either side of it (1e-5 L away, same draws: Philox key seed ^
 *                           0x9E3779B97F4A7C15, counter (edge * M + point, direction, bounce,
 *                           design)), the jump of their deposit times the edge's normal image
 *                           velocity (silhouettes against the background or other surfaces,
 *                           occlusion, edges between facets).  Edges are numbered by first
 *                           appearance over the facets; coincident edges count once.  An edge
 *                           across which the surface continues in one plane (every facet on it
 *                           riding its hinge, one facet on each side of each layer) with equal
 *                           rho_s, rho_d and p_spec on both sides carries no jump and is skipped,
 *                           keeping its number (the first edge-sampled call after a change of the
 *                           scene synchronises `stream` once to classify the edges).  Left out:
 *                           visibility edges of reflected light, and the dependence of the grid
 *                           frame on the design (the estimator's expectation does not depend on
 *                           it).  With edge terms, at most 65535 directions per call.
 * Gradients are summed in FP64 (wavefront-aggregated atomics per facet, fixed-order sums per
 * direction for the hinges) and rounded to float for g_rho_s and g_rho_d.  Uses scene workspace;
 * calls on the same scene must be ordered on one stream. */
srp_status srp_trace_adjoint(srp_scene scene, const double* sun_dirs, int64_t D, const srp_trace_params* params,
                             const double* frames, const double* g_force, const double* g_torque, float* g_rho_s,
                             float* g_rho_d, double* g_hinge, void* stream);

/* Path records: the forward keeps the facet sequence of every traced path so that the adjoint
 * (paper Sec. 3.4, same gradients as srp_trace_adjoint) does not walk the BVH a second time.
 *
 * srp_path_record_bytes: size of the record for D directions and these params, host int64:
 *   D x bounces x ceil(nu/8) x ceil(nv/8) x 64 x 4 bytes (one int32 per traced interaction slot;
 *   about 3.2 GB for 1024 directions at 512 x 512 and 3 bounces).
 * srp_trace_recorded: srp_trace (same arguments, same paths; its own kernel, so force and torque
 *   agree with srp_trace's to FP32 rounding, not bit for bit) that also writes the record into
 *   `paths` (device, caller-owned, at least srp_path_record_bytes bytes, layout private to the
 *   library).  Only the slots of paths that were traced are written.
 * srp_trace_adjoint_recorded: srp_trace_adjoint with the same arguments, taking each path's
 *   facets from `paths` and recomputing each hit with the same ray-triangle test: every path adds
 *   the same terms, summed in another order (per workgroup in LDS first, then one FP64 atomic per
 *   facet and workgroup), so the gradients agree with srp_trace_adjoint's to rounding.  `paths`
 *   must come from the LAST srp_trace_recorded on this scene, with no design,
 *   vertex, Phong or BVH change since, and the same sun_dirs pointer, D, params (every field; the
 *   ray_mask pointer) and, with frame_mode 1, frames pointer: otherwise SRP_EINVAL.  The contents
 *   behind those pointers are the caller's to keep unchanged; a record that does not match them
 *   gives wrong gradients (indices are range-checked, so never an out-of-bounds read).
 * Paths of at most 3 interactions (params->bounces <= 3, else SRP_EUNSUPPORTED).
 * Errors as srp_trace / srp_trace_adjoint, plus SRP_EINVAL for a NULL or too small record. */
srp_status srp_path_record_bytes(srp_scene scene, int64_t D, const srp_trace_params* params, int64_t* bytes);
srp_status srp_trace_recorded(srp_scene scene, const double* sun_dirs, int64_t D, const srp_trace_params* params,
                              const double* frames, double* force, double* torque, int32_t* paths,
                              int64_t paths_bytes, void* stream);
srp_status srp_trace_adjoint_recorded(srp_scene scene, const double* sun_dirs, int64_t D,
                                      const srp_trace_params* params, const double* frames, const double* g_force,
                                      const double* g_torque, const int32_t* paths, int64_t paths_bytes,
                                      float* g_rho_s, float* g_rho_d, double* g_hinge, void* stream);

/* Traversal statistics for the bandwidth model: a host-side single-ray depth-first closest-hit
 * traversal (nearer child first) of this scene's BVH on the same rays as srp_trace, for every
 * pixel_stride-th pixel of each direction.  sun_dirs and frames are HOST arrays here.
 * out host double [6]: primary rays, ray segments (traversals), BVH nodes fetched, triangles
 * tested, surface hits, primary rays that hit the scene.  Synchronous; reads the materials back
 * from the device.  A ray_mask in params is rejected (SRP_EUNSUPPORTED). */
srp_status srp_scene_ray_stats(srp_scene scene, const double* sun_dirs, int64_t D, const srp_trace_params* params,
                               const double* frames, int64_t pixel_stride, double* out);

/* Batched designs (paper Sec. 3.2, "Estimation": samples are drawn over many designs at once): one
 * launch traces S scenes for the same D sun directions (device double [D][3]).  Design s uses
 * Philox design index params->design_index + s and its own mesh-derived frames (frame_mode must be
 * 0).  force, torque: device double [S][D][3] (torque may be NULL).  The (design, direction) units
 * are traced design-major, each direction of a design on one XCD and a design's directions spread
 * over all of them, so the XCDs work through the designs together.  Workspace belongs to
 * scenes[0]; all scenes must be on the current device.  The design table is uploaded on `stream`
 * from pinned staging; a call waits for the previous batch upload led by the same scene before
 * reusing the staging. */
srp_status srp_batch_trace(const srp_scene* scenes, int32_t S, const double* sun_dirs, int64_t D,
                           const srp_trace_params* params, double* force, double* torque, void* stream);

/* Surface-sampling estimator (paper Sec. 3.2, "Estimation", and its equation for F): for each of the
 * S scenes and D sun directions (device double [D][3]), n_samples samples, each a facet drawn by area
 * and a uniform point on it whose arriving light is gathered by path tracing with next-event
 * estimation toward the Sun at every vertex (at most bounces - 1 gathered vertices), converted to
 * force with one sampled outgoing event (specular with weight rho_s/p_s, else a cosine direction with
 * rho_d/(1 - p_s)).  Specular events follow each facet's Phong lobe (srp_scene_set_phong: the lobe
 * is importance-sampled about the mirror direction, weight (m + 2)/(m + 1) (n.o)+; sunlight a
 * gathered vertex reflects into its lobe is added by next-event estimation) or the ideal mirror.  force, torque (nullable): device double [S][D][3], sample means.  Scene s uses
 * Philox design index params->design_index + s; counters (sample, global direction, stage,
 * design).  brute_force = 1 tests every ray against every triangle of its scene (any tree depth);
 * 0 walks each scene's BVH (SRP_EUNSUPPORTED for trees deeper than 24).  Sunlight whose first
 * reflection is an ideal mirror is not gathered (a delta light through a delta reflection); all
 * other light has the expectation of srp_trace with the same `bounces` (for scenes of mirrors).  Optional per-sample
 * records, device int32: rec_facet [S][D][n_samples] (original facet), rec_lit [S][D][n_samples]
 * (bit 0: x sunlit, bit k: gathered vertex k sunlit; required with rec_facet), rec_hits
 * [S][D][n_samples][bounces - 1] (original facet of each gathered vertex, -1 none).  params: nu,
 * nv, jitter, frame_mode and tiles_per_wave are ignored.  Scene table staged like srp_batch_trace. */
srp_status srp_surface_estimate(const srp_scene* scenes, int32_t S, const double* sun_dirs, int64_t D,
                                int64_t n_samples, const srp_trace_params* params, int32_t brute_force, double* force,
                                double* torque, int32_t* rec_facet, int32_t* rec_hits, int32_t* rec_lit,
                                void* stream);

/* Multi-world surface sampling (paper Sec. 3.2, "Estimation": the samples are drawn over random
 * designs, so each sample's rays meet a different world and every ray is tested against every
 * triangle): n_pairs (sun direction, design) pairs, each answered by `samples` samples of the
 * estimator of srp_surface_estimate on its own design.  A design turns the scene's hinged parts
 * from the REST pose (srp_scene_create / srp_scene_set_vertices; the scene's own hinge angles,
 * materials and Phong exponents are not used) and gives every facet the materials of its group.
 *   facet_group host int32 [n_tris] (original facet order), groups 0 .. n_groups - 1, n_groups <= 64;
 *   sun_dirs    device double [n_pairs][3];
 *   designs     device float [n_pairs][n_hinges + 3 n_groups]: the hinge angles (rad), then for
 *               each group rho_s, rho_d and the Phong exponent (>= 1, +infinity: ideal mirror);
 *               the specular-sampling probability follows srp_scene_set_design's default rule;
 *   force, torque (nullable): device double [n_pairs][3], each pair's sample mean;
 *   records (optional, as for srp_surface_estimate): rec_facet, rec_lit [n_pairs][samples],
 *   rec_hits [n_pairs][samples][bounces - 1].
 * Pair i draws the samples that srp_surface_estimate draws for direction index dir_index_base + i
 * and design index params->design_index (counters (sample, dir_index_base + i, stage, design)).  A
 * lane turns its rays into each part's rest frame instead of moving the part, so all lanes share
 * the rest-pose records.  params: bounces, flux, seed, dir_index_base, design_index and sampling
 * are used.  Uses scene workspace (24 bytes per sample); synchronises `stream` twice (the check of
 * the designs).  Errors: SRP_EINVAL (sizes, groups, a design's materials out of range or a hinge
 * angle not finite), SRP_EUNSUPPORTED (more than 4 hinges, or a facet spanning a hinge and the
 * body). */
srp_status srp_surface_designs(srp_scene scene, const int32_t* facet_group, int32_t n_groups, const double* sun_dirs,
                               const float* designs, int64_t n_pairs, int32_t samples,
                               const srp_trace_params* params, double* force, double* torque, int32_t* rec_facet,
                               int32_t* rec_hits, int32_t* rec_lit, void* stream);

/* Launch-shape autotuner (not part of the paper's method): traces the given workload once per
 * candidate tiles_per_wave in 8..16 (S == 1: srp_trace of scenes[0]; S > 1: srp_batch_trace), after
 * one warm-up run each, and returns the fastest in *best; ms_out (host double [9], nullable)
 * receives every candidate's time in ms.  params->tiles_per_wave is ignored.  Pass a
 * representative subset of the directions: the call runs 18 traces.  Synchronous; allocates a
 * temporary force buffer.  Errors as for srp_trace / srp_batch_trace. */
srp_status srp_autotune_tiles_per_wave(const srp_scene* scenes, int32_t S, const double* sun_dirs, int64_t D,
                                       const srp_trace_params* params, int32_t* best, double* ms_out,
                                       void* stream);

/* Rebuilds the scene's BVH on the GPU from its current geometry (linear BVH, Karras, HPG 2012:
 * Morton codes of the triangle centroids, radix sort, parallel radix-tree construction, bottom-up
 * boxes; subtrees of at most 4 triangles become leaves; nodes in pre-order).  Replaces the tree
 * built at creation (binned SAH on the host): traces give the same hits, as the closest hit with its
 * index tie-break does not depend on the tree.  Later hinge changes refit the new tree.  At least
 * 8 triangles; SRP_EUNSUPPORTED when the tree would exceed the traversal stack.  Synchronous on
 * `stream`; the build workspace (about 250 bytes per triangle plus the sort's) stays with the scene
 * for later rebuilds.  *n_nodes_out, *depth_out (nullable): the new tree.  The paper's simulation
 * evaluation (BVH-comparison figure) times a linear-BVH build against brute-force intersection
 * per design; this build is what that comparison takes on this GPU. */
srp_status srp_scene_build_gpu(srp_scene scene, int32_t* n_nodes_out, int32_t* depth_out, void* stream);

srp_status srp_scene_destroy(srp_scene scene);

/* ---------------------------------------------------------------------------------------------
 * Force surrogate (paper Sec. 3.3, "Representation": an MLP maps light direction and design
 * parameters to force and is trained with Adam on simulator samples).  Layers:
 * n_in -> width (SiLU) -> ... depth hidden layers ... -> n_out (linear).  Parameters are FP32
 * masters in the flat order W0 [width][n_in], b0 [width], W1, b1, ..., W_out [n_out][width],
 * b_out [n_out].  Products use BF16 operands (round to nearest even) with FP32 accumulation;
 * bias, SiLU and gradients dL/dz are FP32 and are rounded to BF16 where they enter a product.
 * Initial weights: U(-1/sqrt(fan_in), 1/sqrt(fan_in)) from Philox draws keyed by `seed`.
 * ------------------------------------------------------------------------------------------- */
typedef struct srp_mlp_s* srp_mlp;

/* 1 <= n_in, n_out <= 64; 1 <= depth <= 16; width a multiple of 8 in [8, 4096]. */
srp_status srp_mlp_create(int32_t n_in, int32_t width, int32_t depth, int32_t n_out, uint64_t seed, srp_mlp* out);

srp_status srp_mlp_num_params(srp_mlp mlp, int64_t* n);

/* y = MLP(x): x device float [N][n_in], y device float [N][n_out].  keep_activations = 1 keeps
 * the pre-activations and BF16 activations for a following srp_mlp_backward on the same x and N
 * (library-owned workspace); 0 runs the inference path. */
srp_status srp_mlp_forward(srp_mlp mlp, const float* x, int64_t N, float* y, int32_t keep_activations, void* stream);

/* The surrogate as the paper uses its proxy (Sec. 3.3: the network answers force queries in place
 * of the simulator), with the simulator kept as fallback: two independently trained networks a and
 * b of the same shape (n_in >= 3) evaluate x device float [N][n_in] -- the sun unit vector, then the
 * design inputs scaled to [-1, 1] -- and the call writes
 *   y         device float [N][n_out]: out_scale * (y_a + y_b) / 2;
 *   disagree  device float [N] or NULL: ||y_a - y_b|| in network units;
 *   fail_idx  device int32 [N]: in ascending order, the queries that fail the confidence test --
 *             outside the training domain (| ||x[0:3]|| - 1 | > 1e-5 or |x_i| > 1 + 1e-6 for a
 *             design input) or disagreement above `threshold` (NaN fails everything);
 *   n_fail    device int32 [1]: their number (entries of fail_idx beyond it are unspecified).
 * The caller traces the failing queries (srp_trace) and overwrites their rows of y.  Workspace
 * (both networks' outputs, flags, compaction scratch) belongs to network a; calls using a must be
 * ordered.  0 <= N <= 2^30. */
srp_status srp_mlp_ensemble(srp_mlp a, srp_mlp b, const float* x, int64_t N, float threshold, float out_scale,
                            float* y, float* disagree, int32_t* fail_idx, int32_t* n_fail, void* stream);

/* Back-propagates g_y = dL/dy (device float [N][n_out]) through the kept activations: weight and
 * bias gradients are ADDED to the library's gradient buffer; g_x (device float [N][n_in], may be
 * NULL) receives dL/dx. */
srp_status srp_mlp_backward(srp_mlp mlp, const float* g_y, int64_t N, float* g_x, void* stream);

/* Adam (Kingma & Ba 2015) with bias correction on the FP32 masters, then clears the gradients
 * and refreshes the BF16 copies. */
srp_status srp_mlp_adam_step(srp_mlp mlp, float lr, float beta1, float beta2, float eps, void* stream);

srp_status srp_mlp_zero_grad(srp_mlp mlp, void* stream);

/* Mean squared error over the N x n_out entries: loss (device double [1]) and
 * g_y = 2 (y - target) / (N n_out) (device float [N][n_out]). */
srp_status srp_mlp_mse(srp_mlp mlp, const float* y, const float* target, int64_t N, float* g_y, double* loss,
                       void* stream);

/* Checkpoint / resume: host float arrays [n] (n = srp_mlp_num_params; any pointer may be NULL) of
 * the masters, gradients (get only), Adam moments, and the Adam step count.  Synchronous. */
srp_status srp_mlp_get_params(srp_mlp mlp, float* params, float* grads, float* adam_m, float* adam_v, int64_t* step,
                              int64_t n);
srp_status srp_mlp_set_params(srp_mlp mlp, const float* params, const float* adam_m, const float* adam_v,
                              int64_t step, int64_t n);

srp_status srp_mlp_destroy(srp_mlp mlp);

/* ---------------------------------------------------------------------------------------------
 * Orbit integration (paper Sec. 3.4.1, Eq. ODE, translational part; Sec. 3.4.3, adjoint).  Host
 * FP64, classic fourth-order Runge-Kutta with step dt over n_steps steps of
 *   dr/dt = v,  dv/dt = -mu r / |r|^3 + R_k F_k / mass,
 * where F_body [2 n_steps + 1][3] holds the body-frame SRP force at the stage times t_k = k dt / 2
 * (step n uses k = 2n, 2n+1, 2n+1, 2n+2) and R_body_to_inertial [2 n_steps + 1][9] the attitude
 * (row-major 3x3) at those times.  The attitude is a function of time only.
 * ------------------------------------------------------------------------------------------- */

/* z0 [6] = (r, v) in m and m/s; z_all [n_steps + 1][6] may be NULL; z_final [6]. */
srp_status srp_orbit_rk4(const double* z0, double mu, double mass, double dt, int64_t n_steps, const double* F_body,
                         const double* R_body_to_inertial, double* z_all, double* z_final);

/* Discrete adjoint of srp_orbit_rk4: for g_final = dL/dz_N [6] returns g_F = dL/dF_body
 * [2 n_steps + 1][3] (overwritten) and g_z0 = dL/dz0 [6] (may be NULL).  The forward states are
 * kept only every ckpt_every steps; each segment is recomputed from its checkpoint during the
 * reverse sweep. */
srp_status srp_orbit_rk4_adjoint(const double* z0, double mu, double mass, double dt, int64_t n_steps,
                                 const double* F_body, const double* R_body_to_inertial, const double* g_final,
                                 int64_t ckpt_every, double* g_F, double* g_z0);

/* ------------------------------------------------------------------------------------------- *
 * Orbit and attitude together (paper Sec. 3.4.1, Eq. ODE, the 13-D state): many trajectories at
 * once on the GPU, classic RK4 in FP64, with the force AND torque of every stage taken from a
 * network (the proxy of Sec. 3.3) evaluated at the stage's body-frame Sun direction:
 *   dr/dt = v,
 *   dv/dt = -mu r / |r|^3 + nu R(q) F / mass,
 *   dq/dt = 1/2 q (x) (0, w),
 *   dw/dt = I^-1 (nu tau - w x (I w)),
 * with q = (q0, q1, q2, q3) scalar first, R(q) the rotation of q / |q| (body -> inertial; the
 * state quaternion is not renormalised), w the body-frame angular velocity, s_body = R(q)^T sun,
 * network input x = [float(s_body), design row] and output y: F = force_scale y[0..2] (N, body
 * frame), tau = torque_scale y[3..5] (N m, body frame).  nu is the cylinder eclipse factor: 0 when
 * r . sun < 0 and |r - (r . sun) sun| < earth_radius, else 1 (earth_radius 0: always 1).
 * ------------------------------------------------------------------------------------------- */
typedef struct srp_attitude_params {
    double mu;            /* gravitational parameter, m^3 / s^2, > 0 */
    double mass;          /* kg, > 0 */
    double inertia[9];    /* body-frame inertia tensor, kg m^2, row-major, symmetric positive definite */
    double sun[3];        /* direction toward the Sun, inertial frame (normalised here), fixed */
    double force_scale;   /* N per unit of network outputs 0..2 */
    double torque_scale;  /* N m per unit of network outputs 3..5 */
    double earth_radius;  /* m; 0 disables the eclipse */
    double dt;            /* step, s, > 0 */
    int64_t n_steps;      /* >= 0 */
    int64_t steps_per_design; /* 0: one design row per trajectory for the whole run; L > 0: the design
                                 changes over time (e.g. panel angles), row min(n / L, S - 1) of a
                                 [S][B][n_in - 3] schedule, S = max(1, ceil(n_steps / L)), for step n */
} srp_attitude_params;

/* Integrates B trajectories: z0 and z_final device double [B][13] (r, v, q, w; SI units),
 * design device float [B][n_in - 3], or [S][B][n_in - 3] with steps_per_design (NULL when the
 * network has 3 inputs), z_all device double
 * [n_steps + 1][B][13] or NULL.  The network (n_in >= 3, n_out >= 6; extra outputs ignored)
 * answers 4 n_steps batched queries; its inference path is used, and the integration state lives
 * in a workspace the network owns (about 360 + 4 n_in bytes per trajectory), so calls that use one
 * network must be ordered on one stream.  Asynchronous on `stream`; z0 may alias z_final.  Every
 * trajectory must keep r != 0 and q != 0 (no device check).  Errors: SRP_EINVAL (sizes, params,
 * inertia not symmetric positive definite, network shape). */
srp_status srp_attitude_rk4(srp_mlp model, const srp_attitude_params* params, const double* z0,
                            const float* design, int64_t B, double* z_final, double* z_all, void* stream);

/* Waits for `stream` and reports any pending device error as SRP_EDEVICE. */
srp_status srp_sync(void* stream);

const char* srp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SRP_H */
