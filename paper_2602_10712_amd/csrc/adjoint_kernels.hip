// Adjoint of the ray-grid SRP estimator (reverse mode in the reflectances, forward mode in the
// hinge angles), gfx950.
//
// The paper differentiates only its neural proxy and notes that the simulator itself is
// differentiable for continuous parameters away from visibility discontinuities (Sec. 3.3 and
// Sec. 4.2, "differentiable by construction").  This kernel differentiates the ray-grid estimator
// directly.  It replays every path of the forward trace with the same Philox counters, the same
// traversal and the same interaction arithmetic (so it visits the same facets), and for
// L = sum_j gF_j . F_j + gT_j . tau_j accumulates:
//
//  * dL/d rho_s[f], dL/d rho_d[f]: with the counters and the specular-sampling probabilities
//    frozen, a path's contribution is a polynomial in the event factors k_b = rho_s/p_s (mirror) or
//    rho_d/(1 - p_s) (Lambertian) and, at its last interaction, linear in (rho_s, rho_d).  The
//    products that leave one factor out are carried forward per interaction slot, so no division
//    by k occurs.  Per-facet sums use wavefront-aggregated FP64 atomics.
//
//  * dL/d theta_h (hinge angles), pathwise part: forward-mode tangents with each path at its image
//    position and its facet sequence frozen.  Hit points slide along the ray onto the turned facet
//    planes, normals and mirror directions turn, the Lambertian direction follows the basis of the
//    turned normal, and the secondary origin x + eps n follows the hit point and the normal.  The
//    primary-visibility edges of the moving facets add the boundary part (edge_kernels.hip); the
//    secondary-visibility edges and the grid frame's own dependence on the design are excluded.
#include <float.h>

#include "srp_internal.h"
#include "srp_path.h"
#include "srp_traverse.h"

namespace srp {
namespace {


SRP_HD void cross3f(const float a[3], const float b[3], float r[3])
{
    r[0] = a[1] * b[2] - a[2] * b[1];
    r[1] = a[2] * b[0] - a[0] * b[2];
    r[2] = a[0] * b[1] - a[1] * b[0];
}
SRP_HD float dot3f(const float a[3], const float b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Derivative of the Duff et al. basis (b1, b2) of n along the normal's derivative nd.
SRP_HD void duff_basis_tangent(const float n[3], const float nd[3], float b1d[3], float b2d[3])
{
    const float s = n[2] >= 0.0f ? 1.0f : -1.0f;
    const float a = -1.0f / (s + n[2]);
    const float ad = a * a * nd[2];
    b1d[0] = s * (2.0f * n[0] * nd[0] * a + n[0] * n[0] * ad);
    b1d[1] = s * (nd[0] * n[1] * a + n[0] * nd[1] * a + n[0] * n[1] * ad);
    b1d[2] = -s * nd[0];
    b2d[0] = nd[0] * n[1] * a + n[0] * nd[1] * a + n[0] * n[1] * ad;
    b2d[1] = 2.0f * n[1] * nd[1] * a + n[1] * n[1] * ad;
    b2d[2] = -nd[1];
}

// Adds val into base[key] for every lane with `active`.  Lanes of a coherent tile mostly hit the
// same few facets: up to kScatterGroups keys shared by several lanes are summed across the wave
// first (one FP64 atomic per key); the remaining lanes, whose keys are scattered, add their own
// values with one atomic each.
constexpr int kScatterGroups = 4;

__device__ __forceinline__ void wave_scatter_add(double* base, bool active, int key, float val)
{
    const int lane = threadIdx.x & 63;
    uint64_t pending = wave_ballot(active);
    for (int it = 0; it < kScatterGroups && pending; ++it) {
        const int leader = __ffsll(static_cast<unsigned long long>(pending)) - 1;
        const int k = __shfl(key, leader, 64);
        const bool match = active && key == k;
        const uint64_t group = wave_ballot(match);
        if ((group & (group - 1)) == 0) break;  // the leader's key is its own: no sharing to exploit
        const float sum = wave_sum(match ? val : 0.0f);
        if (lane == leader) atomicAdd(base + k, static_cast<double>(sum));
        active = active && !match;
        pending = wave_ballot(active);
    }
    if (active) atomicAdd(base + key, static_cast<double>(val));
}

// Workgroup-level gradient table (used where the adjoint does not walk the BVH, which leaves its
// LDS free): open addressing over kTableSize slots of (key, FP64 sum); the wave's pre-summed values
// are added there with LDS atomics, and the table goes to the global gradient with one FP64 atomic
// per distinct key when the workgroup ends.  A key that finds no slot within kTableProbes probes
// goes straight to the global gradient.
constexpr int kTableSize = 2048;
constexpr int kTableProbes = 8;

struct GradTable {
    int key[kTableSize];
    double val[kTableSize];
};

__device__ __forceinline__ void table_add(GradTable& T, double* base, int key, double v)
{
    uint32_t h = (static_cast<uint32_t>(key) * 0x9E3779B1u) >> (32 - 11);  // 11 bits: kTableSize
    for (int p = 0; p < kTableProbes; ++p) {
        const int slot = static_cast<int>((h + p) & (kTableSize - 1));
        const int prev = atomicCAS(&T.key[slot], -1, key);
        if (prev == -1 || prev == key) {
            atomicAdd(&T.val[slot], v);
            return;
        }
    }
    atomicAdd(base + key, v);
}

// The workgroup's table in LDS (only kernels that use it allocate it).
template <bool REC>
__device__ __forceinline__ GradTable* grad_table()
{
    return nullptr;
}
template <>
__device__ __forceinline__ GradTable* grad_table<true>()
{
    __shared__ GradTable t;
    return &t;
}

// wave_scatter_add into the workgroup table instead of the global gradient.
__device__ __forceinline__ void wave_table_add(GradTable& T, double* base, bool active, int key, float val)
{
    const int lane = threadIdx.x & 63;
    uint64_t pending = wave_ballot(active);
    for (int it = 0; it < kScatterGroups && pending; ++it) {
        const int leader = __ffsll(static_cast<unsigned long long>(pending)) - 1;
        const int k = __shfl(key, leader, 64);
        const bool match = active && key == k;
        const uint64_t group = wave_ballot(match);
        if ((group & (group - 1)) == 0) break;
        const float sum = wave_sum(match ? val : 0.0f);
        if (lane == leader) table_add(T, base, k, static_cast<double>(sum));
        active = active && !match;
        pending = wave_ballot(active);
    }
    if (active) table_add(T, base, key, static_cast<double>(val));
}

// MAXH: hinge tangents carried (0, 2 or 4); NS: non-final interaction slots per path (bounces - 1
// at most), so that paths of up to 3 bounces keep only two slots in registers.
//
// The scene arrays, frames, cotangents and the written gradient arrays also come as separate
// __restrict__ parameters: the atomics then provably leave the inputs untouched, so node and
// triangle records of the coherent walk, the frame and the cotangents can still be fetched through
// the scalar cache into scalar registers.
//
// REC: the facet of every interaction comes from the forward's path record (TraceArgs::path_hit)
// instead of a second BVH walk; the hit distance is recomputed with the same triangle test on the
// same ray, so every quantity equals the walking replay's.  A recorded index outside the scene is
// taken as a miss (the record belongs to another call).
template <int MAXH, int NS, bool REC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_adjoint(
    AdjointArgs A, const BvhNode* __restrict__ nodes,
                                                 const TriRec* __restrict__ tris, const float4* __restrict__ mat,
                                                 const DevFrame* __restrict__ frames,
                                                 const double* __restrict__ g_force,
                                                 const double* __restrict__ g_torque, double* __restrict__ g_rho,
                                                 double* __restrict__ hinge_partials)
{
    const TraceArgs& a = A.t;
    __shared__ int s_stack[REC ? 1 : kWaves][REC ? 1 : kStackDepth];
    __shared__ int s_lane[REC ? 1 : kWaves][REC ? 1 : kLaneStack][64];
    __shared__ float s_red[kWaves][MAXH > 0 ? MAXH : 1];
    __shared__ float4 s_rect[kCullBoxes];
    __shared__ uint64_t s_live;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int64_t j;
    int32_t blk;
    if (!block_unit(a, a.D, blockIdx.x, j, blk)) return;  // whole workgroup: grid padding
    GradTable* table = grad_table<REC>();
    if (REC) {
        for (int i = threadIdx.x; i < kTableSize; i += 64 * kWaves) {
            table->key[i] = -1;
            table->val[i] = 0.0;
        }
        __syncthreads();
    }
    const DevFrame fr = frames[j];
    const uint32_t dir_global = static_cast<uint32_t>(a.dir_index_base + j);
    int* stack = s_stack[REC ? 0 : wave];
    int* lstack = &s_lane[REC ? 0 : wave][0][lane];
    const float gF[3] = {static_cast<float>(g_force[3 * j]), static_cast<float>(g_force[3 * j + 1]),
                         static_cast<float>(g_force[3 * j + 2])};
    float gT[3] = {0.0f, 0.0f, 0.0f};
    if (g_torque)
        for (int c = 0; c < 3; ++c) gT[c] = static_cast<float>(g_torque[3 * j + c]);
    const int H = A.n_hinges < MAXH ? A.n_hinges : MAXH;

    float accH[MAXH > 0 ? MAXH : 1];
    for (int h = 0; h < (MAXH > 0 ? MAXH : 1); ++h) accH[h] = 0.0f;

    // the workgroup's tiles that may contain a hit
    uint64_t live = ~0ull;
    if (a.cull) {
        if (threadIdx.x < kCullBoxes) s_rect[threadIdx.x] = cull_rect(nodes, fr, threadIdx.x);
        __syncthreads();
        if (wave == 0) {
            const uint64_t mk = live_tiles(a, s_rect, static_cast<int64_t>(blk) * a.tiles_per_wave * kWaves,
                                           a.tiles_per_wave * kWaves);
            if (lane == 0) s_live = mk;
        }
        __syncthreads();
        live = s_live;
    }

    for (int m = 0; m < a.tiles_per_wave; ++m) {
        const int64_t tile = (static_cast<int64_t>(blk) * a.tiles_per_wave + m) * kWaves + wave;
        if (tile >= a.tiles_per_dir) break;
        if (((live >> (m * kWaves + wave)) & 1ull) == 0) continue;
        int64_t pixel, rec;
        int32_t pi, pk;
        const bool valid = tile_pixel<false>(a, tile, lane, pixel, rec, pi, pk);
        float o[3], d[3];
        primary_ray(fr, pi, pk, static_cast<uint32_t>(pixel), dir_global, a.design_index, a.seed_lo, a.seed_hi,
                    a.jitter != 0, o, d);
        float w = fr.w;
        bool alive = valid;
        if (a.ray_mask && valid && ray_masked(a, j, pixel)) alive = false;  // a left-out path adds nothing
        int skip = -1;
        // recorded triangles of the path's interactions (at most kRecordBounces), fetched together
        int ph0 = -1, ph1 = -1, ph2 = -1;
        if (REC && alive) {
            ph0 = a.path_hit[path_slot(a, j, 1, tile, lane)];
            if (a.bounces >= 2) ph1 = a.path_hit[path_slot(a, j, 2, tile, lane)];
            if (a.bounces >= 3) ph2 = a.path_hit[path_slot(a, j, 3, tile, lane)];
        }

        // reflectance adjoint state
        float R[NS], Acc[NS], inv[NS];
        int fac[NS], arr[NS];
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            R[i] = 0.0f;
            Acc[i] = 0.0f;
            inv[i] = 0.0f;
            fac[i] = 0;
            arr[i] = 0;
        }
        int K = 0;
        int touched = 0;  // bit h: the path has met a facet that hinge h turns
        int term_f = -1;
        float term_s = 0.0f, term_d = 0.0f;
        // hinge tangents: origin Od, direction Dd, accumulated dL
        float Od[MAXH > 0 ? MAXH : 1][3], Dd[MAXH > 0 ? MAXH : 1][3], Ld[MAXH > 0 ? MAXH : 1];
#pragma unroll
        for (int h = 0; h < (MAXH > 0 ? MAXH : 1); ++h) {
            for (int c = 0; c < 3; ++c) {
                Od[h][c] = 0.0f;
                Dd[h][c] = 0.0f;
            }
            Ld[h] = 0.0f;
        }

        for (int b = 1; b <= a.bounces; ++b) {
            if (wave_ballot(alive) == 0) break;
            float t = -1.0f;
            int hit = -1;
            if (REC) {
                if (alive) {
                    hit = b == 1 ? ph0 : b == 2 ? ph1 : ph2;
                    if (hit >= A.n_tris || hit < -1) hit = -1;
                    if (hit >= 0) {
                        const TriRec* T = tris + hit;
                        t = tri_hit(o, d, T->f[0], T->f[1], T->f[2]);
                    }
                }
            } else if (b == 1) {
                closest_hit_parallel(nodes, tris, o, d, alive, skip, t, hit, stack, fr.d);
            } else if (!a.lane_walk) {
                closest_hit(nodes, tris, o, d, alive, skip, t, hit, stack);
            } else {
                closest_hit_lane(nodes, tris, o, d, alive, skip, t, hit, lstack);
            }
            if (!alive) continue;
            if (hit < 0) {
                alive = false;
                continue;
            }
            const TriRec tr = tris[hit];
            const float4 mt = mat[hit];
            const float n[3] = {tr.f[1].w, tr.f[2].w, tr.f[3].x};
            const float v0[3] = {tr.f[0].x, tr.f[0].y, tr.f[0].z};
            const int fid = __float_as_int(tr.f[0].w);
            const int hid = __float_as_int(tr.f[3].y);
            const float d_in[3] = {d[0], d[1], d[2]};
            float x[3], g[3];
            InteractInfo inf;
            alive = interact_ex(o, d, w, t, n, mt.x, mt.y, mt.z, b, a.bounces, static_cast<uint32_t>(pixel),
                                dir_global, a.design_index, a.seed_lo, a.seed_hi, a.eps, x, g, &inf);
            const float l[3] = {x[0] - a.com[0], x[1] - a.com[1], x[2] - a.com[2]};
            float G[3];
            cross3f(gT, l, G);
            for (int c = 0; c < 3; ++c) G[c] += gF[c];

            // ---- reflectances: coefficient of the current weight W_K from the incident term
            const float cin = dot3f(G, d_in);
#pragma unroll
            for (int i = 0; i < NS; ++i)
                if (i < K) Acc[i] += R[i] * cin;
            if (inf.last) {
                const float tr_ = dot3f(G, inf.r), tn_ = dot3f(G, n);
                const float term = -(mt.x * tr_ + (2.0f / 3.0f) * mt.y * tn_);
#pragma unroll
                for (int i = 0; i < NS; ++i)
                    if (i < K) Acc[i] += R[i] * term;
                term_f = fid;
                term_s = -inf.w_in * tr_;
                term_d = -inf.w_in * (2.0f / 3.0f) * tn_;
            } else {
                // new slot K with factor k; R_i *= k for the older slots, R_K = W before it
#pragma unroll
                for (int i = 0; i < NS; ++i) {
                    if (i < K) R[i] *= inf.k;
                    if (i == K) {
                        R[i] = inf.w_in;
                        fac[i] = fid;
                        arr[i] = inf.mirror ? 0 : 1;
                        inv[i] = inf.mirror ? 1.0f / mt.z : 1.0f / (1.0f - mt.z);
                    }
                }
                const float cout = -dot3f(G, d);  // coefficient of the new weight: -G . o_b (d is o_b now)
#pragma unroll
                for (int i = 0; i < NS; ++i)
                    if (i <= K) Acc[i] += R[i] * cout;
                ++K;
            }

            // ---- hinge tangents.  A path that has met no facet of hinge h carries exactly zero
            // tangents for it and adds a signed zero, so a wave none of whose paths has skips h.
            if (hid >= 0 && hid < MAXH) touched |= 1 << hid;
#pragma unroll
            for (int h = 0; h < (MAXH > 0 ? MAXH : 1); ++h) {
                if (h >= H) continue;
                if (wave_ballot((touched >> h) & 1) == 0) continue;
                float nd[3] = {0.0f, 0.0f, 0.0f}, pd[3] = {0.0f, 0.0f, 0.0f};
                if (hid == h) {
                    const float* ax = A.hinge_axis[h];
                    const float rel[3] = {v0[0] - A.hinge_origin[h][0], v0[1] - A.hinge_origin[h][1],
                                          v0[2] - A.hinge_origin[h][2]};
                    cross3f(ax, n, nd);
                    cross3f(ax, rel, pd);
                }
                const float xp[3] = {x[0] - v0[0], x[1] - v0[1], x[2] - v0[2]};
                float q[3];
                for (int c = 0; c < 3; ++c) q[c] = Od[h][c] + t * Dd[h][c] - pd[c];
                const float td = -(dot3f(nd, xp) + dot3f(n, q)) / dot3f(n, d_in);
                float xd[3];
                for (int c = 0; c < 3; ++c) xd[c] = Od[h][c] + td * d_in[c] + t * Dd[h][c];
                const float cd = -(dot3f(Dd[h], n) + dot3f(d_in, nd));
                float rd[3];
                for (int c = 0; c < 3; ++c) rd[c] = Dd[h][c] + 2.0f * (cd * n[c] + inf.cth * nd[c]);
                float gd[3];
                for (int c = 0; c < 3; ++c) gd[c] = inf.w_in * Dd[h][c];
                float odd[3] = {0.0f, 0.0f, 0.0f};
                if (inf.last) {
                    for (int c = 0; c < 3; ++c) gd[c] -= inf.w_in * (mt.x * rd[c] + (2.0f / 3.0f) * mt.y * nd[c]);
                } else if (inf.mirror) {
                    for (int c = 0; c < 3; ++c) {
                        odd[c] = rd[c];
                        gd[c] -= inf.w_out * rd[c];
                    }
                } else {
                    float b1d[3], b2d[3];
                    duff_basis_tangent(n, nd, b1d, b2d);
                    for (int c = 0; c < 3; ++c) {
                        odd[c] = inf.lam[0] * b1d[c] + inf.lam[1] * b2d[c] + inf.lam[2] * nd[c];
                        gd[c] -= inf.w_out * odd[c];
                    }
                }
                float c1[3], c2[3];
                cross3f(xd, g, c1);
                cross3f(l, gd, c2);
                Ld[h] += dot3f(gF, gd) + gT[0] * (c1[0] + c2[0]) + gT[1] * (c1[1] + c2[1]) + gT[2] * (c1[2] + c2[2]);
                if (!inf.last) {
                    for (int c = 0; c < 3; ++c) {
                        Od[h][c] = xd[c] + a.eps * nd[c];
                        Dd[h][c] = odd[c];
                    }
                }
            }
            skip = hit;
        }

        // ---- scatter the reflectance gradients (original facet order, FP64)
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            const bool act = valid && i < K;
            if (wave_ballot(act) == 0) break;
            if (REC)
                wave_table_add(*table, g_rho, act, arr[i] * A.n_tris + fac[i], Acc[i] * inv[i]);
            else
                wave_scatter_add(g_rho, act, arr[i] * A.n_tris + fac[i], Acc[i] * inv[i]);
        }
        const bool has_term = valid && term_f >= 0;
        if (wave_ballot(has_term)) {
            if (REC) {
                wave_table_add(*table, g_rho, has_term, term_f, term_s);
                wave_table_add(*table, g_rho, has_term, A.n_tris + term_f, term_d);
            } else {
                wave_scatter_add(g_rho, has_term, term_f, term_s);
                wave_scatter_add(g_rho, has_term, A.n_tris + term_f, term_d);
            }
        }
#pragma unroll
        for (int h = 0; h < (MAXH > 0 ? MAXH : 1); ++h)
            if (valid && h < H) accH[h] += Ld[h];
    }

    if (REC) {  // the workgroup's table into the global gradient: one FP64 atomic per distinct key
        __syncthreads();
        for (int i = threadIdx.x; i < kTableSize; i += 64 * kWaves) {
            const int k = table->key[i];
            if (k >= 0) atomicAdd(g_rho + k, table->val[i]);
        }
    }
    if (MAXH > 0) {
#pragma unroll
        for (int h = 0; h < MAXH; ++h) accH[h] = wave_sum(accH[h]);
        if (lane == 0)
            for (int h = 0; h < MAXH; ++h) s_red[wave][h] = accH[h];
        __syncthreads();
        if (threadIdx.x < MAXH) {
            double s = 0.0;
            for (int q = 0; q < kWaves; ++q) s += static_cast<double>(s_red[q][threadIdx.x]);
            hinge_partials[(j * a.blocks_per_dir + blk) * kMaxHinges + threadIdx.x] = s;
        }
    }
}

__global__ void k_fill_f64(double* __restrict__ p, int64_t n, double v)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Per-direction sums of the hinge partials (fixed order over workgroups).
__global__ void k_reduce_hinges(const double* __restrict__ hp, int64_t D, int32_t bpd, double* __restrict__ per_dir)
{
    const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (t >= D * kMaxHinges) return;
    const int64_t j = t / kMaxHinges;
    const int h = static_cast<int>(t % kMaxHinges);
    double s = 0.0;
    for (int32_t b = 0; b < bpd; ++b) s += hp[(j * bpd + b) * kMaxHinges + h];
    per_dir[t] = s;
}

__global__ void k_finish_adjoint(const double* __restrict__ g_rho, int32_t n_tris, float* __restrict__ g_rs,
                                 float* __restrict__ g_rd, const double* __restrict__ per_dir, int64_t D,
                                 int32_t n_hinges, double* __restrict__ g_hinge)
{
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n_tris) {
        if (g_rs) g_rs[i] += static_cast<float>(g_rho[i]);
        if (g_rd) g_rd[i] += static_cast<float>(g_rho[n_tris + i]);
    }
    if (i < n_hinges && g_hinge) {
        double s = 0.0;  // fixed order over directions
        for (int64_t j = 0; j < D; ++j) s += per_dir[j * kMaxHinges + i];
        g_hinge[i] += s;
    }
}

}  // namespace

namespace {

template <int MAXH, bool REC>
void launch_adjoint_h(const AdjointArgs& a, unsigned blocks, hipStream_t stream)
{
    if (a.t.bounces <= 3)
        hipLaunchKernelGGL((k_adjoint<MAXH, 2, REC>), dim3(blocks), dim3(64 * kWaves), 0, stream, a, a.t.nodes,
                           a.t.tris, a.t.mat, a.t.frames, a.g_force, a.g_torque, a.g_rho, a.hinge_partials);
    else
        hipLaunchKernelGGL((k_adjoint<MAXH, kMaxBounces - 1, REC>), dim3(blocks), dim3(64 * kWaves), 0, stream, a,
                           a.t.nodes, a.t.tris, a.t.mat, a.t.frames, a.g_force, a.g_torque, a.g_rho,
                           a.hinge_partials);
}

template <bool REC>
void launch_adjoint_rec(const AdjointArgs& a, unsigned blocks, hipStream_t stream)
{
    if (a.n_hinges == 0)
        launch_adjoint_h<0, REC>(a, blocks, stream);
    else if (a.n_hinges <= 2)
        launch_adjoint_h<2, REC>(a, blocks, stream);
    else
        launch_adjoint_h<kMaxHinges, REC>(a, blocks, stream);
}

}  // namespace

hipError_t launch_adjoint(const AdjointArgs& a, hipStream_t stream)
{
    const int64_t nb = grid_blocks(a.t, a.t.D);
    if (nb == 0) return hipSuccess;
    if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
    const unsigned blocks = static_cast<unsigned>(nb);
    if (a.t.path_hit)
        launch_adjoint_rec<true>(a, blocks, stream);
    else
        launch_adjoint_rec<false>(a, blocks, stream);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, int64_t n, double v, hipStream_t stream)
{
    if (n <= 0) return hipSuccess;
    const int threads = 256;
    hipLaunchKernelGGL(k_fill_f64, dim3(static_cast<unsigned>((n + threads - 1) / threads)), dim3(threads), 0, stream,
                       p, n, v);
    return hipGetLastError();
}

hipError_t launch_reduce_hinges(const double* hinge_partials, int64_t D, int32_t blocks_per_dir, double* per_dir,
                                hipStream_t stream)
{
    const int threads = 256;
    const int64_t nt = D * kMaxHinges;
    if (nt <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_hinges, dim3(static_cast<unsigned>((nt + threads - 1) / threads)), dim3(threads), 0,
                       stream, hinge_partials, D, blocks_per_dir, per_dir);
    return hipGetLastError();
}

hipError_t launch_finish_adjoint(const double* g_rho, int32_t n_tris, float* g_rho_s, float* g_rho_d, int64_t D,
                                 int32_t n_hinges, const double* per_dir, double* g_hinge, hipStream_t stream)
{
    const int threads = 256;
    const int64_t n = n_tris > n_hinges ? n_tris : n_hinges;
    hipLaunchKernelGGL(k_finish_adjoint, dim3(static_cast<unsigned>((n + threads - 1) / threads)), dim3(threads), 0,
                       stream, g_rho, n_tris, g_rho_s, g_rho_d, per_dir, D, n_hinges, g_hinge);
    return hipGetLastError();
}

}  // namespace srp
