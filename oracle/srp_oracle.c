/*
 * srp_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, double-precision CPU reference of the ray-grid Monte Carlo estimate of solar
 * radiation pressure (SRP) force and torque on a triangle mesh.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load this library; the product path never
 * links or calls it.  It shares no code with the GPU library: every formula here is written out
 * again from the paper and from the published methods it names.
 *
 * What it computes (paper, Sec. 3.2 "Radiation Pressure Simulation"):
 *   - Eq. (Force) / the light-to-force map l2f: a photon packet of power P arriving along the
 *     propagation direction d and leaving along o deposits (P/c)(d - o); the clamped cosine
 *     <n, w_in>+ is realised by the ray-grid footprint (rays are spaced on a plane normal to d,
 *     so each ray carries the flux through its pixel: w = Phi * du * dv / c).
 *   - F = integral over the surface, tau = integral of (x - x_COM) x f  (Sec. 3.2, force and
 *     torque integrals): every deposit is added to F and (x - x_COM) x deposit to tau.
 *   - Single distant light from one direction (Sec. 3.2, first paragraph).
 *   - Per-face materials (Sec. 3.2, "Estimation"): here ideal mirror (rho_s), Lambertian (rho_d)
 *     and absorbed (1 - rho_s - rho_d).
 *   - Light followed as a path over several surface interactions (Sec. 3.2, "Estimation").
 *   - Lambertian momentum factor 2/3 (Sec. 5.9, thermal recoil of a Lambertian emitter): the
 *     expected momentum leaving a Lambertian reflector is (2/3) rho_d n per unit incident.
 * Readings where the paper is silent (ray grid, basis, RNG, tie rules, offsets) are listed in the
 * design document; each is restated at the point of use below.
 *
 * Everything is double precision except the per-facet reflectances and specular-sampling
 * probabilities, which arrive as float32 arrays so that the specular/diffuse decision
 * (u_e < p_s) is taken on exactly the same numbers as in the GPU path.
 *
 * Pinned by tests/test_oracle_pins.py (plate and sphere closed forms, dihedral retro-reflection,
 * Lambertian 2/3 mean, invariants, intersection against numpy.linalg.solve, Philox against the
 * rocRAND library implementation).
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_EDEGENERATE (-4)

static const double kSpeedOfLight = 299792458.0; /* m/s, exact by definition */

/* ------------------------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw: "Parallel random numbers: as easy as 1, 2, 3",   */
/* SC'11).  Ten rounds of the 4x32 Philox S-box with the published multipliers and Weyl key    */
/* increments.                                                                                 */
/* ------------------------------------------------------------------------------------------ */
void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t prod_a = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t prod_b = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi_a = (uint32_t)(prod_a >> 32), lo_a = (uint32_t)prod_a;
        uint32_t hi_b = (uint32_t)(prod_b >> 32), lo_b = (uint32_t)prod_b;
        uint32_t n0 = hi_b ^ c1 ^ k0;
        uint32_t n1 = lo_b;
        uint32_t n2 = hi_a ^ c3 ^ k1;
        uint32_t n3 = lo_a;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 24 high bits -> [0, 1): exactly representable in float and double. */
static double u01(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }

static void draw4(uint64_t seed, uint32_t pixel, uint32_t dir, uint32_t bounce, uint32_t design,
                  double u[4])
{
    uint32_t ctr[4] = {pixel, dir, bounce, design};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    oracle_philox4x32_10(ctr, key, r);
    for (int i = 0; i < 4; ++i) u[i] = u01(r[i]);
}

/* ------------------------------------------------------------------------------------------ */
/* small vector helpers (double)                                                               */
/* ------------------------------------------------------------------------------------------ */
static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double a[3], const double b[3], double r[3])
{
    double x = a[1] * b[2] - a[2] * b[1];
    double y = a[2] * b[0] - a[0] * b[2];
    double z = a[0] * b[1] - a[1] * b[0];
    r[0] = x; r[1] = y; r[2] = z;
}
static void sub3(const double a[3], const double b[3], double r[3]) { r[0] = a[0] - b[0]; r[1] = a[1] - b[1]; r[2] = a[2] - b[2]; }

/* Orthonormal basis (b1, b2) completing the unit vector n to a right-handed frame
 * (b1 x b2 = n): Duff, Burgess, Christensen, Hery, Kensler, Liani, Villemin, "Building an
 * Orthonormal Basis, Revisited", JCGT 6(1), 2017.  sign(0) is taken as +1. */
void oracle_basis(const double n[3], double b1[3], double b2[3])
{
    double s = (n[2] >= 0.0) ? 1.0 : -1.0;
    double a = -1.0 / (s + n[2]);
    double b = n[0] * n[1] * a;
    b1[0] = 1.0 + s * n[0] * n[0] * a;
    b1[1] = s * b;
    b1[2] = -s * n[0];
    b2[0] = b;
    b2[1] = s + n[1] * n[1] * a;
    b2[2] = -n[1];
}

/* ------------------------------------------------------------------------------------------ */
/* Grid frame of one sun direction.                                                            */
/* Layout of a frame (12 doubles): u[3], v[3], o0[3], du, dv, unused.                          */
/* Ray origin of pixel (i, k) with in-pixel offsets (a, b):  o0 + (i + a) du u + (k + b) dv v. */
/* The rectangle spans the projections of the 8 corners of the mesh's axis-aligned bounding   */
/* box on (u, v); the entry plane sits 0.01 L in front of the nearest corner, where L is the    */
/* scene size: twice the largest distance of a vertex from the vertex mean (rotation-invariant).*/
/* ------------------------------------------------------------------------------------------ */
static void mesh_aabb(const double* verts, int64_t n_verts, double lo[3], double hi[3])
{
    for (int a = 0; a < 3; ++a) { lo[a] = INFINITY; hi[a] = -INFINITY; }
    for (int64_t i = 0; i < n_verts; ++i)
        for (int a = 0; a < 3; ++a) {
            double x = verts[3 * i + a];
            if (x < lo[a]) lo[a] = x;
            if (x > hi[a]) hi[a] = x;
        }
}

static double scene_size(const double* verts, int64_t n_verts)
{
    double m[3] = {0.0, 0.0, 0.0};
    for (int64_t i = 0; i < n_verts; ++i)
        for (int a = 0; a < 3; ++a) m[a] += verts[3 * i + a];
    for (int a = 0; a < 3; ++a) m[a] /= (double)n_verts;
    double r2 = 0.0;
    for (int64_t i = 0; i < n_verts; ++i) {
        double q[3];
        sub3(verts + 3 * i, m, q);
        double d2 = dot3(q, q);
        if (d2 > r2) r2 = d2;
    }
    return 2.0 * sqrt(r2);
}

static void propagation_dir(const double sun[3], double d[3])
{
    double len = sqrt(dot3(sun, sun));
    d[0] = -sun[0] / len; d[1] = -sun[1] / len; d[2] = -sun[2] / len;
}

static void frame_from_box(const double lo[3], const double hi[3], double L, const double sun[3], int32_t nu,
                           int32_t nv, double fr[12])
{
    double d[3], u[3], v[3];
    propagation_dir(sun, d);
    oracle_basis(d, u, v);
    double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY, smin = INFINITY;
    for (int c = 0; c < 8; ++c) {
        double p[3] = {(c & 1) ? hi[0] : lo[0], (c & 2) ? hi[1] : lo[1], (c & 4) ? hi[2] : lo[2]};
        double pu = dot3(p, u), pv = dot3(p, v), ps = dot3(p, d);
        if (pu < umin) umin = pu;
        if (pu > umax) umax = pu;
        if (pv < vmin) vmin = pv;
        if (pv > vmax) vmax = pv;
        if (ps < smin) smin = ps;
    }
    double s0 = smin - 0.01 * L;
    for (int a = 0; a < 3; ++a) {
        fr[a] = u[a];
        fr[3 + a] = v[a];
        fr[6 + a] = s0 * d[a] + umin * u[a] + vmin * v[a];
    }
    fr[9] = (umax - umin) / (double)nu;
    fr[10] = (vmax - vmin) / (double)nv;
    fr[11] = 0.0;
}

int oracle_frames(const double* verts, int64_t n_verts, const double* sun_dirs, int64_t n_dirs,
                  int32_t nu, int32_t nv, double* frames)
{
    if (!verts || n_verts <= 0 || !sun_dirs || n_dirs < 0 || nu <= 0 || nv <= 0 || !frames)
        return ORC_EINVAL;
    double lo[3], hi[3];
    mesh_aabb(verts, n_verts, lo, hi);
    const double L = scene_size(verts, n_verts);
    for (int64_t j = 0; j < n_dirs; ++j) frame_from_box(lo, hi, L, sun_dirs + 3 * j, nu, nv, frames + 12 * j);
    return ORC_OK;
}

/* Default probability of sampling the specular event at a facet, in float arithmetic:
 * rho_s / (rho_s + rho_d) clamped to [0.01, 0.99] when both are positive, else 1 or 0. */
float oracle_default_pspec(float rs, float rd)
{
    if (rs > 0.0f && rd > 0.0f) {
        float p = rs / (rs + rd);
        if (p < 0.01f) p = 0.01f;
        if (p > 0.99f) p = 0.99f;
        return p;
    }
    return rs > 0.0f ? 1.0f : 0.0f;
}

/* ------------------------------------------------------------------------------------------ */
/* scene                                                                                       */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    int64_t n_tris;
    double* v0;  /* [T][3] */
    double* e1;  /* [T][3] */
    double* e2;  /* [T][3] */
    double* nrm; /* [T][3] unit outward normal, (v1-v0) x (v2-v0) */
    double* pv;  /* [T][9] vertices, for the degeneracy tests */
    const float* rho_s;
    const float* rho_d;
    float* p_spec;
    const float* phong; /* [T] Phong exponents (surface estimator), NULL: every specular event a mirror */
    double com[3];
    double L;  /* scene size (see scene_size) */
} scene_t;

static int scene_init(scene_t* S, const double* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                      const float* rho_s, const float* rho_d, const float* p_spec, const double com[3])
{
    memset(S, 0, sizeof(*S));
    S->n_tris = n_tris;
    S->v0 = malloc(sizeof(double) * 3 * n_tris);
    S->e1 = malloc(sizeof(double) * 3 * n_tris);
    S->e2 = malloc(sizeof(double) * 3 * n_tris);
    S->nrm = malloc(sizeof(double) * 3 * n_tris);
    S->pv = malloc(sizeof(double) * 9 * n_tris);
    S->p_spec = malloc(sizeof(float) * n_tris);
    if (!S->v0 || !S->e1 || !S->e2 || !S->nrm || !S->pv || !S->p_spec) return ORC_ENOMEM;
    for (int64_t f = 0; f < n_tris; ++f) {
        const double* p[3];
        for (int c = 0; c < 3; ++c) {
            int32_t id = tris[3 * f + c];
            if (id < 0 || id >= n_verts) return ORC_EINVAL;
            p[c] = verts + 3 * (int64_t)id;
            for (int a = 0; a < 3; ++a) S->pv[9 * f + 3 * c + a] = p[c][a];
        }
        sub3(p[1], p[0], S->e1 + 3 * f);
        sub3(p[2], p[0], S->e2 + 3 * f);
        for (int a = 0; a < 3; ++a) S->v0[3 * f + a] = p[0][a];
        double n[3];
        cross3(S->e1 + 3 * f, S->e2 + 3 * f, n);
        double len = sqrt(dot3(n, n));
        if (!(len > 0.0) || !isfinite(len)) return ORC_EDEGENERATE;
        for (int a = 0; a < 3; ++a) S->nrm[3 * f + a] = n[a] / len;
        S->p_spec[f] = p_spec ? p_spec[f] : oracle_default_pspec(rho_s[f], rho_d[f]);
    }
    S->rho_s = rho_s;
    S->rho_d = rho_d;
    for (int a = 0; a < 3; ++a) S->com[a] = com ? com[a] : 0.0;
    S->L = scene_size(verts, n_verts);
    return ORC_OK;
}

static void scene_free(scene_t* S)
{
    free(S->v0); free(S->e1); free(S->e2); free(S->nrm); free(S->pv); free(S->p_spec);
}

/* Closest front-facing hit over all triangles, brute force (Moller & Trumbore 1997, "Fast,
 * minimum storage ray-triangle intersection"), one-sided: a hit counts only when the ray meets
 * the outward side (d . n < 0).  Barycentric bounds are inclusive, t must exceed 0, the
 * triangle `skip` (the one the ray leaves) is never hit, and an exact tie in t goes to the lower
 * triangle index. */
static int64_t closest_hit(const scene_t* S, const double o[3], const double d[3], int64_t skip, double* t_out)
{
    int64_t best = -1;
    double tbest = INFINITY;
    for (int64_t f = 0; f < S->n_tris; ++f) {
        if (f == skip) continue;
        const double* e1 = S->e1 + 3 * f;
        const double* e2 = S->e2 + 3 * f;
        double pvec[3];
        cross3(d, e2, pvec);
        double det = dot3(e1, pvec);
        if (!(det > 0.0)) continue;
        double tvec[3];
        sub3(o, S->v0 + 3 * f, tvec);
        double uu = dot3(tvec, pvec);
        if (uu < 0.0 || uu > det) continue;
        double qvec[3];
        cross3(tvec, e1, qvec);
        double vv = dot3(d, qvec);
        if (vv < 0.0 || uu + vv > det) continue;
        double t = dot3(e2, qvec) / det;
        if (!(t > 0.0)) continue;
        if (t < tbest) { tbest = t; best = f; }
    }
    *t_out = tbest;
    return best;
}

/* ---- degeneracy classification of one segment ------------------------------------------- */
/* A segment is flagged when a float32 evaluation could plausibly choose a different closest
 * hit than this double evaluation.  Two uncertainties bound how the float32 ray differs:
 *   u   its position across the ray (metres).  A primary ray carries u = LAT * L.  An interaction
 *       at incidence cos(theta) spreads the hit point's error over the surface by 1/cos(theta)
 *       and the point is rounded again, so the next segment carries u' = u / cos(theta) + LAT * L
 *       (degeneracy_step).
 *   up  the distance of its origin from the plane of a triangle with normal n:
 *       DEPTH * L + u |n x m| for a segment leaving a facet with normal m (the spread error lies in
 *       that facet's plane), DEPTH * L + u for a primary ray.
 * The ray then meets that triangle's plane at a t uncertain by tau = up / |cos|.  The rules:
 *   (i)   another front-facing triangle whose plane the ray meets within tau_f + tau_hit of the
 *         closest hit in t;
 *   (ii)  the ray passes within u (measured in the plane normal to the ray) of an edge of a
 *         triangle whose plane it meets no nearer than -tau_f and no farther than
 *         t_hit + tau_f + tau_hit;
 *   (iii) the closest hit is grazing: cos(theta) < GRAZE;
 *   (iv)  the ray passes through (or within u of) a triangle seen nearly edge-on (|cos| <= GRAZE)
 *         within that depth range;
 *   (v)   the closest hit is at t < tau_hit, or a front-facing triangle containing the ray's
 *         projection (within u) has its plane within tau_f of the origin.
 * (The specular/diffuse event needs no margin: both paths compare the same float32 numbers.)
 * LAT and DEPTH are at least ten times the largest float32 errors measured on the GPU tracer for
 * the 20.6k-triangle satellite (3 bounces): hit points off across the ray by <= 0.101 of a model
 * with LAT = 1e-6, along it by <= 0.231 of that u / cos, and off their facet's plane by <= 2.4e-7 L. */
#define DEG_LAT 1.2e-6
#define DEG_DEPTH 2.5e-6
#define DEG_GRAZE 1e-5

/* LAT and DEPTH (in units of L) and GRAZE (a cosine). */
void oracle_degen_thresholds(double out[3])
{
    out[0] = DEG_LAT;
    out[1] = DEG_DEPTH;
    out[2] = DEG_GRAZE;
}

/* Position uncertainty of the segment after an interaction at incidence cosine c. */
static double degeneracy_step(const scene_t* S, double u, double c)
{
    return u / fmax(c, DEG_GRAZE) + DEG_LAT * S->L;
}

static double point_segment_dist(const double p[3], const double a[3], const double b[3])
{
    double ab[3], ap[3];
    sub3(b, a, ab);
    sub3(p, a, ap);
    double l2 = dot3(ab, ab);
    double s = l2 > 0.0 ? dot3(ap, ab) / l2 : 0.0;
    if (s < 0.0) s = 0.0;
    if (s > 1.0) s = 1.0;
    double q[3] = {a[0] + s * ab[0] - p[0], a[1] + s * ab[1] - p[1], a[2] + s * ab[2] - p[2]};
    return sqrt(dot3(q, q));
}

/* Uncertainty of the origin's distance from the plane of triangle f (see above). */
static double plane_uncertainty(const scene_t* S, int64_t skip, int64_t f, double u)
{
    if (skip < 0) return DEG_DEPTH * S->L + u;
    double c[3];
    cross3(S->nrm + 3 * f, S->nrm + 3 * skip, c);
    return DEG_DEPTH * S->L + u * sqrt(dot3(c, c));
}

static int segment_degenerate(const scene_t* S, const double o[3], const double d[3], int64_t skip, int64_t hit,
                              double thit, double u)
{
    double chit = 1.0, tau_hit = 0.0;
    if (hit >= 0) {
        chit = -dot3(d, S->nrm + 3 * hit);
        if (chit < DEG_GRAZE) return 1;  /* (iii) */
        tau_hit = plane_uncertainty(S, skip, hit, u) / chit;
        if (thit < tau_hit) return 1;    /* (v) */
    }
    const double zero[3] = {0.0, 0.0, 0.0};
    for (int64_t f = 0; f < S->n_tris; ++f) {
        if (f == skip) continue;
        /* project the vertices on the plane through o normal to d */
        double q[3][3], along[3];
        for (int c = 0; c < 3; ++c) {
            double rel[3];
            sub3(S->pv + 9 * f + 3 * c, o, rel);
            along[c] = dot3(rel, d);
            for (int a = 0; a < 3; ++a) q[c][a] = rel[a] - along[c] * d[a];
        }
        const double amin = fmin(along[0], fmin(along[1], along[2]));
        const double amax = fmax(along[0], fmax(along[1], along[2]));
        const double cosn = dot3(d, S->nrm + 3 * f);
        const int edge_on = fabs(cosn) <= DEG_GRAZE;
        /* depth relevance: where (and how uncertainly) the ray meets the triangle's plane */
        double tplane = 0.0, tau = 0.0;
        if (!edge_on) {
            tplane = dot3(S->nrm + 3 * f, (double[3]){S->pv[9 * f] - o[0], S->pv[9 * f + 1] - o[1],
                                                      S->pv[9 * f + 2] - o[2]}) / cosn;
            tau = plane_uncertainty(S, skip, f, u) / fabs(cosn);
            if (tplane < -tau) continue;                                /* behind the origin */
            if (hit >= 0 && tplane > thit + tau + tau_hit) continue;     /* beyond the hit */
        } else {
            if (amax < -u) continue;
            if (hit >= 0 && amin > thit + tau_hit) continue;
        }
        const double emin = fmin(point_segment_dist(zero, q[0], q[1]),
                                 fmin(point_segment_dist(zero, q[1], q[2]), point_segment_dist(zero, q[2], q[0])));
        /* is the projected ray point inside the projected triangle? (signed areas) */
        double n1[3], n2[3], n3[3];
        double a0[3], a1[3], a2[3];
        sub3(q[1], q[0], a0); sub3(q[2], q[1], a1); sub3(q[0], q[2], a2);
        double m0[3], m1[3], m2[3];
        sub3(zero, q[0], m0); sub3(zero, q[1], m1); sub3(zero, q[2], m2);
        cross3(a0, m0, n1); cross3(a1, m1, n2); cross3(a2, m2, n3);
        double s1 = dot3(n1, d), s2 = dot3(n2, d), s3 = dot3(n3, d);
        int inside = (s1 >= 0 && s2 >= 0 && s3 >= 0) || (s1 <= 0 && s2 <= 0 && s3 <= 0);
        if (!inside && emin >= u) continue;
        if (emin < u) return 1;   /* (ii) near an edge of a triangle it meets or narrowly misses */
        if (edge_on) return 1;    /* (iv) through a triangle seen edge-on */
        if (cosn < 0.0) {
            /* (i) a second front-facing hit close to the closest one */
            if (f != hit && hit >= 0 && fabs(tplane - thit) < tau + tau_hit) return 1;
            /* (v) a front-facing plane crossing very near the origin */
            if (fabs(tplane) < tau) return 1;
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------------------------ */
/* one path                                                                                    */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    int32_t nu, nv, bounces, jitter;
    double flux;
    uint64_t seed;
    int64_t dir_index_base;
    uint32_t design_index;
} params_t;

/* Follows one path from origin o along d with ray-tube force w over up to P->bounces surface
 * interactions and returns the force and torque it deposits.  Random draws use the Philox
 * counter (ctr0, dir_global, bounce, design index) with key `seed`.  Optionally records, per
 * interaction, the hit triangle (-1 = the path escaped), the degeneracy flag and the hit point. */
static void follow_path(const scene_t* S, double o[3], double d[3], double w, const params_t* P, uint64_t seed,
                        uint32_t ctr0, uint32_t dir_global, double F[3], double T[3], int32_t* hits, uint8_t* degen,
                        double* hx)
{
    if (hx)
        for (int q = 0; q < 3 * P->bounces; ++q) hx[q] = NAN;
    const double eps = 1e-5 * S->L;
    int64_t skip = -1;
    F[0] = F[1] = F[2] = 0.0;
    T[0] = T[1] = T[2] = 0.0;
    int deg = 0;
    double unc = DEG_LAT * S->L; /* position uncertainty of the segment (degeneracy rules) */
    for (int bnc = 1; bnc <= P->bounces; ++bnc) {
        double t;
        int64_t f = closest_hit(S, o, d, skip, &t);
        if (degen) {
            if (!deg) deg = segment_degenerate(S, o, d, skip, f, t, unc);
            degen[bnc - 1] = (uint8_t)deg;
        }
        if (hits) hits[bnc - 1] = (int32_t)f;
        if (f < 0) {
            for (int rest = bnc; rest < P->bounces; ++rest) {
                if (hits) hits[rest] = -1;
                if (degen) degen[rest] = (uint8_t)deg;
            }
            break;
        }
        const double* n = S->nrm + 3 * f;
        double x[3], lever[3];
        for (int c = 0; c < 3; ++c) {
            x[c] = o[c] + t * d[c];
            lever[c] = x[c] - S->com[c];
        }
        if (hx)
            for (int c = 0; c < 3; ++c) hx[3 * (bnc - 1) + c] = x[c];
        const double cth = -dot3(d, n);
        unc = degeneracy_step(S, unc, cth);
        double r[3];
        for (int c = 0; c < 3; ++c) r[c] = d[c] + 2.0 * cth * n[c];
        const double rs = (double)S->rho_s[f], rd = (double)S->rho_d[f];
        /* incoming momentum */
        double dep[3] = {w * d[0], w * d[1], w * d[2]};
        double tq[3];
        for (int c = 0; c < 3; ++c) F[c] += dep[c];
        cross3(lever, dep, tq);
        for (int c = 0; c < 3; ++c) T[c] += tq[c];
        if (bnc == P->bounces || (S->rho_s[f] == 0.0f && S->rho_d[f] == 0.0f)) {
            /* last traced interaction: the expected outgoing momentum leaves the body */
            double out[3];
            for (int c = 0; c < 3; ++c) out[c] = w * (rs * r[c] + (2.0 / 3.0) * rd * n[c]);
            for (int c = 0; c < 3; ++c) F[c] -= out[c];
            cross3(lever, out, tq);
            for (int c = 0; c < 3; ++c) T[c] -= tq[c];
            for (int rest = bnc; rest < P->bounces; ++rest) {
                if (hits) hits[rest] = -1;
                if (degen) degen[rest] = (uint8_t)deg;
            }
            break;
        }
        double ev[4];
        draw4(seed, ctr0, dir_global, (uint32_t)bnc, P->design_index, ev);
        const float ps = S->p_spec[f];
        double odir[3], w2;
        if ((float)ev[0] < ps) {
            for (int c = 0; c < 3; ++c) odir[c] = r[c];
            w2 = w * rs / (double)ps;
        } else {
            /* cosine-weighted direction about n (Malley's method) */
            double rad = sqrt(ev[1]);
            double phi = 2.0 * M_PI * ev[2];
            double lx = rad * cos(phi), ly = rad * sin(phi), lz = sqrt(fmax(0.0, 1.0 - ev[1]));
            double t1[3], t2[3];
            oracle_basis(n, t1, t2);
            for (int c = 0; c < 3; ++c) odir[c] = lx * t1[c] + ly * t2[c] + lz * n[c];
            w2 = w * rd / (1.0 - (double)ps);
        }
        double out[3] = {w2 * odir[0], w2 * odir[1], w2 * odir[2]};
        for (int c = 0; c < 3; ++c) F[c] -= out[c];
        cross3(lever, out, tq);
        for (int c = 0; c < 3; ++c) T[c] -= tq[c];
        for (int c = 0; c < 3; ++c) {
            o[c] = x[c] + eps * n[c];
            d[c] = odir[c];
        }
        w = w2;
        skip = f;
    }
}

/* Traces primary pixel `pixel` of direction j (global index dir_global) and returns the force
 * and torque it deposits, with the optional per-interaction records of follow_path. */
static void trace_path(const scene_t* S, const double fr[12], const double sun[3], const params_t* P, int64_t pixel,
                       uint32_t dir_global, double F[3], double T[3], int32_t* hits, uint8_t* degen, double* hx)
{
    const int32_t nu = P->nu;
    const int64_t i = pixel % nu, k = pixel / nu;
    double a = 0.5, b = 0.5;
    if (P->jitter) {
        double r[4];
        draw4(P->seed, (uint32_t)pixel, dir_global, 0u, P->design_index, r);
        a = r[0];
        b = r[1];
    }
    const double* u = fr;
    const double* v = fr + 3;
    const double* o0 = fr + 6;
    const double du = fr[9], dv = fr[10];
    double o[3], d[3];
    for (int c = 0; c < 3; ++c) o[c] = o0[c] + ((double)i + a) * du * u[c] + ((double)k + b) * dv * v[c];
    propagation_dir(sun, d);
    const double w = P->flux * du * dv / kSpeedOfLight; /* force carried by the ray tube, N */
    follow_path(S, o, d, w, P, P->seed, (uint32_t)pixel, dir_global, F, T, hits, degen, hx);
}

/* ------------------------------------------------------------------------------------------ */
/* threaded driver                                                                             */
/* ------------------------------------------------------------------------------------------ */
typedef struct {
    const scene_t* S;
    const params_t* P;
    const double* frames;
    const double* sun_dirs;
    int64_t n_dirs;
    const int64_t* pix;
    int64_t n_pix;
    double* part_f; /* [D][chunks][3] per-chunk sums, added in chunk order afterwards */
    double* part_t;
    int64_t n_chunks;
    int32_t* hit_prim;
    uint8_t* degen;
    double* ray_force;
    double* ray_torque;
    double* hit_x;
    int64_t next; /* work counter (rows of 64 pixels) */
    pthread_mutex_t lock;
    int32_t n_threads;
} job_t;

typedef struct {
    job_t* J;
    int32_t tid;
} worker_arg_t;

#define CHUNK 64

static void* worker(void* argp)
{
    worker_arg_t* A = (worker_arg_t*)argp;
    job_t* J = A->J;
    const int64_t per_dir = (J->n_pix + CHUNK - 1) / CHUNK;
    const int64_t total = per_dir * J->n_dirs;
    const int32_t B = J->P->bounces;
    for (;;) {
        pthread_mutex_lock(&J->lock);
        int64_t item = J->next++;
        pthread_mutex_unlock(&J->lock);
        if (item >= total) break;
        int64_t j = item / per_dir;
        int64_t p0 = (item % per_dir) * CHUNK;
        int64_t p1 = p0 + CHUNK < J->n_pix ? p0 + CHUNK : J->n_pix;
        double* pf = J->part_f + 3 * item;
        double* pt = J->part_t + 3 * item;
        for (int64_t q = p0; q < p1; ++q) {
            int64_t pixel = J->pix ? J->pix[q] : q;
            int64_t rec = j * J->n_pix + q;
            double F[3], T[3];
            trace_path(J->S, J->frames + 12 * j, J->sun_dirs + 3 * j, J->P, pixel,
                       (uint32_t)(J->P->dir_index_base + j), F, T,
                       J->hit_prim ? J->hit_prim + rec * B : NULL, J->degen ? J->degen + rec * B : NULL,
                       J->hit_x ? J->hit_x + rec * B * 3 : NULL);
            for (int c = 0; c < 3; ++c) {
                pf[c] += F[c];
                pt[c] += T[c];
            }
            if (J->ray_force)
                for (int c = 0; c < 3; ++c) J->ray_force[3 * rec + c] = F[c];
            if (J->ray_torque)
                for (int c = 0; c < 3; ++c) J->ray_torque[3 * rec + c] = T[c];
        }
    }
    return NULL;
}

/*
 * oracle_trace: ray-grid SRP estimate for n_dirs sun directions.
 *   verts [n_verts][3] (m, body frame), tris [n_tris][3] (counter-clockwise seen from outside),
 *   rho_s, rho_d [n_tris] float32, p_spec [n_tris] float32 or NULL (default rule),
 *   com [3] or NULL (origin), sun_dirs [n_dirs][3] unit vectors toward the Sun,
 *   frames [n_dirs][12] or NULL (computed from the mesh bounding box),
 *   pix [n_pix] explicit pixel list (pixel = i + k*nu) or NULL (all nu*nv pixels; n_pix ignored),
 *   force, torque [n_dirs][3] sums over the traced pixels (N, N m),
 *   hit_prim, degen [n_dirs][n_pix][bounces], ray_force, ray_torque [n_dirs][n_pix][3], hit_x
 *   [n_dirs][n_pix][bounces][3] (hit points, NaN where the path has ended): optional per-ray
 *   records.  Pixels are summed sequentially within chunks of 64; chunk sums are added in chunk
 *   order, so the result does not depend on the thread count.
 */
int oracle_trace(const double* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris, const float* rho_s,
                 const float* rho_d, const float* p_spec, const double* com, const double* sun_dirs, int64_t n_dirs,
                 const double* frames, int32_t nu, int32_t nv, int32_t bounces, int32_t jitter, double flux,
                 uint64_t seed, int64_t dir_index_base, uint32_t design_index, const int64_t* pix, int64_t n_pix,
                 double* force, double* torque, int32_t* hit_prim, uint8_t* degen, double* ray_force,
                 double* ray_torque, double* hit_x, int32_t n_threads)
{
    if (!verts || n_verts <= 0 || !tris || n_tris <= 0 || !rho_s || !rho_d || !sun_dirs || n_dirs < 0 || nu <= 0 ||
        nv <= 0 || bounces < 1 || !force || !torque)
        return ORC_EINVAL;
    if (!pix) n_pix = (int64_t)nu * nv;
    if (n_pix < 0) return ORC_EINVAL;
    for (int64_t f = 0; f < n_tris; ++f)
        if (!(rho_s[f] >= 0.0f) || !(rho_d[f] >= 0.0f) || rho_s[f] + rho_d[f] > 1.0f) return ORC_EINVAL;
    scene_t S;
    int st = scene_init(&S, verts, n_verts, tris, n_tris, rho_s, rho_d, p_spec, com);
    if (st != ORC_OK) {
        scene_free(&S);
        return st;
    }
    double* fr = NULL;
    if (!frames) {
        fr = malloc(sizeof(double) * 12 * (n_dirs > 0 ? n_dirs : 1));
        if (!fr) { scene_free(&S); return ORC_ENOMEM; }
        oracle_frames(verts, n_verts, sun_dirs, n_dirs, nu, nv, fr);
        frames = fr;
    }
    params_t P = {nu, nv, bounces, jitter, flux, seed, dir_index_base, design_index};
    if (n_threads < 1) n_threads = 1;
    job_t J;
    memset(&J, 0, sizeof(J));
    J.S = &S; J.P = &P; J.frames = frames; J.sun_dirs = sun_dirs; J.n_dirs = n_dirs;
    J.pix = pix; J.n_pix = n_pix; J.hit_prim = hit_prim; J.degen = degen;
    J.ray_force = ray_force; J.ray_torque = ray_torque; J.hit_x = hit_x; J.n_threads = n_threads;
    J.n_chunks = (n_pix + CHUNK - 1) / CHUNK;
    J.part_f = calloc((size_t)3 * J.n_chunks * (n_dirs > 0 ? n_dirs : 1) + 3, sizeof(double));
    J.part_t = calloc((size_t)3 * J.n_chunks * (n_dirs > 0 ? n_dirs : 1) + 3, sizeof(double));
    if (!J.part_f || !J.part_t) {
        free(J.part_f); free(J.part_t); free(fr); scene_free(&S);
        return ORC_ENOMEM;
    }
    pthread_mutex_init(&J.lock, NULL);
    pthread_t* th = malloc(sizeof(pthread_t) * n_threads);
    worker_arg_t* args = malloc(sizeof(worker_arg_t) * n_threads);
    for (int32_t t = 0; t < n_threads; ++t) {
        args[t].J = &J;
        args[t].tid = t;
        pthread_create(&th[t], NULL, worker, &args[t]);
    }
    for (int32_t t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
    for (int64_t j = 0; j < n_dirs; ++j)
        for (int c = 0; c < 3; ++c) {
            double sf = 0.0, stq = 0.0;
            for (int64_t q = 0; q < J.n_chunks; ++q) {
                sf += J.part_f[3 * (j * J.n_chunks + q) + c];
                stq += J.part_t[3 * (j * J.n_chunks + q) + c];
            }
            force[3 * j + c] = sf;
            torque[3 * j + c] = stq;
        }
    pthread_mutex_destroy(&J.lock);
    free(th); free(args); free(J.part_f); free(J.part_t); free(fr);
    scene_free(&S);
    return ORC_OK;
}

/* ========================================================================================== */
/* Gradients.                                                                                 */
/*                                                                                            */
/* With every Philox counter and the specular-sampling probabilities p_s frozen, the estimator */
/* is a polynomial in the per-facet reflectances: along a path with interactions b = 1..K the */
/* weights are W_b = w k_1 ... k_b with k_b = rho_s/p_s (mirror event) or rho_d/(1 - p_s)      */
/* (Lambertian event); interaction b < K deposits W_{b-1} d_{b-1} - W_b o_b and the last one    */
/* W_{K-1} (d_{K-1} - rho_s r_K - (2/3) rho_d n_K).  For a loss L = sum_j gF_j . F_j +           */
/* gT_j . tau_j every deposit v at x contributes v . (gF + gT x (x - x_COM)).                  */
/* oracle_trace_adjoint_rho returns dL/d rho_s[f], dL/d rho_d[f] of that polynomial, written   */
/* out per path in FP64 (no division by k: products leaving k_i out are formed directly).       */
/* ========================================================================================== */

typedef struct {
    int32_t facet;
    int32_t mirror; /* 1: mirror event, 0: Lambertian event */
    double k;       /* weight factor of the event */
    double c;       /* loss coefficient of the W_b term: -(G_b . o_b) */
} grad_step_t;

/* Adds one path's gradient terms and returns 1 when the path is degenerate (a segment flagged by
 * segment_degenerate, classified as in trace_path).  With drop_degenerate set, a degenerate path
 * adds nothing. */
static int adjoint_path(const scene_t* S, const double fr[12], const double sun[3], const params_t* P, int64_t pixel,
                        uint32_t dir_global, const double gF[3], const double gT[3], double* g_rs, double* g_rd,
                        int drop_degenerate)
{
    const int32_t nu = P->nu;
    const int64_t i = pixel % nu, k = pixel / nu;
    double a = 0.5, b = 0.5;
    if (P->jitter) {
        double r[4];
        draw4(P->seed, (uint32_t)pixel, dir_global, 0u, P->design_index, r);
        a = r[0];
        b = r[1];
    }
    const double* u = fr;
    const double* v = fr + 3;
    const double* o0 = fr + 6;
    double o[3], d[3];
    for (int c = 0; c < 3; ++c) o[c] = o0[c] + ((double)i + a) * fr[9] * u[c] + ((double)k + b) * fr[10] * v[c];
    propagation_dir(sun, d);
    const double w = P->flux * fr[9] * fr[10] / kSpeedOfLight;
    const double eps = 1e-5 * S->L;
    grad_step_t st[16];
    int K = 0;            /* non-terminal interactions recorded */
    double coef0 = 0.0;   /* coefficient of W_0 = w */
    int64_t skip = -1;
    /* terminal data */
    int have_term = 0;
    int64_t tf = -1;
    double tg = 0.0, td = 0.0; /* G . r and G . n at the terminal interaction */
    double W_in = w;           /* current weight (for the terminal coefficients) */
    int deg = 0;
    double unc = DEG_LAT * S->L;
    for (int bnc = 1; bnc <= P->bounces; ++bnc) {
        double t;
        int64_t f = closest_hit(S, o, d, skip, &t);
        if (drop_degenerate && !deg) deg = segment_degenerate(S, o, d, skip, f, t, unc);
        if (f < 0) break;
        const double* n = S->nrm + 3 * f;
        double x[3], lever[3], G[3], gx[3];
        for (int c = 0; c < 3; ++c) {
            x[c] = o[c] + t * d[c];
            lever[c] = x[c] - S->com[c];
        }
        cross3(gT, lever, gx);
        for (int c = 0; c < 3; ++c) G[c] = gF[c] + gx[c];
        const double cth = -dot3(d, n);
        unc = degeneracy_step(S, unc, cth);
        double r[3];
        for (int c = 0; c < 3; ++c) r[c] = d[c] + 2.0 * cth * n[c];
        /* incoming term: W_{b-1} (G . d_{b-1}) */
        const double gin = dot3(G, d);
        if (K == 0) coef0 += gin; else st[K - 1].c += gin;
        if (bnc == P->bounces || (S->rho_s[f] == 0.0f && S->rho_d[f] == 0.0f)) {
            have_term = 1;
            tf = f;
            tg = dot3(G, r);
            td = dot3(G, n);
            break;
        }
        double ev[4];
        draw4(P->seed, (uint32_t)pixel, dir_global, (uint32_t)bnc, P->design_index, ev);
        const float ps = S->p_spec[f];
        double odir[3], kf;
        int mirror;
        if ((float)ev[0] < ps) {
            for (int c = 0; c < 3; ++c) odir[c] = r[c];
            kf = (double)S->rho_s[f] / (double)ps;
            mirror = 1;
        } else {
            double rad = sqrt(ev[1]);
            double phi = 2.0 * M_PI * ev[2];
            double lx = rad * cos(phi), ly = rad * sin(phi), lz = sqrt(fmax(0.0, 1.0 - ev[1]));
            double t1[3], t2[3];
            oracle_basis(n, t1, t2);
            for (int c = 0; c < 3; ++c) odir[c] = lx * t1[c] + ly * t2[c] + lz * n[c];
            kf = (double)S->rho_d[f] / (1.0 - (double)ps);
            mirror = 0;
        }
        st[K].facet = (int32_t)f;
        st[K].mirror = mirror;
        st[K].k = kf;
        st[K].c = -dot3(G, odir);
        ++K;
        W_in *= kf;
        for (int c = 0; c < 3; ++c) {
            o[c] = x[c] + eps * n[c];
            d[c] = odir[c];
        }
        skip = f;
    }
    (void)W_in;
    if (deg) return 1;
    /* L = w coef0 + sum_b W_b c_b + W_K (-(rho_s G.r + 2/3 rho_d G.n)) at the terminal one */
    double term_c = 0.0;
    if (have_term) term_c = -((double)S->rho_s[tf] * tg + (2.0 / 3.0) * (double)S->rho_d[tf] * td);
    for (int q = 0; q < K; ++q) {
        /* dL/dk_q = sum over m >= q of (W_m / k_q) c_m  (+ terminal) */
        double acc = 0.0;
        for (int m = q; m < K; ++m) {
            double prod = w;
            for (int l = 0; l <= m; ++l)
                if (l != q) prod *= st[l].k;
            acc += prod * st[m].c;
        }
        if (have_term) {
            double prod = w;
            for (int l = 0; l < K; ++l)
                if (l != q) prod *= st[l].k;
            acc += prod * term_c;
        }
        const int32_t f = st[q].facet;
        const float ps = S->p_spec[f];
        if (st[q].mirror) g_rs[f] += acc / (double)ps;
        else g_rd[f] += acc / (1.0 - (double)ps);
    }
    if (have_term) {
        double WK = w;
        for (int l = 0; l < K; ++l) WK *= st[l].k;
        g_rs[tf] += -WK * tg;
        g_rd[tf] += -WK * (2.0 / 3.0) * td;
    }
    return 0;
}

typedef struct {
    const scene_t* S;
    const params_t* P;
    const double* frames;
    const double* sun_dirs;
    int64_t n_dirs;
    const int64_t* pix;
    int64_t n_pix;
    const double* gF;
    const double* gT;
    double* g_rs; /* [threads][T] */
    double* g_rd;
    int32_t n_threads;
    int32_t drop_degenerate;
    uint8_t* path_degen; /* [D][n_pix] or NULL */
} adj_job_t;

typedef struct {
    adj_job_t* J;
    int32_t tid;
} adj_arg_t;

static void* adj_worker(void* argp)
{
    adj_arg_t* A = (adj_arg_t*)argp;
    adj_job_t* J = A->J;
    const int64_t per_dir = (J->n_pix + CHUNK - 1) / CHUNK;
    const int64_t total = per_dir * J->n_dirs;
    const int64_t T = J->S->n_tris;
    double* gs = J->g_rs + (int64_t)A->tid * T;
    double* gd = J->g_rd + (int64_t)A->tid * T;
    for (int64_t item = A->tid; item < total; item += J->n_threads) { /* static assignment: deterministic */
        int64_t j = item / per_dir;
        int64_t p0 = (item % per_dir) * CHUNK;
        int64_t p1 = p0 + CHUNK < J->n_pix ? p0 + CHUNK : J->n_pix;
        for (int64_t q = p0; q < p1; ++q) {
            int64_t pixel = J->pix ? J->pix[q] : q;
            const int dg = adjoint_path(J->S, J->frames + 12 * j, J->sun_dirs + 3 * j, J->P, pixel,
                                        (uint32_t)(J->P->dir_index_base + j), J->gF + 3 * j, J->gT + 3 * j, gs, gd,
                                        J->drop_degenerate);
            if (J->path_degen) J->path_degen[j * J->n_pix + q] = (uint8_t)dg;
        }
    }
    return NULL;
}

/* oracle_trace_adjoint_rho: dL/d rho_s and dL/d rho_d per facet (ADDED to g_rho_s, g_rho_d
 * [n_tris]) for L = sum_j gF[j] . F_j + gT[j] . tau_j, with the inputs of oracle_trace.
 * gT may be NULL (zero).  drop_degenerate != 0 leaves out every path with a degenerate segment
 * (the rule of the hit records) and marks it in path_degen [n_dirs][n_pix] (may be NULL). */
int oracle_trace_adjoint_rho(const double* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                             const float* rho_s, const float* rho_d, const float* p_spec, const double* com,
                             const double* sun_dirs, int64_t n_dirs, const double* frames, int32_t nu, int32_t nv,
                             int32_t bounces, int32_t jitter, double flux, uint64_t seed, int64_t dir_index_base,
                             uint32_t design_index, const int64_t* pix, int64_t n_pix, const double* gF,
                             const double* gT, double* g_rho_s, double* g_rho_d, int32_t drop_degenerate,
                             uint8_t* path_degen, int32_t n_threads)
{
    if (!verts || !tris || !rho_s || !rho_d || !sun_dirs || !gF || !g_rho_s || !g_rho_d || nu <= 0 || nv <= 0 ||
        bounces < 1 || bounces > 15 || n_dirs < 0)
        return ORC_EINVAL;
    if (!pix) n_pix = (int64_t)nu * nv;
    scene_t S;
    int st = scene_init(&S, verts, n_verts, tris, n_tris, rho_s, rho_d, p_spec, com);
    if (st != ORC_OK) {
        scene_free(&S);
        return st;
    }
    double* fr = NULL;
    if (!frames) {
        fr = malloc(sizeof(double) * 12 * (n_dirs > 0 ? n_dirs : 1));
        oracle_frames(verts, n_verts, sun_dirs, n_dirs, nu, nv, fr);
        frames = fr;
    }
    double* zero = NULL;
    if (!gT) {
        zero = calloc(3 * (size_t)(n_dirs > 0 ? n_dirs : 1), sizeof(double));
        gT = zero;
    }
    params_t P = {nu, nv, bounces, jitter, flux, seed, dir_index_base, design_index};
    if (n_threads < 1) n_threads = 1;
    adj_job_t J = {&S, &P, frames, sun_dirs, n_dirs, pix, n_pix, gF, gT, NULL, NULL, n_threads, drop_degenerate,
                   path_degen};
    J.g_rs = calloc((size_t)n_threads * n_tris, sizeof(double));
    J.g_rd = calloc((size_t)n_threads * n_tris, sizeof(double));
    pthread_t* th = malloc(sizeof(pthread_t) * n_threads);
    adj_arg_t* args = malloc(sizeof(adj_arg_t) * n_threads);
    for (int32_t t = 0; t < n_threads; ++t) {
        args[t].J = &J;
        args[t].tid = t;
        pthread_create(&th[t], NULL, adj_worker, &args[t]);
    }
    for (int32_t t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
    for (int32_t t = 0; t < n_threads; ++t)
        for (int64_t f = 0; f < n_tris; ++f) {
            g_rho_s[f] += J.g_rs[(int64_t)t * n_tris + f];
            g_rho_d[f] += J.g_rd[(int64_t)t * n_tris + f];
        }
    free(J.g_rs); free(J.g_rd); free(th); free(args); free(fr); free(zero);
    scene_free(&S);
    return ORC_OK;
}

/* ========================================================================================== */
/* Frozen-visibility estimator (for hinge-angle gradients).                                   */
/*                                                                                            */
/* Each path keeps the facet sequence it had at the reference design (ref_hits, from           */
/* oracle_trace records at theta_0); at the current vertices each segment meets the PLANE of   */
/* its frozen facet, so hit points move with the facets, normals and mirror directions turn,    */
/* and the Lambertian direction is rebuilt in the basis of the turned normal from the same      */
/* draws.  Its derivative at theta_0 is the pathwise part of the hinge-angle gradient: each     */
/* path keeps its image position and its facet sequence.  With `footprint` set, the path's     */
/* deposits are also scaled by P_f(theta)/P_f(theta_0), where P_f is the area of the primary    */
/* facet projected on the grid plane (1/2 ((v1-v0) x (v2-v0)) . (-d)): the first-order change   */
/* of the facet's share of the grid for a facet no other facet shadows (an approximation of   */
/* the visibility-edge terms that oracle_edge_term estimates exactly).                          */
/* ========================================================================================== */
static double proj_area(const double* pv, const double d[3])
{
    double e1[3], e2[3], cr[3];
    sub3(pv + 3, pv, e1);
    sub3(pv + 6, pv, e2);
    cross3(e1, e2, cr);
    return -0.5 * dot3(cr, d);
}

int oracle_trace_frozen(const double* verts, const double* verts0, int64_t n_verts, const int32_t* tris,
                        int64_t n_tris, const float* rho_s, const float* rho_d, const float* p_spec, const double* com,
                        const double* sun_dirs, int64_t n_dirs, const double* frames, int32_t nu, int32_t nv,
                        int32_t bounces, int32_t jitter, double flux, uint64_t seed, int64_t dir_index_base,
                        uint32_t design_index, const int64_t* pix, int64_t n_pix, const int32_t* ref_hits,
                        int32_t footprint, double* force, double* torque)
{
    if (!verts || !verts0 || !tris || !rho_s || !rho_d || !sun_dirs || !frames || !ref_hits || !force || !torque ||
        nu <= 0 || nv <= 0 || bounces < 1)
        return ORC_EINVAL;
    if (!pix) n_pix = (int64_t)nu * nv;
    scene_t S, S0;
    int st = scene_init(&S, verts, n_verts, tris, n_tris, rho_s, rho_d, p_spec, com);
    int st0 = scene_init(&S0, verts0, n_verts, tris, n_tris, rho_s, rho_d, p_spec, com);
    if (st != ORC_OK || st0 != ORC_OK) {
        scene_free(&S);
        scene_free(&S0);
        return st != ORC_OK ? st : st0;
    }
    /* the offset scale is taken at the reference design (its derivative is excluded) */
    const double eps = 1e-5 * S0.L;
    for (int64_t j = 0; j < n_dirs; ++j) {
        const double* fr = frames + 12 * j;
        double Fj[3] = {0, 0, 0}, Tj[3] = {0, 0, 0};
        const uint32_t dir_global = (uint32_t)(dir_index_base + j);
        for (int64_t q = 0; q < n_pix; ++q) {
            const int64_t pixel = pix ? pix[q] : q;
            const int32_t* hits = ref_hits + (j * n_pix + q) * bounces;
            if (hits[0] < 0) continue;
            const int64_t i = pixel % nu, k = pixel / nu;
            double a = 0.5, b = 0.5;
            if (jitter) {
                double r[4];
                draw4(seed, (uint32_t)pixel, dir_global, 0u, design_index, r);
                a = r[0];
                b = r[1];
            }
            double o[3], d[3];
            for (int c = 0; c < 3; ++c)
                o[c] = fr[6 + c] + ((double)i + a) * fr[9] * fr[c] + ((double)k + b) * fr[10] * fr[3 + c];
            propagation_dir(sun_dirs + 3 * j, d);
            const double scale =
                footprint ? proj_area(S.pv + 9 * hits[0], d) / proj_area(S0.pv + 9 * hits[0], d) : 1.0;
            double w = flux * fr[9] * fr[10] / kSpeedOfLight;
            double PF[3] = {0, 0, 0}, PT[3] = {0, 0, 0};
            for (int bnc = 1; bnc <= bounces; ++bnc) {
                const int32_t f = hits[bnc - 1];
                if (f < 0) break;
                const double* n = S.nrm + 3 * f;
                double rel[3];
                sub3(S.v0 + 3 * f, o, rel);
                const double t = dot3(n, rel) / dot3(n, d);
                double x[3], lever[3];
                for (int c = 0; c < 3; ++c) {
                    x[c] = o[c] + t * d[c];
                    lever[c] = x[c] - S.com[c];
                }
                const double cth = -dot3(d, n);
                double r[3];
                for (int c = 0; c < 3; ++c) r[c] = d[c] + 2.0 * cth * n[c];
                const double rs = (double)rho_s[f], rd = (double)rho_d[f];
                double dep[3] = {w * d[0], w * d[1], w * d[2]}, tq[3];
                if (bnc == bounces || (rho_s[f] == 0.0f && rho_d[f] == 0.0f)) {
                    for (int c = 0; c < 3; ++c) dep[c] -= w * (rs * r[c] + (2.0 / 3.0) * rd * n[c]);
                    for (int c = 0; c < 3; ++c) PF[c] += dep[c];
                    cross3(lever, dep, tq);
                    for (int c = 0; c < 3; ++c) PT[c] += tq[c];
                    break;
                }
                double ev[4];
                draw4(seed, (uint32_t)pixel, dir_global, (uint32_t)bnc, design_index, ev);
                const float ps = S.p_spec[f];
                double odir[3], w2;
                if ((float)ev[0] < ps) {
                    for (int c = 0; c < 3; ++c) odir[c] = r[c];
                    w2 = w * rs / (double)ps;
                } else {
                    double rad = sqrt(ev[1]);
                    double phi = 2.0 * M_PI * ev[2];
                    double lx = rad * cos(phi), ly = rad * sin(phi), lz = sqrt(fmax(0.0, 1.0 - ev[1]));
                    double t1[3], t2[3];
                    oracle_basis(n, t1, t2);
                    for (int c = 0; c < 3; ++c) odir[c] = lx * t1[c] + ly * t2[c] + lz * n[c];
                    w2 = w * rd / (1.0 - (double)ps);
                }
                for (int c = 0; c < 3; ++c) dep[c] -= w2 * odir[c];
                for (int c = 0; c < 3; ++c) PF[c] += dep[c];
                cross3(lever, dep, tq);
                for (int c = 0; c < 3; ++c) PT[c] += tq[c];
                for (int c = 0; c < 3; ++c) {
                    o[c] = x[c] + eps * n[c];
                    d[c] = odir[c];
                }
                w = w2;
            }
            for (int c = 0; c < 3; ++c) {
                Fj[c] += scale * PF[c];
                Tj[c] += scale * PT[c];
            }
        }
        for (int c = 0; c < 3; ++c) {
            force[3 * j + c] = Fj[c];
            torque[3 * j + c] = Tj[c];
        }
    }
    scene_free(&S);
    scene_free(&S0);
    return ORC_OK;
}

/* ========================================================================================== */
/* Visibility-edge terms of the hinge-angle gradient, by edge sampling.                         */
/*                                                                                            */
/* Per sun direction the ray grid estimates F = (Phi/c) int g(y) dy over the grid plane, where  */
/* g(y) is the momentum that a unit-weight path started at image point y deposits (all its      */
/* interactions).  Turning hinge k moves the images of the edges of the facets it carries, and  */
/* g jumps across them (silhouettes against the background or against other surfaces, edges     */
/* between facets of different material, occlusion of one part by another).  The derivative    */
/* of the integral is the pathwise part (oracle_trace_frozen without footprint factor: every    */
/* path keeps its image position and facet sequence) plus, for every moving edge,              */
/*     (Phi/c) int_edge (g(y - delta n) - g(y + delta n)) v_n dl,                              */
/* n the edge's unit normal in the grid plane, v_n = n . (the image velocity of the edge point  */
/* under the rotation about the hinge axis), delta -> 0.  Edges hidden behind other surfaces    */
/* contribute nothing because g is the same on both sides.                                     */
/*                                                                                            */
/* Estimator: the moving edges are the distinct edges of facets whose three vertices the hinge */
/* carries, numbered by first appearance in facet order (an edge coincident with an earlier    */
/* one -- the two layers of a two-sided sheet, the shared edge of two facets -- counts once).   */
/* Edge e takes M stratified points s = (m + xi)/M along it; both side points y -+ delta n with */
/* delta = 1e-5 L start a full path with the same draws (Philox key seed ^ EDGE_KEY, counter   */
/* (e M + m, direction, bounce, design); xi is the first uniform of bounce 0), and the edge's   */
/* contribution is (Phi/c) (len/M) sum_m v_n(s_m) (deposit(y-) - deposit(y+)).  Secondary       */
/* visibility edges (reflected light crossing an edge) are not included.                       */
/*                                                                                            */
/* The caller may pass a keep mask over the edges in that numbering and leave out edges across */
/* which g is continuous (a flat continuation of the surface with the same material): there    */
/* the two side paths meet facets of one plane and material, leave in the same direction with  */
/* the same draws, and their deposits differ by O(delta) only.                                 */
/* ========================================================================================== */
#define EDGE_KEY 0x9E3779B97F4A7C15ULL

typedef struct {
    double key[6]; /* the two endpoint positions, lexicographically ordered */
    int64_t order; /* facet * 3 + edge slot */
    int32_t a, b;  /* vertex indices (a, b in the facet's winding order) */
    int32_t hinge;
} edge_rec_t;

static int cmp_edge_key(const void* pa, const void* pb)
{
    const edge_rec_t* x = (const edge_rec_t*)pa;
    const edge_rec_t* y = (const edge_rec_t*)pb;
    for (int c = 0; c < 6; ++c) {
        if (x->key[c] < y->key[c]) return -1;
        if (x->key[c] > y->key[c]) return 1;
    }
    return (x->order > y->order) - (x->order < y->order);
}

static int cmp_edge_order(const void* pa, const void* pb)
{
    const edge_rec_t* x = (const edge_rec_t*)pa;
    const edge_rec_t* y = (const edge_rec_t*)pb;
    return (x->order > y->order) - (x->order < y->order);
}

static int pos_less(const double* p, const double* q)
{
    for (int c = 0; c < 3; ++c) {
        if (p[c] < q[c]) return 1;
        if (p[c] > q[c]) return 0;
    }
    return 0;
}

/* Distinct moving edges, in order of first appearance; returns the count (or -1). */
static int64_t moving_edges(const double* verts, const int32_t* tris, int64_t n_tris, const int32_t* vert_hinge,
                            edge_rec_t** out)
{
    edge_rec_t* all = malloc(sizeof(edge_rec_t) * (size_t)(3 * n_tris + 1));
    if (!all) return -1;
    int64_t n = 0;
    for (int64_t f = 0; f < n_tris; ++f) {
        const int32_t* t = tris + 3 * f;
        const int32_t k = vert_hinge[t[0]];
        if (k < 0 || vert_hinge[t[1]] != k || vert_hinge[t[2]] != k) continue;
        for (int e = 0; e < 3; ++e) {
            edge_rec_t r;
            r.a = t[e];
            r.b = t[(e + 1) % 3];
            r.hinge = k;
            r.order = 3 * f + e;
            const double* pa = verts + 3 * r.a;
            const double* pb = verts + 3 * r.b;
            const double* lo = pos_less(pb, pa) ? pb : pa;
            const double* hi = lo == pa ? pb : pa;
            for (int c = 0; c < 3; ++c) {
                r.key[c] = lo[c];
                r.key[3 + c] = hi[c];
            }
            all[n++] = r;
        }
    }
    qsort(all, (size_t)n, sizeof(edge_rec_t), cmp_edge_key);
    int64_t m = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (i > 0 && memcmp(all[i].key, all[i - 1].key, sizeof(all[i].key)) == 0) continue;
        all[m++] = all[i];
    }
    qsort(all, (size_t)m, sizeof(edge_rec_t), cmp_edge_order);
    *out = all;
    return m;
}

typedef struct {
    const scene_t* S;
    const params_t* P;
    const edge_rec_t* E;
    int64_t n_edges;
    const double* verts;
    const double* hinge_origin;
    const double* hinge_axis;
    int32_t n_hinges;
    const double* frames;
    const double* sun_dirs;
    int64_t n_dirs;
    int32_t samples;
    const uint8_t* keep; /* [n_edges] or NULL (all) */
    double* out;         /* [n_dirs][n_hinges][6] */
    int32_t n_threads;
    int32_t tid;
} edge_job_t;

static void* edge_worker(void* argp)
{
    edge_job_t* J = (edge_job_t*)argp;
    const scene_t* S = J->S;
    const params_t* P = J->P;
    const double delta = 1e-5 * S->L;
    const uint64_t key = P->seed ^ EDGE_KEY;
    const int32_t M = J->samples;
    for (int64_t j = J->tid; j < J->n_dirs; j += J->n_threads) { /* whole directions: deterministic sums */
        const double* fr = J->frames + 12 * j;
        const double* u = fr;
        const double* v = fr + 3;
        const double* o0 = fr + 6;
        const uint32_t dir_global = (uint32_t)(P->dir_index_base + j);
        double d[3];
        propagation_dir(J->sun_dirs + 3 * j, d);
        double* acc = J->out + (size_t)j * J->n_hinges * 6;
        for (int64_t e = 0; e < J->n_edges; ++e) {
            if (J->keep && !J->keep[e]) continue;
            const edge_rec_t* r = J->E + e;
            const double* p0 = J->verts + 3 * r->a;
            const double* p1 = J->verts + 3 * r->b;
            double rel0[3], rel1[3];
            sub3(p0, o0, rel0);
            sub3(p1, o0, rel1);
            const double y0[2] = {dot3(rel0, u), dot3(rel0, v)};
            const double y1[2] = {dot3(rel1, u), dot3(rel1, v)};
            const double ty[2] = {y1[0] - y0[0], y1[1] - y0[1]};
            const double len = sqrt(ty[0] * ty[0] + ty[1] * ty[1]);
            if (!(len > 0.0)) continue; /* an edge seen end-on sweeps no area */
            const double nrm[2] = {ty[1] / len, -ty[0] / len};
            const double* ho = J->hinge_origin + 3 * r->hinge;
            const double* ha = J->hinge_axis + 3 * r->hinge;
            double sum[6] = {0, 0, 0, 0, 0, 0};
            for (int32_t m = 0; m < M; ++m) {
                const uint32_t ctr0 = (uint32_t)(e * M + m);
                double xi[4];
                draw4(key, ctr0, dir_global, 0u, P->design_index, xi);
                const double sp = ((double)m + xi[0]) / (double)M;
                /* the edge point, its image and its image velocity under the rotation */
                double x[3], rx[3], xd[3];
                for (int c = 0; c < 3; ++c) x[c] = p0[c] + sp * (p1[c] - p0[c]);
                sub3(x, ho, rx);
                cross3(ha, rx, xd);
                const double vn = dot3(xd, u) * nrm[0] + dot3(xd, v) * nrm[1];
                const double y[2] = {y0[0] + sp * ty[0], y0[1] + sp * ty[1]};
                double Fm[3], Tm[3], Fp[3], Tp[3];
                for (int side = 0; side < 2; ++side) {
                    const double sgn = side == 0 ? -1.0 : 1.0;
                    const double yy[2] = {y[0] + sgn * delta * nrm[0], y[1] + sgn * delta * nrm[1]};
                    double o[3], dd[3] = {d[0], d[1], d[2]};
                    for (int c = 0; c < 3; ++c) o[c] = o0[c] + yy[0] * u[c] + yy[1] * v[c];
                    follow_path(S, o, dd, 1.0, P, key, ctr0, dir_global, side == 0 ? Fm : Fp, side == 0 ? Tm : Tp,
                                NULL, NULL, NULL);
                }
                for (int c = 0; c < 3; ++c) {
                    sum[c] += vn * (Fm[c] - Fp[c]);
                    sum[3 + c] += vn * (Tm[c] - Tp[c]);
                }
            }
            const double scale = P->flux / kSpeedOfLight * len / (double)M;
            for (int c = 0; c < 6; ++c) acc[6 * r->hinge + c] += scale * sum[c];
        }
    }
    return NULL;
}

/*
 * oracle_edge_term: the visibility-edge part of d(F, tau)/d(hinge angle) for n_dirs sun
 * directions (see above).  verts [n_verts][3] are the current vertices, vert_hinge [n_verts] the
 * hinge carrying each vertex (-1: rigid), hinge_origin/hinge_axis [n_hinges][3] (axis unit) the
 * hinge lines, frames [n_dirs][12] the grid frames, `samples` = M points per edge, keep
 * [n_keep] (NULL: every edge) the edges taken, in the numbering above (n_keep must equal the edge
 * count).  Writes dF [n_dirs][n_hinges][6] (force then torque, per radian).  Also returns the
 * edge count in *n_edges_out (may be NULL).
 */
int oracle_edge_term(const double* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                     const int32_t* vert_hinge, const double* hinge_origin, const double* hinge_axis, int32_t n_hinges,
                     const float* rho_s, const float* rho_d, const float* p_spec, const double* com,
                     const double* sun_dirs, int64_t n_dirs, const double* frames, int32_t bounces, double flux,
                     uint64_t seed, int64_t dir_index_base, uint32_t design_index, int32_t samples,
                     const uint8_t* keep, int64_t n_keep, double* dF, int64_t* n_edges_out, int32_t n_threads)
{
    if (!verts || !tris || !vert_hinge || (n_hinges > 0 && (!hinge_origin || !hinge_axis)) || !rho_s || !rho_d ||
        !sun_dirs || !frames || !dF || bounces < 1 || samples < 1 || n_dirs < 0 || n_hinges < 0)
        return ORC_EINVAL;
    scene_t S;
    int st = scene_init(&S, verts, n_verts, tris, n_tris, rho_s, rho_d, p_spec, com);
    if (st != ORC_OK) {
        scene_free(&S);
        return st;
    }
    edge_rec_t* E = NULL;
    const int64_t ne = moving_edges(verts, tris, n_tris, vert_hinge, &E);
    if (ne < 0) {
        scene_free(&S);
        return ORC_ENOMEM;
    }
    if (n_edges_out) *n_edges_out = ne;
    if (keep && n_keep != ne) {
        free(E);
        scene_free(&S);
        return ORC_EINVAL;
    }
    memset(dF, 0, sizeof(double) * 6 * (size_t)(n_dirs * n_hinges));
    params_t P = {1, 1, bounces, 0, flux, seed, dir_index_base, design_index};
    if (n_threads < 1) n_threads = 1;
    pthread_t* th = malloc(sizeof(pthread_t) * n_threads);
    edge_job_t* jobs = malloc(sizeof(edge_job_t) * n_threads);
    for (int32_t t = 0; t < n_threads; ++t) {
        edge_job_t J = {&S, &P, E, ne, verts, hinge_origin, hinge_axis, n_hinges, frames, sun_dirs, n_dirs, samples,
                        keep, dF, n_threads, t};
        jobs[t] = J;
        pthread_create(&th[t], NULL, edge_worker, &jobs[t]);
    }
    for (int32_t t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
    free(th);
    free(jobs);
    free(E);
    scene_free(&S);
    return ORC_OK;
}

/* ========================================================================================== */
/* Surface-sampling estimator (paper Sec. 3.2, "Estimation", and its equation for F).          */
/*                                                                                            */
/* Every sample picks a facet with probability proportional to its area and a uniform point x */
/* on it (square-root barycentric mapping), gathers the light arriving at x by path tracing     */
/* with next-event estimation toward the Sun at every path vertex, and converts it to momentum  */
/* at x with one sampled outgoing event: with probability p_s the specular event of weight      */
/* rho_s/p_s, else a cosine-distributed direction o of weight rho_d/(1 - p_s).  The sample's    */
/* force is the total area A times the force density at x; the estimate is the sample mean.    */
/*                                                                                            */
/* Materials (the paper's per-face Phong parameters): BRDF rho_d/pi + rho_s (m + 2)/(2 pi)      */
/* ((r.o)+)^m, r the mirror direction of the arriving light (the modified Phong model of        */
/* Lafortune and Willems 1994), exponent m >= 1 per facet; m infinite is the ideal mirror.  A   */
/* specular event samples the lobe about r (BRDF importance sampling: cos(alpha) =               */
/* u^(1/(m+1)), pdf (m+1)/(2 pi) cos^m alpha), so a lobe direction o carries the weight         */
/* (m + 2)/(m + 1) (n.o)+ per unit rho_s (0 below the horizon).  Sunlight reflected into a lobe */
/* is gathered by next-event estimation like the Lambertian share.                             */
/*                                                                                            */
/* Light reaching x (force units per area, propagation p, deposit W (p - R(p))):               */
/*   direct     W = Phi (n.s)/c if n.s > 0 and no sun-facing facet blocks the ray x -> s;       */
/*   gathered   one cosine-distributed direction w1 about n (pdf cos/pi) leads to the closest   */
/*              front-facing facet v1; the radiance it sends to x is the BRDF share of its own  */
/*              sunlight, (rho_d/pi + lobe toward x) Phi (n1.s)+ (unblocked), plus what it      */
/*              reflects of light from further vertices v2, ... (event sampled at each vertex:  */
/*              specular continuation with weight rho_s/p_s times the lobe weight, or cosine    */
/*              continuation with rho_d/(1-p_s)), so W = pi/c * radiance and p = -w1.  Light    */
/*              reaching x has met at most B - 1 surfaces before x: vertices v1 .. v_{B-1}.     */
/* Sunlight whose first reflection is an ideal mirror is not gathered (a delta light seen       */
/* through a delta reflection has zero probability of being sampled); everything else has the  */
/* same expectation as the ray-grid estimator with `bounces` = B (which has ideal mirrors only). */
/*                                                                                            */
/* Random numbers: Philox counter (sample, global direction, stage, design); stage 0: facet,   */
/* two barycentric uniforms, the event at x; stage 1: the outgoing direction at x (2) and the   */
/* first gathering direction (2); stage k + 1: the event at v_k and its continuation direction. */
/*                                                                                            */
/* Variance-reduction options (the paper's convergence study compares plain MC, BRDF importance */
/* sampling, stratified surface sampling and both; Sec. 4, simulation results):                 */
/*   sampling bit 0  stratified surface: sample i of N uses (i + u)/N for the area coordinate,  */
/*                   one sample per 1/N of the total area;                                      */
/*   sampling bit 1  every sampled direction (outgoing, gathering, continuation) uniform over   */
/*                   the hemisphere, weighted by 2 cos(theta) -- plain MC; without it, cosine     */
/*                   sampling (the Lambertian BRDF's importance sampling), weight 1.  A lobe      */
/*                   direction is then uniform too, weighted by (m + 2) ((r.o)+)^m (n.o).        */
/* ========================================================================================== */

/* Sunlight reaching o along -s is blocked by any facet other than `skip` whose outward side
 * faces the Sun (n.s > 0) and that the ray o + t s (t > 0) crosses.  *deg flags a ray passing
 * within u (its position uncertainty, see segment_degenerate) of such a facet's edge, crossing
 * one nearly edge-on, or meeting its plane within u / cos of the origin. */
static int sun_blocked(const scene_t* S, const double o[3], const double s[3], int64_t skip, double u, int* deg)
{
    /* (the origin lies just off the plane of facet `skip`: see segment_degenerate for the
       uncertainty of its distance from another plane) */
    const double zero[3] = {0.0, 0.0, 0.0};
    int blocked = 0;
    for (int64_t f = 0; f < S->n_tris; ++f) {
        if (f == skip) continue;
        const double cosn = dot3(s, S->nrm + 3 * f);
        if (!(cosn > 0.0)) continue;
        /* projection of the facet on the plane through o normal to s */
        double q[3][3], along[3];
        for (int c = 0; c < 3; ++c) {
            double rel[3];
            sub3(S->pv + 9 * f + 3 * c, o, rel);
            along[c] = dot3(rel, s);
            for (int a = 0; a < 3; ++a) q[c][a] = rel[a] - along[c] * s[a];
        }
        const double amax = fmax(along[0], fmax(along[1], along[2]));
        if (amax < -plane_uncertainty(S, skip, f, u)) continue; /* entirely behind the origin */
        /* signed areas of the projected point against the three edges */
        double cr1[3], cr2[3], cr3[3], m0[3], m1[3], m2[3], e0[3], e1v[3], e2v[3];
        sub3(zero, q[0], m0); sub3(zero, q[1], m1); sub3(zero, q[2], m2);
        sub3(q[1], q[0], e0); sub3(q[2], q[1], e1v); sub3(q[0], q[2], e2v);
        cross3(e0, m0, cr1); cross3(e1v, m1, cr2); cross3(e2v, m2, cr3);
        const double s1 = dot3(cr1, s), s2 = dot3(cr2, s), s3 = dot3(cr3, s);
        const int inside = (s1 >= 0 && s2 >= 0 && s3 >= 0) || (s1 <= 0 && s2 <= 0 && s3 <= 0);
        const double emin = fmin(point_segment_dist(zero, q[0], q[1]),
                                 fmin(point_segment_dist(zero, q[1], q[2]), point_segment_dist(zero, q[2], q[0])));
        if (emin < u) *deg = 1;
        if (cosn < DEG_GRAZE && (inside || emin < u)) *deg = 1;
        if (!inside) continue;
        /* distance along s to the facet's plane */
        const double tplane = dot3(S->nrm + 3 * f, (double[3]){S->pv[9 * f] - o[0], S->pv[9 * f + 1] - o[1],
                                                             S->pv[9 * f + 2] - o[2]}) / cosn;
        if (fabs(tplane) < plane_uncertainty(S, skip, f, u) / fmax(cosn, DEG_GRAZE)) *deg = 1;
        if (tplane > 0.0) blocked = 1;
    }
    return blocked;
}

/* cosine-distributed direction about the unit normal n from two uniforms (Malley's method) */
static void cosine_dir(const double n[3], double u1, double u2, double out[3])
{
    double rad = sqrt(u1);
    double phi = 2.0 * M_PI * u2;
    double lx = rad * cos(phi), ly = rad * sin(phi), lz = sqrt(fmax(0.0, 1.0 - u1));
    double t1[3], t2[3];
    oracle_basis(n, t1, t2);
    for (int c = 0; c < 3; ++c) out[c] = lx * t1[c] + ly * t2[c] + lz * n[c];
}

/* A direction on the hemisphere of n and its weight relative to cosine sampling: the cosine
 * distribution (the Lambertian BRDF's importance sampling, weight 1) or, with `uniform`, the uniform
 * distribution over solid angle (cos theta = u1, weight 2 cos theta = pi cos / (pi * 1 / (2 pi))). */
static double hemi_dir(const double n[3], double u1, double u2, int uniform, double out[3])
{
    if (!uniform) {
        cosine_dir(n, u1, u2, out);
        return 1.0;
    }
    double rad = sqrt(fmax(0.0, 1.0 - u1 * u1));
    double phi = 2.0 * M_PI * u2;
    double lx = rad * cos(phi), ly = rad * sin(phi), lz = u1;
    double t1[3], t2[3];
    oracle_basis(n, t1, t2);
    for (int c = 0; c < 3; ++c) out[c] = lx * t1[c] + ly * t2[c] + lz * n[c];
    return 2.0 * u1;
}

/* The specular event for light of propagation p at a point with normal n: the outgoing direction
 * and its weight per unit rho_s.  An ideal mirror (m infinite) reflects into r = p - 2 (p.n) n with
 * weight 1; a Phong lobe of exponent m draws o about r from (u1, u2) (weight (m + 2)/(m + 1) (n.o)+)
 * or, with `uniform`, over the hemisphere of n (weight (m + 2) ((r.o)+)^m (n.o)). */
static double specular_dir(const double p[3], const double n[3], double m, double u1, double u2, int uniform,
                           double out[3])
{
    double r[3];
    const double pn = dot3(p, n);
    for (int c = 0; c < 3; ++c) r[c] = p[c] - 2.0 * pn * n[c];
    if (isinf(m)) {
        for (int c = 0; c < 3; ++c) out[c] = r[c];
        return 1.0;
    }
    if (uniform) {
        hemi_dir(n, u1, u2, 1, out);
        return (m + 2.0) * pow(fmax(0.0, dot3(r, out)), m) * dot3(n, out);
    }
    const double ca = pow(u1, 1.0 / (m + 1.0));
    const double sa = sqrt(fmax(0.0, 1.0 - ca * ca));
    const double phi = 2.0 * M_PI * u2;
    double t1[3], t2[3];
    oracle_basis(r, t1, t2);
    for (int c = 0; c < 3; ++c) out[c] = sa * cos(phi) * t1[c] + sa * sin(phi) * t2[c] + ca * r[c];
    return (m + 2.0) / (m + 1.0) * fmax(0.0, dot3(n, out));
}

/* Whether the specular weight of direction o is nonzero by the model (as opposed to by rounding):
 * always for the ideal mirror; for a lobe, o above the horizon and, when drawn uniformly, inside
 * the lobe's half-space r.o > 0. */
static int lobe_open(const double p[3], const double n[3], double m, int uniform, const double o[3])
{
    if (isinf(m)) return 1;
    double r[3];
    const double pn = dot3(p, n);
    for (int c = 0; c < 3; ++c) r[c] = p[c] - 2.0 * pn * n[c];
    return dot3(n, o) > 0.0 && (!uniform || dot3(r, o) > 0.0);
}

typedef struct {
    uint64_t seed;
    uint32_t design_index;
    int32_t bounces;
    double flux;
    const double* cum; /* [T] cumulative facet areas, facet order */
    double area;       /* total area */
    int32_t sampling;  /* bit 0: stratified surface; bit 1: uniform hemisphere directions */
    int64_t n_samples;
} gather_params_t;

/* One sample of the surface-sampling estimator for direction `sun` (global index dir_global).
 * Returns the sample's force and torque (area already applied) and, optionally, its record:
 * facet, gathered vertices (B - 1 facets, -1 = none), sunlit flags (bit 0: x, bit k: v_k) and
 * the degeneracy flag. */
static void gather_sample(const scene_t* S, const gather_params_t* G, const double sun[3], uint32_t dir_global,
                          uint32_t sample, double F[3], double T[3], int32_t* rec_facet, int32_t* rec_hits,
                          int32_t* rec_lit, uint8_t* rec_deg)
{
    const int32_t B = G->bounces;
    const double eps = 1e-5 * S->L;
    int deg = 0;
    double u0[4], u1[4];
    draw4(G->seed, sample, dir_global, 0u, G->design_index, u0);
    draw4(G->seed, sample, dir_global, 1u, G->design_index, u1);
    /* facet by area: the first f with u A < cum[f]; stratified, sample i takes u = (i + u0) / N */
    const double uf = (G->sampling & 1) ? ((double)sample + u0[0]) / (double)G->n_samples : u0[0];
    const double target = uf * G->area;
    int64_t lo = 0, hi = S->n_tris - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (target < G->cum[mid]) hi = mid; else lo = mid + 1;
    }
    const int64_t f = lo;
    if (fabs(target - G->cum[f]) < 1e-12 * G->area || (f > 0 && fabs(target - G->cum[f - 1]) < 1e-12 * G->area))
        deg = 1;
    /* uniform point: x = v0 + sqrt(u1)(1 - u2) e1 + sqrt(u1) u2 e2 */
    const double sq = sqrt(u0[1]);
    const double b1 = sq * (1.0 - u0[2]), b2 = sq * u0[2];
    double x[3];
    for (int c = 0; c < 3; ++c) x[c] = S->v0[3 * f + c] + b1 * S->e1[3 * f + c] + b2 * S->e2[3 * f + c];
    const double* n = S->nrm + 3 * f;
    const double rs = (double)S->rho_s[f], rd = (double)S->rho_d[f];
    const float ps = S->p_spec[f];
    const double mx = S->phong ? (double)S->phong[f] : INFINITY;
    /* the outgoing event at x: specular (about each arriving contribution's mirror direction,
       drawn from the same two uniforms) or one cosine direction for all contributions */
    const int uniform = (G->sampling & 2) != 0;
    const int spec = (float)u0[3] < ps;
    double odir[3];
    const double wo = hemi_dir(n, u1[0], u1[1], uniform, odir);
    const double kdif = rd > 0.0 ? rd / (1.0 - (double)ps) * wo : 0.0;
    double s[3] = {sun[0], sun[1], sun[2]};
    double dep[3] = {0.0, 0.0, 0.0};
    int32_t lit = 0;
    double o[3];
    for (int c = 0; c < 3; ++c) o[c] = x[c] + eps * n[c];
    /* direct sunlight at x */
    const double cs = dot3(n, s);
    double unc = DEG_LAT * S->L; /* position uncertainty of the sample point (degeneracy rules) */
    if (cs > 0.0 && !sun_blocked(S, o, s, f, unc, &deg)) {
        lit |= 1;
        const double W = G->flux * cs / kSpeedOfLight;
        double p[3] = {-s[0], -s[1], -s[2]};
        double od[3];
        double k = kdif;
        if (spec) k = rs / (double)ps * specular_dir(p, n, mx, u1[0], u1[1], uniform, od);
        for (int c = 0; c < 3; ++c) dep[c] += W * (p[c] - k * (spec ? od[c] : odir[c]));
    }
    if (rec_hits)
        for (int k = 0; k < B - 1; ++k) rec_hits[k] = -1;
    if (B >= 2) {
        /* gathered light: vertices v1 .. v_{B-1} */
        double w[3];
        const double wg = hemi_dir(n, u1[2], u1[3], uniform, w);
        double p1[3] = {-w[0], -w[1], -w[2]};
        double radiance = 0.0; /* pi x radiance toward x, in units of Phi */
        double beta = 1.0;
        double ro[3] = {o[0], o[1], o[2]}, rdir[3] = {w[0], w[1], w[2]};
        int64_t skip = f;
        for (int k = 1; k <= B - 1; ++k) {
            double t;
            int64_t g = closest_hit(S, ro, rdir, skip, &t);
            if (!deg) deg = segment_degenerate(S, ro, rdir, skip, g, t, unc);
            if (g < 0) break;
            if (rec_hits) rec_hits[k - 1] = (int32_t)g;
            const double* ng = S->nrm + 3 * g;
            unc = degeneracy_step(S, unc, -dot3(rdir, ng));
            double y[3], oy[3];
            for (int c = 0; c < 3; ++c) {
                y[c] = ro[c] + t * rdir[c];
                oy[c] = y[c] + eps * ng[c];
            }
            const double rsg = (double)S->rho_s[g], rdg = (double)S->rho_d[g];
            const double mg = S->phong ? (double)S->phong[g] : INFINITY;
            const int lobe = rsg > 0.0 && !isinf(mg);
            const double cg = dot3(ng, s);
            if ((rdg > 0.0 || lobe) && cg > 0.0 && !sun_blocked(S, oy, s, g, unc, &deg)) {
                lit |= 1 << k;
                double add = rdg * cg;
                if (lobe) {
                    /* pi times the lobe's radiance toward the previous vertex (along -rdir) for
                       sunlight of propagation -s: rho_s (m + 2)/2 ((r.(-rdir))+)^m (n.s) */
                    const double sn = dot3(s, ng);
                    double rsun[3];
                    for (int c = 0; c < 3; ++c) rsun[c] = -s[c] + 2.0 * sn * ng[c];
                    add += rsg * (mg + 2.0) * 0.5 * pow(fmax(0.0, -dot3(rsun, rdir)), mg) * cg;
                }
                radiance += beta * add;
            }
            if (k == B - 1) break;
            /* continue from v_k: event, weight and the next gathering direction */
            double ev[4];
            draw4(G->seed, sample, dir_global, (uint32_t)(k + 1), G->design_index, ev);
            const float psg = S->p_spec[g];
            double nd[3];
            int live;
            if ((float)ev[0] < psg) {
                /* light leaving v_k toward the previous vertex travels along -rdir; it comes from
                   about the reflection of rdir (the lobe is symmetric in its two directions) */
                beta *= rsg / (double)psg * specular_dir(rdir, ng, mg, ev[1], ev[2], uniform, nd);
                live = rsg > 0.0 && lobe_open(rdir, ng, mg, uniform, nd);
            } else {
                const double wv = hemi_dir(ng, ev[1], ev[2], uniform, nd);
                beta *= rdg > 0.0 ? rdg / (1.0 - (double)psg) * wv : 0.0;
                live = rdg > 0.0 && wv > 0.0;
            }
            /* the path ends where its weight is zero by the model (a zero reflectance, a direction on
               or below the horizon or outside the lobe), not where a long product underflows */
            if (!live) break;
            for (int c = 0; c < 3; ++c) {
                ro[c] = oy[c];
                rdir[c] = nd[c];
            }
            skip = g;
        }
        if (radiance > 0.0) {
            const double W = G->flux * radiance * wg / kSpeedOfLight;
            double od[3];
            double k = kdif;
            if (spec) k = rs / (double)ps * specular_dir(p1, n, mx, u1[0], u1[1], uniform, od);
            for (int c = 0; c < 3; ++c) dep[c] += W * (p1[c] - k * (spec ? od[c] : odir[c]));
        }
    }
    double lever[3];
    for (int c = 0; c < 3; ++c) {
        F[c] = G->area * dep[c];
        lever[c] = x[c] - S->com[c];
    }
    cross3(lever, F, T);
    if (rec_facet) *rec_facet = (int32_t)f;
    if (rec_lit) *rec_lit = lit;
    if (rec_deg) *rec_deg = (uint8_t)deg;
}

typedef struct {
    const scene_t* S;
    const gather_params_t* G;
    const double* sun_dirs;
    int64_t n_dirs, n_samples, dir_index_base;
    double* part_f; /* [D][chunks][3] */
    double* part_t;
    int32_t *rec_facet, *rec_hits, *rec_lit;
    uint8_t* rec_deg;
    double* sample_force;
    int64_t next;
    pthread_mutex_t lock;
} gather_job_t;

static void* gather_worker(void* argp)
{
    gather_job_t* J = (gather_job_t*)argp;
    const int64_t per_dir = (J->n_samples + CHUNK - 1) / CHUNK;
    const int64_t total = per_dir * J->n_dirs;
    const int32_t B = J->G->bounces;
    for (;;) {
        pthread_mutex_lock(&J->lock);
        int64_t item = J->next++;
        pthread_mutex_unlock(&J->lock);
        if (item >= total) break;
        const int64_t j = item / per_dir;
        const int64_t s0 = (item % per_dir) * CHUNK;
        const int64_t s1 = s0 + CHUNK < J->n_samples ? s0 + CHUNK : J->n_samples;
        double* pf = J->part_f + 3 * item;
        double* pt = J->part_t + 3 * item;
        for (int64_t i = s0; i < s1; ++i) {
            const int64_t rec = j * J->n_samples + i;
            double F[3], T[3];
            gather_sample(J->S, J->G, J->sun_dirs + 3 * j, (uint32_t)(J->dir_index_base + j), (uint32_t)i, F, T,
                          J->rec_facet ? J->rec_facet + rec : NULL,
                          J->rec_hits && B > 1 ? J->rec_hits + rec * (B - 1) : NULL,
                          J->rec_lit ? J->rec_lit + rec : NULL, J->rec_deg ? J->rec_deg + rec : NULL);
            for (int c = 0; c < 3; ++c) {
                pf[c] += F[c];
                pt[c] += T[c];
            }
            if (J->sample_force)
                for (int c = 0; c < 3; ++c) J->sample_force[3 * rec + c] = F[c];
        }
    }
    return NULL;
}

/*
 * oracle_surface_estimate: surface-sampling estimate of the force and torque for n_dirs sun
 * directions, n_samples samples each (sample index = Philox counter word 0).
 *   verts, tris, rho_s, rho_d, p_spec, com, sun_dirs as for oracle_trace;
 *   phong [n_tris] Phong exponents, each >= 1 or +infinity (ideal mirror); NULL: all mirrors;
 *   force, torque [n_dirs][3]: sample means (N, N m);
 *   optional per-sample records [n_dirs][n_samples] (hits: [.. ][bounces - 1]) and forces [..][3];
 *   sampling: 0..3, the variance-reduction bits above.
 * Samples are summed in chunks of 64, chunk sums in order: independent of the thread count.
 */
int oracle_surface_estimate(const double* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                            const float* rho_s, const float* rho_d, const float* p_spec, const float* phong,
                            const double* com,
                            const double* sun_dirs, int64_t n_dirs, int64_t n_samples, int32_t bounces, double flux,
                            uint64_t seed, int64_t dir_index_base, uint32_t design_index, double* force,
                            double* torque, int32_t* rec_facet, int32_t* rec_hits, int32_t* rec_lit, uint8_t* rec_deg,
                            double* sample_force, int32_t sampling, int32_t n_threads)
{
    if (!verts || n_verts <= 0 || !tris || n_tris <= 0 || !rho_s || !rho_d || !sun_dirs || n_dirs < 0 ||
        n_samples < 1 || bounces < 1 || !force || !torque || sampling < 0 || sampling > 3)
        return ORC_EINVAL;
    for (int64_t f = 0; f < n_tris; ++f)
        if (!(rho_s[f] >= 0.0f) || !(rho_d[f] >= 0.0f) || rho_s[f] + rho_d[f] > 1.0f) return ORC_EINVAL;
    if (phong)
        for (int64_t f = 0; f < n_tris; ++f)
            if (!(phong[f] >= 1.0f)) return ORC_EINVAL;
    scene_t S;
    int st = scene_init(&S, verts, n_verts, tris, n_tris, rho_s, rho_d, p_spec, com);
    if (st != ORC_OK) {
        scene_free(&S);
        return st;
    }
    S.phong = phong;
    double* cum = malloc(sizeof(double) * n_tris);
    if (!cum) { scene_free(&S); return ORC_ENOMEM; }
    double acc = 0.0;
    for (int64_t f = 0; f < n_tris; ++f) {
        double cr[3];
        cross3(S.e1 + 3 * f, S.e2 + 3 * f, cr);
        acc += 0.5 * sqrt(dot3(cr, cr));
        cum[f] = acc;
    }
    gather_params_t G = {seed, design_index, bounces, flux, cum, acc, sampling, n_samples};
    if (n_threads < 1) n_threads = 1;
    gather_job_t J;
    memset(&J, 0, sizeof(J));
    J.S = &S; J.G = &G; J.sun_dirs = sun_dirs; J.n_dirs = n_dirs; J.n_samples = n_samples;
    J.dir_index_base = dir_index_base; J.rec_facet = rec_facet; J.rec_hits = rec_hits; J.rec_lit = rec_lit;
    J.rec_deg = rec_deg; J.sample_force = sample_force;
    const int64_t chunks = (n_samples + CHUNK - 1) / CHUNK;
    J.part_f = calloc((size_t)3 * chunks * (n_dirs > 0 ? n_dirs : 1), sizeof(double));
    J.part_t = calloc((size_t)3 * chunks * (n_dirs > 0 ? n_dirs : 1), sizeof(double));
    if (!J.part_f || !J.part_t) {
        free(J.part_f); free(J.part_t); free(cum); scene_free(&S);
        return ORC_ENOMEM;
    }
    pthread_mutex_init(&J.lock, NULL);
    pthread_t* th = malloc(sizeof(pthread_t) * n_threads);
    for (int32_t t = 0; t < n_threads; ++t) pthread_create(&th[t], NULL, gather_worker, &J);
    for (int32_t t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
    for (int64_t j = 0; j < n_dirs; ++j)
        for (int c = 0; c < 3; ++c) {
            double sf = 0.0, stq = 0.0;
            for (int64_t q = 0; q < chunks; ++q) {
                sf += J.part_f[3 * (j * chunks + q) + c];
                stq += J.part_t[3 * (j * chunks + q) + c];
            }
            force[3 * j + c] = sf / (double)n_samples;
            torque[3 * j + c] = stq / (double)n_samples;
        }
    pthread_mutex_destroy(&J.lock);
    free(th); free(J.part_f); free(J.part_t); free(cum);
    scene_free(&S);
    return ORC_OK;
}

/* ========================================================================================== */
/* Multi-world surface sampling (paper Sec. 3.2, "Estimation": the samples are drawn over      */
/* random designs, so each sample's rays meet a different world).  Pair i (a sun direction and */
/* a design) rotates the panels of the rest-pose mesh by its hinge angles (Rodrigues' formula,  */
/* FP64, vertex by vertex), gives every facet the materials of its group, and averages K       */
/* samples of the estimator above with the Philox counter (k, dir_index_base + i, stage,       */
/* design_index): the same samples the single-design estimator draws for that world when its  */
/* direction index is dir_index_base + i.                                                      */
/* ========================================================================================== */

typedef struct {
    const double* verts;
    int64_t n_verts;
    const int32_t* tris;
    int64_t n_tris;
    const int32_t* vert_hinge;
    const double* hinge_origin;
    const double* hinge_axis;
    int32_t n_hinges;
    const int32_t* group;
    int32_t n_groups;
    const double* designs; /* [N][H + 3 G] */
    const double* sun;     /* [N][3] */
    int64_t n_pairs, samples;
    int32_t bounces, sampling;
    double flux;
    uint64_t seed;
    int64_t dir_index_base;
    uint32_t design_index;
    const double* com;
    double *force, *torque;
    int32_t *rec_facet, *rec_hits, *rec_lit;
    uint8_t* rec_deg;
    int64_t next;
    int status;
    pthread_mutex_t lock;
} designs_job_t;

/* Vertex positions of one design: every vertex carried by hinge h rotates by its angle about
 * (origin_h, axis_h), right-hand rule. */
static void design_vertices(const designs_job_t* J, const double* angles, double* out)
{
    for (int64_t v = 0; v < J->n_verts; ++v) {
        const double* p = J->verts + 3 * v;
        const int32_t h = J->vert_hinge ? J->vert_hinge[v] : -1;
        if (h < 0) {
            for (int c = 0; c < 3; ++c) out[3 * v + c] = p[c];
            continue;
        }
        const double* o = J->hinge_origin + 3 * h;
        const double* k = J->hinge_axis + 3 * h;
        const double ct = cos(angles[h]), st = sin(angles[h]);
        double r[3], kr[3];
        sub3(p, o, r);
        cross3(k, r, kr);
        const double kd = dot3(k, r);
        for (int c = 0; c < 3; ++c) out[3 * v + c] = o[c] + r[c] * ct + kr[c] * st + k[c] * kd * (1.0 - ct);
    }
}

static void* designs_worker(void* argp)
{
    designs_job_t* J = (designs_job_t*)argp;
    const int64_t T = J->n_tris;
    const int32_t H = J->n_hinges, B = J->bounces;
    double* V = malloc(sizeof(double) * 3 * J->n_verts);
    float* rs = malloc(sizeof(float) * T);
    float* rd = malloc(sizeof(float) * T);
    float* ph = malloc(sizeof(float) * T);
    double* cum = malloc(sizeof(double) * T);
    if (!V || !rs || !rd || !ph || !cum) {
        pthread_mutex_lock(&J->lock);
        J->status = ORC_ENOMEM;
        pthread_mutex_unlock(&J->lock);
        free(V); free(rs); free(rd); free(ph); free(cum);
        return NULL;
    }
    for (;;) {
        pthread_mutex_lock(&J->lock);
        const int64_t i = J->next++;
        pthread_mutex_unlock(&J->lock);
        if (i >= J->n_pairs) break;
        const double* dsg = J->designs + (int64_t)i * (H + 3 * J->n_groups);
        design_vertices(J, dsg, V);
        for (int64_t f = 0; f < T; ++f) {
            const double* mg = dsg + H + 3 * J->group[f];
            rs[f] = (float)mg[0];
            rd[f] = (float)mg[1];
            ph[f] = (float)mg[2];
        }
        scene_t S;
        int st = scene_init(&S, V, J->n_verts, J->tris, T, rs, rd, NULL, J->com);
        if (st != ORC_OK) {
            scene_free(&S);
            pthread_mutex_lock(&J->lock);
            J->status = st;
            pthread_mutex_unlock(&J->lock);
            break;
        }
        S.phong = ph;
        double acc = 0.0;
        for (int64_t f = 0; f < T; ++f) {
            double cr[3];
            cross3(S.e1 + 3 * f, S.e2 + 3 * f, cr);
            acc += 0.5 * sqrt(dot3(cr, cr));
            cum[f] = acc;
        }
        gather_params_t G = {J->seed, J->design_index, B, J->flux, cum, acc, J->sampling, J->samples};
        double sf[3] = {0.0, 0.0, 0.0}, stq[3] = {0.0, 0.0, 0.0};
        for (int64_t k = 0; k < J->samples; ++k) {
            const int64_t rec = i * J->samples + k;
            double F[3], Tq[3];
            gather_sample(&S, &G, J->sun + 3 * i, (uint32_t)(J->dir_index_base + i), (uint32_t)k, F, Tq,
                          J->rec_facet ? J->rec_facet + rec : NULL,
                          J->rec_hits && B > 1 ? J->rec_hits + rec * (B - 1) : NULL,
                          J->rec_lit ? J->rec_lit + rec : NULL, J->rec_deg ? J->rec_deg + rec : NULL);
            for (int c = 0; c < 3; ++c) {
                sf[c] += F[c];
                stq[c] += Tq[c];
            }
        }
        for (int c = 0; c < 3; ++c) {
            J->force[3 * i + c] = sf[c] / (double)J->samples;
            J->torque[3 * i + c] = stq[c] / (double)J->samples;
        }
        scene_free(&S);
    }
    free(V); free(rs); free(rd); free(ph); free(cum);
    return NULL;
}

/*
 * oracle_surface_designs: the surface-sampling estimator for n_pairs (sun direction, design) pairs.
 *   verts [n_verts][3] rest pose; tris; vert_hinge [n_verts] (-1 rigid, NULL all rigid);
 *   hinge_origin, hinge_axis [n_hinges][3] (axes of unit length); group [n_tris] in [0, n_groups);
 *   designs [n_pairs][n_hinges + 3 n_groups]: hinge angles (rad), then per group rho_s, rho_d and
 *   the Phong exponent (>= 1, or +infinity for the ideal mirror); sun [n_pairs][3];
 *   samples per pair; com [3] or NULL; force, torque [n_pairs][3]: per-pair sample means;
 *   optional records [n_pairs][samples] as for oracle_surface_estimate.
 */
int oracle_surface_designs(const double* verts, int64_t n_verts, const int32_t* tris, int64_t n_tris,
                           const int32_t* vert_hinge, const double* hinge_origin, const double* hinge_axis,
                           int32_t n_hinges, const int32_t* group, int32_t n_groups, const double* designs,
                           const double* sun, int64_t n_pairs, int64_t samples, int32_t bounces, double flux,
                           uint64_t seed, int64_t dir_index_base, uint32_t design_index, int32_t sampling,
                           const double* com, double* force, double* torque, int32_t* rec_facet, int32_t* rec_hits,
                           int32_t* rec_lit, uint8_t* rec_deg, int32_t n_threads)
{
    if (!verts || n_verts <= 0 || !tris || n_tris <= 0 || n_hinges < 0 || (n_hinges > 0 && (!hinge_origin ||
        !hinge_axis)) || !group || n_groups < 1 || !designs || !sun || n_pairs < 0 || samples < 1 || bounces < 1 ||
        !force || !torque || sampling < 0 || sampling > 3)
        return ORC_EINVAL;
    for (int64_t f = 0; f < n_tris; ++f)
        if (group[f] < 0 || group[f] >= n_groups) return ORC_EINVAL;
    if (vert_hinge)
        for (int64_t v = 0; v < n_verts; ++v)
            if (vert_hinge[v] < -1 || vert_hinge[v] >= n_hinges) return ORC_EINVAL;
    const int64_t P = n_hinges + 3 * n_groups;
    for (int64_t i = 0; i < n_pairs; ++i)
        for (int32_t g = 0; g < n_groups; ++g) {
            const double* m = designs + i * P + n_hinges + 3 * g;
            const float a = (float)m[0], b = (float)m[1];
            if (!(a >= 0.0f) || !(b >= 0.0f) || !(a + b <= 1.0f) || !((float)m[2] >= 1.0f)) return ORC_EINVAL;
        }
    designs_job_t J;
    memset(&J, 0, sizeof(J));
    J.verts = verts; J.n_verts = n_verts; J.tris = tris; J.n_tris = n_tris; J.vert_hinge = vert_hinge;
    J.hinge_origin = hinge_origin; J.hinge_axis = hinge_axis; J.n_hinges = n_hinges; J.group = group;
    J.n_groups = n_groups; J.designs = designs; J.sun = sun; J.n_pairs = n_pairs; J.samples = samples;
    J.bounces = bounces; J.sampling = sampling; J.flux = flux; J.seed = seed; J.dir_index_base = dir_index_base;
    J.design_index = design_index; J.com = com; J.force = force; J.torque = torque; J.rec_facet = rec_facet;
    J.rec_hits = rec_hits; J.rec_lit = rec_lit; J.rec_deg = rec_deg; J.status = ORC_OK;
    pthread_mutex_init(&J.lock, NULL);
    if (n_threads < 1) n_threads = 1;
    pthread_t* th = malloc(sizeof(pthread_t) * n_threads);
    for (int32_t t = 0; t < n_threads; ++t) pthread_create(&th[t], NULL, designs_worker, &J);
    for (int32_t t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
    free(th);
    pthread_mutex_destroy(&J.lock);
    return J.status;
}
