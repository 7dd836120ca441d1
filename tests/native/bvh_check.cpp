// Host check of the BVH builder and refit (built with g++ against the library's sources by the
// test-suite; no GPU).  Reads "n_verts n_tris pad" then vertices and triangles on stdin, builds the
// tree, optionally refits it to a second vertex set, and prints one line per check:
//   nodes depth max_leaf covered_once boxes_contain_tris children_inside_parent
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../paper_2602_10712_amd/csrc/bvh_build.h"

using namespace srp;

static bool check(const std::vector<BvhNode>& nodes, const std::vector<int32_t>& perm, const std::vector<double>& V,
                  const std::vector<int32_t>& T, int64_t nt, int depth)
{
    std::vector<int> seen(nt, 0);
    int max_leaf = 0;
    bool contain = true, nested = true;
    // box of node i's child slot s
    auto child_box = [&](int i, int s, float lo[3], float hi[3]) {
        const BvhNode& n = nodes[i];
        if (s == 0) {
            lo[0] = n.f[0].x; hi[0] = n.f[0].y; lo[1] = n.f[0].z; hi[1] = n.f[0].w; lo[2] = n.f[2].x; hi[2] = n.f[2].y;
        } else {
            lo[0] = n.f[1].x; hi[0] = n.f[1].y; lo[1] = n.f[1].z; hi[1] = n.f[1].w; lo[2] = n.f[2].z; hi[2] = n.f[2].w;
        }
    };
    for (size_t i = 0; i < nodes.size(); ++i) {
        int32_t codes[2];
        std::memcpy(codes, &nodes[i].f[3], 8);
        for (int s = 0; s < 2; ++s) {
            float lo[3], hi[3];
            child_box(static_cast<int>(i), s, lo, hi);
            const int32_t c = codes[s];
            if (c >= 0) {
                if (c <= static_cast<int32_t>(i) || c >= static_cast<int32_t>(nodes.size())) nested = false;
                for (int q = 0; q < 2; ++q) {
                    float l2[3], h2[3];
                    child_box(c, q, l2, h2);
                    int32_t cc[2];
                    std::memcpy(cc, &nodes[c].f[3], 8);
                    if (cc[q] < 0 && ((~cc[q]) & 7) == 0) continue;
                    for (int a = 0; a < 3; ++a)
                        if (l2[a] < lo[a] || h2[a] > hi[a]) nested = false;
                }
            } else {
                const int32_t code = ~c;
                const int32_t first = code >> 3, cnt = code & 7;
                if (cnt > max_leaf) max_leaf = cnt;
                for (int32_t q = first; q < first + cnt; ++q) {
                    if (q < 0 || q >= nt) return false;
                    const int32_t f = perm[q];
                    seen[f]++;
                    for (int k = 0; k < 3; ++k)
                        for (int a = 0; a < 3; ++a) {
                            const double x = V[3 * T[3 * f + k] + a];
                            if (!(x >= lo[a] && x <= hi[a])) contain = false;
                        }
                }
            }
        }
    }
    bool once = true;
    for (int64_t f = 0; f < nt; ++f)
        if (seen[f] != 1) once = false;
    std::printf("%zu %d %d %d %d %d\n", nodes.size(), depth, max_leaf, once ? 1 : 0, contain ? 1 : 0, nested ? 1 : 0);
    return once && contain && nested;
}

int main()
{
    long long nv, nt;
    double pad;
    int refit;
    if (std::scanf("%lld %lld %lf %d", &nv, &nt, &pad, &refit) != 4) return 2;
    std::vector<double> V(3 * nv), V2(3 * nv);
    std::vector<int32_t> T(3 * nt);
    for (auto& x : V) std::scanf("%lf", &x);
    for (auto& t : T) std::scanf("%d", &t);
    BvhBuildResult r = build_bvh(V.data(), T.data(), nt, pad);
    bool ok = check(r.nodes, r.perm, V, T, nt, r.depth);
    if (refit) {
        for (auto& x : V2) std::scanf("%lf", &x);
        refit_bvh(r.nodes, r.perm, V2.data(), T.data(), pad);
        ok = check(r.nodes, r.perm, V2, T, nt, r.depth) && ok;
    }
    return ok ? 0 : 1;
}
