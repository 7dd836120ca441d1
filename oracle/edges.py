"""Which moving edges the oracle's visibility-edge estimator takes (test infrastructure: only the
tests, the smoke check and the benchmark's CPU leg use this package).

The edge part of the hinge-angle gradient integrates (g(y - delta n) - g(y + delta n)) v_n along
the image of every moving edge (paper Sec. 3.3: the visibility discontinuities the gradient must
account for), g(y) the momentum a path started at image point y deposits.  Across an edge where
the moving surface simply continues in the same plane with the same material, g is continuous:
the two side paths meet facets of one plane and material, leave in the same direction with the
same draws, and their deposits differ only by O(delta) (the torque lever arm, and later bounces
that separate with probability O(delta)).  Such edges contribute nothing as delta -> 0 and are
left out; every other moving edge (silhouettes, creases, material boundaries, edges shared with
facets another hinge or the rigid body carries) is kept.

The rule, per distinct moving edge (the numbering of oracle_edge_term: edges of facets whose
three vertices one hinge carries, by first appearance over facets and edge slots, coincident
edges counted once):
  * every facet of the mesh that contains the edge (both endpoint positions) must be carried by
    the edge's hinge (a facet of the rigid body or of another hinge moves differently);
  * those facets are grouped by unit normal (components equal within `tol`); there are at most
    two groups, and two only with opposite normals (the two layers of a two-sided sheet, each
    checked on its own; planes that cross at the edge are a visibility discontinuity);
  * every group holds exactly two facets, whose third vertices lie on opposite sides of the edge,
    with equal rho_s, rho_d and (when given) p_spec.
"""
import numpy as np


def _carrier(vh, t):
    """The hinge carrying all three vertices of facet t, else -1."""
    k = int(vh[t[0]])
    return k if k >= 0 and vh[t[1]] == k and vh[t[2]] == k else -1


def moving_edges(verts, tris, vert_hinge):
    """Distinct edges of hinge-carried facets in order of first appearance.

    Returns a list of (a, b, hinge, incident), incident = [(facet, opposite vertex), ...] over all
    facets of the mesh containing the edge (matched by the two endpoint positions)."""
    V = np.asarray(verts, dtype=np.float64)
    T = np.asarray(tris)
    vh = np.asarray(vert_hinge)
    index = {}
    out = []
    for f, t in enumerate(T):
        k = _carrier(vh, t)
        if k < 0:
            continue
        for slot in range(3):
            a, b = int(t[slot]), int(t[(slot + 1) % 3])
            key = tuple(sorted([tuple(V[a]), tuple(V[b])]))
            if key not in index:
                index[key] = len(out)
                out.append((a, b, k, []))
    for f, t in enumerate(T):
        for slot in range(3):
            a, b, c = int(t[slot]), int(t[(slot + 1) % 3]), int(t[(slot + 2) % 3])
            key = tuple(sorted([tuple(V[a]), tuple(V[b])]))
            if key in index:
                out[index[key]][3].append((f, c))
    return out


def smooth_edge_mask(verts, tris, vert_hinge, rho_s, rho_d, p_spec=None, tol=1e-9):
    """Boolean per moving edge (numbering of moving_edges): True where the grid integrand is
    continuous across the edge and the edge term leaves it out."""
    V = np.asarray(verts, dtype=np.float64)
    T = np.asarray(tris)
    rs = np.asarray(rho_s, dtype=np.float32)
    rd = np.asarray(rho_d, dtype=np.float32)
    ps = None if p_spec is None else np.asarray(p_spec, dtype=np.float32)
    vh = np.asarray(vert_hinge)
    edges = moving_edges(V, T, vh)
    out = np.zeros(len(edges), dtype=bool)
    for e, (a, b, k, incident) in enumerate(edges):
        if any(_carrier(vh, T[f]) != k for f, _ in incident):
            continue
        groups = []
        for f, c in incident:
            p = V[T[f]]
            n = np.cross(p[1] - p[0], p[2] - p[0])
            n = n / np.linalg.norm(n)
            for g in groups:
                if np.abs(g[0] - n).max() <= tol:
                    g[1].append((f, c))
                    break
            else:
                groups.append((n, [(f, c)]))
        if len(groups) > 2 or (len(groups) == 2 and np.abs(groups[0][0] + groups[1][0]).max() > tol):
            continue
        smooth = True
        for n, members in groups:
            if len(members) != 2:
                smooth = False
                break
            (f0, c0), (f1, c1) = members
            ab = V[b] - V[a]
            side0 = np.dot(np.cross(ab, V[c0] - V[a]), n)
            side1 = np.dot(np.cross(ab, V[c1] - V[a]), n)
            same = rs[f0] == rs[f1] and rd[f0] == rd[f1] and (ps is None or ps[f0] == ps[f1])
            if not (side0 * side1 < 0.0 and same):
                smooth = False
                break
        out[e] = smooth
    return out
