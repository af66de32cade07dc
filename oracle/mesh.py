"""Surface triangulations and uniform refinement with projected midpoints.

Follows Sec. 3 of the paper (first paragraphs and Fig. 2): the fine mesh T_h is
the uniform refinement of T_H, the new vertices are the midpoints of the coarse
edges, and those midpoints are moved onto the continuous surface Gamma (the
closest-point lift of eq. (lift) in Sec. 2.2).  All vertices therefore lie on
Gamma (Sec. 2.1), and the spaces on consecutive levels are not nested.

Conventions (the paper is silent on numbering; these readings are shared by the
library only through this written statement, not through code):
  * coarse edges (a, b) with a < b are enumerated in lexicographic order; the
    midpoint of edge e becomes vertex  N_coarse + e;
  * triangle (a, b, c) is split into (a, ab, ca), (ab, b, bc), (ca, bc, c),
    (ab, bc, ca), in the order of the parent triangles;
  * sphere: the projection is normalisation (the closest-point lift);
  * ellipsoid (semi-axes a0, a1, a2): the unit-sphere hierarchy mapped vertex by
    vertex, x -> (a0 x, a1 y, a2 z); vertices lie on the ellipsoid but the new
    ones are not closest-point lifts;
  * torus (R, r): 64 x 32 parametric grid; vertex (i, j) has index 32 i + j;
    quad (i, j) splits along the (i,j)-(i+1,j+1) diagonal; the projection is
    the closest-point map onto the torus.
"""
import numpy as np

PHI = (1.0 + 5.0 ** 0.5) / 2.0


def _orient_outward(xyz, tri):
    """Reorder each triangle so that its normal points away from the origin."""
    out = tri.copy()
    for t in range(len(tri)):
        a, b, c = tri[t]
        n = np.cross(xyz[b] - xyz[a], xyz[c] - xyz[a])
        if np.dot(n, xyz[a] + xyz[b] + xyz[c]) < 0:
            out[t] = (a, c, b)
    return out


def _rotate_min_first(tri):
    out = tri.copy()
    for t in range(len(tri)):
        k = int(np.argmin(tri[t]))
        out[t] = np.roll(tri[t], -k)
    return out


def icosahedron():
    """Regular icosahedron inscribed in the unit sphere: (xyz[12,3], tri[20,3]).

    Faces are the vertex triples that are pairwise at (unnormalised) distance 2,
    oriented outward, rotated so the smallest index is first, and sorted.
    """
    p = PHI
    v = np.array([(-1, p, 0), (1, p, 0), (-1, -p, 0), (1, -p, 0),
                  (0, -1, p), (0, 1, p), (0, -1, -p), (0, 1, -p),
                  (p, 0, -1), (p, 0, 1), (-p, 0, -1), (-p, 0, 1)], dtype=np.float64)
    faces = []
    n = len(v)
    d = np.linalg.norm(v[:, None, :] - v[None, :, :], axis=2)
    for a in range(n):
        for b in range(a + 1, n):
            for c in range(b + 1, n):
                if abs(d[a, b] - 2) < 1e-9 and abs(d[b, c] - 2) < 1e-9 and abs(d[a, c] - 2) < 1e-9:
                    faces.append((a, b, c))
    tri = np.array(faces, dtype=np.int64)
    tri = _rotate_min_first(_orient_outward(v, tri))
    tri = tri[np.lexsort((tri[:, 2], tri[:, 1], tri[:, 0]))]
    xyz = v / np.linalg.norm(v, axis=1, keepdims=True)
    return xyz, tri


def edges(tri):
    """Unique undirected edges (a < b) of a triangulation in lexicographic order."""
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    e = np.sort(e, axis=1)
    return np.unique(e, axis=0)


def refine(xyz, tri, project):
    """One uniform refinement step (Sec. 3, Fig. 2).

    Returns (xyz_fine, tri_fine, parents) where parents[e] = (a, b) are the two
    coarse vertices whose midpoint became fine vertex N_coarse + e.
    """
    n = len(xyz)
    E = edges(tri)
    eid = {(int(a), int(b)): n + i for i, (a, b) in enumerate(E)}

    def mid(a, b):
        return eid[(a, b) if a < b else (b, a)]

    new_pts = np.array([project(0.5 * (xyz[a] + xyz[b])) for a, b in E])
    xyz_f = np.concatenate([xyz, new_pts.reshape(-1, 3)])
    children = []
    for a, b, c in tri:
        a, b, c = int(a), int(b), int(c)
        ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
        children += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]
    return xyz_f, np.array(children, dtype=np.int64), E.astype(np.int64)


def project_sphere(p):
    """Closest-point lift onto the unit sphere (eq. lift)."""
    return p / np.linalg.norm(p)


def torus_project(R, r):
    def proj(p):
        c = R * np.array([p[0], p[1], 0.0]) / np.hypot(p[0], p[1])
        d = p - c
        return c + r * d / np.linalg.norm(d)
    return proj


def torus_grid(R=1.0, r=0.4, nu=64, nv=32):
    """Coarse torus mesh from an nu x nv parametric grid (vertex index nv*i + j)."""
    xyz = np.zeros((nu * nv, 3))
    for i in range(nu):
        u = 2 * np.pi * i / nu
        for j in range(nv):
            v = 2 * np.pi * j / nv
            xyz[nv * i + j] = ((R + r * np.cos(v)) * np.cos(u),
                               (R + r * np.cos(v)) * np.sin(u), r * np.sin(v))
    tri = []
    for i in range(nu):
        for j in range(nv):
            p00 = nv * i + j
            p10 = nv * ((i + 1) % nu) + j
            p11 = nv * ((i + 1) % nu) + (j + 1) % nv
            p01 = nv * i + (j + 1) % nv
            tri += [(p00, p10, p11), (p00, p11, p01)]
    tri = np.array(tri, dtype=np.int64)
    # outward: normal points away from the tube centre line
    out = tri.copy()
    for t in range(len(tri)):
        a, b, c = tri[t]
        n = np.cross(xyz[b] - xyz[a], xyz[c] - xyz[a])
        cen = (xyz[a] + xyz[b] + xyz[c]) / 3
        core = R * np.array([cen[0], cen[1], 0.0]) / np.hypot(cen[0], cen[1])
        if np.dot(n, cen - core) < 0:
            out[t] = (a, c, b)
    return xyz, out


class Level:
    """One level of the hierarchy: vertices, triangles, parents of new vertices."""

    def __init__(self, xyz, tri, parents=None):
        self.xyz = xyz
        self.tri = tri
        self.parents = parents  # None on level 0


def hierarchy(kind, n_refine, axes=(1.0, 1.0, 1.0), R=1.0, r=0.4, nu=64, nv=32, flat=False):
    """Levels 0..n_refine of a sphere / ellipsoid / torus hierarchy.

    flat=True skips the projection of midpoints (nested meshes; used only by
    the nested-Galerkin identity pin).
    """
    if kind in ("sphere", "ellipsoid"):
        xyz, tri = icosahedron()
        proj = (lambda p: p) if flat else project_sphere
    elif kind == "torus":
        xyz, tri = torus_grid(R, r, nu, nv)
        proj = (lambda p: p) if flat else torus_project(R, r)
    else:
        raise ValueError(kind)
    levels = [Level(xyz, tri)]
    for _ in range(n_refine):
        xyz, tri, par = refine(xyz, tri, proj)
        levels.append(Level(xyz, tri, par))
    if kind == "ellipsoid":
        s = np.asarray(axes, dtype=np.float64)
        for lv in levels:
            lv.xyz = lv.xyz * s[None, :]
    return levels
