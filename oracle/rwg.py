"""RWG basis functions on a closed triangulated surface (eq. 22 and Fig. 4).

For edge n shared by triangles T+ and T-, with free vertices v+ and v-,

    f_n(r) = + l_n / (2 A+) (r - v+)   on T+
    f_n(r) = - l_n / (2 A-) (r - v-)   on T-    (= l_n/(2A-) (v- - r))

so the current flows from T+ across the edge into T-, and its surface
divergence is +l_n/A+ on T+ and -l_n/A- on T-; the total charge of every basis
function is zero.

Canonical edge order and orientation (the library's boundary uses the same
convention, implemented separately): edges are sorted by (smaller vertex id,
larger vertex id); T+ is the triangle whose counter-clockwise vertex order
traverses the edge from the smaller to the larger vertex id.

Multi-region bodies: every edge lies on one interface, i.e. both of its
triangles carry the same (front region, back region) pair.  Its region sign is
+1 for the front region (the one the normal points into) and -1 for the back
region (eqs. 12-13 with the inward normals of each region).
"""

from __future__ import annotations

import dataclasses

import numpy as np

from . import quadrature


@dataclasses.dataclass
class RWGMesh:
    vertices: np.ndarray       # [nv, 3]
    triangles: np.ndarray      # [nt, 3]
    tri_regions: np.ndarray    # [nt, 2]
    # per triangle
    area: np.ndarray           # [nt]
    normal: np.ndarray         # [nt, 3] unit normal (right-hand rule)
    centroid: np.ndarray       # [nt, 3]
    max_edge: np.ndarray       # [nt]
    qpts: np.ndarray           # [nt, 7, 3] quadrature nodes
    # per edge (canonical order)
    edge_v: np.ndarray         # [ne, 2] (min id, max id)
    tri_p: np.ndarray          # [ne] T+
    tri_m: np.ndarray          # [ne] T-
    free_p: np.ndarray         # [ne] free vertex id of T+
    free_m: np.ndarray         # [ne] free vertex id of T-
    length: np.ndarray         # [ne]
    regions: np.ndarray        # [ne, 2] (front, back)
    # per triangle, for each local vertex i (0..2): the edge opposite to it and
    # the sign of that edge's basis function on this triangle (+1 on T+).
    tri_edge: np.ndarray       # [nt, 3]
    tri_sign: np.ndarray       # [nt, 3]

    @property
    def n_edges(self):
        return len(self.edge_v)

    def region_sign(self, r):
        """[ne] region sign of every edge for region r (0 where r is not adjacent)."""
        return np.where(self.regions[:, 0] == r, 1.0, np.where(self.regions[:, 1] == r, -1.0, 0.0))


class MeshError(ValueError):
    pass


def build(vertices, triangles, tri_regions) -> RWGMesh:
    v = np.asarray(vertices, dtype=np.float64)
    t = np.asarray(triangles, dtype=np.int64)
    reg = np.asarray(tri_regions, dtype=np.int64)
    p0, p1, p2 = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    cr = np.cross(p1 - p0, p2 - p0)
    two_a = np.linalg.norm(cr, axis=1)
    if np.any(two_a <= 0):
        raise MeshError("degenerate triangle")
    area = 0.5 * two_a
    normal = cr / two_a[:, None]
    el = np.stack([np.linalg.norm(p1 - p0, axis=1), np.linalg.norm(p2 - p1, axis=1),
                   np.linalg.norm(p0 - p2, axis=1)], axis=1)

    # directed edges of every triangle: local vertex i is free for the edge
    # running from vertex (i+1) to vertex (i+2) in CCW order
    plus, minus = {}, {}
    for ti, (a, b, c) in enumerate(t):
        for free, (x, y) in zip((a, b, c), ((b, c), (c, a), (a, b))):
            key = (min(x, y), max(x, y))
            side = plus if x < y else minus
            if key in side:
                raise MeshError(f"edge {key} traversed twice in the same direction (orientation or non-manifold)")
            side[key] = (ti, free)
    if set(plus) != set(minus):
        raise MeshError("open surface or inconsistent orientation")
    keys = sorted(plus)
    ne = len(keys)
    edge_v = np.array(keys, dtype=np.int64).reshape(ne, 2)
    tri_p = np.array([plus[k][0] for k in keys], dtype=np.int64)
    free_p = np.array([plus[k][1] for k in keys], dtype=np.int64)
    tri_m = np.array([minus[k][0] for k in keys], dtype=np.int64)
    free_m = np.array([minus[k][1] for k in keys], dtype=np.int64)
    if np.any(np.any(reg[tri_p] != reg[tri_m], axis=1)):
        raise MeshError("edge between triangles of different interfaces (junctions are not supported here)")
    length = np.linalg.norm(v[edge_v[:, 0]] - v[edge_v[:, 1]], axis=1)

    tri_edge = np.full((len(t), 3), -1, dtype=np.int64)
    tri_sign = np.zeros((len(t), 3))
    index = {k: i for i, k in enumerate(keys)}
    for ti, (a, b, c) in enumerate(t):
        for li, (x, y) in enumerate(((b, c), (c, a), (a, b))):
            e = index[(min(x, y), max(x, y))]
            tri_edge[ti, li] = e
            tri_sign[ti, li] = 1.0 if x < y else -1.0
    return RWGMesh(v, t, reg, area, normal, (p0 + p1 + p2) / 3.0, el.max(axis=1),
                   quadrature.points(p0, p1, p2), edge_v, tri_p, tri_m, free_p, free_m, length,
                   reg[tri_p], tri_edge, tri_sign)


def from_body(body) -> RWGMesh:
    return build(body.vertices, body.triangles, body.tri_regions)


def basis_at(mesh: RWGMesh, n: int, tri: int, r):
    """Value of basis n at points r ([..., 3]) of triangle tri (for tests)."""
    r = np.asarray(r, dtype=float)
    if tri == mesh.tri_p[n]:
        return mesh.length[n] / (2 * mesh.area[tri]) * (r - mesh.vertices[mesh.free_p[n]])
    if tri == mesh.tri_m[n]:
        return -mesh.length[n] / (2 * mesh.area[tri]) * (r - mesh.vertices[mesh.free_m[n]])
    return np.zeros_like(r)
