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

Multi-region bodies: the region sign of a triangle for region r is +1 if its
normal points into r (r is its front region), -1 if r lies behind it and 0 if
it does not border r (eqs. 12-13 with the inward normals of each region).
The basis function of an edge restricted to region r consists of its halves on
the triangles that border r, each weighted by that triangle's region sign; eq.
16 sums the regions' operators over these restrictions.

An interface edge has two triangles of one interface.  A junction edge, where
three regions meet along a line (the rim of an internal interface of a stacked
body), has three triangles, one per interface, and one basis function made of
three halves: on a triangle that runs along the edge from the smaller to the
larger vertex id it is + l/(2A)(r - v), on the others - l/(2A)(r - v).  Every
region sees two of the three triangles; the mesh must orient each region's
closed boundary consistently (seen from the region the two triangles run along
the edge in opposite directions), and then the two signed halves form an
ordinary RWG function of that boundary.  The unknown is the tangential field
along the junction line, which all three regions share.
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
    # every half of every basis function: triangle, free vertex and sign
    # (+1 on T+), [ne, 3], padded with -1 / -1 / 0 on interface edges
    side_tri: np.ndarray
    side_free: np.ndarray
    side_sign: np.ndarray

    @property
    def n_edges(self):
        return len(self.edge_v)

    def region_sign(self, r):
        """[ne] region sign of every edge for region r (0 where r is not
        adjacent), from the interface of the edge's T+ triangle."""
        return np.where(self.regions[:, 0] == r, 1.0, np.where(self.regions[:, 1] == r, -1.0, 0.0))

    def tri_region_sign(self, r):
        """[nt] region sign of every triangle for region r."""
        t = self.tri_regions
        return np.where(t[:, 0] == r, 1.0, np.where(t[:, 1] == r, -1.0, 0.0))

    def restricted_halves(self, r):
        """Halves of every basis function restricted to region r: arrays
        (edge, triangle, free vertex, coefficient) with coefficient = side
        sign * region sign of the triangle, for every half whose triangle
        borders r."""
        trs = self.tri_region_sign(r)
        e, i = np.nonzero(self.side_tri >= 0)
        t = self.side_tri[e, i]
        c = self.side_sign[e, i] * trs[t]
        keep = c != 0
        return e[keep], t[keep], self.side_free[e, i][keep], c[keep]


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
    sides = {}
    for ti, (a, b, c) in enumerate(t):
        for li, (free, (x, y)) in enumerate(zip((a, b, c), ((b, c), (c, a), (a, b)))):
            sides.setdefault((min(x, y), max(x, y)), []).append((1 if x < y else -1, ti, free, li))
    keys = sorted(sides)
    ne = len(keys)
    side_tri = np.full((ne, 3), -1, dtype=np.int64)
    side_free = np.full((ne, 3), -1, dtype=np.int64)
    side_sign = np.zeros((ne, 3))
    tri_edge = np.full((len(t), 3), -1, dtype=np.int64)
    tri_sign = np.zeros((len(t), 3))
    for e, k in enumerate(keys):
        sd = sorted(sides[k], key=lambda q: (-q[0], q[1]))      # T+ halves first
        if len(sd) < 2:
            raise MeshError("open surface or inconsistent orientation")
        if len(sd) > 3:
            raise MeshError(f"edge {k} shared by more than three triangles")
        regions = {int(r) for q in sd for r in reg[q[1]]}
        for r in regions:
            s_r = [(1 if reg[q[1], 0] == r else -1) * q[0] for q in sd if r in reg[q[1]]]
            if len(s_r) != 2:
                raise MeshError(f"edge {k}: region {r} sees {len(s_r)} of its triangles"
                                + (" (triangles of different interfaces)" if len(sd) == 2 else ""))
            if sum(s_r) != 0:
                raise MeshError(f"edge {k} traversed twice in the same direction by region {r}'s boundary "
                                "(orientation or non-manifold)")
        for i, (sg, ti, free, li) in enumerate(sd):
            side_tri[e, i], side_free[e, i], side_sign[e, i] = ti, free, sg
            tri_edge[ti, li] = e
            tri_sign[ti, li] = sg
    edge_v = np.array(keys, dtype=np.int64).reshape(ne, 2)
    # first T+ and first T- half of every edge (the two halves of an interface edge)
    first_m = np.argmax(side_sign < 0, axis=1)
    tri_p, free_p = side_tri[:, 0], side_free[:, 0]
    tri_m = side_tri[np.arange(ne), first_m]
    free_m = side_free[np.arange(ne), first_m]
    length = np.linalg.norm(v[edge_v[:, 0]] - v[edge_v[:, 1]], axis=1)
    return RWGMesh(v, t, reg, area, normal, (p0 + p1 + p2) / 3.0, el.max(axis=1),
                   quadrature.points(p0, p1, p2), edge_v, tri_p, tri_m, free_p, free_m, length,
                   reg[tri_p], tri_edge, tri_sign, side_tri, side_free, side_sign)


def from_body(body) -> RWGMesh:
    return build(body.vertices, body.triangles, body.tri_regions)


def basis_at(mesh: RWGMesh, n: int, tri: int, r):
    """Value of basis n at points r ([..., 3]) of triangle tri (for tests)."""
    r = np.asarray(r, dtype=float)
    for i in range(3):
        if mesh.side_tri[n, i] == tri:
            return mesh.side_sign[n, i] * mesh.length[n] / (2 * mesh.area[tri]) * \
                (r - mesh.vertices[mesh.side_free[n, i]])
    return np.zeros_like(r)
