"""Closed triangle meshes for the scatterers studied with the surface integral method.

Every body is described the way the library's C interface takes it: vertex
coordinates in metres, triangles as vertex triples ordered counter-clockwise
about the surface normal, and for every triangle the pair
``(region the normal points into, region behind it)``.  Region 0 is the
unbounded background (free space).  Material parameters are relative
permittivity and permeability per region under the e^{+j omega t} convention,
so a lossy medium has a negative imaginary part.

The free-space wavelength is fixed at 1 m, so lengths are in wavelengths.
"""

from __future__ import annotations

import dataclasses
import itertools

import numpy as np

C0 = 299792458.0          # speed of light in vacuum, m/s (exact, SI)
WAVELENGTH = 1.0          # free-space wavelength used by every workload, m
FREQUENCY = C0 / WAVELENGTH


@dataclasses.dataclass
class Body:
    """One scatterer: a closed (possibly multi-region) triangulated surface."""

    vertices: np.ndarray      # [nv, 3] float64, metres
    triangles: np.ndarray     # [nt, 3] int32, CCW about the normal
    tri_regions: np.ndarray   # [nt, 2] int32: (region in front of normal, region behind)
    eps_r: np.ndarray         # [nr] complex128, region 0 first
    mu_r: np.ndarray          # [nr] complex128
    frequency: float = FREQUENCY
    name: str = ""

    @property
    def n_regions(self) -> int:
        return int(len(self.eps_r))

    def mean_edge_length(self) -> float:
        tri = self.triangles
        e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
        e = np.unique(np.sort(e, axis=1), axis=0)
        d = self.vertices[e[:, 0]] - self.vertices[e[:, 1]]
        return float(np.sqrt((d * d).sum(1)).mean())


def _icosahedron():
    """Unit icosahedron: 12 vertices, 20 faces with outward CCW orientation."""
    g = (1.0 + 5.0 ** 0.5) / 2.0
    v = []
    for a, b in itertools.product((-1.0, 1.0), repeat=2):
        v += [(0.0, a, b * g), (a, b * g, 0.0), (b * g, 0.0, a)]
    v = np.array(v)
    # faces are the vertex triples that are pairwise at the edge length 2
    faces = []
    for i, j, k in itertools.combinations(range(12), 3):
        if all(abs(np.linalg.norm(v[p] - v[q]) - 2.0) < 1e-9 for p, q in ((i, j), (j, k), (i, k))):
            n = np.cross(v[j] - v[i], v[k] - v[i])
            faces.append((i, j, k) if n @ (v[i] + v[j] + v[k]) > 0 else (i, k, j))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v, np.array(faces, dtype=np.int64)


def icosphere(subdivisions: int, radius: float = 1.0):
    """Icosphere: each subdivision splits every triangle into four through the
    edge midpoints, pushed out onto the sphere.  Vertices lie on the sphere
    (an inscribed polyhedron); faces keep the outward CCW orientation.

    Returns ``(vertices [nv,3] float64, triangles [nt,3] int32)`` with
    30*4**s edges, 20*4**s triangles and 10*4**s + 2 vertices.
    """
    v, f = _icosahedron()
    verts = [tuple(p) for p in v]
    for _ in range(subdivisions):
        mid = {}

        def midpoint(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in mid:
                p = np.add(verts[a], verts[b])
                p /= np.linalg.norm(p)
                mid[key] = len(verts)
                verts.append(tuple(p))
            return mid[key]

        nf = []
        for a, b, c in f:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        f = np.array(nf, dtype=np.int64)
    return np.array(verts) * radius, f.astype(np.int32)


def sphere_body(radius: float, eps_r: complex, subdivisions: int, mu_r: complex = 1.0,
                name: str = "") -> Body:
    """Homogeneous dielectric sphere (region 1) in free space (region 0)."""
    v, t = icosphere(subdivisions, radius)
    reg = np.tile(np.array([[0, 1]], dtype=np.int32), (len(t), 1))
    return Body(v, t, reg, np.array([1.0, eps_r], dtype=complex), np.array([1.0, mu_r], dtype=complex),
                name=name or f"sphere r={radius} eps={eps_r} s={subdivisions}")


def coated_sphere_body(core_radius: float, core_eps: complex, core_sub: int,
                       shell_radius: float, shell_eps: complex, shell_sub: int,
                       name: str = "") -> Body:
    """Two-layer sphere: core (region 2) inside a shell (region 1) in free space.

    The outer surface separates regions (0, 1) and the inner one (1, 2); both
    normals point outward, i.e. into the lower-numbered region.
    """
    vo, to = icosphere(shell_sub, shell_radius)
    vi, ti = icosphere(core_sub, core_radius)
    v = np.concatenate([vo, vi])
    t = np.concatenate([to, ti + len(vo)]).astype(np.int32)
    reg = np.concatenate([np.tile([[0, 1]], (len(to), 1)), np.tile([[1, 2]], (len(ti), 1))]).astype(np.int32)
    eps = np.array([1.0, shell_eps, core_eps], dtype=complex)
    return Body(v, t, reg, eps, np.ones(3, dtype=complex),
                name=name or f"coated sphere core {core_radius}/{core_eps} shell {shell_radius}/{shell_eps}")


def ellipsoid_batch(n_bodies: int = 48, seed: int = 0, edge_rule: float = 1.0 / 12.0,
                    subdivision_choices=(3, 4, 5)):
    """Seeded batch of homogeneous dielectric ellipsoids.

    Semi-axes are drawn uniform in [0.3, 1.5] wavelengths (all 3*n first), then
    relative permittivities uniform in [2, 10].  Each body is an icosphere
    scaled per axis, at the smallest subdivision whose mean edge length is at
    most ``edge_rule`` wavelengths.
    """
    rng = np.random.default_rng(seed)
    axes = rng.uniform(0.3, 1.5, size=(n_bodies, 3))
    eps = rng.uniform(2.0, 10.0, size=n_bodies)
    bodies = []
    for i in range(n_bodies):
        for s in subdivision_choices:
            v, t = icosphere(s, 1.0)
            v = v * axes[i]
            reg = np.tile(np.array([[0, 1]], dtype=np.int32), (len(t), 1))
            b = Body(v, t, reg, np.array([1.0, eps[i]], dtype=complex), np.ones(2, dtype=complex),
                     name=f"ellipsoid {i} axes {axes[i].round(3).tolist()} eps {eps[i]:.3f} s={s}")
            if b.mean_edge_length() <= edge_rule or s == subdivision_choices[-1]:
                bodies.append(b)
                break
    return bodies


def _disc_mesh(radius: float, z: float, ring: np.ndarray, n_phi: int, target_edge: float):
    """Triangulated disc at height z whose boundary uses the given ring nodes.

    Concentric rings with node counts decreasing towards the centre; returns
    (vertices, triangles with normal +z) using local indices where the first
    n_phi vertices are the outer ring (same order as ``ring``).
    """
    n_rings = max(1, int(round(radius / target_edge)))
    verts = [p for p in ring]
    rings = [list(range(n_phi))]
    for i in range(1, n_rings):
        r = radius * (n_rings - i) / n_rings
        m = max(6, int(round(2 * np.pi * r / target_edge)))
        start = len(verts)
        phase = 0.5 * (i % 2) * 2 * np.pi / m
        for j in range(m):
            a = 2 * np.pi * j / m + phase
            verts.append((r * np.cos(a), r * np.sin(a), z))
        rings.append(list(range(start, start + m)))
    centre = len(verts)
    verts.append((0.0, 0.0, z))
    verts = np.array(verts, dtype=float)
    tris = []

    def angle(k):
        return np.arctan2(verts[k, 1], verts[k, 0]) % (2 * np.pi)

    for outer, inner in zip(rings[:-1], rings[1:]):
        # advancing front between two rings, both sorted by angle
        o = sorted(outer, key=angle)
        n = sorted(inner, key=angle)
        i = j = 0
        while i < len(o) or j < len(n):
            a_o = angle(o[(i + 1) % len(o)]) + (2 * np.pi if i + 1 >= len(o) else 0.0)
            a_n = angle(n[(j + 1) % len(n)]) + (2 * np.pi if j + 1 >= len(n) else 0.0)
            if j >= len(n) or (i < len(o) and a_o <= a_n):
                tris.append((o[i % len(o)], o[(i + 1) % len(o)], n[j % len(n)]))
                i += 1
            else:
                tris.append((o[i % len(o)], n[(j + 1) % len(n)], n[j % len(n)]))
                j += 1
    last = sorted(rings[-1], key=angle)
    for j in range(len(last)):
        tris.append((last[j], last[(j + 1) % len(last)], centre))
    tris = np.array(tris, dtype=np.int64)
    # orient every triangle with normal +z
    e1 = verts[tris[:, 1]] - verts[tris[:, 0]]
    e2 = verts[tris[:, 2]] - verts[tris[:, 0]]
    flip = np.cross(e1, e2)[:, 2] < 0
    tris[flip] = tris[flip][:, [0, 2, 1]]
    return verts, tris


def stacked_cylinder_body(radius: float = 1.0, height: float = 3.0, eps_layers=(2.2, 4.4, 10.2),
                          target_edge: float = 0.05, name: str = "", merge_layers: bool = False) -> Body:
    """Stack of equal-height dielectric cylinder layers (regions 1..n, bottom up).

    The side wall and the two end caps separate the layers from free space; the
    internal discs separate neighbouring layers (normal +z, i.e. pointing into
    the upper layer).  Every surface shares its boundary ring nodes, so the
    rings where a side wall meets an internal disc carry edges bordered by three
    triangles (junction edges).

    merge_layers=True builds the same outer surface (identical vertices and
    triangles) without the internal discs, as one homogeneous region of
    permittivity eps_layers[0].
    """
    n_layers = len(eps_layers)
    n_phi = int(round(2 * np.pi * radius / target_edge))
    layer_h = height / n_layers
    n_z = max(1, int(round(layer_h / (target_edge * np.sqrt(3) / 2))))
    verts = []
    ring_ids = []       # vertex ids of every ring from bottom to top
    z_levels = []
    for il in range(n_layers):
        for iz in range(n_z + (1 if il == n_layers - 1 else 0)):
            z = il * layer_h + iz * layer_h / n_z - height / 2
            phase = 0.5 * ((il * n_z + iz) % 2) * 2 * np.pi / n_phi
            ids = []
            for j in range(n_phi):
                a = 2 * np.pi * j / n_phi + phase
                ids.append(len(verts))
                verts.append((radius * np.cos(a), radius * np.sin(a), z))
            ring_ids.append(ids)
            z_levels.append(z)
    tris, regs = [], []
    for r in range(len(ring_ids) - 1):
        layer = min(r // n_z, n_layers - 1) + 1
        lo, hi = ring_ids[r], ring_ids[r + 1]
        shifted = (r % 2) == 0   # the upper ring is rotated by +half a step
        for j in range(n_phi):
            j1 = (j + 1) % n_phi
            if shifted:
                tris += [(lo[j], lo[j1], hi[j]), (lo[j1], hi[j1], hi[j])]
            else:
                tris += [(lo[j], lo[j1], hi[j1]), (lo[j], hi[j1], hi[j])]
            regs += [(0, layer), (0, layer)]
    verts = np.array(verts, dtype=float)
    tris = np.array(tris, dtype=np.int64)
    # outward orientation of the side wall (normal away from the axis)
    cen = verts[tris].mean(1)
    nrm = np.cross(verts[tris[:, 1]] - verts[tris[:, 0]], verts[tris[:, 2]] - verts[tris[:, 0]])
    flip = (nrm[:, 0] * cen[:, 0] + nrm[:, 1] * cen[:, 1]) < 0
    tris[flip] = tris[flip][:, [0, 2, 1]]
    all_v = [verts]
    all_t = [tris]
    all_r = [np.array(regs, dtype=np.int64)]
    nv = len(verts)
    # discs: bottom cap, internal interfaces, top cap
    for k in range(n_layers + 1):
        if merge_layers and 0 < k < n_layers:
            continue
        ring = ring_ids[k * n_z] if k < n_layers else ring_ids[-1]
        z = verts[ring[0], 2]
        dv, dt = _disc_mesh(radius, z, verts[ring], n_phi, target_edge)
        # map local ids: first n_phi are the shared ring nodes
        gid = np.empty(len(dv), dtype=np.int64)
        gid[:n_phi] = ring
        gid[n_phi:] = nv + np.arange(len(dv) - n_phi)
        nv += len(dv) - n_phi
        all_v.append(dv[n_phi:])
        tri = gid[dt]
        if k == 0:
            tri = tri[:, [0, 2, 1]]              # bottom cap: normal -z into free space
            reg = (0, 1)
        elif k == n_layers:
            reg = (0, n_layers)                  # top cap: normal +z into free space
        else:
            reg = (k + 1, k)                     # normal +z points into the upper layer
        all_t.append(tri)
        all_r.append(np.tile(np.array([reg]), (len(tri), 1)))
    v = np.concatenate(all_v)
    t = np.concatenate(all_t).astype(np.int32)
    rg = np.concatenate(all_r).astype(np.int32)
    if merge_layers:
        rg = np.minimum(rg, 1)
        eps = np.array([1.0, eps_layers[0]], dtype=complex)
        return Body(v, t, rg, eps, np.ones(2, dtype=complex),
                    name=name or f"cylinder r={radius} h={height} eps={eps_layers[0]}")
    eps = np.array([1.0] + list(eps_layers), dtype=complex)
    return Body(v, t, rg, eps, np.ones(n_layers + 1, dtype=complex),
                name=name or f"stacked cylinder r={radius} h={height} eps={list(eps_layers)}")
