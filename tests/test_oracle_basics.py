"""Pins of the oracle's building blocks against mathematics that does not
depend on the oracle: exactness of the triangle rule, RWG invariants,
closed-form triangle integrals against brute-force adaptive quadrature, and
the octree/ordering invariants."""

import math

import numpy as np
import pytest

from oracle import octree, potentials, quadrature, rwg
from workloads import icosphere, sphere_body, coated_sphere_body


# --- quadrature ------------------------------------------------------------

def _ref_triangle_monomial(a, b):
    # int over the unit right triangle of x^a y^b = a! b! / (a + b + 2)!
    return math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)


def test_seven_point_rule_exact_to_degree_five():
    p0, p1, p2 = np.array([0.0, 0, 0]), np.array([1.0, 0, 0]), np.array([0.0, 1, 0])
    pts = quadrature.points(p0, p1, p2)
    assert abs(quadrature.WEIGHTS.sum() - 1.0) < 1e-15
    for a in range(6):
        for b in range(6 - a):
            q = 0.5 * np.sum(quadrature.WEIGHTS * pts[:, 0] ** a * pts[:, 1] ** b)
            assert abs(q - _ref_triangle_monomial(a, b)) < 1e-15, (a, b)
    # degree 6 is not integrated exactly (the rule is not of higher degree)
    q = 0.5 * np.sum(quadrature.WEIGHTS * pts[:, 0] ** 6)
    assert abs(q - _ref_triangle_monomial(6, 0)) > 1e-6


# --- RWG ---------------------------------------------------------------------

@pytest.mark.parametrize("s", [0, 1, 2])
def test_icosphere_rwg_invariants(s):
    v, t = icosphere(s, 0.7)
    reg = np.tile([[0, 1]], (len(t), 1))
    m = rwg.build(v, t, reg)
    assert len(v) - m.n_edges + len(t) == 2                    # Euler, closed genus 0
    assert m.n_edges == 30 * 4 ** s
    assert np.all(m.edge_v[:, 0] < m.edge_v[:, 1])
    assert np.all(np.diff(m.edge_v[:, 0] * len(v) + m.edge_v[:, 1]) > 0)   # canonical order
    # outward normals on a sphere
    assert np.all(np.sum(m.normal * m.centroid, axis=1) > 0)
    # T+ traverses the edge min -> max counter-clockwise
    for e in range(0, m.n_edges, 7):
        tri = list(m.triangles[m.tri_p[e]])
        i = tri.index(m.edge_v[e, 0])
        assert tri[(i + 1) % 3] == m.edge_v[e, 1]
    # the normal component of f_n across its edge is 1 from both sides, and
    # the total charge is zero
    for e in range(0, m.n_edges, 5):
        a, b = m.vertices[m.edge_v[e]]
        mid = 0.5 * (a + b)
        for tri, sgn in ((m.tri_p[e], 1.0), (m.tri_m[e], -1.0)):
            c = m.centroid[tri]
            s_hat = (b - a) / np.linalg.norm(b - a)
            out = (mid - c) - np.dot(mid - c, s_hat) * s_hat
            out /= np.linalg.norm(out)
            f = rwg.basis_at(m, e, tri, mid)
            assert abs(np.dot(f, out) - sgn) < 1e-12
        q = m.length[e] / m.area[m.tri_p[e]] * m.area[m.tri_p[e]] - m.length[e] / m.area[m.tri_m[e]] * m.area[m.tri_m[e]]
        assert abs(q) < 1e-15


def test_open_or_misoriented_mesh_is_rejected():
    v, t = icosphere(1)
    reg = np.tile([[0, 1]], (len(t), 1))
    with pytest.raises(rwg.MeshError):
        rwg.build(v, t[1:], reg[1:])
    t2 = t.copy()
    t2[0] = t2[0, [0, 2, 1]]
    with pytest.raises(rwg.MeshError):
        rwg.build(v, t2, reg)


def test_coated_sphere_interfaces():
    b = coated_sphere_body(0.5, 6 - 0.5j, 1, 0.8, 2.56, 1)
    m = rwg.from_body(b)
    assert m.n_edges == 2 * 120
    assert set(map(tuple, m.regions)) == {(0, 1), (1, 2)}
    s1 = m.region_sign(1)
    assert np.all(s1[m.regions[:, 0] == 1] == 1) and np.all(s1[m.regions[:, 1] == 1] == -1)


# --- closed-form triangle integrals vs brute force ---------------------------

TRI = np.array([[0.0, 0.0, 0.0], [1.0, 0.1, 0.0], [0.3, 0.9, 0.0]])


def _brute(r, tri, ncomp=14):
    """The six integrals by brute-force Gauss quadrature on the three
    sub-triangles (rho, a, b) around the projection rho (signed areas), with
    r' = rho + u (a - rho + v (b - a)), dS' = u |..| du dv; the u direction is
    split geometrically towards u = 0 on the scale |h| / |a - rho| so that the
    near-singular behaviour is resolved."""
    n = np.cross(tri[1] - tri[0], tri[2] - tri[0])
    n /= np.linalg.norm(n)
    h = (r - tri[0]) @ n
    rho = r - h * n
    gx, gw = np.polynomial.legendre.leggauss(40)
    total = np.zeros(ncomp)
    for i in range(3):
        a, b = tri[i], tri[(i + 1) % 3]
        c = np.cross(a - rho, b - rho) @ n
        if abs(c) < 1e-14:
            continue
        # v: uniform split into 8 panels
        vb = np.linspace(0.0, 1.0, 9)
        scale = abs(h) / max(np.linalg.norm(a - rho), np.linalg.norm(b - rho))
        ub = [0.0]
        if scale > 0:
            t = scale / 1024
            while t < 1.0:
                ub.append(t)
                t *= 2.0
        ub.append(1.0)
        for v0, v1 in zip(vb[:-1], vb[1:]):
            v = v0 + (v1 - v0) * 0.5 * (gx + 1)
            wv = (v1 - v0) * 0.5 * gw
            for u0, u1 in zip(ub[:-1], ub[1:]):
                u = u0 + (u1 - u0) * 0.5 * (gx + 1)
                wu = (u1 - u0) * 0.5 * gw
                w = (a - rho)[None, :] + v[:, None] * (b - a)[None, :]          # [nv, 3]
                p = rho + u[None, :, None] * w[:, None, :]                      # [nv, nu, 3]
                d = r - p
                R = np.linalg.norm(d, axis=-1)[..., None]
                vals = [1 / R, R, (p - rho) / R, (p - rho) * R]
                if ncomp == 14:
                    vals += [-d / R ** 3, d / R]
                f = np.concatenate(vals, axis=-1) * u[None, :, None]
                total += c * np.einsum("v,u,vuc->c", wv, wu, f)
    return total


@pytest.mark.parametrize("r", [
    [0.3, 0.3, 0.2],        # above the interior
    [0.3, 0.3, 0.01],       # close above the interior
    [0.5, 0.05, -0.002],    # very close below, near an edge
    [-0.5, 1.2, -0.3],      # below, projection outside
    [1.2, 1.1, 0.05],       # slightly above, projection outside
])
def test_closed_form_integrals_match_brute_force(r):
    r = np.array(r)
    res = potentials.triangle_integrals(r, *TRI)
    bf = _brute(r, TRI)
    got = np.concatenate([[res["inv_r"], res["r1"]], res["vinv_r"], res["vr1"], res["grad_inv_r"], res["grad_r1"]])
    assert np.allclose(got, bf, rtol=1e-9, atol=1e-10), np.abs(got - bf).max()


def test_closed_form_coplanar_points():
    # in-plane observation point inside (weakly singular) and outside (regular)
    r_in = np.array([0.4, 0.3, 0.0])
    res = potentials.triangle_integrals(r_in, *TRI)
    bf = _brute(r_in, TRI, ncomp=8)
    got = np.concatenate([[res["inv_r"], res["r1"]], res["vinv_r"], res["vr1"]])
    assert np.allclose(got, bf, rtol=1e-9, atol=1e-10)
    # outside: plain Gauss on the triangle is enough (no singularity)
    r_out = np.array([1.8, -0.4, 0.0])
    gx, gw = np.polynomial.legendre.leggauss(60)
    acc = np.zeros(14)
    for x, wx in zip(0.5 * (gx + 1), 0.5 * gw):
        for y, wy in zip(0.5 * (gx + 1), 0.5 * gw):
            p = TRI[0] + x * (TRI[1] - TRI[0]) + x * y * (TRI[2] - TRI[1])
            jac = x * np.linalg.norm(np.cross(TRI[1] - TRI[0], TRI[2] - TRI[1]))
            d = r_out - p
            R = np.linalg.norm(d)
            rho = r_out
            acc += wx * wy * jac * np.concatenate([[1 / R, R], (p - rho) / R, (p - rho) * R, -d / R ** 3, d / R])
    res = potentials.triangle_integrals(r_out, *TRI)
    got = np.concatenate([[res["inv_r"], res["r1"]], res["vinv_r"], res["vr1"], res["grad_inv_r"], res["grad_r1"]])
    assert np.allclose(got, acc, rtol=1e-9, atol=1e-11)


def test_solid_angle_jump():
    # the normal component of int grad(1/R) tends to -/+ 2 pi on either side
    res_p = potentials.triangle_integrals(np.array([0.4, 0.3, 1e-9]), *TRI)
    res_m = potentials.triangle_integrals(np.array([0.4, 0.3, -1e-9]), *TRI)
    assert abs(res_p["grad_inv_r"][2] + 2 * np.pi) < 1e-6
    assert abs(res_m["grad_inv_r"][2] - 2 * np.pi) < 1e-6
    res_0 = potentials.triangle_integrals(np.array([0.4, 0.3, 1e-9]), *TRI, coplanar=True)
    assert res_0["grad_inv_r"][2] == 0.0


# --- octree ------------------------------------------------------------------

def test_octree_keys_near_and_colours():
    b = sphere_body(0.3, 4.0, 2)
    m = rwg.from_body(b)
    assert octree.auto_levels(m, 0.15) == 3
    keys = octree.finest_keys(m, 0.15, 3)
    assert keys.min() >= 0 and keys.max() <= 3
    near = octree.near_mask(keys)
    assert np.array_equal(near, near.T) and near.diagonal().all()
    colour = (keys[:, 0] & 1) * 4 + (keys[:, 1] & 1) * 2 + (keys[:, 2] & 1)
    same_box = (keys[:, None, :] == keys[None, :, :]).all(-1)
    same_colour = colour[:, None] == colour[None, :]
    assert not np.any(near & same_colour & ~same_box)
    p = octree.unknown_order(keys)
    assert np.array_equal(np.sort(p), np.arange(2 * m.n_edges))
    ne = m.n_edges
    assert np.all(p[1::2] == p[0::2] + ne)
    c = colour[p[0::2]]
    assert np.all(np.diff(c) >= 0)


# --- junction edges (three regions along a line) ------------------------------

def test_junction_edges_restrict_to_rwg_functions_of_every_region():
    from workloads import stacked_cylinder_body
    b = stacked_cylinder_body(0.3, 0.6, (2.2, 4.4), 0.1)
    m = rwg.from_body(b)
    junction = np.nonzero(m.side_tri[:, 2] >= 0)[0]
    assert len(junction) == 19                       # one ring of 19 edges
    assert len(b.vertices) - m.n_edges + len(b.triangles) == 2 + 1   # two closed layers share a disc
    for r in range(3):
        e, tri, free, c = m.restricted_halves(r)
        # every edge touching the region has exactly two halves there ...
        cnt = np.bincount(e, minlength=m.n_edges)
        assert set(np.unique(cnt)) <= {0, 2}
        # ... and they form an RWG function of the region's closed boundary:
        # flux +1 out of one half and +1 into the other, zero total charge
        for k in np.nonzero(cnt == 2)[0][::3]:
            sel = np.nonzero(e == k)[0]
            assert sorted(c[sel]) == [-1.0, 1.0]
            a, bb = m.vertices[m.edge_v[k]]
            mid = 0.5 * (a + bb)
            s_hat = (bb - a) / np.linalg.norm(bb - a)
            flux = []
            for h in sel:
                cen = m.centroid[tri[h]]
                out = (mid - cen) - np.dot(mid - cen, s_hat) * s_hat
                out /= np.linalg.norm(out)
                f = c[h] * m.length[k] / (2 * m.area[tri[h]]) * (mid - m.vertices[free[h]])
                flux.append(np.dot(f, out))
            assert abs(flux[0] + flux[1]) < 1e-12 and abs(abs(flux[0]) - 1) < 1e-12
    # the merged body (no internal disc) has no junctions
    mm = rwg.from_body(stacked_cylinder_body(0.3, 0.6, (2.2, 4.4), 0.1, merge_layers=True))
    assert np.all(mm.side_tri[:, 2] < 0)


def test_junction_orientation_errors_are_rejected():
    from workloads import stacked_cylinder_body
    b = stacked_cylinder_body(0.3, 0.6, (2.2, 4.4), 0.1)
    t = b.triangles.copy()
    disc = np.nonzero((b.tri_regions[:, 0] == 2) & (b.tri_regions[:, 1] == 1))[0]
    t[disc] = t[disc][:, [0, 2, 1]]          # flip the internal disc only
    with pytest.raises(rwg.MeshError):
        rwg.build(b.vertices, t, b.tri_regions)
