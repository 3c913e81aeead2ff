"""Pins of the oracle's moment matrix, right-hand side and RCS: exact symmetry
of the Galerkin matrix on well-separated pairs, convergence of the symmetry
defect on touching pairs under outer-rule refinement, the Mie series, the
transparent-body limit and reciprocity."""

import numpy as np
import pytest

from oracle import farfield, mie, mom, octree, potentials, quadrature, rwg
from workloads import coated_sphere_body, sphere_body

THETA = np.deg2rad(np.arange(181.0))


@pytest.fixture(scope="module")
def sphere960():
    b = sphere_body(0.3, 4.0, 2)
    m = rwg.from_body(b)
    Z = mom.pmchwt_dense(m, b.eps_r, b.mu_r, b.frequency)
    return b, m, Z


def _far_pairs(m):
    ne = m.n_edges
    far = np.ones((ne, ne), bool)
    for a in (m.tri_p, m.tri_m):
        for b in (m.tri_p, m.tri_m):
            d = np.linalg.norm(m.centroid[a][:, None] - m.centroid[b][None], axis=-1)
            lim = 2 * np.maximum(m.max_edge[a][:, None], m.max_edge[b][None])
            shared = np.array([[len(set(m.triangles[i]) & set(m.triangles[j])) > 0 for j in b] for i in a])
            far &= (d >= lim) & ~shared
    return far


def test_galerkin_symmetry_on_separated_pairs(sphere960):
    # L and K are symmetric, so Z^T = D Z D with D = diag(I, -I); on pairs
    # computed with the plain 7x7 rule this holds to rounding.
    b, m, Z = sphere960
    ne = m.n_edges
    far = np.tile(_far_pairs(m), (2, 2))
    D = np.r_[np.ones(ne), -np.ones(ne)]
    defect = np.abs(Z.T - D[:, None] * Z * D[None, :])
    assert far.mean() > 0.5
    assert defect[far].max() < 1e-12 * np.abs(Z).max()
    # touching pairs only carry quadrature-level asymmetry
    assert defect.max() < 5e-3 * np.abs(Z).max()


def _refined_pair(m, P, Q, k, nsub):
    """L_loc, K_loc of triangles (P, Q) with the outer integral over P split
    into 4**nsub sub-triangles (inner integrals as in the oracle)."""
    tris = [m.vertices[m.triangles[P]]]
    for _ in range(nsub):
        nt = []
        for a, b, c in tris:
            ab, bc, ca = (a + b) / 2, (b + c) / 2, (c + a) / 2
            nt += [np.array(x) for x in ((a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca))]
        tris = nt
    pv = m.vertices[m.triangles[P]]
    qv = m.vertices[m.triangles[Q]]
    AP, AQ = m.area[P], m.area[Q]
    L = np.zeros((3, 3), complex)
    K = np.zeros((3, 3), complex)
    rb = m.qpts[Q]
    wb = quadrature.WEIGHTS * AQ
    for t in tris:
        ra = quadrature.points(*t)
        wa = quadrature.WEIGHTS * 0.5 * np.linalg.norm(np.cross(t[1] - t[0], t[2] - t[0]))
        I = potentials.triangle_integrals(ra, qv[0][None], qv[1][None], qv[2][None])
        d = ra[:, None, :] - rb[None]
        R = np.linalg.norm(d, axis=-1)
        Gr = mom._green_remainder(k, R)
        gr = mom._grad_factor_remainder(k, R)
        sc = (I["inv_r"] - 0.5 * k * k * I["r1"]) / (4 * np.pi) + Gr @ wb
        vec = (I["vinv_r"] - 0.5 * k * k * I["vr1"] + I["rho"] * (I["inv_r"] - 0.5 * k * k * I["r1"])[:, None]) / (4 * np.pi) \
            + np.einsum("ab,b,bx->ax", Gr, wb, rb)
        g = (I["grad_inv_r"] - 0.5 * k * k * I["grad_r1"]) / (4 * np.pi) + np.einsum("ab,b,abx->ax", gr, wb, d)
        for i in range(3):
            for j in range(3):
                L[i, j] += np.sum(wa * (np.einsum("ax,ax->a", ra - pv[i], vec - qv[j] * sc[:, None]) - 4 / k ** 2 * sc))
                K[i, j] += np.sum(wa * np.einsum("ax,ax->a", ra - pv[i], np.cross(g, ra - qv[j])))
    return -1j * k / (4 * AP * AQ) * L, K / (4 * AP * AQ)


def test_touching_pair_symmetry_converges_under_refinement(sphere960):
    b, m, _ = sphere960
    k = mom.wavenumber(b.frequency, 4.0, 1.0)
    e = 100
    P, Q = m.tri_p[e], m.tri_m[e]          # edge-adjacent pair
    L7, K7 = mom.pair_interactions(m, P, np.array([Q]), k)
    Lr0, Kr0 = _refined_pair(m, P, Q, k, 0)
    assert np.allclose(L7[0], Lr0, rtol=1e-12, atol=1e-14 * np.abs(Lr0).max())
    assert np.allclose(K7[0], Kr0, rtol=1e-12, atol=1e-14 * np.abs(Kr0).max())
    defects = []
    for ns in (0, 2, 4):
        Lpq, Kpq = _refined_pair(m, P, Q, k, ns)
        Lqp, Kqp = _refined_pair(m, Q, P, k, ns)
        defects.append((np.abs(Lpq - Lqp.T).max() / np.abs(Lpq).max(), np.abs(Kpq - Kqp.T).max() / np.abs(Kpq).max()))
    dl, dk = np.array(defects).T
    assert dl[-1] < dl[0] / 10 and dk[-1] < dk[0] / 3
    assert dl[-1] < 1e-4 and dk[-1] < 2e-2


def _solve_rcs(b, m, Z, theta_i=0.0, phi_i=0.0):
    kh, eh = mom.incidence(theta_i, phi_i)
    x = np.linalg.solve(Z, mom.planewave_rhs(m, b.frequency, kh, eh))
    sE, _ = farfield.rcs(m, b.frequency, x, THETA, 0 * THETA)
    _, sH = farfield.rcs(m, b.frequency, x, THETA, 0 * THETA + np.pi / 2)
    return x, sE, sH


def test_oracle_matches_mie_on_the_small_sphere(sphere960):
    b, m, Z = sphere960
    _, sE, sH = _solve_rcs(b, m, Z)
    mE, mH = mie.sphere_rcs(0.3, 4.0, THETA)
    dE = 10 * np.log10(sE / mE)
    dH = 10 * np.log10(sH / mH)
    # 480 edges (interior wavelength / 5.6): facetting-limited agreement
    assert np.sqrt(np.mean(dE ** 2)) < 0.5 and np.abs(dE).max() < 1.0
    assert np.sqrt(np.mean(dH ** 2)) < 0.6 and np.abs(dH).max() < 1.6


def test_transparent_sphere_scatters_nothing(sphere960):
    b, m, Z = sphere960
    bt = sphere_body(0.3, 1.0, 2)
    Zt = mom.pmchwt_dense(m, bt.eps_r, bt.mu_r, bt.frequency)
    _, sE, sH = _solve_rcs(bt, m, Zt)
    _, sE4, sH4 = _solve_rcs(b, m, Z)
    assert np.all(10 * np.log10(sE / sE4) < -30)
    assert np.all(10 * np.log10(sH / sH4) < -30)


def test_bistatic_reciprocity(sphere960):
    b, m, Z = sphere960
    ti, pi_, ts, ps = 0.3, 0.2, 1.9, 2.5
    ki, ei = mom.incidence(ti, pi_)
    ks, es = mom.incidence(ts, ps)
    # scattered far field toward -k_s from incidence k_i, and vice versa
    xi = np.linalg.solve(Z, mom.planewave_rhs(m, b.frequency, ki, ei))
    xs = np.linalg.solve(Z, mom.planewave_rhs(m, b.frequency, ks, es))
    Fi = farfield.far_field(m, b.frequency, xi, ts, ps)[0]
    Fs = farfield.far_field(m, b.frequency, xs, ti, pi_)[0]
    a1 = np.dot(es, Fi)
    a2 = np.dot(ei, Fs)
    assert abs(a1 - a2) < 5e-3 * abs(a1)


# --- near-field matrix and several interfaces (eq. 16) -----------------------

def _cuts(b, m, Z):
    _, sE, sH = _solve_rcs(b, m, Z)
    return sE, sH


def _db_rms_max(s, ref):
    floor = 1e-3 * ref.max()
    d = np.abs(10 * np.log10((s + floor) / (ref + floor)))
    return float(np.sqrt(np.mean(d ** 2))), float(d.max())


def test_near_matrix_is_the_dense_matrix_on_the_near_pattern(sphere960):
    # the near-field fill integrates only the triangle pairs of near edge
    # pairs; every near entry must equal the dense fill's, every other be zero
    b, m, Z = sphere960
    keys = octree.finest_keys(m, 0.15, 3)
    mask = octree.near_mask(keys)
    Zn = mom.pmchwt_near(m, b.eps_r, b.mu_r, b.frequency, mask)
    pat = octree.near_pattern(keys)
    assert 0.05 < pat.mean() < 0.95
    assert np.abs(Zn - np.where(pat, Z, 0)).max() <= 1e-14 * np.abs(Z).max()


@pytest.fixture(scope="module")
def coated1200():
    b = coated_sphere_body(0.15, 6 - 0.5j, 1, 0.3, 2.56, 2)
    m = rwg.from_body(b)
    return b, m, mom.pmchwt_dense(m, b.eps_r, b.mu_r, b.frequency)


def test_near_matrix_of_two_interfaces(coated1200):
    b, m, Z = coated1200
    keys = octree.finest_keys(m, 0.15, 3)
    Zn = mom.pmchwt_near(m, b.eps_r, b.mu_r, b.frequency, octree.near_mask(keys))
    pat = octree.near_pattern(keys)
    # both interfaces and the pairs between them are in the pattern
    inner = m.regions[:, 1] == 2
    assert pat[:m.n_edges, :m.n_edges][np.ix_(inner, ~inner)].any()
    assert np.abs(Zn - np.where(pat, Z, 0)).max() <= 1e-14 * np.abs(Z).max()


def test_equal_media_across_the_inner_interface(coated1200):
    # eq. 16 with the core made of the shell material: the inner interface
    # separates identical media, so the body scatters like the homogeneous
    # sphere of the outer mesh.  A wrong region sign on either interface, or a
    # missing cross-interface block, breaks this by dBs.
    b, m, _ = coated1200
    be = coated_sphere_body(0.15, 2.56, 1, 0.3, 2.56, 2)
    Ze = mom.pmchwt_dense(m, be.eps_r, be.mu_r, be.frequency)
    bh = sphere_body(0.3, 2.56, 2)
    mh = rwg.from_body(bh)
    Zh = mom.pmchwt_dense(mh, bh.eps_r, bh.mu_r, bh.frequency)
    eE, eH = _cuts(be, m, Ze)
    hE, hH = _cuts(bh, mh, Zh)
    for s, ref in ((eE, hE), (eH, hH)):
        rms, mx = _db_rms_max(s, ref)
        assert rms < 0.03 and mx < 0.1


@pytest.mark.slow
def test_coated_sphere_converges_to_the_coated_mie_series(coated1200):
    # lossy core (eps 6 - 0.5j, r = 0.15) in a shell (eps 2.56, r = 0.3): the
    # oracle's RCS approaches the Aden-Kerker series as both surfaces are
    # refined (1,200 -> 4,800 unknowns)
    mE, mH = mie.coated_sphere_rcs(0.15, 6 - 0.5j, 0.3, 2.56, THETA)
    errs = []
    for (cs, ss), pre in (((1, 2), coated1200), ((2, 3), None)):
        if pre is None:
            b = coated_sphere_body(0.15, 6 - 0.5j, cs, 0.3, 2.56, ss)
            m = rwg.from_body(b)
            Z = mom.pmchwt_dense(m, b.eps_r, b.mu_r, b.frequency)
        else:
            b, m, Z = pre
        sE, sH = _cuts(b, m, Z)
        errs.append(_db_rms_max(sE, mE) + _db_rms_max(sH, mH))
    (e1, x1, h1, y1), (e2, x2, h2, y2) = errs
    assert e1 < 0.6 and h1 < 0.7
    assert e2 < 0.15 and h2 < 0.2 and x2 < 0.3 and y2 < 0.6
    assert e2 < e1 / 3 and h2 < h1 / 3


def test_equal_layers_of_a_stacked_cylinder_match_the_homogeneous_cylinder():
    # junction edges (eq. 16 with three regions meeting along the rim of the
    # internal disc): with both layers of one material the internal disc
    # separates identical media and the stack must scatter like the same outer
    # mesh without it.  A wrong sign on a junction half breaks this by dBs.
    from workloads import stacked_cylinder_body
    bs = stacked_cylinder_body(0.3, 0.6, (2.2, 2.2), 0.1)
    bh = stacked_cylinder_body(0.3, 0.6, (2.2, 2.2), 0.1, merge_layers=True)
    cuts = []
    for b in (bs, bh):
        m = rwg.from_body(b)
        Z = mom.pmchwt_dense(m, b.eps_r, b.mu_r, b.frequency)
        kh, eh = mom.incidence(0.6, 0.0)
        x = np.linalg.solve(Z, mom.planewave_rhs(m, b.frequency, kh, eh))
        sE, _ = farfield.rcs(m, b.frequency, x, THETA, 0 * THETA)
        _, sH = farfield.rcs(m, b.frequency, x, THETA, 0 * THETA + np.pi / 2)
        cuts.append((sE, sH))
    for s, ref in zip(cuts[0], cuts[1]):
        rms, mx = _db_rms_max(s, ref)
        assert rms < 0.05 and mx < 0.2
    # with different layers the stack scatters measurably differently
    bd = stacked_cylinder_body(0.3, 0.6, (2.2, 10.2), 0.1)
    m = rwg.from_body(bd)
    Z = mom.pmchwt_dense(m, bd.eps_r, bd.mu_r, bd.frequency)
    kh, eh = mom.incidence(0.6, 0.0)
    x = np.linalg.solve(Z, mom.planewave_rhs(m, bd.frequency, kh, eh))
    sE, _ = farfield.rcs(m, bd.frequency, x, THETA, 0 * THETA)
    assert _db_rms_max(sE, cuts[1][0])[0] > 1.0
