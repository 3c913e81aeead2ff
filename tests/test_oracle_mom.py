"""Pins of the oracle's moment matrix, right-hand side and RCS: exact symmetry
of the Galerkin matrix on well-separated pairs, convergence of the symmetry
defect on touching pairs under outer-rule refinement, the Mie series, the
transparent-body limit and reciprocity."""

import numpy as np
import pytest

from oracle import farfield, mie, mom, potentials, quadrature, rwg
from workloads import sphere_body

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
