"""Galerkin (RWG) moment matrix of the PMCHWT surface integral equation and
plane-wave right-hand sides, written as their plain definitions.

Operators (eqs. 3-7, e^{+j omega t}, G_r = exp(-j k_r R)/(4 pi R)):

    L_r[m,n] = -j k_r  int int [ f_m . f_n - k_r^-2 (div f_m)(div' f_n) ] G_r dS' dS
    K_r[m,n] =         int int   f_m(r) . [ grad G_r(r,r') x f_n(r') ]       dS' dS

so that <f_m, E^scat> = eta L J - K M and <f_m, H^scat> = K J + L M / eta
(eqs. 3-4; the printed eq. 5 has a garbled sign and the printed RWG forms
eqs. 23-26 are not usable, so these are derived from eqs. 3-6 with the
surface divergence theorem).  K is the principal value; its half-jump terms
cancel in the PMCHWT sum below.

PMCHWT (T-EFIE and T-MFIE of eqs. 10-11 summed over the two regions at every
interface, with J1 = -J2, M2 = -M1 from eqs. 12-13, extended to several
interfaces as in eq. 16): for interfaces i, j and every region r bordering
both, with region signs s (rwg module),

    Z_ij = sum_r s_ri s_rj [[ et_r L_r , -K_r ], [ K_r , L_r / et_r ]]

acting on [J ; M~] with M~ = M / eta0 and et_r = eta_r / eta0 (the E-rows are
divided by eta0, the H-rows are unchanged), so both unknowns and both rows
carry A/m and A.  The right-hand side is b_i = -s_0i [<f, E_inc>/eta0 ;
<f, H_inc>], non-zero only on interfaces that touch free space (region 0).
The region signs are carried per triangle (rwg module), which also covers
junction edges whose halves lie on different interfaces.
The boundary layout is [J_1..J_E, M~_1..M~_E] in canonical edge order.

Integration (the paper is silent): 7-point rule for outer and inner integrals.
For a triangle pair that shares a vertex or whose centroids are closer than
twice the longer of the two triangles' longest edges, (1/R - k^2 R/2)/(4 pi)
and its gradient are integrated in closed form over the source triangle
(potentials module) and only the remainder goes to the 7-point inner rule.
K of a triangle with itself is zero (all three vectors lie in its plane).
"""

from __future__ import annotations

import numpy as np

from . import potentials, quadrature
from .rwg import RWGMesh

C0 = 299792458.0
MU0 = 4e-7 * np.pi * 1.00000000055        # CODATA 2018 magnetic constant, H/m
ETA0 = MU0 * C0                           # free-space impedance, ohm


def wavenumber(frequency, eps_r, mu_r):
    """k_r = k0 sqrt(eps_r mu_r) with Im k_r <= 0 (principal branch)."""
    k0 = 2 * np.pi * frequency / C0
    return k0 * np.sqrt(complex(eps_r) * complex(mu_r))


def rel_impedance(eps_r, mu_r):
    """eta_r / eta0 = sqrt(mu_r / eps_r), principal branch."""
    return np.sqrt(complex(mu_r) / complex(eps_r))


def _close_pairs(mesh: RWGMesh, P: int, Qs: np.ndarray):
    share = np.isin(mesh.triangles[Qs], mesh.triangles[P]).any(axis=1)
    d = np.linalg.norm(mesh.centroid[Qs] - mesh.centroid[P], axis=1)
    lim = 2.0 * np.maximum(mesh.max_edge[Qs], mesh.max_edge[P])
    return share | (d < lim)


def _green_remainder(k, R):
    """G - (1/R - k^2 R/2)/(4 pi); limit -jk/(4 pi) at R = 0."""
    with np.errstate(divide="ignore", invalid="ignore"):
        v = (np.exp(-1j * k * R) - 1.0 + 0.5 * (k * R) ** 2) / (4 * np.pi * R)
    return np.where(R > 0, v, -1j * k / (4 * np.pi))


def _grad_factor_remainder(k, R):
    """g - g_s with grad G = (r - r') g(R), g_s from (1/R - k^2 R/2)/(4 pi);
    its product with (r - r') vanishes at R = 0."""
    with np.errstate(divide="ignore", invalid="ignore"):
        v = (-(1.0 + 1j * k * R) * np.exp(-1j * k * R) + 1.0 + 0.5 * (k * R) ** 2) / (4 * np.pi * R ** 3)
    return np.where(R > 0, v, 0.0)


def _green(k, R):
    return np.exp(-1j * k * R) / (4 * np.pi * R)


def _grad_factor(k, R):
    return -(1.0 + 1j * k * R) * np.exp(-1j * k * R) / (4 * np.pi * R ** 3)


def _inner_integrals(mesh: RWGMesh, P: int, Qs: np.ndarray, k: complex):
    """At the 7 outer nodes r_a of test triangle P, over each source triangle
    Q: I_sc = int_Q G, I_vec = int_Q r' G, g = int_Q grad G (grad w.r.t. r),
    with the singular parts integrated in closed form for close pairs.
    Returns (r_a [7, 3], I_sc [7, nQ], I_vec [7, nQ, 3], g [7, nQ, 3])."""
    Qs = np.asarray(Qs, dtype=np.int64)
    w = quadrature.WEIGHTS
    ra = mesh.qpts[P]                                    # [7, 3] outer nodes
    rb = mesh.qpts[Qs]                                   # [nQ, 7, 3] inner nodes
    AQ = mesh.area[Qs]
    d = ra[:, None, None, :] - rb[None, :, :, :]         # [7a, nQ, 7b, 3]  r - r'
    R = np.linalg.norm(d, axis=-1)
    close = _close_pairs(mesh, P, Qs)

    with np.errstate(divide="ignore", invalid="ignore"):
        Gf = np.where(close[None, :, None], _green_remainder(k, R), _green(k, R))
        gf = np.where(close[None, :, None], _grad_factor_remainder(k, R), _grad_factor(k, R))
    wq = (w[None, None, :] * AQ[None, :, None])          # [1, nQ, 7b]
    I_sc = np.sum(wq * Gf, axis=2)                               # [7a, nQ]
    I_vec = np.sum((wq * Gf)[..., None] * rb[None], axis=2)      # [7a, nQ, 3]
    g = np.sum((wq * gf)[..., None] * d, axis=2)                 # [7a, nQ, 3]

    ci = np.nonzero(close)[0]
    if len(ci):
        V = mesh.vertices[mesh.triangles[Qs[ci]]]                # [nc, 3, 3]
        same = (Qs[ci] == P)
        res = potentials.triangle_integrals(ra[:, None, :], V[None, :, 0], V[None, :, 1], V[None, :, 2],
                                            coplanar=np.broadcast_to(same[None, :], (7, len(ci))))
        s_sc = (res["inv_r"] - 0.5 * k * k * res["r1"]) / (4 * np.pi)
        s_vec = (res["vinv_r"] - 0.5 * k * k * res["vr1"] + res["rho"] * (res["inv_r"] - 0.5 * k * k * res["r1"])[..., None]) / (4 * np.pi)
        s_grad = (res["grad_inv_r"] - 0.5 * k * k * res["grad_r1"]) / (4 * np.pi)
        I_sc[:, ci] += s_sc
        I_vec[:, ci] += s_vec
        g[:, ci] += s_grad
    return ra, I_sc, I_vec, g


def pair_interactions(mesh: RWGMesh, P: int, Qs: np.ndarray, k: complex):
    """Local interactions of the three half-basis functions of test triangle P
    with those of source triangles Qs for wavenumber k.

    On triangle T the half-basis of local vertex i is (r - v_i)/(2 A_T) with
    divergence 1/A_T; a basis function is (sign * edge length) times it.

    Returns L_loc, K_loc of shape [len(Qs), 3, 3] (test local i, source local j).
    """
    Qs = np.asarray(Qs, dtype=np.int64)
    w = quadrature.WEIGHTS
    AQ = mesh.area[Qs]
    AP = mesh.area[P]
    ra, I_sc, I_vec, g = _inner_integrals(mesh, P, Qs, k)
    pv = mesh.vertices[mesh.triangles[P]]                # [3i, 3]
    qv = mesh.vertices[mesh.triangles[Qs]]               # [nQ, 3j, 3]
    wa = w * AP                                          # outer weights
    ri = ra[:, None, :] - pv[None, :, :]                 # [7a, 3i, 3] r - p_i
    # L: (r - p_i).(I_vec - q_j I_sc) - 4/k^2 I_sc
    vec_j = I_vec[:, :, None, :] - qv[None, :, :, :] * I_sc[:, :, None, None]   # [7a, nQ, 3j, 3]
    dot = np.einsum("aix,aqjx->aqij", ri, vec_j)
    integrand = dot - (4.0 / (k * k)) * I_sc[:, :, None, None]
    L_loc = (-1j * k / (4 * AP * AQ))[:, None, None] * np.einsum("a,aqij->qij", wa, integrand)
    # K: (r - p_i).(g x (r - q_j))
    rj = ra[:, None, None, :] - qv[None, :, :, :]                               # [7a, nQ, 3j, 3]
    cr = np.cross(g[:, :, None, :], rj)                                          # [7a, nQ, 3j, 3]
    kint = np.einsum("aix,aqjx->aqij", ri, cr)
    K_loc = (1.0 / (4 * AP * AQ))[:, None, None] * np.einsum("a,aqij->qij", wa, kint)
    K_loc[Qs == P] = 0.0
    return L_loc, K_loc


def pair_interactions_n(mesh: RWGMesh, P: int, Qs: np.ndarray, k: complex):
    """As pair_interactions with the test half-bases rotated by the normal of
    P, t_i = n_P x (r - p_i) / (2 A_P) (the "N" testing of eqs. 8-9).  The
    rotated function is not divergence-conforming, so the scalar-potential
    part of L keeps its gradient:

        (L h_j)(r) = -j k int_Q h_j G dS' - (j / k) (1 / A_Q) int_Q grad G dS'
        (K h_j)(r) = int_Q grad G x h_j dS'   (principal value; 0 on Q = P)

    Returns LN_loc, KN_loc [len(Qs), 3, 3]."""
    Qs = np.asarray(Qs, dtype=np.int64)
    w = quadrature.WEIGHTS
    AQ = mesh.area[Qs]
    AP = mesh.area[P]
    ra, I_sc, I_vec, g = _inner_integrals(mesh, P, Qs, k)
    pv = mesh.vertices[mesh.triangles[P]]
    qv = mesh.vertices[mesh.triangles[Qs]]
    wa = w * AP
    ti = np.cross(mesh.normal[P][None, None, :], ra[:, None, :] - pv[None, :, :])   # [7a, 3i, 3]
    Lh = (-1j * k / 2) * (I_vec[:, :, None, :] - qv[None, :, :, :] * I_sc[:, :, None, None]) \
        - (1j / k) * g[:, :, None, :]                                                  # [7a, nQ, 3j, 3] x A_Q
    LN_loc = (1.0 / (2 * AP * AQ))[:, None, None] * np.einsum("a,aix,aqjx->qij", wa, ti, Lh)
    rj = ra[:, None, None, :] - qv[None, :, :, :]
    cr = np.cross(g[:, :, None, :], rj)                                                # [7a, nQ, 3j, 3]
    KN_loc = (1.0 / (4 * AP * AQ))[:, None, None] * np.einsum("a,aix,aqjx->qij", wa, ti, cr)
    KN_loc[Qs == P] = 0.0
    return LN_loc, KN_loc


def gram_local(mesh: RWGMesh, P: int):
    """G[i, j] = int_P h_i . h_j and GN[i, j] = int_P h_i . (n_P x h_j) for the
    half-bases of triangle P (the 7-point rule is exact: quadratics)."""
    w = quadrature.WEIGHTS * mesh.area[P]
    ra = mesh.qpts[P]
    h = (ra[:, None, :] - mesh.vertices[mesh.triangles[P]][None, :, :]) / (2 * mesh.area[P])   # [7, 3, 3]
    nh = np.cross(mesh.normal[P][None, None, :], h)
    return np.einsum("a,aix,ajx->ij", w, h, h), np.einsum("a,aix,ajx->ij", w, h, nh)


def operator_rows(mesh: RWGMesh, k: complex, region: int, test_edges):
    """Rows ``test_edges`` of L_r and K_r between the basis functions
    restricted to ``region`` (columns in canonical order): only triangles that
    border the region take part, each half weighted by its triangle's region
    sign, so the result already carries the sign products of eq. 16."""
    test_edges = np.asarray(test_edges, dtype=np.int64)
    ne = mesh.n_edges
    L = np.zeros((len(test_edges), ne), dtype=complex)
    K = np.zeros((len(test_edges), ne), dtype=complex)
    trs = mesh.tri_region_sign(region)
    border = np.nonzero(trs)[0]
    edge_pos = {e: i for i, e in enumerate(test_edges)}
    tris = sorted({int(t) for e in test_edges for t in mesh.side_tri[e] if t >= 0})
    for P in tris:
        if trs[P] == 0:
            continue
        L_loc, K_loc = pair_interactions(mesh, P, border, k)
        for i in range(3):
            m = mesh.tri_edge[P, i]
            if m not in edge_pos:
                continue
            sm = trs[P] * mesh.tri_sign[P, i] * mesh.length[m]
            row = edge_pos[m]
            for j in range(3):
                n = mesh.tri_edge[border, j]
                sn = trs[border] * mesh.tri_sign[border, j] * mesh.length[n]
                np.add.at(L[row], n, sm * sn * L_loc[:, i, j])
                np.add.at(K[row], n, sm * sn * K_loc[:, i, j])
    return L, K


def operator_near(mesh: RWGMesh, k: complex, region: int, near):
    """As operator_rows for all rows, restricted to the boolean edge-pair
    pattern ``near`` ([ne, ne]); entries outside the pattern are zero.  Only
    the triangle pairs that contribute to pattern entries are integrated."""
    ne = mesh.n_edges
    L = np.zeros((ne, ne), dtype=complex)
    K = np.zeros((ne, ne), dtype=complex)
    trs = mesh.tri_region_sign(region)
    border = trs != 0
    for P in np.nonzero(border)[0]:
        edges_P = mesh.tri_edge[P]
        cols = np.nonzero(near[edges_P].any(axis=0))[0]
        Qs = mesh.side_tri[cols].ravel()
        Qs = np.unique(Qs[Qs >= 0])
        Qs = Qs[border[Qs]]
        if len(Qs) == 0:
            continue
        L_loc, K_loc = pair_interactions(mesh, P, Qs, k)
        for i in range(3):
            m = edges_P[i]
            sm = trs[P] * mesh.tri_sign[P, i] * mesh.length[m]
            for j in range(3):
                n = mesh.tri_edge[Qs, j]
                keep = near[m, n]
                sn = trs[Qs] * mesh.tri_sign[Qs, j] * mesh.length[n]
                np.add.at(L[m], n[keep], (sm * sn * L_loc[:, i, j])[keep])
                np.add.at(K[m], n[keep], (sm * sn * K_loc[:, i, j])[keep])
    return L, K


def pmchwt_near(mesh: RWGMesh, eps_r, mu_r, frequency, near):
    """Scaled PMCHWT matrix [2 ne, 2 ne] restricted to the edge-pair pattern
    ``near`` (the near-field matrix when ``near`` is the octree's near mask)."""
    ne = mesh.n_edges
    Z = np.zeros((2 * ne, 2 * ne), dtype=complex)
    for r in range(len(eps_r)):
        if not np.any(mesh.tri_region_sign(r)):
            continue
        k = wavenumber(frequency, eps_r[r], mu_r[r])
        et = rel_impedance(eps_r[r], mu_r[r])
        L, K = operator_near(mesh, k, r, near)
        Z[:ne, :ne] += et * L
        Z[:ne, ne:] += -K
        Z[ne:, :ne] += K
        Z[ne:, ne:] += L / et
    return Z


def pmchwt_rows(mesh: RWGMesh, eps_r, mu_r, frequency, test_edges):
    """Rows of the scaled PMCHWT matrix for the E-equations and H-equations of
    ``test_edges``.  Returns (Z_E, Z_H), each [len(test_edges), 2 ne]."""
    test_edges = np.asarray(test_edges, dtype=np.int64)
    ne = mesh.n_edges
    ZE = np.zeros((len(test_edges), 2 * ne), dtype=complex)
    ZH = np.zeros((len(test_edges), 2 * ne), dtype=complex)
    for r in range(len(eps_r)):
        trs = mesh.tri_region_sign(r)
        touched = np.any(trs[mesh.side_tri[test_edges].clip(0)] * (mesh.side_tri[test_edges] >= 0))
        if not touched:
            continue
        k = wavenumber(frequency, eps_r[r], mu_r[r])
        et = rel_impedance(eps_r[r], mu_r[r])
        L, K = operator_rows(mesh, k, r, test_edges)
        ZE[:, :ne] += et * L
        ZE[:, ne:] += -K
        ZH[:, :ne] += K
        ZH[:, ne:] += L / et
    return ZE, ZH


def pmchwt_dense(mesh: RWGMesh, eps_r, mu_r, frequency):
    """The full scaled PMCHWT matrix [2 ne, 2 ne] in boundary layout."""
    ne = mesh.n_edges
    ZE, ZH = pmchwt_rows(mesh, eps_r, mu_r, frequency, np.arange(ne))
    return np.concatenate([ZE, ZH], axis=0)


def incidence(theta, phi):
    """Propagation direction and theta-polarisation of a plane wave coming from
    (theta, phi): k_hat = -r_hat(theta, phi), e_hat = theta_hat(theta, phi)."""
    st, ct, sp, cp = np.sin(theta), np.cos(theta), np.sin(phi), np.cos(phi)
    k_hat = -np.array([st * cp, st * sp, ct])
    e_hat = np.array([ct * cp, ct * sp, -st])
    return k_hat, e_hat


def planewave_rhs(mesh: RWGMesh, frequency, k_hat, e_hat, E0=1.0):
    """Scaled right-hand side [-<f,E_inc>/eta0 ; -<f,H_inc>] (eqs. 20-21 with
    the plane wave of eq. 30 read as E_inc = e E0 exp(-j k0 k_hat.r),
    H_inc = k_hat x E_inc / eta0), region sign of free space applied."""
    k0 = 2 * np.pi * frequency / C0
    k_hat = np.asarray(k_hat, dtype=float)
    e_hat = np.asarray(e_hat, dtype=complex)
    h_hat = np.cross(k_hat, e_hat)
    w = quadrature.WEIGHTS
    ne = mesh.n_edges
    bE = np.zeros(ne, dtype=complex)
    bH = np.zeros(ne, dtype=complex)
    # basis functions restricted to free space (region 0), region sign included
    e, tri, free, c = mesh.restricted_halves(0)
    pts = mesh.qpts[tri]                                               # [nh, 7, 3]
    f = (c * mesh.length[e] / (2 * mesh.area[tri]))[:, None, None] * (pts - mesh.vertices[free][:, None, :])
    phase = E0 * np.exp(-1j * k0 * pts @ k_hat)                        # [nh, 7]
    np.add.at(bE, e, mesh.area[tri] * np.sum(w * (f @ e_hat) * phase, axis=1))
    np.add.at(bH, e, mesh.area[tri] * np.sum(w * (f @ h_hat) * phase, axis=1))
    return np.concatenate([-bE / ETA0, -bH / ETA0])


# --- JMCFIE and CNF (eqs. 8-9, 14-16) -----------------------------------------
#
# Per region r (fields of the restricted currents J^r, M^r in the unbounded
# medium r, its inward normal n_r = +-n_P on a triangle P), tested with RWG
# functions, with the jump terms of the principal-value K made explicit
# (n_r x K X -> X / 2 + n_r x K_pv X, (K X)_tan -> K_pv X_tan - n_r x X / 2 on
# the region's side):
#   T-EFIE(r): eta L J - K M - (1/2) n x M = -E_inc        (tangential E)
#   T-MFIE(r): K J + L M / eta + (1/2) n x J = -H_inc      (tangential H)
#   N-EFIE(r): eta n x L J - n x K M + M / 2 = -n x E_inc   (eq. 8)
#   N-MFIE(r): n x K J - J / 2 + n x L M / eta = -n x H_inc (eq. 9)
# JMCFIE (eq. 14): J-row = sum_r T-EFIE(r) / eta_r + (-1)^r N-MFIE(r),
# M-row = sum_r eta_r T-MFIE(r) - (-1)^r N-EFIE(r).  The figure that numbers
# the two media is not available; region 1 is taken as the one behind the
# normal (the interior of a single body), so (-1)^r = +1 on the side the
# normal points into and -1 behind it.  Both numberings give systems with
# the same solution (the T and N parts hold separately); this one lets the
# identity terms of the two parts reinforce each other (condition number 6.6
# against 55 on a 960-unknown sphere of eps_r 4) and is the one for which
# JMCFIE needs fewer iterations than the T parts alone and than PMCHWT, as
# the paper reports.  The rows below are the combination times -1, so that
# the Gram identity enters the diagonal blocks with a positive sign, as in
# CNF: JMCFIE = (N parts) - (T parts).
# The T parts are tested with the region-restricted basis (region sign on the
# test half, as in PMCHWT); in the N parts the sign (-1)^r cancels the sign
# of n_r, so the test halves carry no region sign and are rotated by the
# triangle's own normal.  The code integrates the fields against the rotated
# halves, <n x f, X> = -<f, n x X>.  The identity terms become Gram
# matrices: J and M (one half from each region) and, with the T parts' jump
# terms, -(1/eta_o - 1/eta_p) <f, n x M> / 2 and +(eta_o - eta_p) <f, n x J> / 2
# per triangle between front region o and back region p.
# Scaled as PMCHWT: unknowns [J ; M~ = M / eta0], J-row in A/m, M-row / eta0.
# CNF (the normal equations alone, eqs. 8-9): the N parts only.

def operator_rows_n(mesh: RWGMesh, k: complex, region: int, test_edges):
    """Rows ``test_edges`` of n x L_r and n x K_r with unsigned test halves
    rotated by their triangle's normal and region-restricted source bases."""
    test_edges = np.asarray(test_edges, dtype=np.int64)
    ne = mesh.n_edges
    LN = np.zeros((len(test_edges), ne), dtype=complex)
    KN = np.zeros((len(test_edges), ne), dtype=complex)
    trs = mesh.tri_region_sign(region)
    border = np.nonzero(trs)[0]
    edge_pos = {e: i for i, e in enumerate(test_edges)}
    tris = sorted({int(t) for e in test_edges for t in mesh.side_tri[e] if t >= 0})
    for P in tris:
        if trs[P] == 0:
            continue
        L_loc, K_loc = pair_interactions_n(mesh, P, border, k)
        for i in range(3):
            m = mesh.tri_edge[P, i]
            if m not in edge_pos:
                continue
            sm = mesh.tri_sign[P, i] * mesh.length[m]
            row = edge_pos[m]
            for j in range(3):
                n = mesh.tri_edge[border, j]
                sn = trs[border] * mesh.tri_sign[border, j] * mesh.length[n]
                np.add.at(LN[row], n, sm * sn * L_loc[:, i, j])
                np.add.at(KN[row], n, sm * sn * K_loc[:, i, j])
    return LN, KN


def gram_rows(mesh: RWGMesh, eta_rel, test_edges):
    """Rows of the Gram matrix G = <f_m, f_n> and of the T-part jump terms
    GJ = sum_P (eta_o - eta_p) <f_m, n x f_n>_P / 2 and
    GM = -sum_P (1/eta_o - 1/eta_p) <f_m, n x f_n>_P / 2 (unsigned halves)."""
    test_edges = np.asarray(test_edges, dtype=np.int64)
    ne = mesh.n_edges
    G = np.zeros((len(test_edges), ne))
    GJ = np.zeros((len(test_edges), ne), dtype=complex)
    GM = np.zeros((len(test_edges), ne), dtype=complex)
    edge_pos = {e: i for i, e in enumerate(test_edges)}
    tris = sorted({int(t) for e in test_edges for t in mesh.side_tri[e] if t >= 0})
    for P in tris:
        g, gn = gram_local(mesh, P)
        o, p = mesh.tri_regions[P]
        wj = 0.5 * (eta_rel[o] - eta_rel[p])
        wm = -0.5 * (1 / eta_rel[o] - 1 / eta_rel[p])
        for i in range(3):
            m = mesh.tri_edge[P, i]
            if m not in edge_pos:
                continue
            sm = mesh.tri_sign[P, i] * mesh.length[m]
            for j in range(3):
                n = mesh.tri_edge[P, j]
                sn = mesh.tri_sign[P, j] * mesh.length[n]
                G[edge_pos[m], n] += sm * sn * g[i, j]
                GJ[edge_pos[m], n] += wj * sm * sn * gn[i, j]
                GM[edge_pos[m], n] += wm * sm * sn * gn[i, j]
    return G, GJ, GM


def combined_rows(mesh: RWGMesh, eps_r, mu_r, frequency, test_edges, tangential=True):
    """Rows (Z_J, Z_M) of the scaled JMCFIE matrix (tangential=True) or of
    the CNF matrix (tangential=False) for ``test_edges``, each [n, 2 ne]."""
    test_edges = np.asarray(test_edges, dtype=np.int64)
    ne = mesh.n_edges
    ZJ = np.zeros((len(test_edges), 2 * ne), dtype=complex)
    ZM = np.zeros((len(test_edges), 2 * ne), dtype=complex)
    eta = [rel_impedance(eps_r[r], mu_r[r]) for r in range(len(eps_r))]
    for r in range(len(eps_r)):
        trs = mesh.tri_region_sign(r)
        st = mesh.side_tri[test_edges]
        if not np.any(trs[st.clip(0)] * (st >= 0)):
            continue
        k = wavenumber(frequency, eps_r[r], mu_r[r])
        LN, KN = operator_rows_n(mesh, k, r, test_edges)
        ZJ[:, :ne] += KN
        ZJ[:, ne:] += LN / eta[r]
        ZM[:, :ne] += -eta[r] * LN
        ZM[:, ne:] += KN
        if tangential:
            L, K = operator_rows(mesh, k, r, test_edges)
            ZJ[:, :ne] -= L
            ZJ[:, ne:] -= -K / eta[r]
            ZM[:, :ne] -= eta[r] * K
            ZM[:, ne:] -= L
    G, GJ, GM = gram_rows(mesh, eta, test_edges)
    ZJ[:, :ne] += G
    ZM[:, ne:] += G
    if tangential:
        ZJ[:, ne:] -= GM
        ZM[:, :ne] -= GJ
    return ZJ, ZM


def combined_dense(mesh: RWGMesh, eps_r, mu_r, frequency, tangential=True):
    """The full scaled JMCFIE (or CNF) matrix [2 ne, 2 ne]."""
    ZJ, ZM = combined_rows(mesh, eps_r, mu_r, frequency, np.arange(mesh.n_edges), tangential)
    return np.concatenate([ZJ, ZM], axis=0)


def combined_rhs(mesh: RWGMesh, frequency, k_hat, e_hat, tangential=True, E0=1.0):
    """Right-hand side of the scaled JMCFIE (or CNF) system for a plane wave
    in free space (region 0, eta_0 = 1):
        J-row: -<n x f, H_inc> + <f^0, E_inc>/eta0,  M-row: <n x f, E_inc>/eta0 + <f^0, H_inc>
    (f^0: region-0-restricted basis; n x f: unsigned halves on the triangles
    bordering free space, rotated by their normals); the T terms (those of
    PMCHWT, entering JMCFIE with the sign -1) only for JMCFIE."""
    k0 = 2 * np.pi * frequency / C0
    k_hat = np.asarray(k_hat, dtype=float)
    e_hat = np.asarray(e_hat, dtype=complex)
    h_hat = np.cross(k_hat, e_hat)
    w = quadrature.WEIGHTS
    ne = mesh.n_edges
    e, tri, free, c = mesh.restricted_halves(0)
    pts = mesh.qpts[tri]
    f = (mesh.length[e] / (2 * mesh.area[tri]))[:, None, None] * (pts - mesh.vertices[free][:, None, :])
    phase = E0 * np.exp(-1j * k0 * pts @ k_hat)
    unsigned = (c * mesh.tri_region_sign(0)[tri])[:, None, None]      # side sign alone
    t = np.cross(mesh.normal[tri][:, None, :], unsigned * f)
    aw = mesh.area[tri][:, None] * w[None, :]
    bJ = np.zeros(ne, dtype=complex)
    bM = np.zeros(ne, dtype=complex)
    np.add.at(bJ, e, -np.sum(aw * (t @ h_hat) * phase, axis=1) / ETA0)
    np.add.at(bM, e, np.sum(aw * (t @ e_hat) * phase, axis=1) / ETA0)
    if tangential:
        fr = c[:, None, None] * f
        np.add.at(bJ, e, np.sum(aw * (fr @ e_hat) * phase, axis=1) / ETA0)
        np.add.at(bM, e, np.sum(aw * (fr @ h_hat) * phase, axis=1) / ETA0)
    return np.concatenate([bJ, bM])
