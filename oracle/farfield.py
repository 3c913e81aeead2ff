"""Far-field pattern and radar cross section (eqs. 27-29).

The printed eqs. 27-28 drop the transverse projection and the r_hat x of the
magnetic-current term; the form below follows from eqs. 3-6 in the far zone,
where G -> exp(-j k0 r)/(4 pi r) exp(+j k0 r_hat.r') and grad G -> -j k0 r_hat G:

    E_scat = F(r_hat) exp(-j k0 r) / r
    F(r_hat) = (-j k0 / 4 pi) [ eta0 (I - r_hat r_hat) J_hat - r_hat x M_hat ]
    J_hat = int J(r') exp(+j k0 r_hat.r') dS'   (likewise M_hat)

over the interfaces that face free space (each half basis weighted by its
triangle's region-0 sign).  With M = eta0 M~ the bracket becomes eta0 [(I - r r) J_hat - r x M~_hat].
RCS (eq. 29): sigma_pp = 4 pi |p_hat . F|^2 / |E0|^2 in m^2.
"""

import numpy as np

from . import quadrature
from .mom import C0, ETA0
from .rwg import RWGMesh


def spherical_units(theta, phi):
    st, ct, sp, cp = np.sin(theta), np.cos(theta), np.sin(phi), np.cos(phi)
    r = np.stack([st * cp, st * sp, ct], axis=-1)
    th = np.stack([ct * cp, ct * sp, -st], axis=-1)
    ph = np.stack([-sp, cp, np.zeros_like(sp)], axis=-1)
    return r, th, ph


def basis_transforms(mesh: RWGMesh, frequency, r_hat):
    """T[d, n, 3] = int f_n(r') exp(+j k0 r_hat_d . r') dS' for every direction
    d, f_n restricted to free space with its region-0 sign."""
    k0 = 2 * np.pi * frequency / C0
    r_hat = np.atleast_2d(r_hat)
    w = quadrature.WEIGHTS
    T = np.zeros((len(r_hat), mesh.n_edges, 3), dtype=complex)
    e, tri, free, c = mesh.restricted_halves(0)
    pts = mesh.qpts[tri]                                                         # [nh, 7, 3]
    f = (c * mesh.length[e] / (2 * mesh.area[tri]))[:, None, None] * (pts - mesh.vertices[free][:, None, :])
    ph = np.exp(1j * k0 * np.einsum("dx,nqx->dnq", r_hat, pts))                  # [d, nh, 7]
    part = np.einsum("nq,dnq,nqx->dnx", w[None, :] * mesh.area[tri][:, None], ph, f)
    for d in range(len(r_hat)):
        np.add.at(T[d], e, part[d])
    return T


def far_field(mesh: RWGMesh, frequency, x, theta, phi, T=None):
    """F(theta, phi) [..., 3] for the scaled unknowns x = [J ; M~] (one RHS);
    T: basis_transforms of these directions if already computed."""
    k0 = 2 * np.pi * frequency / C0
    ne = mesh.n_edges
    J = x[:ne]
    Mt = x[ne:]
    r, th, ph = spherical_units(np.atleast_1d(theta), np.atleast_1d(phi))
    if T is None:
        T = basis_transforms(mesh, frequency, r)
    Jh = np.einsum("dnx,n->dx", T, J)
    Mh = np.einsum("dnx,n->dx", T, Mt)
    Jt = Jh - r * np.sum(r * Jh, axis=-1, keepdims=True)
    return (-1j * k0 * ETA0 / (4 * np.pi)) * (Jt - np.cross(r, Mh))


def rcs(mesh: RWGMesh, frequency, x, theta, phi, E0=1.0):
    """(sigma_theta, sigma_phi) in m^2 at the given directions."""
    F = far_field(mesh, frequency, x, theta, phi)
    _, th, ph = spherical_units(np.atleast_1d(theta), np.atleast_1d(phi))
    st = 4 * np.pi * np.abs(np.sum(th * F, axis=-1)) ** 2 / abs(E0) ** 2
    sp = 4 * np.pi * np.abs(np.sum(ph * F, axis=-1)) ** 2 / abs(E0) ** 2
    return st, sp
