"""Closed-form integrals over a flat triangle of R^q (q = -1, 1), of
(rho' - rho) R^q, and of the gradients of R^-1 and R with respect to the
observation point.

They carry the 1/R and R terms of the Taylor expansion of the Green's function
of eq. 7, G = exp(-jkR)/(4 pi R) = (1/R - k^2 R / 2)/(4 pi) + smooth, so that
only a smooth remainder is left to the quadrature rule when source and
observation triangles touch or are close.  The paper does not state how it
integrates these terms; the formulas below are the standard ones (Wilton et
al., IEEE TAP 32(3), 1984; Graglia, IEEE TAP 41(10), 1993), rederived from the
two-dimensional divergence and gradient theorems:

For an observation point r with projection rho onto the plane of triangle T
and signed height h = (r - rho).n, and for every edge i of T (CCW about n,
unit tangent s_i, outward in-plane normal m_i = s_i x n, endpoints at
tangential coordinates s-, s+ relative to rho, signed distance t_i of rho
from the edge line, R0^2 = t_i^2 + h^2):

    edge integrals      E_i^q = int_edge R^q dl
        E^-1 = ln((R+ + s+)/(R- + s-))
        E^1  = (s+ R+ - s- R- + R0^2 E^-1) / 2
        E^3  = (s+ R+^3 - s- R-^3 + 3 R0^2 E^1) / 4
    solid-angle term    beta_i = atan(t s+ / (R0^2 + |h| R+)) - atan(t s- / (R0^2 + |h| R-))

    int_T 1/R          = sum_i t_i E_i^-1 - |h| sum_i beta_i
    int_T R            = ( sum_i t_i E_i^1 + h^2 int_T 1/R ) / 3
    int_T (rho'-rho)/R = sum_i m_i E_i^1
    int_T (rho'-rho) R = sum_i m_i E_i^3 / 3
    int_T grad(1/R)    = -sum_i m_i E_i^-1 - n sign(h) sum_i beta_i
    int_T grad R       = -int_T (rho'-rho)/R + n h int_T 1/R

All arrays broadcast over leading dimensions.
"""

import numpy as np


def _dot(a, b):
    return np.sum(a * b, axis=-1)


def _log_ratio(rp, sp, rm, sm):
    """ln((R+ + s+)/(R- + s-)) using whichever of the two equal forms has the
    larger denominators (they agree whenever R0 > 0)."""
    num1, den1 = rp + sp, rm + sm
    num2, den2 = rm - sm, rp - sp
    use1 = np.minimum(num1, den1) >= np.minimum(num2, den2)
    with np.errstate(divide="ignore", invalid="ignore"):
        a = np.log(np.where(use1, num1, num2) / np.where(use1, den1, den2))
    return np.where(np.isfinite(a), a, 0.0)


def triangle_integrals(r, p0, p1, p2, coplanar=None):
    """Closed-form integrals over triangles (p0, p1, p2) for observation points r.

    ``coplanar`` (bool array, optional) forces h = 0 where the observation
    point is known to lie in the triangle's plane (e.g. on the same triangle),
    so that the principal value of the normal gradient is taken.

    Returns a dict with keys
        inv_r   int 1/R               [...]
        r1      int R                 [...]
        vinv_r  int (rho'-rho)/R      [..., 3]
        vr1     int (rho'-rho) R      [..., 3]
        grad_inv_r  int grad_r (1/R)  [..., 3]
        grad_r1     int grad_r R      [..., 3]
        rho     projection of r       [..., 3]
    """
    r = np.asarray(r, dtype=float)
    verts = [np.asarray(p, dtype=float) for p in (p0, p1, p2)]
    cr = np.cross(verts[1] - verts[0], verts[2] - verts[0])
    n = cr / np.linalg.norm(cr, axis=-1, keepdims=True)
    h = _dot(r - verts[0], n)
    if coplanar is not None:
        h = np.where(coplanar, 0.0, h)
    rho = r - h[..., None] * n
    ah = np.abs(h)

    inv_r = 0.0
    sum_t_e1 = 0.0
    vinv_r = 0.0
    vr1 = 0.0
    sum_m_em1 = 0.0
    sum_beta = 0.0
    for i in range(3):
        a, b = verts[i], verts[(i + 1) % 3]
        ln = np.linalg.norm(b - a, axis=-1, keepdims=True)
        s = (b - a) / ln
        m = np.cross(s, n)
        sm = _dot(a - rho, s)
        sp = _dot(b - rho, s)
        t = _dot(a - rho, m)
        r0sq = t * t + h * h
        rm = np.linalg.norm(r - a, axis=-1)
        rp = np.linalg.norm(r - b, axis=-1)
        em1 = _log_ratio(rp, sp, rm, sm)
        e1 = 0.5 * (sp * rp - sm * rm + r0sq * em1)
        e3 = 0.25 * (sp * rp ** 3 - sm * rm ** 3 + 3.0 * r0sq * e1)
        with np.errstate(divide="ignore", invalid="ignore"):
            bp = np.arctan2(t * sp, r0sq + ah * rp)
            bm = np.arctan2(t * sm, r0sq + ah * rm)
        beta = np.where(r0sq + ah * np.minimum(rp, rm) > 0, bp - bm, 0.0)
        inv_r = inv_r + t * em1
        sum_beta = sum_beta + beta
        sum_t_e1 = sum_t_e1 + t * e1
        vinv_r = vinv_r + m * e1[..., None]
        vr1 = vr1 + m * (e3[..., None] / 3.0)
        sum_m_em1 = sum_m_em1 + m * em1[..., None]
    inv_r = inv_r - ah * sum_beta
    r1 = (sum_t_e1 + h * h * inv_r) / 3.0
    grad_inv_r = -sum_m_em1 - n * (np.sign(h) * sum_beta)[..., None]
    grad_r1 = -vinv_r + n * (h * inv_r)[..., None]
    return dict(inv_r=inv_r, r1=r1, vinv_r=vinv_r, vr1=vr1, grad_inv_r=grad_inv_r,
                grad_r1=grad_r1, rho=rho)
