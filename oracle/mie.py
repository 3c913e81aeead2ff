"""Mie series for a homogeneous and for a coated (two-layer) dielectric sphere,
used to validate the surface-integral solution (the paper validates its
two-layer sphere and its coated nanoparticle against Mie results).

Written from Bohren & Huffman, "Absorption and Scattering of Light by Small
Particles" (1983), ch. 4 (homogeneous sphere) and sec. 8.1 (coated sphere,
Aden-Kerker), with Riccati-Bessel functions psi_n(z) = z j_n(z),
chi_n(z) = -z y_n(z), xi_n = psi_n - i chi_n evaluated through scipy's
spherical Bessel functions.  That book uses exp(-i omega t); for the
exp(+j omega t) permittivities used here the refractive index is
m = conj(sqrt(eps_r)) (mu_r = 1).

Geometry of the bistatic cuts used by the tests: the plane wave comes from
theta = 0 (propagates along -z) polarised along x.  The observation angle theta
then corresponds to the scattering angle pi - theta, and

    sigma_theta(theta, phi = 0)  = 4 pi |S2(pi - theta)|^2 / k^2   (E-plane)
    sigma_phi(theta, phi = 90 deg) = 4 pi |S1(pi - theta)|^2 / k^2 (H-plane)
"""

import numpy as np
from scipy.special import spherical_jn, spherical_yn


def _psi(n, z):
    return z * spherical_jn(n, z)


def _dpsi(n, z):
    return spherical_jn(n, z) + z * spherical_jn(n, z, derivative=True)


def _chi(n, z):
    return -z * spherical_yn(n, z)


def _dchi(n, z):
    return -(spherical_yn(n, z) + z * spherical_yn(n, z, derivative=True))


def _xi(n, z):
    return _psi(n, z) - 1j * _chi(n, z)


def _dxi(n, z):
    return _dpsi(n, z) - 1j * _dchi(n, z)


def n_terms(x):
    """Series length: Wiscombe's x + 4 x^(1/3) + 2, plus a margin of 8 terms."""
    return int(np.ceil(x + 4.0 * x ** (1.0 / 3.0) + 2.0)) + 8


def index_from_eps(eps_r):
    """Refractive index in Bohren & Huffman's convention for an exp(+j w t) eps_r."""
    return np.conj(np.sqrt(complex(eps_r)))


def coefficients_homogeneous(x, m, nmax=None):
    """a_n, b_n (n = 1..nmax) of a homogeneous sphere, size parameter x, index m."""
    nmax = nmax or n_terms(x)
    n = np.arange(1, nmax + 1)
    mx = m * x
    a = (m * _psi(n, mx) * _dpsi(n, x) - _psi(n, x) * _dpsi(n, mx)) / \
        (m * _psi(n, mx) * _dxi(n, x) - _xi(n, x) * _dpsi(n, mx))
    b = (_psi(n, mx) * _dpsi(n, x) - m * _psi(n, x) * _dpsi(n, mx)) / \
        (_psi(n, mx) * _dxi(n, x) - m * _xi(n, x) * _dpsi(n, mx))
    return a, b


def coefficients_coated(x, y, m1, m2, nmax=None):
    """a_n, b_n of a coated sphere: core size parameter x (index m1), outer size
    parameter y (shell index m2)."""
    nmax = nmax or n_terms(y)
    n = np.arange(1, nmax + 1)
    A = (m2 * _psi(n, m2 * x) * _dpsi(n, m1 * x) - m1 * _dpsi(n, m2 * x) * _psi(n, m1 * x)) / \
        (m2 * _chi(n, m2 * x) * _dpsi(n, m1 * x) - m1 * _dchi(n, m2 * x) * _psi(n, m1 * x))
    B = (m2 * _psi(n, m1 * x) * _dpsi(n, m2 * x) - m1 * _psi(n, m2 * x) * _dpsi(n, m1 * x)) / \
        (m2 * _dchi(n, m2 * x) * _psi(n, m1 * x) - m1 * _dpsi(n, m1 * x) * _chi(n, m2 * x))
    pA = _psi(n, m2 * y) - A * _chi(n, m2 * y)
    dpA = _dpsi(n, m2 * y) - A * _dchi(n, m2 * y)
    pB = _psi(n, m2 * y) - B * _chi(n, m2 * y)
    dpB = _dpsi(n, m2 * y) - B * _dchi(n, m2 * y)
    a = (_psi(n, y) * dpA - m2 * _dpsi(n, y) * pA) / (_xi(n, y) * dpA - m2 * _dxi(n, y) * pA)
    b = (m2 * _psi(n, y) * dpB - _dpsi(n, y) * pB) / (m2 * _xi(n, y) * dpB - _dxi(n, y) * pB)
    return a, b


def amplitudes(a, b, scattering_angle):
    """S1, S2 at the given scattering angles (radians)."""
    mu = np.cos(np.atleast_1d(scattering_angle))
    nmax = len(a)
    pi_prev = np.zeros_like(mu)
    pi_cur = np.ones_like(mu)
    S1 = np.zeros(mu.shape, dtype=complex)
    S2 = np.zeros(mu.shape, dtype=complex)
    for n in range(1, nmax + 1):
        if n > 1:
            pi_prev, pi_cur = pi_cur, ((2 * n - 1) * mu * pi_cur - n * pi_prev) / (n - 1)
        tau = n * mu * pi_cur - (n + 1) * pi_prev
        c = (2 * n + 1) / (n * (n + 1))
        S1 += c * (a[n - 1] * pi_cur + b[n - 1] * tau)
        S2 += c * (a[n - 1] * tau + b[n - 1] * pi_cur)
    return S1, S2


def efficiencies(a, b, x):
    """(Q_ext, Q_sca) normalised by the geometric cross section of radius x/k."""
    n = np.arange(1, len(a) + 1)
    qext = 2.0 / x ** 2 * np.sum((2 * n + 1) * np.real(a + b))
    qsca = 2.0 / x ** 2 * np.sum((2 * n + 1) * (np.abs(a) ** 2 + np.abs(b) ** 2))
    return qext, qsca


def bistatic_rcs(k0, theta, a, b):
    """(sigma_E(theta), sigma_H(theta)) in m^2 for incidence from theta = 0:
    E-plane theta-theta (phi = 0) and H-plane phi-phi (phi = 90 deg) cuts."""
    S1, S2 = amplitudes(a, b, np.pi - np.atleast_1d(theta))
    return 4 * np.pi * np.abs(S2) ** 2 / k0 ** 2, 4 * np.pi * np.abs(S1) ** 2 / k0 ** 2


def sphere_rcs(radius, eps_r, theta, wavelength=1.0):
    k0 = 2 * np.pi / wavelength
    a, b = coefficients_homogeneous(k0 * radius, index_from_eps(eps_r))
    return bistatic_rcs(k0, theta, a, b)


def coated_sphere_rcs(core_radius, core_eps, shell_radius, shell_eps, theta, wavelength=1.0):
    k0 = 2 * np.pi / wavelength
    a, b = coefficients_coated(k0 * core_radius, k0 * shell_radius, index_from_eps(core_eps),
                               index_from_eps(shell_eps))
    return bistatic_rcs(k0, theta, a, b)
