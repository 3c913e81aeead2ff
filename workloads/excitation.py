"""Incidence-angle lists and seeded random test vectors.

An incidence "angle (theta_i, phi_i)" names the direction the plane wave comes
from; the propagation direction is the opposite unit vector.  Conversions from
angles to vectors belong to each consumer; this module only lists angles.
"""

from __future__ import annotations

import numpy as np


def theta_sweep(n: int, phi: float = 0.0, theta_max_deg: float = 180.0):
    """``n`` incidence angles with theta uniform in [0, theta_max] (inclusive)
    at fixed phi.  Returns an [n, 2] float64 array of (theta, phi) in radians."""
    th = np.deg2rad(np.linspace(0.0, theta_max_deg, n)) if n > 1 else np.zeros(1)
    return np.stack([th, np.full_like(th, phi)], axis=1)


def random_complex_vector(n: int, n_rhs: int = 1, seed: int = 1234):
    """Complex Gaussian test vectors of unit variance, shape [n_rhs, n]."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((n_rhs, n))
    im = rng.standard_normal((n_rhs, n))
    return (re + 1j * im) / np.sqrt(2.0)
