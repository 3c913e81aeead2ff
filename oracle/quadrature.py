"""Seven-point, degree-5 symmetric triangle rule (Radon's rule, as tabulated by
Hammer, Marlowe and Stroud).  The paper fixes no rule for the surface integrals
of eqs. 16-26; this oracle uses this rule for every outer and inner integral.

Nodes are barycentric coordinates (l0, l1, l2); weights sum to 1 and multiply
the triangle area.
"""

import numpy as np

_S15 = np.sqrt(15.0)
_A1 = (6.0 - _S15) / 21.0
_B1 = (9.0 + 2.0 * _S15) / 21.0
_A2 = (6.0 + _S15) / 21.0
_B2 = (9.0 - 2.0 * _S15) / 21.0
_W0 = 9.0 / 40.0
_W1 = (155.0 - _S15) / 1200.0
_W2 = (155.0 + _S15) / 1200.0

BARY = np.array([
    [1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0],
    [_A1, _A1, _B1], [_A1, _B1, _A1], [_B1, _A1, _A1],
    [_A2, _A2, _B2], [_A2, _B2, _A2], [_B2, _A2, _A2],
])
WEIGHTS = np.array([_W0, _W1, _W1, _W1, _W2, _W2, _W2])


def points(p0, p1, p2):
    """Quadrature nodes of triangles with vertices p0, p1, p2 ([..., 3]).

    Returns [..., 7, 3]."""
    p0, p1, p2 = (np.asarray(p)[..., None, :] for p in (p0, p1, p2))
    b = BARY
    return b[:, 0:1] * p0 + b[:, 1:2] * p1 + b[:, 2:3] * p2
