"""Octree boxes, near-field pairs and the unknown ordering used by ILU(0).

The paper only says that the MLFMM of its ref. [17] is used and that an ILU
preconditioner suits it; these definitions are the readings adopted for the
near-field matrix and the preconditioner:

* one root cube per body, centred on the centre of the vertex bounding box,
  with side  finest_box * 2^(n_levels - 1)  (n_levels counts the root);
* a basis function belongs to the finest box holding its edge midpoint:
  integer key = floor((midpoint - corner) / finest_box), clamped to the grid,
  so a point on a box face goes to the higher box;
* a pair of basis functions is *near* when their finest keys differ by at most
  one in every coordinate (27-box stencil); the near-field matrix is the
  full matrix restricted to near pairs;
* ILU(0) ordering: boxes by colour (x&1)*4 + (y&1)*2 + (z&1) of the finest
  key, then by Morton code within a colour, then canonical edge index inside a
  box, with J of an edge before its M~.  Same-colour boxes are never near, so
  the factors do not depend on the order of boxes inside a colour.
"""

import numpy as np

from .rwg import RWGMesh


def auto_levels(mesh: RWGMesh, finest_box: float) -> int:
    ext = float(np.max(mesh.vertices.max(0) - mesh.vertices.min(0)))
    n = 1
    while finest_box * 2 ** (n - 1) < ext * (1.0 - 1e-12):
        n += 1
    return n


def finest_keys(mesh: RWGMesh, finest_box: float, n_levels: int):
    lo, hi = mesh.vertices.min(0), mesh.vertices.max(0)
    side = finest_box * 2 ** (n_levels - 1)
    corner = 0.5 * (lo + hi) - 0.5 * side
    mid = 0.5 * (mesh.vertices[mesh.edge_v[:, 0]] + mesh.vertices[mesh.edge_v[:, 1]])
    key = np.floor((mid - corner) / finest_box).astype(np.int64)
    return np.clip(key, 0, 2 ** (n_levels - 1) - 1)


def near_mask(keys):
    """[ne, ne] bool: basis pairs whose finest boxes touch or coincide."""
    d = np.abs(keys[:, None, :] - keys[None, :, :]).max(axis=-1)
    return d <= 1


def morton(keys):
    code = np.zeros(len(keys), dtype=np.int64)
    for bit in range(21):
        for axis, shift in ((0, 2), (1, 1), (2, 0)):
            code |= ((keys[:, axis] >> bit) & 1) << (3 * bit + shift)
    return code


def unknown_order(keys):
    """Permutation p of the 2 ne unknowns (boundary layout [J ; M~]) into ILU
    order: p[i] = boundary index of the i-th unknown in ILU order."""
    ne = len(keys)
    colour = (keys[:, 0] & 1) * 4 + (keys[:, 1] & 1) * 2 + (keys[:, 2] & 1)
    edges = np.lexsort((np.arange(ne), morton(keys), colour))
    p = np.empty(2 * ne, dtype=np.int64)
    p[0::2] = edges
    p[1::2] = edges + ne
    return p


def near_pattern(keys):
    """[2 ne, 2 ne] bool near pattern in boundary layout."""
    m = near_mask(keys)
    return np.block([[m, m], [m, m]])


def natural_order(keys):
    """Permutation of the 2 ne unknowns into the natural (uncoloured) order:
    boxes by Morton code, canonical edge index inside a box, J before M~.
    Used only to measure what the colouring of unknown_order costs ILU(0)."""
    ne = len(keys)
    edges = np.lexsort((np.arange(ne), morton(keys)))
    p = np.empty(2 * ne, dtype=np.int64)
    p[0::2] = edges
    p[1::2] = edges + ne
    return p
