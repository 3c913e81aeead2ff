"""ILU(0) iteration counts in coloured and natural unknown order.

The paper preconditions its Krylov solver with an incomplete LU of the
near-field matrix (Simulation Results) without naming the variant or the
ordering.  ILU(0) depends on the elimination order; this study measures
GMRES(m) iterations to a relative residual tol on a dielectric sphere with
ILU(0) of the near-field matrix in the coloured box order (octree.unknown_order)
and in the natural Morton order (octree.natural_order), beside no
preconditioner and the exact inverse of the near-field matrix.

Plain FP64; the factorisation is the IKJ form of ILU(0) over sparse rows
(ilu0_sparse, equal to krylov.ilu0 on the same pattern).  Run from the
repository root:

    python -m oracle.ilu_order RADIUS SUBDIVISION [processes]

e.g. 1.0 3 (3,840 unknowns) or 2.0 4 (15,360 unknowns).
"""

from __future__ import annotations

import os
import sys
import time
from multiprocessing import Pool

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import spsolve_triangular

from . import krylov, mom, octree, rwg


def ilu0_sparse(A, pattern):
    """ILU(0) of A on the boolean pattern (elimination order = index order),
    row by row: for every row i and every pattern column k < i in ascending
    order, l_ik = a_ik / u_kk and a_ij -= l_ik u_kj for the pattern columns
    j > k of row i.  Returns (L unit lower, U upper) as CSR matrices."""
    n = A.shape[0]
    upper_cols, upper_vals, diag = [None] * n, [None] * n, np.zeros(n, dtype=complex)
    Lr, Lc, Lv = [], [], []
    mask = np.zeros(n, dtype=bool)
    for i in range(n):
        cols = np.nonzero(pattern[i])[0]
        row = np.zeros(n, dtype=complex)
        row[cols] = A[i, cols]
        mask[cols] = True
        for k in cols[cols < i]:
            row[k] /= diag[k]
            uc = upper_cols[k]
            keep = mask[uc]
            row[uc[keep]] -= row[k] * upper_vals[k][keep]
        lo = cols[cols < i]
        Lr.append(np.full(len(lo), i))
        Lc.append(lo)
        Lv.append(row[lo])
        diag[i] = row[i]
        up = cols[cols > i]
        upper_cols[i] = up
        upper_vals[i] = row[up]
        mask[cols] = False
    L = sp.csr_matrix((np.concatenate(Lv + [np.ones(n)]),
                       (np.concatenate(Lr + [np.arange(n)]), np.concatenate(Lc + [np.arange(n)]))), shape=(n, n))
    Ur = np.concatenate([np.full(len(upper_cols[i]) + 1, i) for i in range(n)])
    Uc = np.concatenate([np.r_[i, upper_cols[i]] for i in range(n)])
    Uv = np.concatenate([np.r_[diag[i], upper_vals[i]] for i in range(n)])
    return L, sp.csr_matrix((Uv, (Ur, Uc)), shape=(n, n))


def ilu_solver(L, U):
    def apply(v):
        y = spsolve_triangular(L, v, lower=True, unit_diagonal=True)
        return spsolve_triangular(U, y, lower=False)
    return apply


_MESH = None


def _rows(args):
    body, lo, hi = args
    global _MESH
    if _MESH is None:
        _MESH = rwg.from_body(body)
    return lo, mom.pmchwt_rows(_MESH, body.eps_r, body.mu_r, body.frequency, np.arange(lo, hi))


def dense_matrix(body, procs):
    mesh = rwg.from_body(body)
    ne = mesh.n_edges
    Z = np.empty((2 * ne, 2 * ne), dtype=complex)
    spans = [(body, lo, min(ne, lo + 64)) for lo in range(0, ne, 64)]
    with Pool(procs) as pool:
        for lo, (ZE, ZH) in pool.imap_unordered(_rows, spans):
            Z[lo:lo + len(ZE)] = ZE
            Z[ne + lo:ne + lo + len(ZH)] = ZH
    return mesh, Z


def study(radius, subdivision, eps_r=2.56, finest_box=0.25, restart=50, tol=1e-4, max_iters=1000, procs=None):
    from workloads import sphere_body

    body = sphere_body(radius, eps_r, subdivision)
    t0 = time.time()
    mesh, Z = dense_matrix(body, procs or os.cpu_count())
    nlev = octree.auto_levels(mesh, finest_box)
    keys = octree.finest_keys(mesh, finest_box, nlev)
    pat = octree.near_pattern(keys)
    kh, eh = mom.incidence(0.0, 0.0)
    b = mom.planewave_rhs(mesh, body.frequency, kh, eh)
    out = {"unknowns": 2 * mesh.n_edges, "levels": nlev, "fill_s": round(time.time() - t0, 1)}

    def run(name, precond):
        t = time.time()
        _, info = krylov.gmres(lambda v: Z @ v, b, precond, restart=restart, tol=tol, max_iters=max_iters)
        out[name] = {"iterations": info.iterations, "converged": info.converged,
                     "true_residual": float(info.true_residual), "s": round(time.time() - t, 1)}
        print(name, out[name], flush=True)

    run("none", None)
    for name, perm in (("ilu0_colour", octree.unknown_order(keys)), ("ilu0_natural", octree.natural_order(keys))):
        Ap = Z[np.ix_(perm, perm)]
        L, U = ilu0_sparse(np.where(pat[np.ix_(perm, perm)], Ap, 0), pat[np.ix_(perm, perm)])
        solve = ilu_solver(L, U)
        inv = np.empty_like(perm)
        inv[perm] = np.arange(len(perm))

        def precond(v, solve=solve, perm=perm, inv=inv):
            return solve(v[perm])[inv]

        run(name, precond)
    Zn = np.where(pat, Z, 0)
    lu = __import__("scipy.linalg", fromlist=["lu_factor"])
    F = lu.lu_factor(Zn)
    run("exact_near_inverse", lambda v: lu.lu_solve(F, v))
    return out


if __name__ == "__main__":
    r, s = float(sys.argv[1]), int(sys.argv[2])
    procs = int(sys.argv[3]) if len(sys.argv) > 3 else None
    print(study(r, s, procs=procs))
