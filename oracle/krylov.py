"""ILU(0) and right-preconditioned restarted GMRES(m).

The paper accelerates its Krylov solver with an incomplete LU preconditioner
(Simulation Results, Fig. 7 discussion) but does not name the variant; the
reading adopted is ILU(0) of the near-field matrix in the ordering of the
octree module: no pivoting, no fill outside the near pattern.  The Krylov
method is restarted GMRES(m) (Saad & Schultz, SIAM J. Sci. Stat. Comput. 7,
1986) with right preconditioning, classical Gram-Schmidt applied twice, and
complex Givens rotations; convergence is declared only when the true residual
||b - A x|| / ||b|| is at most the tolerance.
"""

from __future__ import annotations

import dataclasses

import numpy as np
from scipy.linalg import solve_triangular


def ilu0(A, pattern):
    """ILU(0) of the dense matrix A restricted to the boolean pattern (both in
    the elimination order).  Returns the packed factors: unit lower L strictly
    below the diagonal, U on and above it."""
    n = A.shape[0]
    F = np.where(pattern, A, 0).astype(complex)
    for i in range(1, n):
        for k in np.nonzero(pattern[i, :i])[0]:
            F[i, k] /= F[k, k]
            cols = np.nonzero(pattern[i, k + 1:])[0] + k + 1
            F[i, cols] -= F[i, k] * F[k, cols]
    return F


def ilu_apply(F, v):
    """z = U^-1 L^-1 v for packed ILU factors."""
    y = solve_triangular(F, v, lower=True, unit_diagonal=True)
    return solve_triangular(F, y, lower=False)


@dataclasses.dataclass
class GmresInfo:
    converged: bool
    iterations: int          # Arnoldi steps (one preconditioned product each)
    restarts: int
    true_residual: float     # ||b - A x|| / ||b|| at exit
    history: list            # estimated relative residual after every step


def _givens(a, b):
    """c (real), s with [[c, s], [-conj(s), c]] [a; b] = [r; 0]."""
    na, nb = abs(a), abs(b)
    if nb == 0.0:
        return 1.0, 0.0
    if na == 0.0:
        return 0.0, np.conj(b) / nb
    rho = np.hypot(na, nb)
    return na / rho, (a / na) * np.conj(b) / rho


def gmres(matvec, b, precond=None, restart=30, tol=1e-6, max_iters=1000, x0=None):
    """Solve A x = b with A M^-1 u = b, x = M^-1 u (right preconditioning)."""
    precond = precond or (lambda v: v)
    b = np.asarray(b, dtype=complex)
    nb = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=complex)
    if nb == 0.0:
        return np.zeros_like(b), GmresInfo(True, 0, 0, 0.0, [])
    its, restarts, hist = 0, 0, []
    while True:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        if beta / nb <= tol:
            return x, GmresInfo(True, its, restarts, beta / nb, hist)
        if its >= max_iters:
            return x, GmresInfo(False, its, restarts, beta / nb, hist)
        m = restart
        V = np.zeros((m + 1, len(b)), dtype=complex)
        H = np.zeros((m + 1, m), dtype=complex)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=complex)
        g = np.zeros(m + 1, dtype=complex)
        g[0] = beta
        V[0] = r / beta
        j_end = 0
        for j in range(m):
            w = matvec(precond(V[j]))
            its += 1
            h = V[: j + 1].conj() @ w
            w = w - V[: j + 1].T @ h
            h2 = V[: j + 1].conj() @ w
            w = w - V[: j + 1].T @ h2
            H[: j + 1, j] = h + h2
            H[j + 1, j] = np.linalg.norm(w)
            breakdown = H[j + 1, j] == 0
            if not breakdown:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j] = _givens(H[j, j], H[j + 1, j])
            H[j, j] = cs[j] * H[j, j] + sn[j] * H[j + 1, j]
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            hist.append(abs(g[j + 1]) / nb)
            j_end = j + 1
            if abs(g[j + 1]) / nb <= tol or its >= max_iters or breakdown:
                break
        y = solve_triangular(H[:j_end, :j_end], g[:j_end], lower=False)
        x = x + precond(V[:j_end].T @ y)
        restarts += 1
