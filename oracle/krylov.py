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


# --- polynomial preconditioner ---------------------------------------------
#
# Reading adopted for the paper's near-field preconditioner when ILU(0) of the
# PMCHWT near field is too poor an approximation of its inverse: a fixed
# polynomial p with p(Z_near) ~ Z_near^-1, namely the residual polynomial of
# d GMRES steps on Z_near (Loe & Morgan, Numer. Linear Algebra Appl. 2022).
# Its roots are the harmonic Ritz values of d Arnoldi steps from the
# deterministic start vector v0[i] = exp(2 pi j frac(i g)), g = (sqrt 5 - 1)/2,
# and it is applied in Leja order in product form.

def golden_start(n):
    g = 0.5 * (np.sqrt(5.0) - 1.0)
    i = np.arange(n, dtype=np.float64)
    t = i * g - np.floor(i * g)
    return np.exp(2j * np.pi * t)


def harmonic_ritz(matvec, v0, d):
    """Harmonic Ritz values of d Arnoldi steps (CGS2) from v0: eigenvalues of
    H_d + |h_{d+1,d}|^2 H_d^-H e_d e_d^T."""
    n = len(v0)
    V = np.zeros((d + 1, n), dtype=complex)
    H = np.zeros((d + 1, d), dtype=complex)
    V[0] = v0 / np.linalg.norm(v0)
    for j in range(d):
        w = matvec(V[j])
        for _ in range(2):
            h = V[: j + 1].conj() @ w
            w = w - V[: j + 1].T @ h
            H[: j + 1, j] += h
        H[j + 1, j] = np.linalg.norm(w)
        V[j + 1] = w / H[j + 1, j]
    Hd = H[:d, :d]
    ed = np.zeros(d)
    ed[-1] = 1.0
    f = np.linalg.solve(Hd.conj().T, ed)
    return np.linalg.eigvals(Hd + abs(H[d, d - 1]) ** 2 * np.outer(f, ed))


def leja_order(theta):
    """Largest modulus first, then each next root maximises the product of
    distances to the roots already chosen."""
    rest = list(theta)
    first = max(rest, key=abs)
    out = [first]
    rest.remove(first)
    while rest:
        nxt = max(rest, key=lambda t: np.sum(np.log(np.abs(t - np.array(out)) + 1e-300)))
        out.append(nxt)
        rest.remove(nxt)
    return np.array(out)


def poly_apply(matvec, roots, v):
    """y = p(A) v with 1 - z p(z) = prod_k (1 - z / roots_k)."""
    y = np.zeros_like(v)
    q = np.array(v, dtype=complex)
    for t in roots:
        y = y + q / t
        q = q - matvec(q) / t
    return y


# ---------------------------------------------------------------------------
# Edge-block scaling of the polynomial preconditioner.  Every RWG edge m owns
# the 2x2 self block D_m = [[Z_EJ(m,m), Z_EM(m,m)], [Z_HJ(m,m), Z_HM(m,m)]] of
# the near matrix (boundary layout: J/E rows 0..E-1, M/H rows E..2E-1).  The
# polynomial is built for D^-1 Z_near, which puts the J and M unknowns of
# every interface on a common scale, and applied as p(D^-1 Z_near) D^-1.

def edge_blocks_inverse(Zn):
    """[E, 2, 2] inverses of the edge self blocks of Zn (boundary layout)."""
    ne = Zn.shape[0] // 2
    i = np.arange(ne)
    D = np.empty((ne, 2, 2), dtype=complex)
    D[:, 0, 0] = Zn[i, i]
    D[:, 0, 1] = Zn[i, ne + i]
    D[:, 1, 0] = Zn[ne + i, i]
    D[:, 1, 1] = Zn[ne + i, ne + i]
    return np.linalg.inv(D)


def edge_blocks_apply(Dinv, v):
    ne = Dinv.shape[0]
    a, c = v[:ne], v[ne:]
    return np.concatenate([Dinv[:, 0, 0] * a + Dinv[:, 0, 1] * c, Dinv[:, 1, 0] * a + Dinv[:, 1, 1] * c])


def near_poly_preconditioner(Zn, degree):
    """v -> p(D^-1 Zn) D^-1 v with p the degree-d GMRES residual polynomial
    of D^-1 Zn (roots: harmonic Ritz values from golden_start, Leja order)."""
    Dinv = edge_blocks_inverse(Zn)

    def op(u):
        return edge_blocks_apply(Dinv, Zn @ u)

    th = leja_order(harmonic_ritz(op, golden_start(Zn.shape[0]), degree))
    return lambda v: poly_apply(op, th, edge_blocks_apply(Dinv, v))


# --- BiCGStab and CGS --------------------------------------------------------
#
# The paper compares ILU-preconditioned BiCGStab and CGS, and BiCGStab without
# a preconditioner (Simulation Results, Fig. 7 discussion).  Both are written
# here with right preconditioning (A M^-1 u = b, the iterate x = M^-1 u kept
# directly), an iteration being two preconditioned products; convergence is
# declared on the true residual, and a vanishing inner product or a
# recurrence residual that the true residual does not confirm restarts the
# method from the current iterate.

def _bicg_family(matvec, b, precond, tol, max_iters, x0, squared):
    precond = precond or (lambda v: v)
    b = np.asarray(b, dtype=complex)
    nb = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=complex)
    if nb == 0.0:
        return np.zeros_like(b), GmresInfo(True, 0, 0, 0.0, [])
    its, restarts, hist = 0, 0, []
    r = b - matvec(x)
    while True:
        if np.linalg.norm(r) / nb <= tol:
            return x, GmresInfo(True, its, restarts, np.linalg.norm(r) / nb, hist)
        if its >= max_iters:
            return x, GmresInfo(False, its, restarts, np.linalg.norm(r) / nb, hist)
        rh = r.copy()
        p = np.zeros_like(b)
        v = np.zeros_like(b)            # BiCGStab: A p^ ; CGS: q
        rho_old = alpha = omega = 1.0
        first = True
        while its < max_iters:
            rho = np.vdot(rh, r)
            if squared:                 # Sonneveld's CGS
                beta = 0.0 if first else rho / rho_old
                u = r + beta * v
                p = u + beta * (v + beta * p)
                ph = precond(p)
                vh = matvec(ph)
                sigma = np.vdot(rh, vh)
                alpha = rho / sigma if sigma != 0 else 0.0
                v = u - alpha * vh
                uh = precond(u + v)
                x = x + alpha * uh
                r = r - alpha * matvec(uh)
                broke = rho == 0 or sigma == 0
            else:                       # van der Vorst's BiCGStab
                beta = 0.0 if first else (rho / rho_old) * (alpha / omega)
                p = r + beta * (p - omega * v)
                ph = precond(p)
                v = matvec(ph)
                sigma = np.vdot(rh, v)
                alpha = rho / sigma if sigma != 0 else 0.0
                s = r - alpha * v
                sh = precond(s)
                t = matvec(sh)
                tt = np.vdot(t, t)
                omega = np.vdot(t, s) / tt if tt != 0 else 0.0
                x = x + alpha * ph + omega * sh
                r = s - omega * t
                broke = rho == 0 or sigma == 0 or omega == 0
            rho_old = rho
            first = False
            its += 1
            est = np.linalg.norm(r) / nb
            hist.append(est)
            if est <= tol or broke or not np.isfinite(est):
                break
        r = b - matvec(x)               # the true residual decides
        if np.linalg.norm(r) / nb > tol and its < max_iters:
            restarts += 1


def bicgstab(matvec, b, precond=None, tol=1e-6, max_iters=1000, x0=None):
    """Right-preconditioned BiCGStab (van der Vorst, SIAM J. Sci. Stat.
    Comput. 13, 1992)."""
    return _bicg_family(matvec, b, precond, tol, max_iters, x0, squared=False)


def cgs(matvec, b, precond=None, tol=1e-6, max_iters=1000, x0=None):
    """Right-preconditioned CGS (Sonneveld, SIAM J. Sci. Stat. Comput. 10,
    1989)."""
    return _bicg_family(matvec, b, precond, tol, max_iters, x0, squared=True)
