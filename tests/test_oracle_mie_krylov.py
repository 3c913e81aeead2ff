"""Pins of the Mie series (Rayleigh limit, optical theorem, coated-sphere
limits) and of ILU(0)/GMRES (LU limit, pattern property, direct solve)."""

import numpy as np
import pytest

from oracle import krylov, mie


def test_rayleigh_limit():
    a, eps = 0.002, 4.0
    k = 2 * np.pi
    th = np.linspace(0, np.pi, 19)
    sE, sH = mie.sphere_rcs(a, eps, th)
    pol = abs((eps - 1) / (eps + 2)) ** 2
    ref = 4 * np.pi * k ** 4 * a ** 6 * pol
    assert np.allclose(sE, ref * np.cos(th) ** 2, rtol=2e-3, atol=1e-6 * ref)
    assert np.allclose(sH, ref * np.ones_like(th), rtol=1e-3)


def test_optical_theorem_and_angular_integral():
    x, m = 5.0, 1.6
    a, b = mie.coefficients_homogeneous(x, m)
    qext, qsca = mie.efficiencies(a, b, x)
    assert abs(qext - qsca) < 1e-10 * qext
    g, w = np.polynomial.legendre.leggauss(400)
    gam = np.arccos(g)
    S1, S2 = mie.amplitudes(a, b, gam)
    q_int = np.sum(w * (np.abs(S1) ** 2 + np.abs(S2) ** 2)) / x ** 2
    assert abs(q_int - qsca) < 1e-9 * qsca
    # lossy sphere absorbs
    a, b = mie.coefficients_homogeneous(x, mie.index_from_eps(6 - 0.5j))
    qext, qsca = mie.efficiencies(a, b, x)
    assert qext > qsca * 1.01


def test_coated_sphere_limits():
    k = 2 * np.pi
    th = np.linspace(0, np.pi, 37)
    # transparent shell: only the core scatters
    s1 = mie.coated_sphere_rcs(0.4, 6 - 0.5j, 0.7, 1.0, th)
    s2 = mie.sphere_rcs(0.4, 6 - 0.5j, th)
    assert np.allclose(s1, s2, rtol=1e-8)
    # core of the shell material: homogeneous sphere of the outer radius
    s1 = mie.coated_sphere_rcs(0.4, 2.56, 0.7, 2.56, th)
    s2 = mie.sphere_rcs(0.7, 2.56, th)
    assert np.allclose(s1, s2, rtol=1e-8)
    # lossless coated sphere conserves energy
    a, b = mie.coefficients_coated(k * 0.4, k * 0.7, mie.index_from_eps(6.0), mie.index_from_eps(2.56))
    qext, qsca = mie.efficiencies(a, b, k * 0.7)
    assert abs(qext - qsca) < 1e-9 * qext


def _test_matrix(n, seed=3):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return A / np.sqrt(n) + 3 * np.eye(n)


def test_ilu0_full_pattern_is_lu_and_gmres_takes_one_step():
    A = _test_matrix(40)
    F = krylov.ilu0(A, np.ones_like(A, dtype=bool))
    L = np.tril(F, -1) + np.eye(40)
    U = np.triu(F)
    assert np.allclose(L @ U, A, atol=1e-12)
    b = np.arange(40) + 1j
    x, info = krylov.gmres(lambda v: A @ v, b, lambda v: krylov.ilu_apply(F, v), restart=10, tol=1e-10)
    assert info.converged and info.iterations == 1
    assert np.allclose(x, np.linalg.solve(A, b), atol=1e-10)


def test_ilu0_matches_on_pattern():
    n = 60
    A = _test_matrix(n)
    rng = np.random.default_rng(7)
    pat = rng.random((n, n)) < 0.25
    pat |= pat.T
    np.fill_diagonal(pat, True)
    F = krylov.ilu0(A, pat)
    L = np.tril(F, -1) + np.eye(n)
    U = np.triu(F)
    assert np.all(F[~pat] == 0)
    assert np.allclose((L @ U)[pat], A[pat], atol=1e-12)


def test_gmres_solves_and_reports():
    n = 80
    A = _test_matrix(n, seed=11)
    b = np.exp(1j * np.arange(n))
    x, info = krylov.gmres(lambda v: A @ v, b, restart=15, tol=1e-12, max_iters=2000)
    assert info.converged and info.true_residual <= 1e-12
    assert np.allclose(x, np.linalg.solve(A, b), atol=1e-10)
    # an exact initial guess needs no iteration
    x2, info2 = krylov.gmres(lambda v: A @ v, b, restart=15, tol=1e-10, x0=np.linalg.solve(A, b))
    assert info2.converged and info2.iterations == 0
    # an iteration cap reports non-convergence and the true residual
    _, info3 = krylov.gmres(lambda v: A @ v, b, restart=5, tol=1e-14, max_iters=3)
    assert not info3.converged and info3.iterations == 3 and info3.true_residual > 1e-14
    # unrestarted GMRES converges in at most n steps
    _, info4 = krylov.gmres(lambda v: A @ v, b, restart=n, tol=1e-10, max_iters=n)
    assert info4.converged and info4.iterations <= n


def test_full_degree_polynomial_is_the_inverse():
    # the residual polynomial of n GMRES steps vanishes on the whole spectrum
    n = 12
    A = _test_matrix(n, seed=21)
    th = krylov.leja_order(krylov.harmonic_ritz(lambda v: A @ v, krylov.golden_start(n), n))
    assert np.allclose(np.sort_complex(th), np.sort_complex(np.linalg.eigvals(A)), atol=1e-8)
    v = np.cos(np.arange(n)) + 1j
    y = krylov.poly_apply(lambda u: A @ u, th, v)
    assert np.allclose(y, np.linalg.solve(A, v), atol=1e-8)


def test_polynomial_preconditioner_reduces_iterations():
    n = 120
    rng = np.random.default_rng(5)
    A = np.diag(np.linspace(1, 50, n) * np.exp(0.3j * rng.standard_normal(n))) + \
        0.05 * (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    b = np.ones(n, dtype=complex)
    th = krylov.leja_order(krylov.harmonic_ritz(lambda v: A @ v, krylov.golden_start(n), 10))
    _, i0 = krylov.gmres(lambda v: A @ v, b, restart=20, tol=1e-8, max_iters=2000)
    _, i1 = krylov.gmres(lambda v: A @ v, b, lambda v: krylov.poly_apply(lambda u: A @ u, th, v),
                         restart=20, tol=1e-8, max_iters=2000)
    assert i1.converged and i1.iterations * 3 < i0.iterations
    # order of the roots does not change the operator
    v = np.sin(np.arange(n)) + 0j
    y1 = krylov.poly_apply(lambda u: A @ u, th, v)
    y2 = krylov.poly_apply(lambda u: A @ u, th[::-1], v)
    assert np.allclose(y1, y2, rtol=1e-8)


def test_golden_start_is_unit_modulus_and_deterministic():
    v = krylov.golden_start(5)
    assert np.allclose(np.abs(v), 1) and v[0] == 1
    g = (np.sqrt(5) - 1) / 2
    assert np.isclose(np.angle(v[1]), 2 * np.pi * g - 2 * np.pi)


def test_edge_block_scaling_pins():
    rng = np.random.default_rng(12)
    ne = 40
    # a matrix made of 2x2 edge blocks only: the scaled operator is I and the
    # degree-1 polynomial is exact
    D = rng.standard_normal((ne, 2, 2)) + 1j * rng.standard_normal((ne, 2, 2)) + 3 * np.eye(2)
    Zb = np.zeros((2 * ne, 2 * ne), dtype=complex)
    i = np.arange(ne)
    Zb[i, i], Zb[i, ne + i], Zb[ne + i, i], Zb[ne + i, ne + i] = D[:, 0, 0], D[:, 0, 1], D[:, 1, 0], D[:, 1, 1]
    Dinv = krylov.edge_blocks_inverse(Zb)
    v = rng.standard_normal(2 * ne) + 1j * rng.standard_normal(2 * ne)
    assert np.allclose(Zb @ krylov.edge_blocks_apply(Dinv, v), v, atol=1e-12)
    assert np.allclose(krylov.near_poly_preconditioner(Zb, 1)(v), np.linalg.solve(Zb, v), atol=1e-12)
    # badly scaled J/M halves plus a weak coupling: the scaled polynomial is
    # far closer to the inverse than the unscaled one of the same degree
    s = np.concatenate([np.full(ne, 1e-2), np.full(ne, 1e2)])
    Zs = s[:, None] * (Zb + 0.05 * (rng.standard_normal((2 * ne, 2 * ne)) + 1j * rng.standard_normal((2 * ne, 2 * ne))) / np.sqrt(2 * ne))
    ref = np.linalg.solve(Zs, v)
    e_scaled = np.linalg.norm(krylov.near_poly_preconditioner(Zs, 8)(v) - ref) / np.linalg.norm(ref)
    th = krylov.leja_order(krylov.harmonic_ritz(lambda u: Zs @ u, krylov.golden_start(2 * ne), 8))
    e_plain = np.linalg.norm(krylov.poly_apply(lambda u: Zs @ u, th, v) - ref) / np.linalg.norm(ref)
    assert e_scaled < 1e-3 and e_scaled < 1e-2 * e_plain


@pytest.mark.parametrize("method", ["bicgstab", "cgs"])
def test_bicg_family_terminates_and_solves(method):
    solve = getattr(krylov, method)
    rng = np.random.default_rng(17)
    n = 60
    # a diagonalisable matrix with three distinct eigenvalues: the BiCG
    # residual polynomial (and its square, and its product with the
    # stabilising factors) annihilates it after three steps
    Q = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    lam = np.repeat([2.0 + 1j, -1.5, 4.0 - 2j], n // 3)
    A = Q @ np.diag(lam) @ np.linalg.inv(Q)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, info = solve(lambda v: A @ v, b, tol=1e-10, max_iters=50)
    assert info.converged and info.iterations <= 3
    assert np.linalg.norm(A @ x - b) <= 1e-9 * np.linalg.norm(b)
    # the exact inverse as preconditioner: one iteration
    Ainv = np.linalg.inv(A)
    x, info = solve(lambda v: A @ v, b, lambda v: Ainv @ v, tol=1e-10, max_iters=50)
    assert info.converged and info.iterations == 1
    # a general non-normal system: the direct solution, the true residual
    A = _test_matrix(80, seed=23)
    x, info = solve(lambda v: A @ v, b[:1].repeat(80) * np.exp(1j * np.arange(80)), tol=1e-12, max_iters=500)
    ref = np.linalg.solve(A, b[:1].repeat(80) * np.exp(1j * np.arange(80)))
    assert info.converged and np.allclose(x, ref, atol=1e-9 * np.abs(ref).max())
    # an iteration cap is reported with the true residual of the last iterate
    _, info = solve(lambda v: A @ v, np.ones(80, dtype=complex), tol=1e-14, max_iters=2)
    assert not info.converged and info.iterations == 2 and info.true_residual > 1e-14


def test_sparse_ilu0_equals_dense_ilu0_and_orders_are_permutations():
    from oracle import octree
    from oracle.ilu_order import ilu0_sparse
    n = 70
    A = _test_matrix(n, seed=31)
    rng = np.random.default_rng(31)
    pat = rng.random((n, n)) < 0.2
    pat |= pat.T
    np.fill_diagonal(pat, True)
    F = krylov.ilu0(A, pat)
    L, U = ilu0_sparse(np.where(pat, A, 0), pat)
    assert np.abs((L.toarray() - np.eye(n)) + U.toarray() - F).max() < 1e-12
    keys = rng.integers(0, 8, size=(40, 3))
    for perm in (octree.unknown_order(keys), octree.natural_order(keys)):
        assert sorted(perm) == list(range(80))
        assert np.all(perm[1::2] == perm[0::2] + 40)          # J then M~ of one edge
    nat = octree.natural_order(keys)[0::2]
    assert np.all(np.diff(octree.morton(keys)[nat]) >= 0)     # boxes in Morton order
