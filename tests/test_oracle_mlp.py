"""Pins of the FP64 reference of the learned guess: backpropagation against
central finite differences, Adam against its closed form on a 1-parameter
problem, the POD basis against its definition (orthonormal, captures the
span), the linear path against the defining property of the minimum-norm
least-squares fit (it reproduces any linear map on the span of the training
features and ignores the orthogonal complement), the radiation-pattern
features against the rotation of the body (a rotation about z by one phi step
shifts the features by one phi column), and the whole pipeline against the
dense moment matrix of a small sphere (the guess's true residual)."""

import numpy as np
import pytest

from oracle import krylov, mlp, mom, rwg
from workloads import Body, sphere_body, theta_sweep


def test_gradients_match_central_differences():
    rng = np.random.default_rng(0)
    params = mlp.init([7, 9, 6, 4], seed=1)
    for layer in params:
        layer[1] = rng.standard_normal(layer[1].shape) * 0.1
    X = rng.standard_normal((5, 7))
    Y = rng.standard_normal((5, 4))
    _, grads = mlp.loss_and_grads(params, X, Y)
    h = 1e-6
    for li, layer in enumerate(params):
        for k in range(2):
            p = layer[k]
            it = np.nditer(p, flags=["multi_index"])
            for _ in it:
                idx = it.multi_index
                old = p[idx]
                p[idx] = old + h
                lp, _ = mlp.loss_and_grads(params, X, Y)
                p[idx] = old - h
                lm, _ = mlp.loss_and_grads(params, X, Y)
                p[idx] = old
                fd = (lp - lm) / (2 * h)
                g = grads[li][k][idx]
                assert abs(fd - g) <= 1e-6 * max(1.0, abs(fd)), (li, k, idx, fd, g)


def test_adam_first_step_is_signed_learning_rate():
    # with zero moments, the bias-corrected first step is -lr * g/(|g| + eps)
    params = [[np.array([[2.0]]), np.array([0.5])]]
    grads = [[np.array([[3.0]]), np.array([-0.25])]]
    state = {}
    mlp.adam(params, grads, state, lr=0.01)
    assert np.isclose(params[0][0][0, 0], 2.0 - 0.01 * 3.0 / (3.0 + 1e-8))
    assert np.isclose(params[0][1][0], 0.5 + 0.01 * 0.25 / (0.25 + 1e-8))


def test_training_fits_a_smooth_map():
    rng = np.random.default_rng(2)
    X = rng.uniform(-1, 1, (64, 3))
    Y = np.stack([np.sin(2 * X[:, 0]) * X[:, 1], np.cos(X[:, 2]) + X[:, 0] ** 2], axis=1)
    params = mlp.init([3, 32, 32, 2], seed=3)
    state = {}
    l0, _ = mlp.loss_and_grads(params, X, Y)
    for _ in range(1500):
        loss, g = mlp.loss_and_grads(params, X, Y)
        mlp.adam(params, g, state, lr=3e-3)
    assert loss < 0.02 * l0


def test_pod_basis():
    rng = np.random.default_rng(4)
    basis = rng.standard_normal((200, 3)) + 1j * rng.standard_normal((200, 3))
    coeff = rng.standard_normal((10, 3)) + 1j * rng.standard_normal((10, 3))
    X = coeff @ basis.T
    U = mlp.pod_basis(X, 3)
    assert np.allclose(U.conj().T @ U, np.eye(3), atol=1e-12)
    # every solution lies in span(U)
    assert np.allclose(U @ (U.conj().T @ X.T), X.T, atol=1e-10)


def test_output_layer_starts_at_zero():
    params = mlp.init([5, 7, 7, 3], seed=2, zero_last=True)
    out, _ = mlp.forward(params, np.random.default_rng(0).standard_normal((4, 5)))
    assert np.all(out == 0.0)
    assert np.all(params[0][0] != 0.0)


def test_min_norm_lstsq_reproduces_linear_maps_on_the_span():
    rng = np.random.default_rng(6)
    Zp = rng.standard_normal((12, 40))
    M = rng.standard_normal((40, 5))
    Ws = mlp.min_norm_lstsq(Zp, Zp @ M)
    # every combination of training features maps like the linear map
    alpha = rng.standard_normal((3, 12))
    z = alpha @ Zp
    assert np.allclose(z @ Ws, z @ M, rtol=0, atol=1e-10 * np.abs(z @ M).max())
    # directions orthogonal to the training features map to zero (minimum norm)
    q, _ = np.linalg.qr(Zp.T, mode="complete")
    perp = q[:, 12:].T
    assert np.abs(perp @ Ws).max() < 1e-10 * np.abs(Ws).max()
    # training rows are reproduced
    assert np.allclose(Zp @ Ws, Zp @ M, atol=1e-10 * np.abs(Zp @ M).max())


def test_pattern_features_rotate_with_the_body():
    b = sphere_body(0.3, 4.0, 2)
    m = rwg.from_body(b)
    n_theta, n_phi = 5, 12
    phi0 = 2 * np.pi / n_phi
    c, s = np.cos(phi0), np.sin(phi0)
    Rz = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
    # same vertex ids, so the same edge numbering and the same current vector
    br = Body(b.vertices @ Rz.T, b.triangles, b.tri_regions, b.eps_r, b.mu_r, name="rotated")
    mr = rwg.from_body(br)
    rng = np.random.default_rng(8)
    x = rng.standard_normal((2, 2 * m.n_edges)) + 1j * rng.standard_normal((2, 2 * m.n_edges))
    f = mlp.pattern_features(m, b.frequency, x, n_theta, n_phi).reshape(2, n_theta, n_phi, 4)
    fr = mlp.pattern_features(mr, b.frequency, x, n_theta, n_phi).reshape(2, n_theta, n_phi, 4)
    assert np.allclose(fr, np.roll(f, 1, axis=2), rtol=0, atol=1e-10 * np.abs(f).max())
    # and the features are not trivially invariant
    assert np.abs(f - np.roll(f, 1, axis=2)).max() > 1e-3 * np.abs(f).max()


@pytest.fixture(scope="module")
def small_sweep():
    b = sphere_body(0.3, 4.0, 2)
    m = rwg.from_body(b)
    Z = mom.pmchwt_dense(m, b.eps_r, b.mu_r, b.frequency)
    ang = theta_sweep(25, phi=0.3)
    B = np.array([mom.planewave_rhs(m, b.frequency, *mom.incidence(t, p)) for t, p in ang])
    X = np.linalg.solve(Z, B.T).T
    return b, m, Z, ang, B, X


@pytest.mark.parametrize("epochs", [0, 150])
def test_learned_guess_pipeline_on_a_small_sphere(small_sweep, epochs):
    b, m, Z, ang, B, X = small_sweep
    tr = np.arange(0, 25, 2)                      # both ends of the sweep included
    te = np.setdiff1d(np.arange(25), tr)
    model = mlp.fit_guess(m, b.frequency, ang[tr], B[tr], X[tr], hidden=32, epochs=epochs, lr=3e-3)
    r = model["U"].shape[1]
    assert r == len(tr)
    # the MLP starts at zero on unit-RMS targets (loss r); Adam lowers it
    # (measured 6.8 of 13)
    assert model["loss"] <= r * (1 + 1e-12) and (epochs == 0 or model["loss"] < 0.8 * r)
    # the training currents are reproduced (measured 1.8e-5 and 1.3e-5)
    X0tr = mlp.predict_guess(model, ang[tr], B[tr])
    assert np.linalg.norm(X0tr - X[tr]) < 1e-4 * np.linalg.norm(X[tr])
    # true residual of the guess between the training angles (measured median
    # 5.3e-5 / 3.8e-5, max 3.1e-4)
    X0 = mlp.predict_guess(model, ang[te], B[te])
    res = np.linalg.norm(B[te] - X0 @ Z.T, axis=1) / np.linalg.norm(B[te], axis=1)
    assert np.median(res) < 2e-4 and np.max(res) < 1e-3, res
    # the guess lies in the span of the training solutions
    U = model["U"]
    assert np.allclose(U @ (U.conj().T @ X0.T), X0.T, atol=1e-10 * np.abs(X0).max())
    # and GMRES from it needs fewer iterations than from zero
    x, info0 = krylov.gmres(lambda v: Z @ v, B[te[3]], restart=30, tol=1e-8)
    x, info1 = krylov.gmres(lambda v: Z @ v, B[te[3]], restart=30, tol=1e-8, x0=X0[3])
    assert info0.converged and info1.converged
    assert info1.iterations < 0.7 * info0.iterations, (info0.iterations, info1.iterations)
