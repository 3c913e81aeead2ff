"""Pins of the FP64 reference MLP: backpropagation against central finite
differences, Adam against its closed form on a 1-parameter problem, and the
POD basis against the definition (orthonormal, captures the span)."""

import numpy as np

from oracle import mlp


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


def _family(n_pts=240, seed=5):
    """A smooth family of systems Z x(theta) = b(theta): plane-wave-like
    right-hand sides sampled at random points, a non-normal Z."""
    rng = np.random.default_rng(seed)
    pts = rng.uniform(-1, 1, (n_pts, 2))
    lam = 1.0 + 2.0 * np.arange(n_pts) / n_pts * np.exp(1j * np.pi * np.arange(n_pts) / n_pts)
    Z = np.diag(lam) + 0.3 * (rng.standard_normal((n_pts, n_pts)) + 1j * rng.standard_normal((n_pts, n_pts))) / np.sqrt(n_pts)

    def rhs(theta):
        return np.exp(-4j * (np.cos(theta)[:, None] * pts[:, 0] + np.sin(theta)[:, None] * pts[:, 1]))

    return Z, rhs


def test_learned_guess_pipeline_cuts_iterations():
    from oracle import krylov
    Z, rhs = _family()
    th = np.linspace(0, np.pi, 73)
    tr = np.arange(0, 73, 2)
    te = np.setdiff1d(np.arange(73), tr)
    ang = np.stack([th, np.zeros_like(th)], axis=1)
    B = rhs(th)
    X = np.linalg.solve(Z, B.T).T
    model = mlp.fit_guess(ang[tr], B[tr], X[tr], rank=24, harmonics=4, hidden=32, epochs=2000, lr=3e-3)
    X0 = mlp.predict_guess(model, ang[te], B[te])
    res = np.linalg.norm(B[te] - X0 @ Z.T, axis=1) / np.linalg.norm(B[te], axis=1)
    assert np.median(res) < 0.06   # measured 0.025
    # the guess lies in the span of the training solutions
    U = model["U"]
    assert np.allclose(U @ (U.conj().T @ X0.T), X0.T, atol=1e-10 * np.abs(X0).max())
    its0 = its1 = 0
    for i in range(0, len(te), 6):
        x, info0 = krylov.gmres(lambda v: Z @ v, B[te[i]], restart=30, tol=1e-4)
        x, info1 = krylov.gmres(lambda v: Z @ v, B[te[i]], restart=30, tol=1e-4, x0=X0[i])
        assert info0.converged and info1.converged
        its0 += info0.iterations
        its1 += info1.iterations
    assert its1 < 0.75 * its0   # measured 144 vs 245
