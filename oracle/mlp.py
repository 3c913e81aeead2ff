"""FP64 reference of the learned initial guess for GMRES.

The paper has no learned component; this module is the reference for an
addition to the method: a small network, trained on solved currents, that
predicts the GMRES initial guess for a new incidence angle.  Plain numpy:

* POD basis: U = the first r left singular vectors of the matrix of solved
  currents X = [x_1 .. x_n] (complex); coefficients c = U^H x.
* features of an incidence (theta, phi) with right-hand side b:
  [cos(m theta), sin(m theta), cos(m phi), sin(m phi)] for m = 1..M, then
  Re/Im of U^H b scaled by 1/||b||.
* network: two tanh hidden layers, linear output of the 2r real coefficients
  (Re then Im), mean-squared error 0.5/B sum ||y_hat - y||^2, Adam
  (Kingma & Ba 2015) with bias correction.
* guess x0 = U (y_re + j y_im) * ||b||; the solver keeps it only if its true
  residual is below ||b|| (otherwise it starts from zero).
"""

import numpy as np


def pod_basis(X, r):
    """X: [n, N] complex solutions (rows). Returns U [N, r] orthonormal."""
    u, s, vh = np.linalg.svd(X.T, full_matrices=False)
    return u[:, :r]


def features(theta, phi, b, U, M):
    """[n, 4M + 2r] feature rows for incidences (theta, phi) with RHS rows b."""
    th = np.atleast_1d(theta)[:, None]
    ph = np.atleast_1d(phi)[:, None]
    m = np.arange(1, M + 1)[None, :]
    nb = np.linalg.norm(b, axis=1, keepdims=True)
    proj = (b @ U.conj()) / nb
    return np.concatenate([np.cos(m * th), np.sin(m * th), np.cos(m * ph), np.sin(m * ph),
                           proj.real, proj.imag], axis=1)


def targets(X, b, U):
    """[n, 2r] real targets: Re/Im of U^H x scaled by 1/||b||."""
    nb = np.linalg.norm(b, axis=1, keepdims=True)
    c = (X @ U.conj()) / nb
    return np.concatenate([c.real, c.imag], axis=1)


def init(sizes, seed=0):
    """Weights W_l [in, out] uniform(+-sqrt(6/(in+out))), biases zero."""
    rng = np.random.default_rng(seed)
    params = []
    for a, b in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / (a + b))
        params.append([rng.uniform(-lim, lim, size=(a, b)), np.zeros(b)])
    return params


def forward(params, X):
    """Returns output and the list of layer activations (inputs of each layer)."""
    acts = [X]
    h = X
    for i, (W, b) in enumerate(params):
        z = h @ W + b
        h = np.tanh(z) if i < len(params) - 1 else z
        acts.append(h)
    return h, acts


def loss_and_grads(params, X, Y):
    """0.5/B sum ||f(X) - Y||^2 and its gradients (backpropagation)."""
    B = X.shape[0]
    out, acts = forward(params, X)
    diff = out - Y
    loss = 0.5 * np.sum(diff ** 2) / B
    grads = [None] * len(params)
    delta = diff / B                               # dL/d(output pre-activation)
    for i in range(len(params) - 1, -1, -1):
        W, _ = params[i]
        grads[i] = [acts[i].T @ delta, delta.sum(axis=0)]
        if i > 0:
            delta = (delta @ W.T) * (1.0 - acts[i] ** 2)   # tanh' = 1 - tanh^2
    return loss, grads


def adam(params, grads, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step in place; state = {'t': int, 'm': [...], 'v': [...]}."""
    if not state:
        state["t"] = 0
        state["m"] = [[np.zeros_like(p) for p in layer] for layer in params]
        state["v"] = [[np.zeros_like(p) for p in layer] for layer in params]
    state["t"] += 1
    t = state["t"]
    for layer, g_layer, m_layer, v_layer in zip(params, grads, state["m"], state["v"]):
        for k in range(2):
            m_layer[k] = b1 * m_layer[k] + (1 - b1) * g_layer[k]
            v_layer[k] = b2 * v_layer[k] + (1 - b2) * g_layer[k] ** 2
            mh = m_layer[k] / (1 - b1 ** t)
            vh = v_layer[k] / (1 - b2 ** t)
            layer[k] = layer[k] - lr * mh / (np.sqrt(vh) + eps)
    return params


def standardize(Y):
    """Per-output mean and standard deviation (floored at 1e-6 of the largest)."""
    mu = Y.mean(axis=0)
    sd = Y.std(axis=0)
    top = sd.max() if sd.size else 0.0
    sd = np.maximum(sd, 1e-6 * top if top > 0 else 1.0)
    return mu, sd


def fit_guess(angles, B, X, rank=16, harmonics=4, hidden=64, epochs=6000, lr=3e-3, seed=0):
    """Whole training pipeline in FP64: POD basis, features, standardised
    targets, full-batch Adam with the step decayed as lr (1 + cos(pi e / E)) / 2.
    angles [n, 2] (theta, phi); B, X [n, N] right-hand sides and solutions."""
    r = min(rank, X.shape[0])
    U = pod_basis(X, r)
    F = features(angles[:, 0], angles[:, 1], B, U, harmonics)
    Y = targets(X, B, U)
    mu, sd = standardize(Y)
    params = init([F.shape[1], hidden, hidden, 2 * r], seed)
    state = {}
    for e in range(epochs):
        _, grads = loss_and_grads(params, F, (Y - mu) / sd)
        adam(params, grads, state, lr=lr * 0.5 * (1.0 + np.cos(np.pi * e / epochs)))
    loss, _ = loss_and_grads(params, F, (Y - mu) / sd)
    return dict(U=U, mu=mu, sd=sd, params=params, harmonics=harmonics, loss=loss)


def predict_guess(model, angles, B):
    """x0 = U c ||b|| with c decoded from the network output."""
    U, r = model["U"], model["U"].shape[1]
    F = features(angles[:, 0], angles[:, 1], B, U, model["harmonics"])
    out, _ = forward(model["params"], F)
    Yp = out * model["sd"] + model["mu"]
    nb = np.linalg.norm(B, axis=1, keepdims=True)
    return ((Yp[:, :r] + 1j * Yp[:, r:]) * nb) @ U.T
