"""FP64 reference of the learned initial guess for GMRES.

The paper has no learned component; this module is the reference for an
addition to the method: a network, trained on solved currents, that predicts
the GMRES initial guess for a new incidence.  Plain numpy:

* POD basis: U = the r leading left singular vectors of the matrix of solved
  currents X = [x_1 .. x_n] (complex, r clamped to the resolved rank);
  coefficients c = U^H x.
* radiation-pattern features of a right-hand side b: b read as the surface
  currents [J ; M~] and its far field F (eqs. 27-29, `farfield.far_field`)
  sampled on a coarse direction grid (theta at the midpoints of n_theta
  bands of [0, pi], phi at n_phi uniform points of [0, 2 pi), theta-major);
  per direction Re/Im of theta.F then Re/Im of phi.F, divided by ||b||.
* network input z = [cos(m theta), sin(m theta), cos(m phi), sin(m phi) for
  m = 1..M ; s_p * pattern features], s_p one scalar (the inverse RMS of the
  training features).
* network: a linear path from the pattern part z_p of z straight to the
  output plus two tanh hidden layers with a linear output layer that starts
  at zero:   y(z) = Ws^T z_p + MLP(z) / s_r.
  Targets y = s_y [Re c ; Im c] / ||b||, s_y one scalar.  The map from a
  right-hand side to its currents is linear, so the linear path is fitted
  first, in closed form: the minimum-norm least-squares Ws = Z_p^T (Z_p
  Z_p^T)^+ Y (eigenvalues of the Gram matrix below `cutoff` times the largest
  dropped).  The MLP then learns what the linear path leaves, R = Y - Z_p Ws,
  scaled to unit RMS (s_r), by full-batch Adam (Kingma & Ba 2015,
  bias-corrected) on 0.5/B sum ||MLP(z) - s_r R||^2 with the step decayed as
  lr (1 + cos(pi (t - 1) / E)) / 2.
* guess x0 = U (y_re + j y_im) ||b|| / s_y; the solver keeps it only if its
  true residual is below ||b|| (otherwise it starts from zero).
"""

import numpy as np

from . import farfield


def pod_basis(X, r, resolved=1e-14):
    """X: [n, N] complex solutions (rows). Returns U [N, r'] orthonormal, r' <=
    r the number of squared singular values above `resolved` times the largest."""
    u, s, vh = np.linalg.svd(X.T, full_matrices=False)
    w = s ** 2
    keep = int(np.sum(w > resolved * w[0])) if w.size and w[0] > 0 else 0
    return u[:, :max(1, min(r, keep))]


def pattern_directions(n_theta, n_phi):
    """[n_theta * n_phi, 2] (theta, phi), theta-major."""
    th = (np.arange(n_theta) + 0.5) * np.pi / n_theta
    ph = np.arange(n_phi) * 2.0 * np.pi / n_phi
    T, P = np.meshgrid(th, ph, indexing="ij")
    return np.stack([T.ravel(), P.ravel()], axis=1)


def pattern_features(mesh, frequency, B, n_theta, n_phi):
    """[n, 4 nd] radiation-pattern features of the right-hand sides B [n, 2E]
    (not yet divided by ||b||)."""
    d = pattern_directions(n_theta, n_phi)
    r, th, ph = farfield.spherical_units(d[:, 0], d[:, 1])
    T = farfield.basis_transforms(mesh, frequency, r)
    out = np.zeros((len(B), 4 * len(d)))
    for i, b in enumerate(B):
        F = farfield.far_field(mesh, frequency, b, d[:, 0], d[:, 1], T)
        ft = np.sum(th * F, axis=-1)
        fp = np.sum(ph * F, axis=-1)
        out[i] = np.stack([ft.real, ft.imag, fp.real, fp.imag], axis=1).ravel()
    return out


def angle_harmonics(theta, phi, M):
    th = np.atleast_1d(theta)[:, None]
    ph = np.atleast_1d(phi)[:, None]
    m = np.arange(1, M + 1)[None, :]
    return np.concatenate([np.cos(m * th), np.sin(m * th), np.cos(m * ph), np.sin(m * ph)], axis=1)


def init(sizes, seed=0, zero_last=False):
    """Weights W_l [in, out] uniform(+-sqrt(6/(in+out))), biases zero; with
    zero_last the output layer starts at zero."""
    rng = np.random.default_rng(seed)
    params = []
    for i, (a, b) in enumerate(zip(sizes[:-1], sizes[1:])):
        lim = np.sqrt(6.0 / (a + b))
        W = rng.uniform(-lim, lim, size=(a, b))
        if zero_last and i == len(sizes) - 2:
            W = np.zeros((a, b))
        params.append([W, np.zeros(b)])
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


def min_norm_lstsq(Zp, R, cutoff=1e-12):
    """Ws = Zp^T G^+ R, G = Zp Zp^T, eigenvalues at or below cutoff * the
    largest dropped: the minimum-norm W with Zp W = R on the resolved span."""
    G = Zp @ Zp.T
    w, V = np.linalg.eigh(G)
    keep = w > cutoff * w.max() if w.size and w.max() > 0 else np.zeros(w.shape, bool)
    Gp = (V[:, keep] / w[keep]) @ V[:, keep].T
    return Zp.T @ (Gp @ R)


def fit_guess(mesh, frequency, angles, B, X, rank=72, harmonics=4, hidden=768, epochs=300, lr=1e-3, seed=0,
              n_theta=16, n_phi=31, cutoff=1e-12):
    """Whole training pipeline in FP64.  angles [n, 2] (theta, phi); B, X
    [n, N] right-hand sides and solutions."""
    U = pod_basis(X, min(rank, X.shape[0]))
    r = U.shape[1]
    nb = np.linalg.norm(B, axis=1, keepdims=True)
    P = pattern_features(mesh, frequency, B, n_theta, n_phi) / nb
    s_p = 1.0 / np.sqrt(np.mean(P ** 2))
    Zp = s_p * P
    Z = np.concatenate([angle_harmonics(angles[:, 0], angles[:, 1], harmonics), Zp], axis=1)
    c = (X @ U.conj()) / nb
    Y = np.concatenate([c.real, c.imag], axis=1)
    s_y = 1.0 / np.sqrt(np.mean(Y ** 2))
    Y = s_y * Y
    Ws = min_norm_lstsq(Zp, Y, cutoff)
    R = Y - Zp @ Ws
    rms = np.sqrt(np.mean(R ** 2))
    s_r = 1.0 / rms if rms > 0 else 1.0
    params = init([Z.shape[1], hidden, hidden, 2 * r], seed, zero_last=True)
    state = {}
    for e in range(epochs):
        _, grads = loss_and_grads(params, Z, s_r * R)
        adam(params, grads, state, lr=lr * 0.5 * (1.0 + np.cos(np.pi * e / epochs)))
    loss, _ = loss_and_grads(params, Z, s_r * R)
    return dict(U=U, s_p=s_p, s_y=s_y, s_r=s_r, params=params, Ws=Ws, harmonics=harmonics, n_theta=n_theta,
                n_phi=n_phi, mesh=mesh, frequency=frequency, loss=loss)


def predict_guess(model, angles, B):
    """x0 = U c ||b|| with c decoded from the network output."""
    U, r = model["U"], model["U"].shape[1]
    nb = np.linalg.norm(B, axis=1, keepdims=True)
    Zp = model["s_p"] * pattern_features(model["mesh"], model["frequency"], B, model["n_theta"],
                                         model["n_phi"]) / nb
    Z = np.concatenate([angle_harmonics(angles[:, 0], angles[:, 1], model["harmonics"]), Zp], axis=1)
    out, _ = forward(model["params"], Z)
    Yp = (Zp @ model["Ws"] + out / model["s_r"]) / model["s_y"]
    return ((Yp[:, :r] + 1j * Yp[:, r:]) * nb) @ U.T
