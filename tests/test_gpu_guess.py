"""GPU checks of the learned initial guess.

* The network kernels (matrix-core GEMMs with bf16-split operands, FP32
  accumulation) against the FP64 oracle MLP on the same parameters: outputs,
  loss and gradients within 1e-4 relative (bf16-split keeps about 16
  significant bits per operand); Adam steps and a short training run follow
  the oracle's.
* The whole fit/predict pipeline with the linear path alone (no Adam steps:
  deterministic) against the oracle's on the same angles and the same seeded
  training currents: radiation-pattern features, POD basis, minimum-norm
  least squares and the decode, within 1e-6.
* The trained guess on a theta sweep of a dielectric ellipsoid: it lies in the
  span of the training solutions, it reproduces them, it starts GMRES near
  the tolerance between the training angles, and every solve still meets the
  tolerance on its true residual.
* The solver's judge: a guess worse than zero is dropped.
"""

import numpy as np
import pytest

from oracle import mlp, rwg
from workloads import Body, icosphere, random_complex_vector, theta_sweep

pytestmark = pytest.mark.gpu

sfmm = pytest.importorskip("paper_1704_06862_amd.sfmm")

SIZES = [20, 48, 48, 10]


def flatten(params):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params]).astype(np.float32)


def unflatten(vec, sizes):
    out, off = [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        W = vec[off:off + a * b].reshape(a, b).astype(np.float64)
        off += a * b
        out.append([W, vec[off:off + b].astype(np.float64)])
        off += b
    return out


def problem(seed=0):
    rng = np.random.default_rng(seed)
    params = mlp.init(SIZES, seed=seed + 1)
    for layer in params:
        layer[1] = 0.1 * rng.standard_normal(layer[1].shape)
    p32 = flatten(params)
    X = rng.standard_normal((37, SIZES[0])).astype(np.float32)
    Y = rng.standard_normal((37, SIZES[-1])).astype(np.float32)
    return p32, X, Y


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_forward_and_gradients_match_oracle():
    print("mlp forward/backward parity", flush=True)
    p32, X, Y = problem()
    loss, grads, out = sfmm.sfmm_mlp_train(SIZES, p32.copy(), X, Y, steps=0)
    ref_params = unflatten(p32, SIZES)
    ref_out, _ = mlp.forward(ref_params, X.astype(np.float64))
    ref_loss, ref_grads = mlp.loss_and_grads(ref_params, X.astype(np.float64), Y.astype(np.float64))
    assert rel(out, ref_out) < 1e-4, rel(out, ref_out)
    assert abs(loss[0] - ref_loss) < 1e-4 * ref_loss
    g = unflatten(grads, SIZES)
    for li in range(len(g)):
        for k in range(2):
            a, b = g[li][k].ravel(), ref_grads[li][k].ravel()
            assert rel(a, b) <= 1e-4, (li, k, rel(a, b))


def test_adam_steps_follow_oracle():
    print("mlp adam parity", flush=True)
    p32, X, Y = problem(1)
    p = p32.copy()
    loss, _, _ = sfmm.sfmm_mlp_train(SIZES, p, X, Y, steps=20, lr=1e-3)
    ref = unflatten(p32, SIZES)
    state, ref_loss = {}, []
    for _ in range(20):
        l, g = mlp.loss_and_grads(ref, X.astype(np.float64), Y.astype(np.float64))
        ref_loss.append(l)
        mlp.adam(ref, g, state, lr=1e-3)
    ref_loss.append(mlp.loss_and_grads(ref, X.astype(np.float64), Y.astype(np.float64))[0])
    d_gpu = p.astype(np.float64) - p32
    d_ref = flatten(ref).astype(np.float64) - p32
    cos = d_gpu @ d_ref / (np.linalg.norm(d_gpu) * np.linalg.norm(d_ref))
    assert cos >= 0.999, cos
    assert np.allclose(loss, ref_loss, rtol=1e-3)


def test_training_reduces_loss_like_oracle():
    print("mlp training", flush=True)
    p32, X, _ = problem(2)
    Xd = X.astype(np.float64)
    Y = np.stack([np.sin(Xd[:, 0]) * Xd[:, 1], np.cos(Xd[:, 2]), Xd[:, 3] ** 2 - 1] + [0.5 * Xd[:, i] for i in range(7)],
                 axis=1).astype(np.float32)
    loss, _, _ = sfmm.sfmm_mlp_train(SIZES, p32.copy(), X, Y, steps=300, lr=3e-3)
    ref = unflatten(p32, SIZES)
    state = {}
    for _ in range(300):
        _, g = mlp.loss_and_grads(ref, Xd, Y.astype(np.float64))
        mlp.adam(ref, g, state, lr=3e-3)
    ref_final = mlp.loss_and_grads(ref, Xd, Y.astype(np.float64))[0]
    assert loss[-1] < 0.1 * loss[0]
    assert loss[-1] < 3.0 * ref_final + 1e-3


def ellipsoid():
    v, t = icosphere(3, 1.0)
    v = v * np.array([0.5, 0.35, 0.25])
    reg = np.tile(np.array([[0, 1]], dtype=np.int32), (len(t), 1))
    return Body(v, t, reg, np.array([1.0, 4.0], dtype=complex), np.ones(2, dtype=complex),
                name="ellipsoid 0.5 x 0.35 x 0.25 wavelengths, eps 4")


@pytest.fixture(scope="module")
def ectx():
    print("setup ellipsoid fp32", flush=True)
    with sfmm.Context([ellipsoid()], precision=sfmm.PREC_FP32, finest_box=0.25, tol=1e-4, gmres_restart=50,
                      max_iters=600) as c:
        yield c


def test_fit_and_predict_match_oracle_on_the_linear_path(ectx):
    print("learned guess pipeline parity (linear path)", flush=True)
    body = ellipsoid()
    m = rwg.from_body(body)
    n = ectx.sfmm_num_unknowns()
    tr = theta_sweep(7, phi=0.2)                               # 30 degree steps
    te = tr[:-1] + np.array([np.deg2rad(15.0), 0.0])           # the midpoints
    # seeded training currents with a smooth angle dependence (any data serve
    # the pipeline; both sides build their own right-hand sides)
    V = random_complex_vector(n, 4, seed=11)
    th = tr[:, 0][:, None]
    X = np.cos(th) * V[0] + np.sin(th) * V[1] + np.cos(2 * th) * V[2] + np.sin(2 * th) * V[3]
    ectx.sfmm_guess_fit(tr, X, epochs=0, n_theta=6, n_phi=11)
    x0 = ectx.sfmm_guess_predict(te, np.zeros((len(te), n), dtype=complex))
    B_tr = ectx.sfmm_planewave_rhs(tr, np.zeros((len(tr), n), dtype=complex))
    B_te = ectx.sfmm_planewave_rhs(te, np.zeros((len(te), n), dtype=complex))
    model = mlp.fit_guess(m, body.frequency, tr, _oracle_rhs(m, body, tr), X, hidden=4, epochs=0,
                          n_theta=6, n_phi=11)
    ref = mlp.predict_guess(model, te, _oracle_rhs(m, body, te))
    err = rel(x0, ref)
    print(f"pipeline parity {err:.2e} (rank {model['U'].shape[1]})", flush=True)
    assert err < 1e-6
    # the library's right-hand sides are the oracle's (the features read them)
    assert rel(B_te, _oracle_rhs(m, body, te)) < 1e-10 and rel(B_tr, _oracle_rhs(m, body, tr)) < 1e-10


def _oracle_rhs(m, body, ang):
    from oracle import mom
    return np.array([mom.planewave_rhs(m, body.frequency, *mom.incidence(t, p)) for t, p in ang])


def test_guess_options_are_checked(ectx):
    n = ectx.sfmm_num_unknowns()
    x = np.zeros((2, n), dtype=complex)
    x[:, 0] = 1.0
    with pytest.raises(sfmm.SfmmError):
        ectx.sfmm_guess_fit(theta_sweep(2), x, n_theta=64, n_phi=65)
    with pytest.raises(sfmm.SfmmError):
        ectx.sfmm_guess_fit(theta_sweep(2), x, hidden=0)


def test_learned_guess_cuts_iterations(ectx):
    print("learned guess sweep", flush=True)
    n = ectx.sfmm_num_unknowns()
    ang = theta_sweep(91)
    tr = np.arange(0, 91, 3)                                   # both ends included
    te = np.setdiff1d(np.arange(91), tr)
    b = ectx.sfmm_planewave_rhs(ang, np.zeros((91, n), dtype=complex))
    x_tr = np.zeros((len(tr), n), dtype=complex)
    info_tr = ectx.sfmm_solve(b[tr].copy(), x_tr)
    assert all(i["converged"] for i in info_tr)
    loss = ectx.sfmm_guess_fit(ang[tr], x_tr)
    r = len(tr)
    # the MLP starts at zero on unit-RMS targets (loss r); Adam lowers it
    assert np.isfinite(loss) and loss < 0.9 * r, loss
    x0 = ectx.sfmm_guess_predict(ang[te], np.zeros((len(te), n), dtype=complex))
    # x0 = U c lies in the span of the training solutions
    coef = np.linalg.lstsq(x_tr.T, x0.T, rcond=None)[0]
    assert rel(x_tr.T @ coef, x0.T) < 1e-6
    # at the training angles the guess reproduces the training solutions
    x0_tr = ectx.sfmm_guess_predict(ang[tr], np.zeros((len(tr), n), dtype=complex))
    assert rel(x0_tr, x_tr) < 1e-3, rel(x0_tr, x_tr)
    x_zero = np.zeros((len(te), n), dtype=complex)
    x_lrn = np.zeros((len(te), n), dtype=complex)
    info0 = ectx.sfmm_solve(b[te].copy(), x_zero)
    info1 = ectx.sfmm_solve(b[te].copy(), x_lrn, x0=x0)
    its0 = np.array([i["iterations"] for i in info0])
    its1 = np.array([i["iterations"] for i in info1])
    r0 = np.array([i["initial_residual"] for i in info1])
    print(f"zero-guess iterations {its0.mean():.1f}, learned {its1.mean():.1f} (max {its1.max()}), "
          f"guess residual median {np.median(r0):.3e} max {r0.max():.3e}, loss {loss:.3e}", flush=True)
    for i0, i1 in zip(info0, info1):
        assert i0["converged"] and i1["converged"]
        assert i0["true_residual"] <= 1e-4 and i1["true_residual"] <= 1e-4
    assert np.mean([i["guess_used"] for i in info1]) >= 0.9
    assert np.median(r0) < 1e-3
    assert its1.mean() < 0.5 * its0.mean()
    # both solutions agree to the solver tolerance
    assert rel(x_lrn, x_zero) < 1e-2
    # the network-free baseline: minimal residual in the same POD span; it
    # also lies in the span, and its residual is about the network's
    xs = ectx.sfmm_span_predict(ang[te], np.zeros((len(te), n), dtype=complex))
    coef = np.linalg.lstsq(x_tr.T, xs.T, rcond=None)[0]
    assert rel(x_tr.T @ coef, xs.T) < 1e-6
    info2 = ectx.sfmm_solve(b[te].copy(), np.zeros((len(te), n), dtype=complex), x0=xs)
    r2 = np.array([i["initial_residual"] for i in info2])
    print(f"span baseline: guess residual median {np.median(r2):.3e}, iterations "
          f"{np.mean([i['iterations'] for i in info2]):.1f}")
    assert np.median(r2) <= 2.0 * np.median(r0) + 1e-4


def test_judge_drops_a_bad_guess(ectx):
    print("judge of the initial guess", flush=True)
    n = ectx.sfmm_num_unknowns()
    ang = theta_sweep(3)
    b = ectx.sfmm_planewave_rhs(ang, np.zeros((3, n), dtype=complex))
    x_ref = np.zeros_like(b)
    info_ref = ectx.sfmm_solve(b.copy(), x_ref)
    bad = 1e3 * random_complex_vector(n, 3, seed=7)
    x = np.zeros_like(b)
    info = ectx.sfmm_solve(b.copy(), x, x0=bad)
    for i, r in zip(info, info_ref):
        assert not i["guess_used"] and i["initial_residual"] > 1.0
        assert i["converged"] and i["iterations"] == r["iterations"]
    # a converged solution as the guess needs no iteration
    x2 = np.zeros_like(b)
    info2 = ectx.sfmm_solve(b.copy(), x2, x0=x_ref)
    for i in info2:
        assert i["guess_used"] and i["converged"] and i["iterations"] == 0
