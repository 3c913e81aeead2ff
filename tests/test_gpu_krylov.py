"""The paper's solver comparison (Simulation Results, Fig. 7 discussion) on
the GPU, through the C ABI: ILU-preconditioned BiCGStab and CGS and
unpreconditioned BiCGStab, against the oracle's BiCGStab / CGS on the dense
FP64 matrix of the 960-unknown validation sphere.  The GPU iterates on the
MLFMM-approximated operator (2.4e-4 from the dense matrix on converged currents), so iteration counts
agree within a few; solutions agree with the oracle's direct solution in RCS."""

import numpy as np
import pytest

from oracle import farfield, krylov, mom, octree, rwg
from workloads import sphere_body, theta_sweep

pytestmark = pytest.mark.gpu

sfmm = pytest.importorskip("paper_1704_06862_amd.sfmm")

THETA = np.deg2rad(np.arange(181.0))
OPTS = dict(precision=2, finest_box=0.2, n_levels=3, extra_multipoles=2, tol=1e-6, max_iters=400)


def _masked_db(s, ref):
    floor = 1e-3 * ref.max()
    return np.abs(10 * np.log10((s + floor) / (ref + floor)))


@pytest.fixture(scope="module")
def sphere():
    b = sphere_body(0.3, 4.0, 2)
    m = rwg.from_body(b)
    Z = mom.pmchwt_dense(m, b.eps_r, b.mu_r, b.frequency)
    keys = octree.finest_keys(m, 0.2, 3)
    pat = octree.near_pattern(keys)
    p = octree.unknown_order(keys)
    F = krylov.ilu0(Z[np.ix_(p, p)], pat[np.ix_(p, p)])

    def ilu(v):
        out = np.empty_like(v)
        out[p] = krylov.ilu_apply(F, v[p])
        return out

    return dict(body=b, mesh=m, Z=Z, ilu=ilu)


@pytest.mark.parametrize("method,precond", [("bicgstab", "ilu0"), ("cgs", "ilu0"), ("bicgstab", "none")])
def test_bicg_family_matches_oracle(sphere, method, precond):
    b, m, Z = sphere["body"], sphere["mesh"], sphere["Z"]
    solver = {"bicgstab": sfmm.SOLVER_BICGSTAB, "cgs": sfmm.SOLVER_CGS}[method]
    pc = sfmm.PRECOND_ILU0 if precond == "ilu0" else sfmm.PRECOND_NONE
    ang = theta_sweep(3, theta_max_deg=120.0)
    rhs = np.stack([mom.planewave_rhs(m, b.frequency, *mom.incidence(t, ph)) for t, ph in ang])
    oracle_its = []
    for r in range(3):
        _, oi = getattr(krylov, method)(lambda v: Z @ v, rhs[r], sphere["ilu"] if precond == "ilu0" else None,
                                        tol=1e-6, max_iters=400)
        assert oi.converged
        oracle_its.append(oi.iterations)
    print(f"setup {method}/{precond}", flush=True)
    with sfmm.Context([b], preconditioner=pc, solver=solver, **OPTS) as ctx:
        xb = np.zeros_like(rhs)
        infos = ctx.sfmm_solve(rhs, xb)
        x1 = np.zeros_like(rhs[:1])
        i1 = ctx.sfmm_solve(np.ascontiguousarray(rhs[1:2]), x1)[0]
        sE = ctx.sfmm_rcs(xb, np.stack([THETA, 0 * THETA], 1))[:, :, 0]
    gpu_its = [i["iterations"] for i in infos]
    print(method, precond, "GPU iterations", gpu_its, "oracle", oracle_its, [i["restarts"] for i in infos])
    # preconditioned: within a few iterations of the oracle.  Without a
    # preconditioner BiCGStab's residual history is erratic, and the 2.4e-4
    # difference between the MLFMM operator and the dense matrix moves its
    # iteration count by up to a third (the paper's point: preconditioning
    # makes it both faster and steadier)
    slack = 0.2 if precond == "ilu0" else 0.5
    for r in range(3):
        assert infos[r]["converged"] and infos[r]["true_residual"] <= 1e-6
        assert abs(gpu_its[r] - oracle_its[r]) <= max(3, slack * oracle_its[r])
        if precond == "none":
            assert gpu_its[r] > 3 * 35      # ILU(0)-BiCGStab needs at most 35 here
        xd = np.linalg.solve(Z, rhs[r])
        rE, _ = farfield.rcs(m, b.frequency, xd, THETA, 0 * THETA)
        assert _masked_db(sE[r], rE).max() < 0.2
    # a batch iterates each right-hand side as it would alone (the batched
    # and single-RHS kernels round differently; unpreconditioned BiCGStab
    # amplifies that into a few per cent of its iteration count)
    assert i1["converged"]
    if precond == "ilu0":
        assert abs(i1["iterations"] - infos[1]["iterations"]) <= 1
        assert np.linalg.norm(x1[0] - xb[1]) <= 1e-5 * np.linalg.norm(xb[1])
    else:
        assert abs(i1["iterations"] - infos[1]["iterations"]) <= 0.15 * infos[1]["iterations"]
        assert np.linalg.norm(x1[0] - xb[1]) <= 1e-4 * np.linalg.norm(xb[1])
