"""GPU parity on a body with junction edges (three regions meeting along a
line, eq. 16): a three-layer stacked dielectric cylinder with the layer
permittivities of the paper-shaped stacked workload (2.2, 4.4, 10.2), small
enough for the dense oracle.  Products against the dense FP64 PMCHWT matrix,
solves and RCS against the oracle's LU solution."""

import numpy as np
import pytest

from oracle import farfield, mom, rwg
from workloads import random_complex_vector, stacked_cylinder_body

pytestmark = pytest.mark.gpu

sfmm = pytest.importorskip("paper_1704_06862_amd.sfmm")

THETA = np.deg2rad(np.arange(181.0))


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _masked_db(s, ref):
    floor = 1e-3 * ref.max()
    return np.abs(10 * np.log10((s + floor) / (ref + floor)))


@pytest.fixture(scope="module")
def stack():
    b = stacked_cylinder_body(0.3, 0.9, (2.2, 4.4, 10.2), 0.1)
    m = rwg.from_body(b)
    print("oracle dense stacked cylinder", 2 * m.n_edges, flush=True)
    Z = mom.pmchwt_dense(m, b.eps_r, b.mu_r, b.frequency)
    return dict(body=b, mesh=m, Z=Z)


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_stacked_cylinder_product_solve_and_rcs(stack, prec):
    b, m, Z = stack["body"], stack["mesh"], stack["Z"]
    assert (m.side_tri[:, 2] >= 0).sum() == 2 * 19      # two junction rings
    p = {"fp64": sfmm.PREC_FP64, "fp32": sfmm.PREC_FP32, "bf16": sfmm.PREC_BF16_SPLIT}[prec]
    opts = dict(finest_box=0.15, extra_multipoles=5, tol=1e-6) if prec == "fp64" else \
        dict(finest_box=0.2, extra_multipoles=1, tol=1e-4)
    print("setup stacked cylinder", prec, flush=True)
    with sfmm.Context([b], precision=p, gmres_restart=50, max_iters=2000, **opts) as ctx:
        assert ctx.sfmm_num_unknowns() == 2 * m.n_edges
        assert np.array_equal(ctx.sfmm_edges(), m.edge_v)
        for R in (1, 16):
            x = random_complex_vector(2 * m.n_edges, R, seed=500 + R)
            y = ctx.sfmm_matvec(x, np.zeros_like(x))
            ref = x @ Z.T
            err = max(rel(y[r], ref[r]) for r in range(R))
            print(prec, R, "stacked cylinder product rel err", err, flush=True)
            assert err < 1e-3
        ang = np.array([[0.0, 0.0], [0.9, 0.0], [2.4, 0.0]])
        rhs = ctx.sfmm_planewave_rhs(ang, np.zeros((3, 2 * m.n_edges), dtype=complex))
        for i, (th, ph) in enumerate(ang):
            assert rel(rhs[i], mom.planewave_rhs(m, b.frequency, *mom.incidence(th, ph))) < 1e-12
        xs = np.zeros_like(rhs)
        info = ctx.sfmm_solve(rhs, xs)
        sE = ctx.sfmm_rcs(xs, np.stack([THETA, 0 * THETA], 1))[:, :, 0]
    xd = np.linalg.solve(Z, rhs.T).T
    for i in range(3):
        print(prec, "angle", i, info[i])
        assert info[i]["converged"]
        rE, _ = farfield.rcs(m, b.frequency, xd[i], THETA, 0 * THETA)
        d = _masked_db(sE[i], rE)
        print(prec, "angle", i, "RCS max dB diff vs oracle LU", d.max())
        assert d.max() < 0.2
