"""GPU parity at the benchmark's full size and for the preconditioner on a
multilevel case, through the C ABI.

The 61,440-unknown sphere is far too large for a dense oracle matrix, so the
oracle computes a sample of full rows of Z (E and H rows of random edges) one
by one and the test compares those entries of the GPU product, in the launch
configuration that bench.py times (FP32, 0.25-wavelength boxes, 5 levels,
3-digit excess-bandwidth truncation)."""

import numpy as np
import pytest

from oracle import krylov, mom, octree, rwg
from workloads import random_complex_vector, sphere_body

pytestmark = pytest.mark.gpu

sfmm = pytest.importorskip("paper_1704_06862_amd.sfmm")

BENCH_OPTS = dict(finest_box=0.25, n_levels=5, digits=3.0, extra_multipoles=0, precision=0)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_bench_configuration_sampled_rows():
    body = sphere_body(2.0, 2.56, 5)
    mesh = rwg.from_body(body)
    ne = mesh.n_edges
    rng = np.random.default_rng(11)
    test = np.sort(rng.choice(ne, 16, replace=False))
    x = random_complex_vector(2 * ne, 1, seed=1234)
    print("oracle rows", flush=True)
    ZE, ZH = mom.pmchwt_rows(mesh, body.eps_r, body.mu_r, body.frequency, test)
    keys = octree.finest_keys(mesh, 0.25, 5)
    near = np.tile(octree.near_mask(keys)[test], (1, 2))
    ref = np.concatenate([ZE @ x[0], ZH @ x[0]])
    ref_near = np.concatenate([np.where(near, ZE, 0) @ x[0], np.where(near, ZH, 0) @ x[0]])
    print("setup bench configuration", flush=True)
    with sfmm.Context([body], **BENCH_OPTS) as ctx:
        assert ctx.sfmm_num_unknowns() == 61440
        yn = ctx.sfmm_matvec(x, np.zeros_like(x), parts=sfmm.PART_NEAR)[0]
        y = ctx.sfmm_matvec(x, np.zeros_like(x))[0]
    pick = np.concatenate([test, ne + test])
    e_near = rel(yn[pick], ref_near)
    e_full = rel(y[pick], ref)
    print("bench config sampled rows: near", e_near, "full", e_full,
          "far share", np.linalg.norm(ref - ref_near) / np.linalg.norm(ref))
    assert e_near < 1e-5
    assert e_full < 1e-3


def test_ilu_preconditioner_multilevel_fp64():
    body = sphere_body(1.0, 2.56, 3)
    mesh = rwg.from_body(body)
    keys = octree.finest_keys(mesh, 0.25, 4)
    near = octree.near_mask(keys)
    print("oracle near matrix", flush=True)
    Zn = mom.pmchwt_near(mesh, body.eps_r, body.mu_r, body.frequency, near)
    p = octree.unknown_order(keys)
    pat = np.tile(near, (2, 2))
    F = krylov.ilu0(Zn[np.ix_(p, p)], pat[np.ix_(p, p)])
    x = random_complex_vector(2 * mesh.n_edges, 1, seed=4)
    ref = np.empty_like(x[0])
    ref[p] = krylov.ilu_apply(F, x[0][p])
    with sfmm.Context([body], precision=2, finest_box=0.25, preconditioner=sfmm.PRECOND_ILU0) as ctx:
        z = ctx.sfmm_precond(x, np.zeros_like(x))[0]
    print("multilevel ILU rel err", rel(z, ref), "gain", np.linalg.norm(ref) / np.linalg.norm(x))
    assert rel(z, ref) < 1e-9


def test_polynomial_preconditioner_multilevel_fp64():
    body = sphere_body(1.0, 2.56, 3)
    mesh = rwg.from_body(body)
    keys = octree.finest_keys(mesh, 0.25, 4)
    near = octree.near_mask(keys)
    Zn = mom.pmchwt_near(mesh, body.eps_r, body.mu_r, body.frequency, near)
    th = krylov.leja_order(krylov.harmonic_ritz(lambda v: Zn @ v, krylov.golden_start(len(Zn)), 16))
    x = random_complex_vector(2 * mesh.n_edges, 1, seed=8)
    ref = krylov.poly_apply(lambda v: Zn @ v, th, x[0])
    with sfmm.Context([body], precision=2, finest_box=0.25, preconditioner=sfmm.PRECOND_POLY,
                      poly_degree=16) as ctx:
        z = ctx.sfmm_precond(x, np.zeros_like(x))[0]
    print("multilevel poly rel err", rel(z, ref))
    assert rel(z, ref) < 1e-9
