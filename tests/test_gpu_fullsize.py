"""GPU parity at the benchmark's full size and for the preconditioner on a
multilevel case, through the C ABI.

The 61,440-unknown sphere is far too large for a dense oracle matrix, so the
oracle computes a sample of full rows of Z (E and H rows of random edges) one
by one and the test compares those entries of the GPU product, in the launch
configuration that bench.py times (FP32, 0.25-wavelength boxes, 5 levels,
3-digit excess-bandwidth truncation)."""

import os

import numpy as np
import pytest

from oracle import krylov, mom, octree, rwg
from workloads import random_complex_vector, sphere_body

pytestmark = pytest.mark.gpu

sfmm = pytest.importorskip("paper_1704_06862_amd.sfmm")

BENCH_OPTS = dict(finest_box=0.25, n_levels=5, digits=3.0, extra_multipoles=0, precision=0)
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def bench_rows():
    body = sphere_body(2.0, 2.56, 5)
    mesh = rwg.from_body(body)
    ne = mesh.n_edges
    rng = np.random.default_rng(11)
    test = np.sort(rng.choice(ne, 16, replace=False))
    print("oracle rows", flush=True)
    ZE, ZH = mom.pmchwt_rows(mesh, body.eps_r, body.mu_r, body.frequency, test)
    keys = octree.finest_keys(mesh, 0.25, 5)
    near = np.tile(octree.near_mask(keys)[test], (1, 2))
    return dict(body=body, ne=ne, test=test, Z=np.concatenate([ZE, ZH]),
                Zn=np.concatenate([np.where(near, ZE, 0), np.where(near, ZH, 0)]))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_bench_configuration_sampled_rows(bench_rows, prec):
    # one right-hand side (vector kernels) and 64 (matrix-core near product)
    body, ne, test = bench_rows["body"], bench_rows["ne"], bench_rows["test"]
    x = random_complex_vector(2 * ne, 1, seed=1234)
    xb = random_complex_vector(2 * ne, 64, seed=77)
    opts = dict(BENCH_OPTS, precision=sfmm.PREC_FP32 if prec == "fp32" else sfmm.PREC_BF16_SPLIT)
    print("setup bench configuration", prec, flush=True)
    with sfmm.Context([body], **opts) as ctx:
        assert ctx.sfmm_num_unknowns() == 61440
        yn = ctx.sfmm_matvec(x, np.zeros_like(x), parts=sfmm.PART_NEAR)[0]
        y = ctx.sfmm_matvec(x, np.zeros_like(x))[0]
        ybn = ctx.sfmm_matvec(xb, np.zeros_like(xb), parts=sfmm.PART_NEAR)
        yb = ctx.sfmm_matvec(xb, np.zeros_like(xb))
        # the batched kernels against the single-RHS ones on the same inputs
        y1 = [ctx.sfmm_matvec(np.ascontiguousarray(xb[r:r + 1]), np.zeros_like(xb[:1]))[0] for r in (0, 37, 63)]
    pick = np.concatenate([test, ne + test])
    e_near = rel(yn[pick], bench_rows["Zn"] @ x[0])
    e_full = rel(y[pick], bench_rows["Z"] @ x[0])
    eb_near = max(rel(ybn[r][pick], bench_rows["Zn"] @ xb[r]) for r in range(64))
    eb_full = max(rel(yb[r][pick], bench_rows["Z"] @ xb[r]) for r in range(64))
    print(prec, "bench config sampled rows: near", e_near, "full", e_full, "| 64 RHS: near", eb_near,
          "full", eb_full)
    assert e_near < 1e-5
    assert e_full < 1e-3
    e_bs = max(rel(yb[r], y) for r, y in zip((0, 37, 63), y1))
    print(prec, "64-RHS batch vs single", e_bs)
    assert eb_near < (1e-5 if prec == "fp32" else 5e-5)
    assert eb_full < 1e-3
    assert e_bs < (1e-5 if prec == "fp32" else 5e-5)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_bench_configuration_stored_oracle_rows(prec):
    # 200 stored oracle rows (E and H rows of 100 seeded edges, written by
    # tests/golden/make_sphere_rows.py) applied to the benchmark's single
    # right-hand side and to a 64-RHS batch: the product in the launch
    # configuration bench.py times, within 1e-3 for every right-hand side
    path = os.path.join(GOLDEN, "sphere61440_rows.txt")
    with open(path) as f:
        f.readline()
        edges = np.array([int(v) for v in f.readline().split()[2:]])
    d = np.loadtxt(path)
    ref = d[:, 0::2] + 1j * d[:, 1::2]                  # [2 * n_edges, 65]
    body = sphere_body(2.0, 2.56, 5)
    opts = dict(BENCH_OPTS, precision=sfmm.PREC_FP32 if prec == "fp32" else sfmm.PREC_BF16_SPLIT)
    print("setup bench configuration", prec, flush=True)
    with sfmm.Context([body], **opts) as ctx:
        n = ctx.sfmm_num_unknowns()
        ne = n // 2
        assert n == 61440 and len(edges) == 100 and ref.shape == (200, 65)
        x = np.concatenate([random_complex_vector(n, 1, seed=1234), random_complex_vector(n, 64, seed=77)])
        y1 = ctx.sfmm_matvec(x[:1].copy(), np.zeros_like(x[:1]))
        yb = ctx.sfmm_matvec(x[1:].copy(), np.zeros_like(x[1:]))
    y = np.concatenate([y1, yb])
    pick = np.concatenate([edges, ne + edges])
    err = [rel(y[r][pick], ref[:, r]) for r in range(65)]
    print(prec, "stored oracle rows: single RHS", err[0], "| 64 RHS max", max(err[1:]), "median",
          np.median(err[1:]))
    assert max(err) < 1e-3


@pytest.mark.parametrize("form", ["jmcfie", "cnf"])
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_bench_sphere_combined_formulations_stored_oracle_rows(form, prec):
    # the JMCFIE and CNF products of the benchmark's sphere and tree: 100
    # stored oracle rows each (J and M test rows of 50 seeded edges, written
    # by tests/golden/make_sphere_combined_rows.py) applied to the single
    # right-hand side and to a 64-RHS batch, within 1e-3 for every one
    path = os.path.join(GOLDEN, f"sphere61440_{form}_rows.txt")
    with open(path) as f:
        f.readline()
        edges = np.array([int(v) for v in f.readline().split()[2:]])
    d = np.loadtxt(path)
    ref = d[:, 0::2] + 1j * d[:, 1::2]                  # [2 * n_edges, 65]
    body = sphere_body(2.0, 2.56, 5)
    opts = dict(BENCH_OPTS, precision=sfmm.PREC_FP32 if prec == "fp32" else sfmm.PREC_BF16_SPLIT,
                formulation=sfmm.FORM_JMCFIE if form == "jmcfie" else sfmm.FORM_CNF)
    print("setup bench configuration", form, prec, flush=True)
    with sfmm.Context([body], **opts) as ctx:
        n = ctx.sfmm_num_unknowns()
        ne = n // 2
        assert n == 61440 and len(edges) == 50 and ref.shape == (100, 65)
        x = np.concatenate([random_complex_vector(n, 1, seed=1234), random_complex_vector(n, 64, seed=77)])
        y1 = ctx.sfmm_matvec(x[:1].copy(), np.zeros_like(x[:1]))
        yb = ctx.sfmm_matvec(x[1:].copy(), np.zeros_like(x[1:]))
    y = np.concatenate([y1, yb])
    pick = np.concatenate([edges, ne + edges])
    err = [rel(y[r][pick], ref[:, r]) for r in range(65)]
    print(form, prec, "stored oracle rows: single RHS", err[0], "| 64 RHS max", max(err[1:]))
    assert max(err) < 1e-3


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
    M = krylov.near_poly_preconditioner(Zn, 16)
    x = random_complex_vector(2 * mesh.n_edges, 1, seed=8)
    ref = M(x[0])
    with sfmm.Context([body], precision=2, finest_box=0.25, preconditioner=sfmm.PRECOND_POLY,
                      poly_degree=16) as ctx:
        z = ctx.sfmm_precond(x, np.zeros_like(x))[0]
    print("multilevel poly rel err", rel(z, ref))
    assert rel(z, ref) < 1e-9


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_polynomial_preconditioner_batched(prec):
    # 64 right-hand sides: every near product of the polynomial runs on the
    # matrix cores (bfloat16 blocks, bf16-split vectors, FP32 accumulation)
    body = sphere_body(1.0, 2.56, 3)
    mesh = rwg.from_body(body)
    keys = octree.finest_keys(mesh, 0.25, 4)
    near = octree.near_mask(keys)
    Zn = mom.pmchwt_near(mesh, body.eps_r, body.mu_r, body.frequency, near)
    M = krylov.near_poly_preconditioner(Zn, 16)
    x = random_complex_vector(2 * mesh.n_edges, 64, seed=9)
    p = sfmm.PREC_FP32 if prec == "fp32" else sfmm.PREC_BF16_SPLIT
    with sfmm.Context([body], precision=p, finest_box=0.25, preconditioner=sfmm.PRECOND_POLY,
                      poly_degree=16) as ctx:
        z = ctx.sfmm_precond(x, np.zeros_like(x))
    err = max(rel(z[r], M(x[r])) for r in range(0, 64, 9))
    print(prec, "batched poly rel err", err)
    # FP32 and bf16-split contexts apply the polynomial with bfloat16
    # copies of the blocks: the reference is the oracle's polynomial
    # applied with the rounded blocks
    def bf16(a):
        def r(v):
            u = v.astype(np.float32).view(np.uint32).astype(np.uint64)
            u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
            return u.view(np.float32).astype(np.float64)
        return r(a.real) + 1j * r(a.imag)
    Dinv = krylov.edge_blocks_inverse(Zn)
    th = krylov.leja_order(krylov.harmonic_ritz(lambda u: krylov.edge_blocks_apply(Dinv, Zn @ u),
                                                krylov.golden_start(Zn.shape[0]), 16))
    Zh = bf16(Zn)
    Mh = lambda v: krylov.poly_apply(lambda u: krylov.edge_blocks_apply(Dinv, Zh @ u), th,  # noqa: E731
                                     krylov.edge_blocks_apply(Dinv, v))
    err_h = max(rel(z[r], Mh(x[r])) for r in range(0, 64, 9))
    print("vs the polynomial with rounded blocks", err_h)
    assert err_h < 1e-4 and err < 2e-2
