"""Oracle parity for the paper's multi-layer example at full size: the
two-layer coated sphere of 307,200 unknowns (lossy core r = 1.5 wavelengths,
eps_r = 6 - 0.5j, icosphere s = 5; shell r = 2.5, eps_r = 2.56, s = 6) in its
benchmark form (0.25-wavelength boxes, 3 digits, bf16-split, 64 right-hand
sides in one batch).

* Products: 200 rows of the dense FP64 PMCHWT matrix (E and H rows of 60
  outer- and 40 inner-interface edges, computed by the oracle alone and stored
  with their products with 64 seeded vectors by
  tests/golden/make_coated_rows.py) against the same rows of the batched GPU
  product, for every right-hand side.
* Solves and RCS: the same tree on coarser icospheres (core s = 3, shell
  s = 4; 19,200 unknowns) against the oracle's dense LU solutions of the 64
  incidences of the sweep (tests/golden/make_coated_rcs.py), the 64 angles
  solved as one bf16-split batch to 1e-4; the bound follows the tree's
  accuracy on these coarse facets (see the test).
* Full-size RCS against the Aden-Kerker series (discretisation-limited)."""

import os

import numpy as np
import pytest

from oracle import mie
from workloads import coated_sphere_body, random_complex_vector

pytestmark = pytest.mark.gpu

sfmm = pytest.importorskip("paper_1704_06862_amd.sfmm")

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
THETA = np.deg2rad(np.arange(181.0))
TREE = dict(finest_box=0.25, digits=3.0, precision=1, gmres_restart=50, tol=1e-4, max_iters=1000,
            poly_degree=48)


def _masked_db(s, ref):
    floor = 1e-3 * ref.max()
    return np.abs(10 * np.log10((s + floor) / (ref + floor)))


def test_coated_307200_sampled_oracle_rows_64_rhs():
    path = os.path.join(GOLDEN, "coated307200_rows.txt")
    with open(path) as f:
        f.readline()
        edges = np.array([int(v) for v in f.readline().split()[2:]])
    d = np.loadtxt(path)
    ref = d[:, 0::2] + 1j * d[:, 1::2]                  # [2 * n_edges, 64]
    body = coated_sphere_body(1.5, 6 - 0.5j, 5, 2.5, 2.56, 6)
    print("setup 307,200-unknown coated sphere, bf16-split", flush=True)
    with sfmm.Context([body], **TREE) as ctx:
        n = ctx.sfmm_num_unknowns()
        ne = n // 2
        assert n == 307200 and len(edges) == 100 and ref.shape == (200, 64)
        x = random_complex_vector(n, 64, seed=3307)
        y = ctx.sfmm_matvec(x, np.zeros_like(x))
    pick = np.concatenate([edges, ne + edges])
    err = [np.linalg.norm(y[r][pick] - ref[:, r]) / np.linalg.norm(ref[:, r]) for r in range(64)]
    print("coated 307,200 sampled-row rel err: max", max(err), "median", np.median(err))
    assert max(err) < 1e-3


def test_coated_19200_sweep_rcs_vs_stored_oracle():
    gold = np.loadtxt(os.path.join(GOLDEN, "coated19200_rcs.txt"))
    assert gold.shape == (181, 65)
    body = coated_sphere_body(1.5, 6 - 0.5j, 3, 2.5, 2.56, 4)
    ang = np.stack([np.deg2rad(180.0 * np.arange(64) / 63), np.zeros(64)], 1)
    print("setup 19,200-unknown coated sphere, bf16-split", flush=True)
    with sfmm.Context([body], **TREE) as ctx:
        n = ctx.sfmm_num_unknowns()
        assert n == 19200
        b = ctx.sfmm_planewave_rhs(ang, np.zeros((64, n), dtype=complex))
        x = np.zeros_like(b)
        info = ctx.sfmm_solve(b, x)
        s = ctx.sfmm_rcs(x, np.stack([THETA, 0 * THETA], 1))[:, :, 0]
    assert all(i["converged"] and i["true_residual"] <= 1e-4 for i in info)
    per = [_masked_db(s[i], gold[:, 1 + i]).max() for i in range(64)]
    worst, med = max(per), float(np.median(per))
    print("coated 19,200: 64 angles, iterations", max(i["iterations"] for i in info), "worst masked dB", worst,
          "median", med)
    # This stand-in's facets are four times coarser than the full-size
    # body's, so the far field carries 0.47 of the product's norm (about 0.1
    # at full size) and the 3-digit tree leaves 1.5e-3 to 2.2e-3 on sampled
    # oracle rows, in FP64 as in bf16-split; pairs of triangles closer than
    # the singular-extraction radius also fall in non-neighbouring boxes
    # here (8e-4 from the oracle rows even with 6 digits in FP64).  Measured:
    # worst 0.65 dB, median 0.25 dB over the 64 angles.  The full-size body
    # meets 1e-3 on sampled rows (test above) and its RCS the series.
    assert worst < 0.75 and med < 0.3


def test_coated_307200_rcs_vs_mie():
    body = coated_sphere_body(1.5, 6 - 0.5j, 5, 2.5, 2.56, 6)
    print("setup 307,200-unknown coated sphere, FP32", flush=True)
    with sfmm.Context([body], **dict(TREE, precision=0)) as ctx:
        n = ctx.sfmm_num_unknowns()
        b = ctx.sfmm_planewave_rhs(np.zeros((1, 2)), np.zeros((1, n), dtype=complex))
        x = np.zeros_like(b)
        info = ctx.sfmm_solve(b, x)[0]
        sE = ctx.sfmm_rcs(x, np.stack([THETA, 0 * THETA], 1))[0, :, 0]
        sH = ctx.sfmm_rcs(x, np.stack([THETA, 0 * THETA + np.pi / 2], 1))[0, :, 1]
    mE, mH = mie.coated_sphere_rcs(1.5, 6 - 0.5j, 2.5, 2.56, THETA)
    dE, dH = _masked_db(sE, mE), _masked_db(sH, mH)
    rE, rH = np.sqrt(np.mean(dE ** 2)), np.sqrt(np.mean(dH ** 2))
    print(info, "vs Mie: E-plane RMS/max dB", rE, dE.max(), "H-plane", rH, dH.max())
    assert info["converged"] and info["true_residual"] <= 1e-4
    # measured 0.011 / 0.007 dB RMS (the s = 5 / 6 facets); a regression of
    # the product or the solve shows as tenths of a dB
    assert rE < 0.05 and rH < 0.05 and dE.max() < 0.1 and dH.max() < 0.1
