"""Oracle reference for a two-layer coated sphere in the tree of the
307,200-unknown workload: the same radii and media (lossy core r = 1.5
wavelengths, eps_r = 6 - 0.5j; shell r = 2.5, eps_r = 2.56) on coarser
icospheres (core s = 3, shell s = 4; 19,200 unknowns).  Dense FP64 PMCHWT
matrix (eq. 16, every row by the oracle's row fill), one LU factorisation,
direct solves for the 64 incidences theta_i = 180 deg * i / 63 at phi = 0,
theta-polarised, and the bistatic theta-theta RCS cut at phi = 0 in 1-degree
steps (eq. 29) of each.

Calls only oracle/ (and the mesh generator of workloads/); writes
tests/golden/coated19200_rcs.txt: column 0 theta in degrees, column 1 + i the
cut of incidence i (m^2).  Run from the repository root:

    python tests/golden/make_coated_rcs.py [processes]

About 10 minutes on 8 cores and 12 GB of memory.
"""

import os
import sys
import time
from multiprocessing import Pool

import numpy as np
import scipy.linalg

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

from oracle import farfield, mom, rwg  # noqa: E402
from workloads import coated_sphere_body  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "coated19200_rcs.txt")
N_ANGLES = 64


def body():
    return coated_sphere_body(1.5, 6 - 0.5j, 3, 2.5, 2.56, 4)


_MESH = None


def _rows(span):
    global _MESH
    b = body()
    if _MESH is None:
        _MESH = rwg.from_body(b)
    lo, hi = span
    return lo, mom.pmchwt_rows(_MESH, b.eps_r, b.mu_r, b.frequency, np.arange(lo, hi))


def main(procs):
    b = body()
    mesh = rwg.from_body(b)
    ne = mesh.n_edges
    Z = np.empty((2 * ne, 2 * ne), dtype=complex)
    spans = [(lo, min(ne, lo + 32)) for lo in range(0, ne, 32)]
    t0 = time.time()
    with Pool(procs) as pool:
        for k, (lo, (ZE, ZH)) in enumerate(pool.imap_unordered(_rows, spans)):
            Z[lo:lo + len(ZE)] = ZE
            Z[ne + lo:ne + lo + len(ZH)] = ZH
            if k % 50 == 0:
                print(f"{k + 1} of {len(spans)} row blocks, {time.time() - t0:.0f} s", flush=True)
    theta_i = np.deg2rad(180.0 * np.arange(N_ANGLES) / (N_ANGLES - 1))
    B = np.stack([mom.planewave_rhs(mesh, b.frequency, *mom.incidence(t, 0.0)) for t in theta_i], 1)
    lu = scipy.linalg.lu_factor(Z, overwrite_a=False, check_finite=False)
    X = scipy.linalg.lu_solve(lu, B)
    res = np.linalg.norm(Z @ X - B, axis=0) / np.linalg.norm(B, axis=0)
    print(f"solved in {time.time() - t0:.0f} s, max relative residual {res.max():.2e}", flush=True)
    theta = np.deg2rad(np.arange(181.0))
    cuts = [farfield.rcs(mesh, b.frequency, X[:, i], theta, 0 * theta)[0] for i in range(N_ANGLES)]
    header = ("oracle dense FP64 PMCHWT LU solutions, coated sphere core r=1.5 eps=6-0.5j s=3, shell r=2.5 "
              f"eps=2.56 s=4 ({2 * ne} unknowns); incidence i = 0..63 from theta = 180*i/63 deg, phi = 0, "
              "theta-polarised; columns: theta_deg, then sigma_theta_theta(phi=0) in m^2 of each incidence; "
              "written by tests/golden/make_coated_rcs.py")
    np.savetxt(OUT, np.column_stack([np.arange(181.0)] + cuts), fmt="%.9e", header=header)
    print("wrote", OUT)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count())
