"""Oracle reference for body 20 of the seeded 48-ellipsoid batch
(workloads.ellipsoid_batch(48): semi-axes 0.785 x 0.538 x 0.409 wavelengths,
eps_r = 8.21, icosphere s = 4, 15,360 unknowns): dense FP64 matrix of the
scaled JMCFIE system (eqs. 8-9 and 14-15, every row by the oracle's row
fill), one LU factorisation, direct solves for the batch's 8 incidences
theta_i = 180 deg * i / 7 at phi = 0 (theta-polarised), and the bistatic
theta-theta RCS cut at phi = 0 in 1-degree steps (eq. 29) of each.

Calls only oracle/ (and the mesh generator of workloads/); writes
tests/golden/ellipsoid20_rcs.txt: column 0 theta in degrees, column 1 + i
the cut of incidence i (m^2).  Run from the repository root:

    python tests/golden/make_ellipsoid_rcs.py [processes]

About 15 minutes on 8 cores and 8 GB of memory.
"""

import os
import sys
import time
from multiprocessing import Pool

import numpy as np
import scipy.linalg

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

from oracle import farfield, mom, rwg  # noqa: E402
from workloads import ellipsoid_batch  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "ellipsoid20_rcs.txt")
BODY, N_ANGLES = 20, 8


def body():
    return ellipsoid_batch(48)[BODY]


_MESH = None


def _rows(span):
    global _MESH
    b = body()
    if _MESH is None:
        _MESH = rwg.from_body(b)
    lo, hi = span
    return lo, mom.combined_rows(_MESH, b.eps_r, b.mu_r, b.frequency, np.arange(lo, hi), True)


def main(procs):
    b = body()
    mesh = rwg.from_body(b)
    ne = mesh.n_edges
    Z = np.empty((2 * ne, 2 * ne), dtype=complex)
    spans = [(lo, min(ne, lo + 32)) for lo in range(0, ne, 32)]
    t0 = time.time()
    with Pool(procs) as pool:
        for k, (lo, (ZJ, ZM)) in enumerate(pool.imap_unordered(_rows, spans)):
            Z[lo:lo + len(ZJ)] = ZJ
            Z[ne + lo:ne + lo + len(ZM)] = ZM
            if k % 20 == 0:
                print(f"{k + 1} of {len(spans)} row blocks, {time.time() - t0:.0f} s", flush=True)
    th_in = np.deg2rad(180.0 * np.arange(N_ANGLES) / (N_ANGLES - 1))
    B = np.stack([mom.combined_rhs(mesh, b.frequency, *mom.incidence(t, 0.0), tangential=True) for t in th_in], 1)
    lu = scipy.linalg.lu_factor(Z, overwrite_a=False, check_finite=False)
    X = scipy.linalg.lu_solve(lu, B)
    res = np.linalg.norm(Z @ X - B, axis=0) / np.linalg.norm(B, axis=0)
    print(f"solves done, relative residuals {res.max():.2e} at most", flush=True)
    theta = np.deg2rad(np.arange(181.0))
    cols = [np.arange(181.0)]
    for i in range(N_ANGLES):
        sE, _ = farfield.rcs(mesh, b.frequency, X[:, i], theta, 0 * theta)
        cols.append(sE)
    header = (f"oracle dense FP64 JMCFIE solutions, {b.name} ({2 * ne} unknowns), plane waves from theta_i = "
              f"180 deg * i / {N_ANGLES - 1} at phi = 0, theta-polarised; written by "
              "tests/golden/make_ellipsoid_rcs.py\ntheta_deg sigma_theta_theta(phi=0)_m2 per incidence")
    np.savetxt(OUT, np.stack(cols, 1), fmt="%.10e", header=header)
    print("wrote", OUT)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count())
