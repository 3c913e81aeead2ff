"""Oracle reference for the 15,360-unknown sphere (radius 2 wavelengths,
eps_r = 2.56, icosphere subdivision 4): dense FP64 PMCHWT matrix (every row by
the oracle's row fill), direct LU solve for the plane wave arriving from
theta = 0 (propagating along -z, x-polarised), and the bistatic RCS cuts
phi = 0 (theta-theta) and phi = 90 deg (phi-phi) at 1-degree steps (eq. 29).

Calls only oracle/ (and the mesh generator of workloads/); writes
tests/golden/sphere15360_rcs.txt.  Run from the repository root:

    python tests/golden/make_sphere_rcs.py [processes]

About 3 minutes on 8 cores and 5 GB of memory.
"""

import os
import sys
import time
from multiprocessing import Pool

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

from oracle import farfield, mom, rwg  # noqa: E402
from workloads import sphere_body  # noqa: E402

RADIUS, EPS_R, SUBDIV = 2.0, 2.56, 4
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sphere15360_rcs.txt")


def _mesh():
    body = sphere_body(RADIUS, EPS_R, SUBDIV)
    return body, rwg.from_body(body)


def _rows(span):
    body, mesh = _mesh()
    lo, hi = span
    return lo, mom.pmchwt_rows(mesh, body.eps_r, body.mu_r, body.frequency, np.arange(lo, hi))


def main(procs):
    body, mesh = _mesh()
    ne = mesh.n_edges
    Z = np.empty((2 * ne, 2 * ne), dtype=complex)
    spans = [(lo, min(ne, lo + 64)) for lo in range(0, ne, 64)]
    t0 = time.time()
    with Pool(procs) as pool:
        for lo, (ZE, ZH) in pool.imap_unordered(_rows, spans):
            Z[lo:lo + len(ZE)] = ZE
            Z[ne + lo:ne + lo + len(ZH)] = ZH
    print(f"fill {time.time() - t0:.0f} s", flush=True)
    k_hat, e_hat = mom.incidence(0.0, 0.0)
    b = mom.planewave_rhs(mesh, body.frequency, k_hat, e_hat)
    x = np.linalg.solve(Z, b)
    print(f"solve done, relative residual {np.linalg.norm(Z @ x - b) / np.linalg.norm(b):.2e}", flush=True)
    theta = np.deg2rad(np.arange(181.0))
    sE, _ = farfield.rcs(mesh, body.frequency, x, theta, 0 * theta)
    _, sH = farfield.rcs(mesh, body.frequency, x, theta, 0 * theta + np.pi / 2)
    header = ("oracle dense FP64 PMCHWT solution, sphere r = 2 lambda0, eps_r = 2.56, icosphere s = 4 "
              f"({2 * ne} unknowns), plane wave from theta = 0 (x-polarised); written by "
              "tests/golden/make_sphere_rcs.py\ntheta_deg sigma_theta_theta(phi=0)_m2 sigma_phi_phi(phi=90)_m2")
    np.savetxt(OUT, np.stack([np.arange(181.0), sE, sH], 1), fmt="%.10e", header=header)
    print("wrote", OUT)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count())
