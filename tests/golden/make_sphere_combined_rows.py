"""Oracle reference rows of the JMCFIE and CNF systems for the 61,440-unknown
sphere of the benchmark (r = 2 wavelengths, eps_r = 2.56, icosphere s = 5):
for 50 seeded edges, the J and M test rows of the scaled JMCFIE matrix and of
the CNF matrix (eqs. 8-9 and 14-15, by the oracle's row fill) applied to
the benchmark's single right-hand side
(workloads.random_complex_vector(61440, 1, seed=1234)) and to 64 seeded
vectors (workloads.random_complex_vector(61440, 64, seed=77)).

Calls only oracle/ (and the input generators of workloads/); writes
tests/golden/sphere61440_jmcfie_rows.txt and sphere61440_cnf_rows.txt: a
header line with the edge indices, then for every row (J rows of the edges
in order, then M rows) the 65 products (the single right-hand side first)
as (re, im) pairs.  Run from the repository root:

    python tests/golden/make_sphere_combined_rows.py [processes]

About three minutes on 8 cores.
"""

import os
import sys
import time
from multiprocessing import Pool

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

from oracle import mom, rwg  # noqa: E402
from workloads import random_complex_vector, sphere_body  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
N_EDGES = 50
FORMS = {"jmcfie": True, "cnf": False}   # tangential part present


def body():
    return sphere_body(2.0, 2.56, 5)


def test_edges(ne):
    return np.sort(np.random.default_rng(61441).choice(ne, N_EDGES, replace=False))


_MESH = None


def _rows(job):
    global _MESH
    e, tangential = job
    b = body()
    if _MESH is None:
        _MESH = rwg.from_body(b)
    ZJ, ZM = mom.combined_rows(_MESH, b.eps_r, b.mu_r, b.frequency, np.array([e]), tangential)
    return e, tangential, ZJ[0], ZM[0]


def main(procs):
    b = body()
    mesh = rwg.from_body(b)
    ne = mesh.n_edges
    edges = test_edges(ne)
    X = np.concatenate([random_complex_vector(2 * ne, 1, seed=1234), random_complex_vector(2 * ne, 64, seed=77)])
    where = {int(e): i for i, e in enumerate(edges)}
    Y = {f: np.zeros((2 * len(edges), X.shape[0]), dtype=complex) for f in FORMS}
    jobs = [(int(e), t) for t in FORMS.values() for e in edges]
    t0 = time.time()
    with Pool(procs) as pool:
        for k, (e, tangential, ZJ, ZM) in enumerate(pool.imap_unordered(_rows, jobs)):
            f = "jmcfie" if tangential else "cnf"
            Y[f][where[e]] = X @ ZJ
            Y[f][len(edges) + where[e]] = X @ ZM
            if k % 10 == 0:
                print(f"{k + 1} of {len(jobs)} rows, {time.time() - t0:.0f} s", flush=True)
    for f in FORMS:
        out = np.empty((Y[f].shape[0], 2 * X.shape[0]))
        out[:, 0::2] = Y[f].real
        out[:, 1::2] = Y[f].imag
        path = os.path.join(HERE, f"sphere61440_{f}_rows.txt")
        header = (f"oracle dense FP64 {f.upper()} rows (J rows then M rows of the edges below) times "
                  f"random_complex_vector({2 * ne}, 1, seed=1234) then random_complex_vector({2 * ne}, 64, seed=77), "
                  "sphere r=2 eps=2.56 s=5; (re, im) per right-hand side; written by "
                  "tests/golden/make_sphere_combined_rows.py\n"
                  "edges " + " ".join(str(int(e)) for e in edges))
        np.savetxt(path, out, fmt="%.8e", header=header)
        print("wrote", path)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count())
