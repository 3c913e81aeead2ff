"""Oracle reference rows for the 61,440-unknown sphere of the benchmark
(r = 2 wavelengths, eps_r = 2.56, icosphere s = 5): for 100 seeded edges, the
E and H rows of the dense FP64 PMCHWT matrix (eq. 16, by the oracle's row
fill) applied to the benchmark's single right-hand side
(workloads.random_complex_vector(61440, 1, seed=1234)) and to 64 seeded
vectors (workloads.random_complex_vector(61440, 64, seed=77)).

Calls only oracle/ (and the input generators of workloads/); writes
tests/golden/sphere61440_rows.txt: a header line with the edge indices, then
for every row (E rows of the edges in order, then H rows) the 65 products
(the single right-hand side first) as (re, im) pairs.  Run from the
repository root:

    python tests/golden/make_sphere_rows.py [processes]

About two minutes on 8 cores.
"""

import os
import sys
import time
from multiprocessing import Pool

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

from oracle import mom, rwg  # noqa: E402
from workloads import random_complex_vector, sphere_body  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "sphere61440_rows.txt")
N_EDGES = 100


def body():
    return sphere_body(2.0, 2.56, 5)


def test_edges(ne):
    return np.sort(np.random.default_rng(61440).choice(ne, N_EDGES, replace=False))


_MESH = None


def _rows(e):
    global _MESH
    b = body()
    if _MESH is None:
        _MESH = rwg.from_body(b)
    ZE, ZH = mom.pmchwt_rows(_MESH, b.eps_r, b.mu_r, b.frequency, np.array([e]))
    return e, ZE[0], ZH[0]


def main(procs):
    b = body()
    mesh = rwg.from_body(b)
    ne = mesh.n_edges
    edges = test_edges(ne)
    X = np.concatenate([random_complex_vector(2 * ne, 1, seed=1234), random_complex_vector(2 * ne, 64, seed=77)])
    yE = np.zeros((len(edges), X.shape[0]), dtype=complex)
    yH = np.zeros_like(yE)
    where = {int(e): i for i, e in enumerate(edges)}
    t0 = time.time()
    with Pool(procs) as pool:
        for k, (e, ZE, ZH) in enumerate(pool.imap_unordered(_rows, [int(e) for e in edges])):
            yE[where[e]] = X @ ZE
            yH[where[e]] = X @ ZH
            if k % 10 == 0:
                print(f"{k + 1} of {len(edges)} edges, {time.time() - t0:.0f} s", flush=True)
    Y = np.concatenate([yE, yH])
    out = np.empty((Y.shape[0], 2 * X.shape[0]))
    out[:, 0::2] = Y.real
    out[:, 1::2] = Y.imag
    header = ("oracle dense FP64 PMCHWT rows (E rows then H rows of the edges below) times "
              f"random_complex_vector({2 * ne}, 1, seed=1234) then random_complex_vector({2 * ne}, 64, seed=77), "
              "sphere r=2 eps=2.56 s=5; (re, im) per right-hand side; written by tests/golden/make_sphere_rows.py\n"
              "edges " + " ".join(str(int(e)) for e in edges))
    np.savetxt(OUT, out, fmt="%.8e", header=header)
    print("wrote", OUT)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count())
