"""Oracle reference rows for the 307,200-unknown two-layer coated sphere
(lossy core r = 1.5 wavelengths, eps_r = 6 - 0.5j, icosphere s = 5; shell
r = 2.5, eps_r = 2.56, s = 6): for 60 seeded edges of the outer interface and
40 of the inner one, the E and H rows of the dense FP64 PMCHWT matrix (eq. 16,
by the oracle's row fill) applied to 64 seeded complex Gaussian vectors
(workloads.random_complex_vector(307200, 64, seed=3307)).

Calls only oracle/ (and the input generators of workloads/); writes
tests/golden/coated307200_rows.txt: a header line with the edge indices, then
for every row (E rows of the edges in order, then H rows) the 64 products as
(re, im) pairs.  Run from the repository root:

    python tests/golden/make_coated_rows.py [processes]

About 10 minutes on 8 cores and 16 GB of memory.
"""

import os
import sys
import time
from multiprocessing import Pool

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))

from oracle import mom, rwg  # noqa: E402
from workloads import coated_sphere_body, random_complex_vector  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "coated307200_rows.txt")
SEED_X, N_RHS = 3307, 64


def body():
    return coated_sphere_body(1.5, 6 - 0.5j, 5, 2.5, 2.56, 6)


def test_edges(mesh):
    rng = np.random.default_rng(307)
    outer = np.nonzero(mesh.regions[:, 1] == 1)[0]
    inner = np.nonzero(mesh.regions[:, 1] == 2)[0]
    return np.sort(np.concatenate([rng.choice(outer, 60, replace=False), rng.choice(inner, 40, replace=False)]))


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
    edges = test_edges(mesh)
    X = random_complex_vector(2 * ne, N_RHS, seed=SEED_X)
    yE = np.zeros((len(edges), N_RHS), dtype=complex)
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
    out = np.empty((Y.shape[0], 2 * N_RHS))
    out[:, 0::2] = Y.real
    out[:, 1::2] = Y.imag
    header = ("oracle dense FP64 PMCHWT rows (E rows then H rows of the edges below) times "
              f"random_complex_vector({2 * ne}, {N_RHS}, seed={SEED_X}), coated sphere core r=1.5 eps=6-0.5j s=5, "
              "shell r=2.5 eps=2.56 s=6; (re, im) per right-hand side; written by tests/golden/make_coated_rows.py\n"
              "edges " + " ".join(str(int(e)) for e in edges))
    np.savetxt(OUT, out, fmt="%.8e", header=header)
    print("wrote", OUT)


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else os.cpu_count())
