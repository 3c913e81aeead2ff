"""Plain FP64 CPU oracle for the MLFMM-accelerated PMCHWT/RWG hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything in this
package.  The HIP library never uses it, and it shares no code with the HIP
library: it builds its own basis functions, integrals, matrices, octree,
preconditioner and Krylov solver from the raw mesh arrays produced by the
``workloads`` package.

What it computes (the plain definitions; every module cites the passage of
H. T. Chorsi, "Surface Integral Formulation with Preconditioned,
Multipole-Accelerated Iterative Method ..." (arXiv:1704.06862) that it
follows):

* ``quadrature`` - 7-point degree-5 triangle rule used for every surface integral.
* ``rwg``        - RWG basis functions on triangle pairs (eq. 22).
* ``potentials`` - closed-form integrals of R^-1, R and their gradients over a
                   flat triangle, used to take the singular part of the Green's
                   function (eq. 7) out of near-singular integrals.
* ``mom``        - Galerkin matrix of the two operators of eqs. 5-6 and the
                   PMCHWT combination of T-EFIE/T-MFIE (eqs. 10-13, 16),
                   plane-wave right-hand sides (eqs. 20-21, 30), dense or
                   row-sampled.
* ``octree``     - finest-level boxes, near pairs and the 8-colour ordering
                   that define the near-field matrix and the ILU(0) pattern.
* ``krylov``     - ILU(0) and right-preconditioned restarted GMRES.
* ``farfield``   - far-field pattern and RCS (eqs. 27-29).
* ``mie``        - Mie series for homogeneous and coated spheres (validation).

All floating-point work is complex128/float64.
"""
