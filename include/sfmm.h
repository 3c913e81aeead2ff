/*
 * sfmm.h - C interface of the MI355X (gfx950) MLFMM solver for dielectric
 * scattering with the PMCHWT, JMCFIE or CNF surface integral equations
 * discretised by RWG functions in a Galerkin method of moments.
 *
 * Method: H. T. Chorsi, "Surface Integral Formulation with Preconditioned,
 * Multipole-Accelerated Iterative Method Applied for the Analysis of RCS of
 * Single and Multi-Layer Dielectric Structures", arXiv:1704.06862.
 *   - equivalent currents J, M on every interface and their fields:   eqs. 1-7
 *   - normal field equations N-EFIE / N-MFIE:                          eqs. 8-9
 *   - tangential field equations T-EFIE / T-MFIE and interface rules:  eqs. 10-13
 *   - the JMCFIE combination:                                          eqs. 14-15
 *   - several interfaces / layered bodies:                              eq. 16
 *   - RWG basis functions, Galerkin testing:                            eq. 22, "Discretization" section
 *   - far field and RCS:                                                eqs. 27-29
 *   - plane-wave excitation:                                            eq. 30
 *   - MLFMM-accelerated products inside an ILU-preconditioned Krylov
 *     solver:                                                           "Simulation Results" section
 *
 * Conventions (all entry points):
 *   - time dependence exp(+j omega t); Green's function exp(-jkR)/(4 pi R);
 *     a lossy medium has Im(eps_r) < 0.
 *   - complex numbers are interleaved (re, im) doubles at this interface.
 *   - unknown vectors are [n_rhs][2E] complex: E electric-current
 *     coefficients J_1..J_E (A/m) followed by E scaled magnetic-current
 *     coefficients M~_n = M_n / eta0 (A/m), in canonical edge order (see
 *     sfmm_edges).  Equation vectors (right-hand sides, products) use the same
 *     layout: the E rows hold <f_m, E>/eta0, the H rows <f_m, H>.
 *   - canonical edges: sorted by (smaller vertex id, larger vertex id); the
 *     basis function on edge (a, b), a < b, flows out of the triangle whose
 *     counter-clockwise vertex order runs a -> b, into the other triangle.
 *   - on_device = 0: vector pointers are host memory; the call copies them
 *     and is synchronous.  on_device = 1: pointers are device memory on the
 *     context's device, and the call is ordered on the context's stream
 *     (sfmm_set_stream); results are ready when that stream is synchronised.
 *   - inputs are borrowed for the duration of the call; outputs are
 *     allocated by the caller.  A context is not thread-safe.
 *   - every call returns an sfmm_status and never throws; on failure
 *     sfmm_last_error(ctx) describes the error (also for a NULL ctx).
 *   - the library owns no global GPU state except per-context allocations;
 *     SFMM_E_DEVICE leaves the context unusable (destroy it).
 */
#ifndef SFMM_H
#define SFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sfmm_ctx sfmm_ctx;

typedef enum {
    SFMM_OK = 0,
    SFMM_E_INVALID_ARG = 1,   /* bad pointer, index, size or option          */
    SFMM_E_MESH = 2,          /* open / non-manifold / mis-oriented mesh     */
    SFMM_E_OOM = 3,           /* host or device allocation failed            */
    SFMM_E_DEVICE = 4,        /* HIP error, or no usable gfx950 device       */
    SFMM_E_NOT_CONVERGED = 5, /* iteration cap hit; best iterate returned    */
    SFMM_E_BREAKDOWN = 6,     /* zero pivot in ILU(0) or Krylov breakdown    */
    SFMM_E_UNSUPPORTED = 7    /* valid request outside what is implemented   */
} sfmm_status;

/* One scatterer: a closed, consistently oriented triangulated surface made
 * of one or more interfaces between homogeneous regions (eq. 16). */
typedef struct {
    int32_t n_vertices;
    const double *vertices;      /* [n_vertices][3], metres                          */
    int32_t n_triangles;
    const int32_t *triangles;    /* [n_triangles][3], 0-based, CCW about the normal  */
    const int32_t *tri_regions;  /* [n_triangles][2]: region the normal points into,
                                    region behind it; region 0 = unbounded exterior  */
    int32_t n_regions;
    const double *eps_r;         /* [n_regions][2] complex relative permittivity     */
    const double *mu_r;          /* [n_regions][2] complex relative permeability     */
    double frequency_hz;
} sfmm_body;

/* Number type of the products.  FP32: complex FP32 storage and arithmetic
 * (matrix cores in FP32 for batches of 16+ right-hand sides).  BF16_SPLIT:
 * as FP32, but the batched near-field product runs on the bf16 matrix cores
 * with every FP32 operand split into hi + lo bf16 parts (hi*hi + hi*lo +
 * lo*hi, FP32 accumulation; about 1e-5 relative per product).  FP64: complex
 * FP64 everywhere (reference mode).  GMRES runs in FP64 in every mode.
 * Single precision limits the truncation order at small boxes: the diagonal
 * translation operator grows like the spherical Hankel function h_L(kX) when
 * kX is small, and its rounding is amplified accordingly.  At 0.15-wavelength
 * boxes (960-unknown sphere, eps_r = 4) one extra multipole keeps the FP32
 * product within 1.2e-3 of the dense matrix, while five give 0.12 (FP64:
 * 4e-4); at 0.25-wavelength boxes and above the excess-bandwidth order is safe
 * in FP32.  FP64 has no such limit at these sizes.  sfmm_setup refuses FP32
 * and BF16_SPLIT (SFMM_E_UNSUPPORTED) where an estimate of this amplification
 * at a level's closest translation offset times the FP32 rounding exceeds 5. */
enum { SFMM_PREC_FP32 = 0, SFMM_PREC_BF16_SPLIT = 1, SFMM_PREC_FP64 = 2 };

typedef struct {
    double finest_box;        /* finest octree box edge in metres; 0 = 0.25 lambda0      */
    int32_t n_levels;         /* octree levels counting the root; 0 = fewest that fit     */
    double digits;            /* excess-bandwidth accuracy digits d0; 0 = 3              */
    int32_t extra_multipoles; /* added to every level's truncation order                */
    int32_t precision;        /* SFMM_PREC_*: number type of the far/near products      */
    int32_t gmres_restart;    /* 0 = 30                                                  */
    int32_t max_iters;        /* 0 = 1000                                                */
    double tol;               /* relative residual target; 0 = 1e-6                      */
    int32_t device;           /* HIP device ordinal; -1 = build host tables only        */
    int32_t verbose;          /* 1: setup statistics to stderr; 2: also GMRES restarts  */
    int32_t preconditioner;   /* SFMM_PRECOND_*                                          */
    int32_t poly_degree;      /* degree of SFMM_PRECOND_POLY; 0 = 16                      */
    int32_t graphs;           /* 1 (default): products and preconditioner applications
                                 are captured once per batch size into HIP graphs and
                                 replayed; 0: launched kernel by kernel                 */
    int32_t autotune;         /* 1: on the first batch of each size, time the vector and
                                 the matrix-core / grouped variant of every stage that
                                 has both (for one RHS also the split interpolation
                                 stages and the shared launches of kernel_plan bits 7
                                 and 8) and keep the faster; 0 (default): fixed
                                 thresholds (matrix-core near product from 3 RHS,
                                 matrix-core aggregation, interpolation and receive
                                 from 6 RHS, grouped translation at 1 RHS and from
                                 16 RHS, the split stages and shared launches at
                                 1 RHS)                                                  */
    int32_t kernel_plan;      /* 0 (default): kernels chosen as `autotune` says; with
                                 bit 0 set, bits 1..5, 7 and 8 fix for every batch size:
                                 matrix-core near product, matrix-core aggregation and
                                 receive, matrix-core interpolation, grouped translation,
                                 split single-RHS interpolation stages; bit 7: single-RHS
                                 coarsest upward phi stage in one launch with the finer
                                 levels' translations; bit 8 (with bit 7): the near-field
                                 product in the level-2 translation launch; bit 9: single-RHS
                                 downward level transitions with the phi and theta stages
                                 fused in one kernel (the default at one RHS).  A variant whose
                                 conditions do not hold (batch size, LDS) falls back to
                                 the vector kernel.  For tests and measurement.         */
    int32_t formulation;      /* SFMM_FORM_*: integral equation; 0 = PMCHWT.  JMCFIE and
                                 CNF use the same kernels with a fourth near-field plane
                                 and a second receive table                               */
    int32_t quad_points;      /* points of the triangle rule for the outer and regular
                                 inner integrals; 0 = 7 (degree 5), the only rule built;
                                 other values: SFMM_E_UNSUPPORTED                         */
    int32_t solver;           /* SFMM_SOLVER_*: Krylov method of sfmm_solve; 0 = GMRES     */
    double ilu_pivot_tol;     /* ILU0 / BLOCK_JACOBI: a pivot whose modulus is at most this
                                 times the largest entry of its diagonal box block counts
                                 as zero (SFMM_E_BREAKDOWN at setup); 0 = 1e-13           */
    int32_t setup_on_device;  /* where the FP64 near-field matrix and the ILU(0)
                                 factorisation are computed: 1 on the device (the same
                                 arithmetic: one thread per stored edge pair for the
                                 fill, one workgroup per box row and one launch per
                                 colour for ILU(0); needs device >= 0,
                                 SFMM_E_INVALID_ARG otherwise), 0 on the host (OpenMP),
                                 -1 (default) on the device when there is one.  The
                                 block-Jacobi inverses and the polynomial's roots are
                                 always computed on the host                              */
} sfmm_options;

/* Integral equations (the paper's "Integral Equation Formulation" section).
 * All three act on the same unknowns [J ; M~ = M / eta0] (RWG coefficients,
 * boundary layout) and give the same currents up to discretisation error:
 *   PMCHWT  tangential EFIE and MFIE of both regions of every interface summed
 *           (eqs. 10-13; several interfaces as in eq. 16).
 *   JMCFIE  the paper's mixed formulation (eqs. 8-9, 14-16): J-rows
 *           sum_r T-EFIE(r) / eta_r + (-1)^r N-MFIE(r), M-rows
 *           sum_r eta_r T-MFIE(r) - (-1)^r N-EFIE(r), Galerkin-tested with the
 *           RWG functions; the N parts are the fields tested with n x f on
 *           each triangle, the half-jump terms become sparse Gram blocks.
 *           (-1)^r = +1 on the side the triangle normal points into, the
 *           numbering of the media for which the identity terms of the N
 *           and T parts reinforce; rows multiplied by -1 so the Gram
 *           identity enters the diagonal blocks positively, as in CNF.
 *           J-rows in A/m, M-rows divided by eta0 as for PMCHWT.
 *   CNF     the normal equations alone (eqs. 8-9, the N parts of JMCFIE): a
 *           second-kind system; its near-field matrix is dominated by the
 *           Gram blocks. */
enum { SFMM_FORM_PMCHWT = 0, SFMM_FORM_JMCFIE = 1, SFMM_FORM_CNF = 2 };

/* Krylov solvers of sfmm_solve (the paper's solver comparison, "Simulation
 * Results", Fig. 7: ILU-preconditioned BiCGStab and CGS, and BiCGStab
 * without preconditioner - SFMM_PRECOND_NONE), all right-preconditioned,
 * FP64 recurrences, right-hand sides in lockstep:
 *   GMRES     restarted flexible GMRES(m), see sfmm_solve; an iteration is
 *             one Arnoldi step (one preconditioned product);
 *   BICGSTAB  van der Vorst's BiCGStab (1992); an iteration is two
 *             preconditioned products;
 *   CGS       Sonneveld's conjugate gradient squared (1989); an iteration is
 *             two preconditioned products.
 * For all three, convergence is declared only on the explicitly recomputed
 * residual; a BiCGStab or CGS breakdown (a vanishing inner product) restarts
 * that right-hand side from its current iterate. */
enum { SFMM_SOLVER_GMRES = 0, SFMM_SOLVER_BICGSTAB = 1, SFMM_SOLVER_CGS = 2 };

/* Preconditioners of sfmm_solve, all built from the near-field matrix Z_near
 * (the paper preconditions with an incomplete LU of it):
 *   ILU0          ILU(0) in colour order (the paper's preconditioner);
 *   NONE          identity;
 *   BLOCK_JACOBI  inverses of the same-box diagonal blocks;
 *   POLY          p(D^-1 Z_near) D^-1 with D the edges' 2x2 self blocks
 *                 [[A_mm, -B_mm], [B_mm, C_mm]] and p the degree-d residual
 *                 polynomial of GMRES on D^-1 Z_near (roots: harmonic Ritz
 *                 values from d FP64 Arnoldi steps from v0[i] =
 *                 exp(2 pi j frac(i (sqrt5-1)/2)), Leja order, product form);
 *                 d near-field products per application (D^-1 fused into
 *                 their epilogue), no reductions.  In FP32 and bf16-split
 *                 contexts these products read the blocks of Z_near rounded
 *                 to bfloat16 (roots and D^-1 from the FP64 blocks): a fixed
 *                 operator within about 1e-2 of the FP64 polynomial, half the
 *                 bytes; the solve still converges on the product itself.
 *                 Default; several interfaces with high-contrast or lossy
 *                 media may need a higher degree (poly_degree). */
enum { SFMM_PRECOND_ILU0 = 0, SFMM_PRECOND_NONE = 1, SFMM_PRECOND_BLOCK_JACOBI = 2, SFMM_PRECOND_POLY = 3 };

typedef struct {
    int32_t converged;        /* 1 if ||b - Z x|| / ||b|| <= tol                        */
    int32_t iterations;       /* iterations of the Krylov method: GMRES Arnoldi steps (one
                                 preconditioned product each), BiCGStab / CGS
                                 iterations (two products each)                        */
    int32_t restarts;         /* GMRES restart cycles; BiCGStab / CGS: restarts after a
                                 breakdown or a failed true-residual check             */
    int32_t guess_used;       /* 1 if the supplied x0 was kept (see sfmm_solve)         */
    double true_residual;     /* ||b - Z x|| / ||b|| at exit, recomputed explicitly     */
    double initial_residual;  /* ||b - Z x0|| / ||b|| of the supplied x0 (1 if none)    */
    double seconds;           /* wall time of the solve                                 */
} sfmm_solve_info;

/* Fill *opt with the defaults listed above. */
void sfmm_default_options(sfmm_options *opt);

/* Problem set-up (the paper's problem statement: a body of homogeneous
 * regions with their eps_r, mu_r at one frequency, "Integral Equation
 * Formulation" section and eq. 16; RWG discretisation, eq. 22 and the
 * "Discretization" section).  Validates the meshes, builds the RWG tables,
 * the octrees, the FP64 near-field matrix of the chosen formulation (singular
 * terms in closed form), the preconditioner chosen by opt->preconditioner
 * (default: the near-field polynomial; ILU0 = the paper's incomplete LU) and
 * the MLFMM tables, and uploads them to the device.  Bodies are independent
 * scatterers.  opt = NULL takes sfmm_default_options.  Errors:
 * SFMM_E_INVALID_ARG (NULL or non-finite inputs, bad options, a non-vacuum
 * region 0), SFMM_E_MESH, SFMM_E_OOM, SFMM_E_DEVICE, SFMM_E_UNSUPPORTED,
 * SFMM_E_BREAKDOWN (zero pivot, see ilu_pivot_tol).  On success *out owns all
 * memory; on failure *out is NULL. */
sfmm_status sfmm_setup(const sfmm_body *bodies, int32_t n_bodies, const sfmm_options *opt,
                       sfmm_ctx **out);

/* Release every host and device allocation of ctx (NULL is accepted). */
void sfmm_destroy(sfmm_ctx *ctx);

/* Message for the last failed call on ctx, or for the last failed
 * sfmm_setup when ctx is NULL.  Valid until the next call on ctx. */
const char *sfmm_last_error(const sfmm_ctx *ctx);

/* Stream for subsequent on_device calls (hipStream_t; NULL = null stream). */
sfmm_status sfmm_set_stream(sfmm_ctx *ctx, void *hip_stream);

/* Number of unknowns 2E of a body, number of edges E. */
sfmm_status sfmm_num_unknowns(const sfmm_ctx *ctx, int32_t body, int64_t *n_unknowns);

/* Canonical edge table: [E][2] vertex ids (smaller first). */
sfmm_status sfmm_edges(const sfmm_ctx *ctx, int32_t body, int32_t *edge_vertices);

/* y = Z x for n_rhs vectors: the product of the moment matrix of the
 * context's formulation (PMCHWT: eqs. 10-13 and 16; JMCFIE: eqs. 8-16; CNF:
 * eqs. 8-9; tested with RWG functions, eqs. 22-26)
 * that the paper's Krylov solver evaluates by the MLFMM ("Simulation
 * Results": the multipole-accelerated product).  Near part exact (stored
 * matrix), far part by aggregation, translation and disaggregation.
 * x, y: [n_rhs][2E] complex in the boundary layout, host or device per
 * on_device; y is overwritten.  parts = 3 for the full product; 1 =
 * near-field matrix only, 2 = far-field (MLFMM) part only (for diagnostics).
 * Errors: SFMM_E_INVALID_ARG (NULL pointers, n_rhs <= 0, parts), SFMM_E_OOM,
 * SFMM_E_DEVICE. */
enum { SFMM_PART_NEAR = 1, SFMM_PART_FAR = 2, SFMM_PART_ALL = 3 };
sfmm_status sfmm_matvec(sfmm_ctx *ctx, int32_t body, int32_t n_rhs, const void *x, void *y,
                        int32_t on_device, int32_t parts);

/* y = M^-1 x with M the context's preconditioner (opt->preconditioner: the
 * near-field polynomial by default, ILU(0) of the near-field matrix in colour
 * ordering for SFMM_PRECOND_ILU0 - the paper's incomplete LU, "Simulation
 * Results" - identity for SFMM_PRECOND_NONE).  Layout as sfmm_matvec. */
sfmm_status sfmm_precond(sfmm_ctx *ctx, int32_t body, int32_t n_rhs, const void *x, void *y,
                         int32_t on_device);

/* Plane-wave right-hand sides (eqs. 20-21 tangential part, eq. 30): for
 * incidence angle i, the wave arrives from direction (theta, phi) =
 * angles[i] (radians), i.e. propagates along -r_hat(theta, phi), with
 * E0 = 1 V/m along pol[i] * theta_hat + (1 - pol[i]) * phi_hat  (pol = 1:
 * theta-polarised, 0: phi-polarised; pol = NULL: all theta-polarised).
 * b is [n_rhs][2E] complex.  Computed on the device in FP64 (7-point rule on
 * both triangles of every edge that faces the exterior region). */
sfmm_status sfmm_planewave_rhs(sfmm_ctx *ctx, int32_t body, int32_t n_rhs, const double *angles,
                               const double *pol, void *b, int32_t on_device);

/* Change the GMRES settings of later sfmm_solve calls (0 keeps a value):
 * restart length (1..1000), iteration cap, relative tolerance. */
sfmm_status sfmm_set_solver(sfmm_ctx *ctx, int32_t gmres_restart, int32_t max_iters, double tol);

/* Change the Krylov method (SFMM_SOLVER_*) of later sfmm_solve calls. */
sfmm_status sfmm_set_krylov(sfmm_ctx *ctx, int32_t solver);

/* Solve Z x = b, the discretised system of the context's formulation with the
 * plane-wave right-hand side of eqs. 20-21 and 30, by the preconditioned
 * Krylov iteration the paper uses ("Simulation Results"; the solver is
 * restarted GMRES here, see sfmm_options.solver).  b, x (and x0): [n_rhs][2E]
 * complex, host or device per on_device.  Restarted flexible GMRES(m) (Saad
 * 1993): Arnoldi with
 * classical Gram-Schmidt applied twice, Givens rotations and the
 * least-squares update in FP64, the preconditioner of sfmm_options applied on
 * the right in the product precision.  Right-hand sides are iterated in
 * lockstep, up to 64 at a time; converged ones leave the batch.  Convergence
 * is declared only on the explicitly recomputed residual ||b - Z x|| / ||b||
 * <= tol.  x0 = NULL starts from zero.  A supplied x0 (for instance from
 * sfmm_guess_predict) is judged by its true residual: if ||b - Z x0|| is not
 * below ||b|| the right-hand side starts from zero instead, so a poor guess
 * never costs more than one product.  info [n_rhs] may be NULL.  Returns
 * SFMM_E_NOT_CONVERGED (x holds the last iterate) if any right-hand side
 * misses the tolerance. */
sfmm_status sfmm_solve(sfmm_ctx *ctx, int32_t body, int32_t n_rhs, const void *b, void *x,
                       const void *x0, sfmm_solve_info *info, int32_t on_device);

/* Solve several bodies of the context at once: body bodies[i] with n_rhs[i]
 * right-hand sides b[i] -> x[i] ([n_rhs[i]][2E_i] each, host or device per
 * on_device), zero initial guess.  The bodies are taken largest-first from a
 * work list by up to 8 host threads, each body on a HIP stream of its own, so
 * uneven bodies overlap on the GPU.  info (may be NULL) is [sum n_rhs] in the
 * order of the list.  Work queued on the context stream before the call is
 * complete before any body starts; the call returns when every body is done.
 * A body may be listed once.  Status: the first hard error of any body, else
 * SFMM_E_NOT_CONVERGED if any right-hand side missed the tolerance.  Must not
 * overlap with other calls on the same context. */
sfmm_status sfmm_solve_bodies(sfmm_ctx *ctx, int32_t n, const int32_t *bodies, const int32_t *n_rhs,
                              const void *const *b, void *const *x, sfmm_solve_info *info, int32_t on_device);

/* Bistatic RCS (eqs. 27-29): sigma[r][d] = (sigma_theta, sigma_phi) in m^2
 * for solution r at direction theta_phi[d] (radians).  x follows on_device;
 * theta_phi and sigma are host arrays.  The far-field sums run on the device
 * in FP64 over the exterior-facing edges. */
sfmm_status sfmm_rcs(sfmm_ctx *ctx, int32_t body, int32_t n_rhs, const void *x, int32_t n_dirs,
                     const double *theta_phi, double *sigma, int32_t on_device);

/* Allocation-free variant of sfmm_rcs, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): same result as sfmm_rcs with
 * on_device = 1.  x_dev: [n_rhs][2E] complex on the context's device;
 * theta_phi [n_dirs][2] and sigma [n_rhs][n_dirs][2] are host arrays, staged
 * through a static device scratch of 262,144 doubles (2 MiB) that the
 * library holds on every GPU it runs on until the process ends.  Requires
 * n_dirs * (2 + 2 n_rhs) <= 262144, else SFMM_E_INVALID_ARG.  Calls no
 * allocating routine.  Every context on a GPU shares that GPU's scratch:
 * calls that overlap on one GPU (other threads, other contexts) race.
 * Synchronous on the context's stream. */
sfmm_status sfmm_rcs_noalloc(sfmm_ctx *ctx, int32_t body, int32_t n_rhs, const void *x_dev, int32_t n_dirs,
                             const double *theta_phi, double *sigma);

/* Learned GMRES initial guess (an addition to the paper's method; the paper
 * starts GMRES from zero).  sfmm_guess_fit trains, on the device, a network
 * that maps an incidence to the currents:
 *   POD basis U: the r leading left singular vectors of the n training
 *     solutions x (Gram matrix on the device, Hermitian Jacobi on the host);
 *   features: cos/sin(m theta), cos/sin(m phi) for m = 1..M, then the
 *     radiation pattern of the right-hand side b read as surface currents
 *     (its far field, as in the RCS of eqs. 27-29, at n_theta x n_phi
 *     directions: theta at band midpoints of [0, pi], phi uniform in
 *     [0, 2 pi); Re/Im of the theta and phi components) / ||b||, scaled by
 *     one scalar;
 *   network: y = Ws^T z_p + MLP(z) / s_r for the scaled Re/Im(U^H x) / ||b||:
 *     a linear path from the pattern features, fitted first as the
 *     minimum-norm least-squares map (FP64), and two tanh hidden layers
 *     trained by Adam (cosine step decay) on what the linear path leaves,
 *     scaled to unit RMS; MLP GEMMs on the matrix cores with bf16-split
 *     operands and FP32 accumulation, FP32 weights.
 * sfmm_guess_predict returns x0 = U c ||b|| for new incidences, to be passed
 * to sfmm_solve, which keeps it only if it lowers the true residual.
 * angles [n][2] (theta, phi) and pol [n] follow sfmm_planewave_rhs; x and x0
 * are [n][2E] complex in boundary order, on the device if on_device.
 * fit: 1 <= n <= 512; *final_loss (may be NULL) receives the MLP's training
 * loss on its unit-RMS targets (0.5/n sum of squares; r at the start).
 * Errors: SFMM_E_INVALID_ARG (sizes, options, predict before fit). */
typedef struct {
    int32_t rank;       /* POD basis size r (clamped to n and to the resolved rank) */
    int32_t harmonics;  /* M angle harmonics                                        */
    int32_t hidden;     /* width of both tanh hidden layers (1..4096)               */
    int32_t epochs;     /* full-batch Adam steps (0: the linear path alone)         */
    double lr;          /* peak Adam step size                                      */
    uint64_t seed;      /* SplitMix64 seed of the uniform weight initialisation     */
    int32_t n_theta;    /* pattern directions: theta bands (n_theta * n_phi <= 4096) */
    int32_t n_phi;      /*                     phi samples                           */
} sfmm_guess_options;

void sfmm_guess_default_options(sfmm_guess_options *opt);
sfmm_status sfmm_guess_fit(sfmm_ctx *ctx, int32_t body, int32_t n, const double *angles, const double *pol,
                           const void *x, const sfmm_guess_options *opt, double *final_loss, int32_t on_device);
sfmm_status sfmm_guess_predict(sfmm_ctx *ctx, int32_t body, int32_t n, const double *angles, const double *pol,
                               void *x0, int32_t on_device);

/* Baseline for the learned guess, without the network: the guess in the span
 * of the POD basis U of the last sfmm_guess_fit that minimises the residual,
 * x0 = U c, c = argmin ||b - Z U c|| (normal equations of W = Z U; W costs r
 * products on the first call after a fit).  Arguments as sfmm_guess_predict. */
sfmm_status sfmm_span_predict(sfmm_ctx *ctx, int32_t body, int32_t n, const double *angles, const double *pol,
                              void *x0, int32_t on_device);

/* The network kernels of the learned guess on their own, for checking: an
 * MLP with layer sizes sizes[0..n_sizes-1] (tanh hidden layers, linear
 * output) and parameters params (host; per layer W [in][out] row-major then
 * b [out], FP32) on a batch X [batch][sizes[0]] with targets
 * Y [batch][sizes[n_sizes-1]].  Computes, on GPU `device`, the output out
 * (may be NULL) and the loss 0.5/batch sum ||f(X) - Y||^2 with its gradient
 * grads (may be NULL) at the given parameters, then takes `steps` Adam steps
 * (beta1 0.9, beta2 0.999, eps 1e-8, step size lr) and writes the new
 * parameters back into params.  loss [steps + 1] receives the loss before
 * each step and after the last.  Errors: SFMM_E_INVALID_ARG, SFMM_E_DEVICE. */
sfmm_status sfmm_mlp_train(int32_t device, int32_t n_sizes, const int32_t *sizes, float *params, int32_t batch,
                           const float *X, const float *Y, int32_t steps, double lr, double *loss, float *grads,
                           float *out);

/* Diagnostics: rows of the FP64 near-field matrix (before the cast to the
 * product precision), in boundary layout: out[i] = [E row; H row] of edge
 * edges[i], each 2E complex, zero outside the near pattern.  Works on a
 * host-only context (device = -1). */
sfmm_status sfmm_near_rows(const sfmm_ctx *ctx, int32_t body, int32_t n_rows, const int32_t *edges,
                           double *out);

/* Diagnostics: the octree and sampling actually used. info[0..3] = levels,
 * finest level boxes, near edge pairs, translation pairs; per region r
 * (0 <= r < n_regions, up to 8) trunc[r*16 + l] = truncation order at level l. */
sfmm_status sfmm_describe(const sfmm_ctx *ctx, int32_t body, int64_t *info, int32_t *trunc);

/* Algorithmic HBM bytes of one single-RHS product y = Z x of a body at the
 * context's storage precision: the least traffic of this stored-table form,
 * every array read or written once per use.  bytes[0] near-field values (three
 * complex numbers per edge pair for the PMCHWT 2x2 block [[A, -B], [B, C]],
 * four for JMCFIE / CNF) and
 * column indices; bytes[1] x read and y written once; bytes[2] radiation
 * patterns read for aggregation and again for receiving (the aggregation and
 * disaggregation steps of the multipole method the paper's solver uses,
 * "Simulation Results"); bytes[3] level arrays,
 * outgoing and incoming patterns each written and read once; bytes[4]
 * translation operators for the offsets in use; bytes[5] interpolation and
 * shift tables; bytes[6] the total; bytes[7] = 0.  `bytes` is a caller array
 * of 8 int64. */
sfmm_status sfmm_product_bytes(const sfmm_ctx *ctx, int32_t body, int64_t *bytes);

/* Average GPU time in milliseconds of each stage over the products and
 * preconditioner applications since the last reset, measured with HIP events
 * on the context's stream: t[0] near product, t[1] aggregation, t[2] upward
 * interpolation, t[3] translation, t[4] downward anterpolation, t[5] receive,
 * t[6] ILU(0) solves, t[7] whole product; n[i] = number of samples.
 * Stage timing is enabled only between sfmm_profile(ctx, 1, ...) and
 * sfmm_profile(ctx, 0, ...); enabling resets the accumulators.  While timing
 * is on, products run kernel by kernel instead of from captured graphs. */
sfmm_status sfmm_profile(sfmm_ctx *ctx, int32_t enable, double *t, int64_t *n);

#ifdef __cplusplus
}
#endif

#endif /* SFMM_H */
