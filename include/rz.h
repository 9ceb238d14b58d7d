/*
 * rz.h -- C ABI of the MI355X library for the p-multigrid solvers of the Riesz
 * maps of the L2 de Rham complex (Brubeck & Farrell, "Multigrid solvers for the
 * de Rham complex with optimal complexity in polynomial degree").
 *
 * Problem (Sec. 1, eqs. hgrad/hcurl/hdiv; Sec. 2.1, eq. common_weak_formulation):
 *   find u_h in V^k_{h,p} with a^k(v,u) = (v, beta u) + (d^k v, alpha d^k u) = F(v)
 *   for k = 0 (H(grad), Q_p), 1 (H(curl), NCE_p), 2 (H(div), NCF_p) on a structured
 *   nx*ny*nz hexahedral mesh, homogeneous Dirichlet traces on the faces selected
 *   by a bit mask.
 *
 * Degrees of freedom are coefficients in the FDM bases of Sec. 2.2-2.4 and sit on
 * a lattice (x fastest).  Q_p: index X + Nx*(Y + Ny*Z), Nx = nx*p + 1.  NCE_p /
 * NCF_p: three component blocks one after the other; component m has extent
 * n_a*p along its broken (DP) axes and n_a*p+1 along its continuous axes.
 * Vectors hold every lattice DoF; Dirichlet rows act as the identity (outputs copy
 * the input there, inputs there are read as zero elsewhere).
 *
 * Several right-hand sides (nrhs > 1 in rz_apply, rz_relax, rz_vcycle, rz_solve,
 * rz_solve_batched): multi-vectors are DoF-major with the right-hand side fastest,
 * value r of DoF g at v[g*nrhs + r] (a row-major ndofs x nrhs array).  The first
 * call with more right-hand sides than before allocates the per-vector workspace
 * (kept until rz_free and reused by later calls with as many or fewer).
 *
 * Ownership: the caller owns every vector (device pointers, e.g. the data of a
 * torch tensor on the library's device).  The library owns tables, factors and
 * workspace, all allocated in rz_setup and released by rz_free.  Host arrays
 * passed to rz_setup are copied before it returns.
 *
 * Ordering / synchronisation: calls are stream-ordered on the stream given to
 * rz_create (NULL = the legacy default stream).  rz_setup, rz_solve and
 * rz_export return after the device work they need has finished.
 *
 * Errors: every call returns an rz_status; rz_last_error(ctx) gives a message.
 * Nothing throws across this boundary.  One host thread per context at a time.
 */
#ifndef RZ_H
#define RZ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rz_ctx rz_ctx;
typedef struct rz_problem rz_problem;

typedef enum { RZ_GRAD = 0, RZ_CURL = 1, RZ_DIV = 2 } rz_space;

typedef enum {
  RZ_OK = 0,
  RZ_ERR_ARG = -1,           /* invalid argument or unsupported combination     */
  RZ_ERR_OOM = -2,           /* device or host allocation failed                */
  RZ_ERR_BREAKDOWN = -3,     /* incomplete Cholesky pivot <= 0, or CG p.Ap <= 0  */
  RZ_ERR_NOT_CONVERGED = -4, /* maxit reached before the tolerance              */
  RZ_ERR_HIP = -5,           /* a HIP runtime call failed                        */
  RZ_ERR_SINGULAR = -6,      /* coarse factorisation met a non-positive pivot   */
  RZ_ERR_NODEVICE = -7       /* compute call on a host-only context             */
} rz_status;

/* Element type of device vectors.  RZ_BF16: bfloat16 (the upper 16 bits of an IEEE
 * binary32, rounded to nearest even), for rz_apply only (FP32 arithmetic). */
typedef enum { RZ_F64 = 0, RZ_F32 = 1, RZ_BF16 = 2 } rz_dtype;

/* Mesh: structured nx*ny*nz hexahedra.  vertex_xyz: host array of
 * (nx+1)(ny+1)(nz+1) points (x,y,z), vertex vx + (nx+1)*(vy + (ny+1)*vz);
 * NULL = uniform mesh of the unit cube.  dirichlet_faces: bit 0 x=0, 1 x=1,
 * 2 y=0, 3 y=1, 4 z=0, 5 z=1 (0x3F = whole boundary). */
typedef struct {
  int32_t nx, ny, nz;
  const double *vertex_xyz;
  uint32_t dirichlet_faces;
} rz_mesh;

/* Coefficients alpha, beta > 0 of a^k.  RZ_COEF_CONST: alpha[0], beta[0].
 * RZ_COEF_CELL: one value per cell (cells cx + nx*(cy + ny*cz)), constant on the
 * cell.  RZ_COEF_SAMPLES: 27 values per cell, the coefficient at the images of the
 * reference points {-1,0,1}^3 (x fastest) under the cell's trilinear map; the
 * coefficient is their triquadratic interpolant on the reference cell.  Host
 * arrays.
 *
 * Cartesian meshes with RZ_COEF_CONST / RZ_COEF_CELL use the exact Kronecker cell
 * matrices (Sec. 3.2 closed form).  Any other mesh (trilinear cells) or
 * RZ_COEF_SAMPLES integrates with q = ceil(3(p+1)/2) Gauss-Lobatto-Legendre points
 * per axis (Sec. 5); the relaxation then uses separable per-cell weights from cell
 * averages of the coefficient-weighted metric, and the p=1 coarse operator is
 * integrated with 3 points per axis. */
enum { RZ_COEF_CONST = 0, RZ_COEF_CELL = 1, RZ_COEF_SAMPLES = 2 };
typedef struct {
  int32_t kind;
  const double *alpha;
  const double *beta;
} rz_coef;

/* Precision protocols of the solve. */
enum {
  RZ_PREC_F64 = 0,   /* FP64 apply, relaxation, coarse solve and Krylov            */
  RZ_PREC_MIXED = 1, /* FP64 apply/coarse/Krylov, FP32 relaxation, flexible CG     */
  RZ_PREC_DEFECT = 2 /* defect correction: FP64 outer residuals and updates; inner  *
                      * FP32 flexible CG (FP32 apply, FP32 V-cycle with FP64 coarse *
                      * correction) to 1e-4 relative; iters = inner iterations      */
};

typedef struct {
  int32_t space;       /* rz_space                                                  */
  int32_t p;           /* polynomial degree, 1 <= p <= 9                            */
  int32_t precision;   /* RZ_PREC_*                                                 */
  int32_t maxit;       /* CG iteration cap (default 200)                            */
  double rtol;         /* relative tolerance on the 2-norm residual (default 1e-8)   */
  double omega;        /* smoother damping; 0 = 2/(1.2*lambda_max) with lambda_max  *
                        * estimated by 10 Lanczos steps on M^{-1}A (FP64 M in every  *
                        * precision protocol)                                        */
  uint64_t lanczos_seed; /* SplitMix64 seed of the Lanczos start vector (default 99) */
  double hdiv_eps;     /* H(div): multiple of the (beta-weighted) mass added to the   *
                        * curl-curl potential problem (remark of Sec. 4.3); 0 = 1e-3 */
  int32_t aux;         /* auxiliary operator of the relaxation on trilinear cells     *
                        * (H(grad)): RZ_AUX_CELL_AVG (default) or RZ_AUX_PAPER_DIAG    */
  int32_t graph;       /* 1: rz_solve / rz_solve_batched run each CG iteration (all    *
                        * right-hand sides of the call active, iteration >= 1) from    *
                        * HIP graphs captured on first use (per parity of the count,   *
                        * vector count and set of x vectors), the cooperative Q_1      *
                        * coarse solve launched between their segments; same kernels,  *
                        * same results as 0 (default).  Not with per-kernel timing.    */
  int32_t patch_solver; /* H(grad) vertex-star solves on the statically condensed       *
                        * patches (Sec. 4.5): RZ_PATCH_IC (default) incomplete Cholesky *
                        * on the static-condensation pattern, or RZ_PATCH_CHOLESKY the  *
                        * exact Cholesky factor (the SC-chol column of Table           *
                        * hgrad-iter), applied as W = L^{-1} dense per patch: memory    *
                        * grows as p^4 per vertex, meant for small meshes (RZ_ERR_ARG   *
                        * past 16 GiB of factors)                                       */
  int32_t decomposition; /* H(grad) relaxation (Sec. 4.3-4.4): RZ_DECOMP_SC (default)  *
                        * SC-PAFW, vertex stars on the statically condensed interface; *
                        * RZ_DECOMP_FULL PAFW without static condensation (eq. pafw):  *
                        * every DoF strictly inside the cells around a vertex, the star *
                        * matrix factored exactly (patch_solver RZ_PATCH_CHOLESKY) or   *
                        * by IC on its pattern (RZ_PATCH_IC), both applied as dense     *
                        * W = L^{-1} (the chol / ICC columns of Table hgrad-iter);      *
                        * (2p-1)^3 rows per star, for small meshes and degrees          *
                        * (RZ_ERR_ARG past 16 GiB of factors or about 5e11 host flops). *
                        * H(curl)/H(div): RZ_DECOMP_SC (default) SC-PH; RZ_DECOMP_FULL   *
                        * PAFW, the vertex stars of the k-forms without condensation;    *
                        * RZ_DECOMP_SC_VERTEX SC-PAFW (Sec. 4.4), those stars restricted *
                        * to the condensed interface, each solved exactly on the         *
                        * assembled interface Schur complement; RZ_DECOMP_FULL_PH PH     *
                        * without condensation (Sec. 4.3 eq. ph): edge (H(curl)) or face *
                        * (H(div)) stars holding every DoF of their cells, plus the      *
                        * potential term through the full vertex stars of Q_p (resp. the *
                        * edge stars of NCE_p) and the full exterior derivative (the     *
                        * PAFW, SC-PAFW and PH columns of Tables hcurl-iter / hdiv-iter; *
                        * all with RZ_PATCH_CHOLESKY, dense W = L^{-1} per star, small   *
                        * meshes)                                                        */
  int32_t norm;        /* stopping rule of rz_solve / rz_solve_batched (FP64 and mixed  *
                        * protocols): RZ_NORM_2 (default) the true 2-norm residual      *
                        * <= rtol ||b||, confirmed by a residual from x; RZ_NORM_NATURAL *
                        * the paper's criterion (Sec. 5.1): CG stops once the natural    *
                        * norm (r^T M^{-1} r)^{1/2} of a residual has dropped by rtol    *
                        * against the first (iters_natural then counts the iterations,   *
                        * rel_res reports the true 2-norm residual at exit)              */
  int32_t coarse;      /* H(grad) solver of the p = 1 problem inside the p-multigrid    *
                        * cycle: RZ_COARSE_DIRECT (default) the exact solve, or          *
                        * RZ_COARSE_HMG geometric h-multigrid on the Q_1 space (the      *
                        * h-hierarchy of Sec. 5.1): meshes with half the cells per axis  *
                        * while every count is even and a level holds more than 512 free *
                        * vertices, trilinear interpolation, Galerkin operators, one     *
                        * V(1,1) cycle with point Jacobi (weight 2/3) from a zero guess, *
                        * the coarsest level solved exactly (dense inverse, at most 4096 *
                        * free vertices, else RZ_ERR_ARG).  The cycle is symmetric       *
                        * positive definite, so CG stays valid; iteration counts may     *
                        * grow slightly against the exact solve.                         */
  int32_t lanczos_steps; /* preconditioned CG steps of the Lanczos estimate behind the   *
                        * default damping (omega = 0), at most 200; 0 = 10, or 40 with   *
                        * RZ_DECOMP_SC_VERTEX, whose spectrum has an outlying top at     *
                        * small beta (10 steps underestimate lambda_max by 30 %, and the *
                        * V(1,1) cycle then loses definiteness: CG reports the breakdown)*/
} rz_opts;

/* Solvers of the p = 1 problem (rz_opts.coarse). */
enum { RZ_COARSE_DIRECT = 0, RZ_COARSE_HMG = 1 };

/* Decompositions of the relaxation (rz_opts.decomposition). */
enum { RZ_DECOMP_SC = 0, RZ_DECOMP_FULL = 1, RZ_DECOMP_SC_VERTEX = 2, RZ_DECOMP_FULL_PH = 3 };

/* Stopping rules (rz_opts.norm). */
enum { RZ_NORM_2 = 0, RZ_NORM_NATURAL = 1 };

/* Vertex-star solvers of the H(grad) relaxation (rz_opts.patch_solver). */
enum { RZ_PATCH_IC = 0, RZ_PATCH_CHOLESKY = 1 };

/* Auxiliary operators P of the relaxation (Sec. 3.2).  On Cartesian cells with
 * cellwise-constant coefficients both equal A exactly (and the library uses its
 * separable form).  On trilinear cells or with sampled coefficients:
 *   RZ_AUX_CELL_AVG   the separable form with six weights per cell, cell averages
 *                     of the coefficient-weighted metric (rz_set_aux replaces them);
 *   RZ_AUX_PAPER_DIAG the paper's auxiliary, eq. sum-factorization_approx: the
 *                     beta- and alpha-weighted mass matrices replaced by their
 *                     diagonals in the broken bases (eq. mass_in_broken_basis),
 *                     (p+1)^3 + 3 p (p+1)^2 values per cell computed at setup with
 *                     the apply's quadrature; P_II stays diagonal. */
enum { RZ_AUX_CELL_AVG = 0, RZ_AUX_PAPER_DIAG = 1 };

/* Results of rz_solve. */
typedef struct {
  int32_t iters;          /* CG iterations                                            */
  int32_t status;         /* rz_status of the solve                                   */
  double rel_res;         /* true ||b - A x||_2 / ||b||_2 at exit                     */
  double omega;           /* smoother damping that was used                           */
  double t_solve_ms;      /* device time of the solve (hipEvents on the stream)       */
  int32_t iters_natural;  /* iterations after which the natural norm (r^T M^{-1} r)^{1/2} *
                           * of the residual had dropped by rtol, the paper's criterion  *
                           * (Sec. 5.1); -1 if it did not within the solve (or for the   *
                           * defect-correction protocol)                                 */
} rz_solve_info;

/* Fill *o with defaults (space grad, p = 4, FP64, maxit 200, rtol 1e-8, omega 0,
 * aux RZ_AUX_CELL_AVG). */
void rz_opts_default(rz_opts *o);

/* Create a context on HIP device `device` and stream `stream` (a hipStream_t, may
 * be NULL).  device = -1 creates a host-only context: rz_setup then builds only
 * the host-side data (numbering, 1-D tables, patch layout, IC pattern) for
 * rz_export, and every compute call returns RZ_ERR_NODEVICE. */
rz_status rz_create(rz_ctx **ctx, int device, void *stream);
/* Destroy a context.  RZ_ERR_ARG (and nothing destroyed) while problems or MLPs
 * created on it have not been freed. */
rz_status rz_destroy(rz_ctx *ctx);
const char *rz_last_error(const rz_ctx *ctx);

/* Build everything a solve needs (Sec. 3.2 auxiliary operator, Sec. 4.4 static
 * condensation, Sec. 4.5 incomplete Cholesky of every vertex-star interface
 * patch on the static-condensation pattern, the p=1 coarse problem of eq.
 * asm-afw and its factorisation).  Cells must have a positive Jacobian
 * determinant at every quadrature point (RZ_ERR_ARG otherwise).  Returns
 * RZ_ERR_BREAKDOWN if an IC pivot is not positive and RZ_ERR_SINGULAR if the
 * coarse factorisation fails. */
rz_status rz_setup(rz_ctx *ctx, const rz_mesh *mesh, const rz_coef *coef,
                   const rz_opts *opts, rz_problem **out);
rz_status rz_free(rz_problem *h);

/* sizes[0] lattice DoFs, [1] free DoFs, [2] cells, [3] vertex-patch slots,
 * [4] coarse (p=1) lattice DoFs, [5] nonzeros of one patch factor (lower),
 * [6] rows of one patch, [7] non-empty patches. */
rz_status rz_sizes(const rz_problem *h, int64_t sizes[8]);

/* y = A x (Sec. 3.2, eq. sum-factorization: matrix-free, per-cell tensor
 * contractions).  x, y: device arrays of sizes[0]*nrhs elements of type t (nrhs >= 1
 * right-hand sides, interleaved as above); x and y must not overlap.
 * RZ_BF16 (H(grad)): BF16 vectors.  On trilinear cells or with sampled coefficients
 * the 1-D contractions run on the matrix cores with BF16 operands and FP32
 * accumulation, every contraction's result rounded to BF16 before the next, the
 * pullback in FP32; on Cartesian cells with cellwise-constant coefficients the sparse
 * FDM line operators run in FP32 on BF16 loads and stores.  The result carries the
 * rounding error of BF16 (about 1e-2 relative; the bench reports it against FP64).
 * RZ_ERR_ARG for H(curl) / H(div). */
rz_status rz_apply(rz_problem *h, const void *x, void *y, rz_dtype t, int32_t nrhs);

/* y = A x exactly as rz_apply with nrhs = 1 (same kernels, same result), for callers that cannot
 * allocate device memory at call time or must not trigger the library's own
 * allocations (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  The call allocates nothing: the apply's workspace (the
 * face-line buffer of the Cartesian H(grad) path, the per-cell outputs of the
 * quadrature path, the contributions to shared entries of the H(curl)/H(div) paths)
 * is a static device array of 64 MiB per GPU, its address taken once per device by
 * rz_create.  RZ_ERR_ARG if the problem needs more workspace than that (ny*nz*4p*Nx
 * elements on the Cartesian H(grad) path, ncells*(p+1)^3 on the quadrature path,
 * 3*ndofs for H(curl), ndofs for H(div)).
 * Every call on one GPU shares that array and it keeps the last call's contents:
 * calls that overlap in time on one GPU (other streams, other contexts or
 * threads) race and give wrong results; calls ordered on one stream are safe. */
rz_status rz_apply_noalloc(rz_problem *h, const void *x, void *y, rz_dtype t);

/* z = M^{-1} r, one application of the statically condensed additive Schwarz
 * relaxation on the auxiliary operator.  H(grad) (Sec. 4.4, eqs. schur and
 * sc-asm-afw; Sec. 4.5): cell-interior solves, vertex-star interface patch solves
 * with the IC factors on the static-condensation pattern, harmonic extension.
 * H(curl) / H(div) (Sec. 4.3-4.4, eqs. sc-ph and sc-asm-hiptmair): edge-star
 * Cholesky solves (curl) or face-star Jacobi (div) on the condensed interface, plus
 * the potential term through the interface exterior derivative.  Device arrays of
 * sizes[0]*nrhs elements of type t (RZ_F32 uses FP32 factors).  With nrhs > 1 the
 * H(grad) vertex-patch solve reads each patch factor once per pair of vectors. */
rz_status rz_relax(rz_problem *h, const void *r, void *z, rz_dtype t, int32_t nrhs);

/* Transfers between the degree-p lattice and the p=1 lattice (sizes[4]) of the
 * two-level method (Sec. 4.3, eq. asm-afw: the coarse space V_{h,1}; Sec. 5):
 * xf += P xc (prolongation, the embedding V_{h,1} in V_{h,p}) and rc = P^T rf.
 * FP64 device arrays; Dirichlet entries of the output are zero (prolong adds 0).
 * H(grad) only (RZ_ERR_ARG otherwise). */
rz_status rz_prolong_add(rz_problem *h, const double *xc, double *xf);
rz_status rz_restrict(rz_problem *h, const double *rf, double *rc);

/* xc = A_0^{-1} rc on the free p=1 DoFs (the coarse problem of eq. asm-afw, Sec.
 * 4.3: the same form at p = 1; FP64 block-tridiagonal LDL^T); Dirichlet entries of
 * xc are zero.  H(grad) only (RZ_ERR_ARG otherwise). */
rz_status rz_coarse_solve(rz_problem *h, const double *rc, double *xc);

/* z = V(r): hybrid V(1,1) cycle of Sec. 5 (damped relaxation, coarse correction
 * of eq. asm-afw, damped relaxation), FP64 device arrays of sizes[0]*nrhs
 * elements. */
rz_status rz_vcycle(rz_problem *h, const double *r, double *z, int32_t nrhs);

/* Solve A x = b by CG preconditioned with the V-cycle (Sec. 5) from x = 0, until
 * the true ||b - A x||_2 <= rtol ||b||_2 for every right-hand side.  b, x: FP64
 * device arrays of sizes[0]*nrhs elements.  The right-hand sides iterate in
 * lockstep (their V-cycles together; one that has converged stops), each with the
 * arithmetic of a solve on its own: the results equal nrhs separate solves.  The
 * defect-correction protocol solves them one after another.  info: NULL or nrhs
 * results.  Returns the first failing status of the right-hand sides;
 * RZ_ERR_NOT_CONVERGED if maxit is reached (x holds the last iterate). */
rz_status rz_solve(rz_problem *h, const double *b, double *x, int32_t nrhs, rz_solve_info *info);

/* Batch of independent solves (the batched workload of many Riesz maps of uneven
 * size and degree).  Problem i (each problem at most once) solves nrhs right-hand
 * sides b[i] into x[i] (device multi-vectors of ndofs_i*nrhs elements, interleaved
 * as above), in lockstep as rz_solve does.  The problems advance from the calling
 * thread: it enqueues one step of every problem whose previous step has finished
 * on its problem's stream, so problems created on different contexts (streams)
 * overlap on the device.  Results equal those of rz_solve.
 * infos: n*nrhs results (may be NULL).  Synchronous; returns the first failing
 * status (the other solves still run to completion). */
rz_status rz_solve_batched(rz_problem *const *hs, int32_t n, const double *const *b, double *const *x,
                           int32_t nrhs, rz_solve_info *infos);

/* ---- Mixed Hodge Laplacians (Sec. 5.3) -------------------------------------------
 * With no essential boundary, find (sigma, u) in V^{k-1} x V^k (k = 1: Q_p x NCE_p,
 * k = 2: NCE_p x NCF_p, k = 3: NCF_p x DQ_{p-1}) with
 *   -(tau, sigma) + (d tau, u) = 0,  (v, d sigma) + (d v, d u) = F(v),
 * i.e. in FDM coefficients K [sigma; u] = [0; f] with
 *   K = [ -M_{k-1}  D^T M_k ; M_k D  S_k ],
 * M_j the beta-weighted mass of V^j, S_k the alpha-weighted (d v, d u) (zero for
 * k = 3), D = d^{k-1} (grad, curl, div; exact in the FDM bases), and the L^2 mass of
 * DQ_{p-1} diagonal (8 / V per value on a box of volume V).  The solver is MINRES
 * (Paige & Saunders) preconditioned by blockdiag(C_{k-1}, C_k): C_j is cheb_steps
 * Chebyshev iterations (the paper uses 4) on the Riesz map of problem j,
 * preconditioned by that problem's p-multigrid V-cycle, over [0.9 lambda_min,
 * 1.1 lambda_max] of the extreme eigenvalues of the Lanczos tridiagonal of 10
 * V-cycle-preconditioned CG steps (start vector: SplitMix64 of the problem's
 * lanczos_seed); for DQ_{p-1} the preconditioner is point Jacobi of the diagonal
 * mass, whose Chebyshev interval is [0.9, 1.1].
 * Vectors are [sigma (ndofs of lo); u (ndofs of hi, or ncells p^3 for k = 3)],
 * FP64 device arrays; DQ_{p-1} numbering: X + n_x p (Y + n_y p Z), x fastest.
 * The object borrows lo and hi (set up with rz_setup for the spaces of form degree
 * k-1 and k, on the same Cartesian mesh and degree, dirichlet = 0, cellwise
 * coefficients, the default decomposition); free it first.  Calls on one object, and
 * on its problems, must not overlap.  The paper's setting is alpha = beta = 1 for
 * both problems.  A problem set up with RZ_PREC_MIXED relaxes in FP32 inside its
 * V-cycles (and uses the FP32 copies of its coarse blocks); MINRES, the block
 * operator, the Chebyshev recurrences and the Lanczos intervals stay FP64, and the
 * preconditioner is then symmetric up to FP32 rounding.  RZ_PREC_DEFECT problems are
 * rejected. */
typedef struct rz_hodge rz_hodge;

/* Build D and D^T (CSR on the device), the mass/stiffness weights, and the Chebyshev
 * intervals (synchronous).  hi must be NULL exactly for k = 3.  RZ_ERR_ARG on a
 * mismatch, RZ_ERR_OOM, RZ_ERR_BREAKDOWN if the Lanczos estimate fails. */
rz_status rz_hodge_create(int32_t k, rz_problem *lo, rz_problem *hi, int32_t cheb_steps, rz_hodge **out);
rz_status rz_hodge_free(rz_hodge *g);
/* sizes[0] = ndofs of V^{k-1}, sizes[1] = of V^k; eig (may be NULL): the Ritz
 * extremes (lo min, lo max, hi min, hi max) behind the Chebyshev intervals. */
rz_status rz_hodge_sizes(const rz_hodge *g, int64_t sizes[2], double eig[4]);
/* y = K x (asynchronous on the problems' stream). */
rz_status rz_hodge_apply(rz_hodge *g, const double *x, double *y);
/* z = blockdiag(C_{k-1}, C_k) r (asynchronous). */
rz_status rz_hodge_precond(rz_hodge *g, const double *r, double *z);
/* MINRES from x = 0 until the natural norm (r^T P^{-1} r)^{1/2} of the residual
 * has dropped by rtol (the paper's criterion, 1e-8).  info (may be NULL): iters =
 * iters_natural = MINRES iterations, rel_res = ||b - K x||_2 / ||b||_2 at exit,
 * t_solve_ms = device time.  Synchronous; RZ_ERR_NOT_CONVERGED after maxit,
 * RZ_ERR_BREAKDOWN if the preconditioner is not positive definite. */
rz_status rz_hodge_solve(rz_hodge *g, const double *b, double *x, double rtol, int32_t maxit, rz_solve_info *info);

/* Wait for the problem's queued work and report a coarse-solve wait that gave up.
 * The coarse solve (inside rz_coarse_solve, rz_vcycle and rz_solve) synchronises
 * its planes through bounded waits on data written in the same launch; a wait that
 * runs out records a flag on the device (the result is then not valid).  rz_solve
 * checks the flag itself; after the asynchronous calls, rz_sync returns RZ_ERR_HIP
 * if it is set (and clears it), RZ_OK otherwise. */
rz_status rz_sync(rz_problem *h);

/* Export host copies of setup products for parity checks.  If buf is NULL, *bytes
 * receives the size needed.  what:
 *   RZ_EXPORT_DOFMAP     int64 (ncells, ncell_dofs) cell -> lattice index
 *   RZ_EXPORT_PATCH      int64 lattice indices of non-empty patch `index`
 *                        (in patch order), preceded by its vertex id
 *   RZ_EXPORT_IC_PATTERN int32 pairs (row, col), row >= col, of non-empty patch
 *                        `index` in patch-local numbering, row-major order
 *   RZ_EXPORT_IC_FACTOR  double values matching RZ_EXPORT_IC_PATTERN (FP64 factor)
 *   RZ_EXPORT_TABLES1D   double: lambda (p-1), B (p+1)^2, A (p+1)^2, D p*(p+1),
 *                        E (p+1)*2 (p=1 embedding), all row-major
 *   RZ_EXPORT_AUXCOEF    double (ncells, 6) separable auxiliary weights
 *   RZ_EXPORT_OMEGA      double: the smoother damping of rz_vcycle / rz_solve
 *   RZ_EXPORT_PATCH_KERNEL int32 pair (FP64, FP32): 1 when the H(grad) patch solve
 *                        keeps a patch's factor in registers between its two sweeps,
 *                        0 when it streams the factor in both sweeps
 *   RZ_EXPORT_STATS      int64 pair (H(grad)): lower non-zeros (diagonal included)
 *                        and rows of the IC factors of all non-empty vertex patches
 *                        (the factor values the patch solve needs, without padding)
 *   RZ_EXPORT_AUTOTUNE   double, per precision (FP64, then FP32) of the streaming
 *                        vertex-patch solve: the number n of candidates the setup
 *                        timed, n pairs (resident wavefronts per CU, ms per launch),
 *                        then the chosen count (n = 0 and 0 where the register
 *                        kernel runs)
 *   RZ_EXPORT_PAPER_DIAG double: the broken diagonals of cell `index` with
 *                        RZ_AUX_PAPER_DIAG, (p+1)^3 (beta-mass, x fastest) then
 *                        3 blocks of p (p+1)^2 (alpha-mass of NCE component m, its
 *                        DP index along axis m)
 *   RZ_EXPORT_GRAPHS     int64 triple: CG iterations captured as HIP graphs, iterations
 *                        run from them, segments per captured iteration (last capture)
 *                        of this problem (rz_opts.graph)
 *   RZ_EXPORT_HMG        int64 per level of the h-multigrid coarse solver (rz_opts.coarse =
 *                        RZ_COARSE_HMG), finest first: its free vertices (rows)
 *   RZ_EXPORT_EDGE_PATCH int64: edge id, then the DoFs (ascending) of non-empty
 *                        edge-star patch `index` of H(curl) (or of the NCE_p
 *                        potential problem of H(div)); edge ids run over the axis
 *                        (x, y, z) then lattice order of (cell along the axis,
 *                        vertices across it)   */
enum {
  RZ_EXPORT_DOFMAP = 0, RZ_EXPORT_PATCH = 1, RZ_EXPORT_IC_PATTERN = 2,
  RZ_EXPORT_IC_FACTOR = 3, RZ_EXPORT_TABLES1D = 4, RZ_EXPORT_AUXCOEF = 5,
  RZ_EXPORT_OMEGA = 6, RZ_EXPORT_PATCH_KERNEL = 7, RZ_EXPORT_EDGE_PATCH = 8, RZ_EXPORT_STATS = 9,
  RZ_EXPORT_PAPER_DIAG = 10, RZ_EXPORT_AUTOTUNE = 11, RZ_EXPORT_GRAPHS = 12, RZ_EXPORT_HMG = 13
};
rz_status rz_export(rz_problem *h, int what, int64_t index, void *buf, int64_t *bytes);

/* Per-kernel device timing for measurement.  While enabled, every launch of the
 * kernels below is bracketed by hipEvents on the context stream; rz_timing_read
 * synchronises, returns the accumulated milliseconds and launch counts per kernel
 * (arrays of RZ_NKERNELS entries) and resets the accumulators. */
enum {
  RZ_K_APPLY = 0,        /* operator apply (init + cell kernel)                       */
  RZ_K_CONDENSE = 1,     /* relaxation: interface right-hand side (R_Gamma r)        */
  RZ_K_PATCH = 2,        /* relaxation: vertex-patch triangular solves               */
  RZ_K_EXPAND = 3,       /* relaxation: patch sum + harmonic extension               */
  RZ_K_TRANSFER = 4,     /* restriction + prolongation                               */
  RZ_K_COARSE = 5,       /* coarse block-tridiagonal solve                            */
  RZ_K_KRYLOV = 6,       /* vector updates and dot products                           */
  RZ_NKERNELS = 7
};
rz_status rz_timing_enable(rz_problem *h, int on);
rz_status rz_timing_read(rz_problem *h, double ms[RZ_NKERNELS], int64_t count[RZ_NKERNELS]);

/* Set rz_opts.graph of a problem after setup (1: CG iterations from captured HIP
 * graphs, 0: launches one by one; turning it off releases the graphs).  Results do
 * not depend on it. */
rz_status rz_set_graph(rz_problem *h, int on);

/* ---- learned auxiliary weights (trilinear cells) ----------------------------------
 * The separable auxiliary of the relaxation uses per-cell weights c = (sigma_1..3,
 * mu, mu, mu).  The least-squares fit of c to the broken diagonals of the paper's
 * auxiliary operator (eq. sum-factorization_approx) is their mean, computed with
 * the quadrature of the operator (Christoffel-factorised).  A small MLP (FP32,
 * nin -> nhid tanh -> nhid tanh -> nout, squared-error loss, Adam) learns
 * log(c_fit / c_avg) from dimensionless per-cell features; c_avg are the default
 * cell-averaged weights. */

/* Host arrays of ncells rows: targets (6) = the least-squares fit, features (51) =
 * corner offsets from the centroid over the mean edge length minus those of a cube
 * (24) and log alpha samples minus their mean (27), base (6) = the cell-averaged
 * weights in use.  Any pointer may be NULL.  Requires the quadrature path
 * (trilinear cells or sampled coefficients); works on host-only contexts. */
rz_status rz_aux_data(const rz_problem *h, double *targets, double *features, double *base);

/* Replace the auxiliary weights (host array ncells x 6, all > 0) and rebuild what
 * depends on them: the patch IC factors and, unless omega was fixed, omega.
 * Quadrature-path problems only (on Cartesian cells with cellwise-constant
 * coefficients the six weights are the operator itself: RZ_ERR_ARG).
 * Synchronous.  RZ_ERR_BREAKDOWN if an IC pivot is not positive; the previous
 * weights and factors are then restored. */
rz_status rz_set_aux(rz_problem *h, const double *coef6);

typedef struct rz_mlp rz_mlp;   /* opaque; parameters on the device of ctx */

/* Create an MLP on ctx's device and stream: Glorot-uniform weights from the
 * SplitMix64 stream `seed` (W1, W2, W3 in turn, row-major out x in), zero biases.
 * Parameters are packed W1 (nhid x nin), b1, W2 (nhid x nhid), b2, W3 (nout x nhid), b3. */
rz_status rz_mlp_create(rz_ctx *ctx, int32_t nin, int32_t nhid, int32_t nout, uint64_t seed, rz_mlp **out);
rz_status rz_mlp_free(rz_mlp *m);
const char *rz_mlp_last_error(const rz_mlp *m);
int64_t rz_mlp_nparams(const rz_mlp *m);
/* Copy the packed parameters to (set = 0) or from (set = 1) a host array; setting
 * restarts the Adam step count. */
rz_status rz_mlp_params(rz_mlp *m, float *host, int32_t set);
/* Y (n x nout) = network(X (n x nin)); device pointers, stream-ordered. */
rz_status rz_mlp_predict(rz_mlp *m, const float *X, float *Y, int64_t n);
/* Loss (mean over rows and outputs of the squared error) and its gradient with
 * respect to the packed parameters (host array of rz_mlp_nparams floats, may be
 * NULL); X, Y device pointers.  Synchronous. */
rz_status rz_mlp_loss_grad(rz_mlp *m, const float *X, const float *Y, int64_t n, double *loss, float *grad_host);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on the full batch X, Y. */
rz_status rz_mlp_adam_step(rz_mlp *m, const float *X, const float *Y, int64_t n, float lr);
/* Minibatch Adam: `epochs` passes over the n rows in an order shuffled by the
 * SplitMix64 stream `seed`, floor(n / batch) steps per epoch; *final_loss = the
 * loss of the last batch.  Synchronous. */
rz_status rz_mlp_train(rz_mlp *m, const float *X, const float *Y, int64_t n, int32_t epochs, int32_t batch,
                       float lr, uint64_t seed, double *final_loss);

#ifdef __cplusplus
}
#endif
#endif /* RZ_H */
