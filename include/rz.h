/* rz.h -- C ABI of the MI355X (gfx950) Riesz-map solver.
 *
 * Method: Brubeck, Farrell, Kirby & Parker, "Fast solvers for the high-order
 * FEM simplicial de Rham complex" (arXiv:2506.17406).
 *
 * Problem (Sec. 2, eq:weak-form): find u in X^k_p(T_h) with
 *     (u, beta v) + (d^k u, alpha d^k v) = F(v)   for all v in X^k_p(T_h),
 * for H(grad) (k = 0, CG_p), H(curl) (k = 1, Ned_p first kind) and H(div)
 * (k = 2 in 3D, k = 1 in 2D; RT_p first kind), on a conforming simplicial
 * mesh (triangles or tetrahedra), with natural (pure Neumann) boundary
 * conditions, or on X^k_{p,D} with a Dirichlet part Gamma_D of the
 * boundary (rz_options.dirichlet_facet; Sec. 5).  F is given as its load
 * vector b_i = F(phi_i) in the paper's orthogonality-promoting basis
 * (Sec. 3, eq:abstract-dofs; Sec. 4,
 * eq:reference-basis).  The discrete system A x = b is solved by
 * preconditioned conjugate gradients (Sec. 7.1) with the interior-interface
 * split additive Schwarz preconditioners of Sec. 6:
 *   H(grad)  PAFW(0)(X^0_Gamma) + J(X^0_I)          (eq:approx-sc-pafw)
 *   H(curl)  PH(X^0_Gamma, X^{1,I}_Gamma) + J(X^1_I) (eq:hcurl-decomp)
 *   H(div)   PAFW(1)(X^2_Gamma) + J(X^2_I)           (eq:hdiv-decomp)
 * In 2D, RT_p is the quarter turn R v = (v_1, -v_0) of Ned_p (the remark
 * after eq:hdiv-dofs: its dofs are the H(curl) ones with n = R t and
 * curl = R grad), so the two 2D spaces have the same numbering, the same
 * matrices and the H(curl) decompositions with the dimensions shifted (an
 * edge star holds the edge's Whitney dof; the vertex-star potentials the
 * vertex function and the CG edge dofs).
 * each with an exact solve on the Whitney coarse space W^k.
 *
 * Numbering (host-exported, see rz_export_topology): each cell's vertices are
 * sorted by global number; edges and faces are the sorted vertex tuples,
 * numbered in lexicographic order; global dofs are entity-major -- all vertex
 * dofs, then edges, faces, and the cell interiors last (contiguous) -- with
 * dof = offset(dim) + entity_id * N_dim + j and, within an entity, the
 * Whitney dof, the type-I dofs, then the type-II dofs.
 *
 * Memory and streams.  Vectors passed to rz_apply_A / rz_apply_P / rz_solve
 * are caller-owned DEVICE pointers to float64, column-major with leading
 * dimension ld >= n_dofs (one column per right-hand side).  The library never
 * retains or frees them.  Work is enqueued on the HIP stream passed in
 * (NULL = the default stream); apply calls return without synchronising,
 * rz_solve returns after the solve has finished.  Mesh arrays are host
 * pointers, copied during rz_setup.  A handle owns all its device memory,
 * is not thread-safe, and distinct handles are independent.
 *
 * Errors.  Every int-returning call returns 0 on success or one of the
 * negative RZ_ERR_* codes; rz_last_error() gives a thread-local message for
 * the last failure.  No C++ exception crosses this interface.
 */
#ifndef RZ_H
#define RZ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  RZ_OK = 0,
  RZ_ERR_ARG = -1,              /* bad pointer, size, alpha < 0, beta <= 0, dim */
  RZ_ERR_UNSUPPORTED = -2,      /* (dim, space, degree) outside CG, Ned, RT in 2D / 3D, NedTwo, BDM in 3D, 1 <= p <= 10 */
  RZ_ERR_MESH = -3,             /* vertex index out of range or repeated in a cell */
  RZ_ERR_DEGENERATE_CELL = -4,  /* |det J_T| <= 1e-12 h^d */
  RZ_ERR_NOT_SPD = -5,          /* non-positive pivot in a patch or coarse Cholesky */
  RZ_ERR_NO_CONVERGENCE = -6,   /* max_iter reached; info is still filled */
  RZ_ERR_BREAKDOWN = -7,        /* p^T A p <= 0 or a non-finite CG scalar */
  RZ_ERR_DEVICE = -8,           /* HIP runtime error */
  RZ_ERR_OOM = -9               /* device allocation failed */
};

/* The space: one of the constants below, passed as a 32-bit integer (an
 * out-of-range value is an argument error, never undefined behaviour).
 * RZ_HCURL2 and RZ_HDIV2 are the second-kind spaces NedTwo_p and BDM_p
 * (eq:second-kind-def; tetrahedra only): all of P_p^3, with the dofs of
 * eq:hcurl-dofs / eq:hdiv-dofs whose type-II moments come from the next-lower
 * space of the second-kind sequence (CG_{p+1} for NedTwo_p, NedTwo_{p+1} for
 * BDM_p, the remark after eq:hdiv-dofs).  They take the decompositions of
 * RZ_HCURL and RZ_HDIV, the potentials from those lower spaces, and the
 * exact coarse solver only (RZ_COARSE_MG -> RZ_ERR_UNSUPPORTED). */
enum { RZ_HGRAD = 0, RZ_HCURL = 1, RZ_HDIV = 2, RZ_HCURL2 = 3, RZ_HDIV2 = 4 };
typedef int32_t rz_space;

typedef struct {
  int32_t dim;            /* 2 or 3 */
  int64_t n_vertices;
  const double *coords;   /* host, n_vertices x dim, row-major */
  int64_t n_cells;
  const int64_t *cells;   /* host, n_cells x (dim+1) vertex numbers, any order */
} rz_mesh;

/* Arithmetic of rz_solve.  RZ_FP64: PCG entirely in FP64.  RZ_FP32_PC: PCG
 * with the FP64 operator and vectors; the preconditioner reads FP32 copies
 * of the patch and coarse inverses (accumulating in FP64), so it is a fixed
 * symmetric operator and no refinement is needed.  RZ_BF16_PC: FP64 PCG
 * (FP64 operator, vectors and inner products) whose preconditioner reads
 * bfloat16 copies of the patch inverses (rounded to nearest through FP32; a
 * quarter of the FP64 bytes; each patch product accumulates in FP32, far
 * below the 2^-9 rounding of the entries), the FP32 coarse copy, and applies
 * the FP32 operator copies inside the hybrid sweep; the preconditioner is
 * then SPD only up to FP32 rounding, which may cost a few iterations.
 * RZ_FP32_IR:
 * iterative refinement -- the residual b - A x and the update x += d are
 * FP64; each correction d solves A d = r by PCG to inner_rtol whose operator
 * and preconditioner applies read FP32 copies of the reference tables,
 * weights, patch inverses and coarse inverse (FP32 MFMA, FP32 accumulation
 * inside a cell, FP64 assembly and FP64 Krylov vectors and inner products).
 * The copies are rounded from the FP64 factors built at setup.  If an outer
 * step contracts the true residual by less than a factor 2 the remaining
 * corrections use the FP64 applies. */
typedef enum { RZ_FP64 = 0, RZ_FP32_IR = 1, RZ_FP32_PC = 2, RZ_BF16_PC = 3 } rz_precision;

/* Preconditioner form (Sec. 6 and Sec. 7.1).  RZ_PC_ADDITIVE: the additive
 * Schwarz method of the theory, Jacobi + interface patches + coarse summed.
 * RZ_PC_HYBRID: the symmetric multiplicative hybrid of the experiments --
 * the groups X_I (point-Jacobi), X_Gamma (the additive interface patches)
 * and W (exact coarse solve) applied in the order I, Gamma, W, Gamma, I, each
 * correction z += rho_m^{-1} B_m (r - A z), with rho_m = (lambda_min +
 * 3 lambda_max) / 4 estimated at setup from 10 CG steps on the group
 * (SplitMix64 right-hand side, seeds 0x5EED1000 interior and 0x5EED2000
 * interface; rho = 1 for the exact coarse solve and for an empty group).
 * Costs about 1.5 extra operator applies and a second patch pass per
 * application; takes 2-3 times fewer PCG iterations. */
typedef enum { RZ_PC_ADDITIVE = 0, RZ_PC_HYBRID = 1 } rz_pc;

/* Space decomposition of the preconditioner (Sec. 6).  RZ_DECOMP_PAPER: the
 * interior-interface split solvers the paper recommends -- H(grad)
 * PAFW(0)(X^0_Gamma) + J(X^0_I) (eq:approx-sc-pafw), H(curl)
 * PH(X^0_Gamma, X^{1,I}_Gamma) + J(X^1_I) (vertex-star potentials through
 * the discrete gradient plus type-I edge stars, eq:hcurl-decomp), H(div)
 * PAFW(1)(X^2_Gamma) + J(X^2_I) (edge stars, eq:hdiv-decomp).
 * RZ_DECOMP_VERTEX: the comparator PAFW(0)(X^k_Gamma) + J(X^k_I) for every
 * space -- one patch per vertex with the dofs of the vertex and of the edges
 * and faces containing it (for H(grad) the same as RZ_DECOMP_PAPER).
 * RZ_DECOMP_VERTEX_FULL: the comparator without the split, PAFW(0)(X^k)
 * (eq:pafw) -- the vertex stars also hold the interior dofs of the cells
 * containing the vertex, and there is no Jacobi group (the hybrid sweep is
 * stars, W, stars).  Its patches grow like p^d rather than p^(d-1): a patch
 * larger than 2048 dofs (3D: H(grad) p > 8, H(curl) and H(div) p > 5) is
 * RZ_ERR_UNSUPPORTED.
 * RZ_DECOMP_PAPER_FULL: RZ_DECOMP_PAPER without the split -- each star also
 * holds the dofs (of the kinds it keeps) of the cells containing its centre,
 * the H(curl) potentials the CG cell interiors, and there is no Jacobi group:
 * H(grad) PAFW(0)(X^0), H(curl) PH(X^0, X^{1,I}), H(div) PAFW(1)(X^2).
 * RZ_DECOMP_HIPTMAIR (H(curl) and H(div); H(grad) -> RZ_ERR_UNSUPPORTED):
 * the standard Hiptmair-Toselli decomposition with the split
 * (eq:pavarino_hiptmair).  H(curl): PH(X^0_Gamma, X^1_Gamma) + J(X^1_I), the
 * vertex-star potentials of RZ_DECOMP_PAPER and edge stars of every kind of
 * interface dof.  3D H(div): PH(X^1_Gamma, X^2_Gamma) + J(X^2_I), face stars
 * X^2|star F (the face's dofs) and edge-star potentials curl X^1|star E with
 * X^1 = NedTwo_p (NedTwo_{p+1} for BDM_p): one column per NedTwo dof of the
 * edge and its faces, the curl in the H(div) basis, and each local matrix
 * regularised by the NedTwo mass times 1e-8 beta
 * (eq:local-potential-problem-added-mass; its condition number is then about
 * 1e8, which the explicit inverse carries); pure Neumann only
 * (dirichlet_facet -> RZ_ERR_UNSUPPORTED).
 * RZ_DECOMP_HIPTMAIR_FULL: PH(X^0, X^1) or PH(X^1, X^2), the same with the
 * cell interiors (their dofs in the stars, their NedTwo dofs in the
 * potentials) and no Jacobi group.
 * RZ_DECOMP_TYPEI / RZ_DECOMP_TYPEI_FULL (H(curl) and H(div), else
 * RZ_ERR_UNSUPPORTED): the type-I Hiptmair-Toselli decomposition
 * PH(X^{k-1,I}, X^{k,I}) (eq:pavarino_hiptmair-novel) with / without the
 * split.  For H(curl) these equal RZ_DECOMP_PAPER / RZ_DECOMP_PAPER_FULL.
 * For H(div), split (eq:hdiv-ph-reduced): W^2 + J(X^2_I) + edge-star
 * potentials curl X^{1,I}_Gamma|star E -- the curl of the Whitney edge
 * function (signed face Whitney dofs) and the RT type-II dofs of the faces
 * containing the edge; full: the potentials also hold the RT type-II dofs of
 * the cells containing the edge, there are face stars X^{2,I}|star F (the
 * face's Whitney dof and the type-I dofs of its two cells), and no Jacobi
 * group.
 * The coarse space W^k is the same in all of them. */
typedef enum {
  RZ_DECOMP_PAPER = 0,
  RZ_DECOMP_VERTEX = 1,
  RZ_DECOMP_VERTEX_FULL = 2,
  RZ_DECOMP_PAPER_FULL = 3,
  RZ_DECOMP_HIPTMAIR = 4,
  RZ_DECOMP_HIPTMAIR_FULL = 5,
  RZ_DECOMP_TYPEI = 6,
  RZ_DECOMP_TYPEI_FULL = 7
} rz_decomposition;

/* Solver on the Whitney space W^k (the coarse space of every decomposition).
 * RZ_COARSE_EXACT: an exact solve with the explicit dense inverse of the
 * Whitney principal submatrix A[W, W] (weight 1 in the hybrid sweep).
 * RZ_COARSE_MG: the geometric multigrid V-cycle of the paper's experiments
 * (Sec. 7.1, fig:solver-diagram-PAFW, fig:solver-diagram-PH) over the mesh
 * hierarchy in rz_options.mg_meshes: Whitney prolongations between the
 * nested meshes (exact, since Whitney forms are nested), Galerkin operators
 * P^T A P below A[W, W], two damped relaxation steps before and after the
 * coarse correction -- point-Jacobi (W^0), Hiptmair-Jacobi, i.e. the
 * vertex-hat gradients plus point-Jacobi on the Whitney edge functions
 * (W^1, eq:hiptmair-smoothing at lowest order), edge-star patches (W^2) --
 * each step x += omega S (b - A x) with omega = 1 / rho, rho = (lambda_min +
 * 3 lambda_max) / 4 of S A from 10 CG steps (SplitMix64 right-hand side
 * seeded 0x5EED3000 + level); an explicit inverse on the coarsest mesh.  In
 * the hybrid sweep the cycle gets its own weight rho_W by the same rule
 * (seed 0x5EED4000).  Tetrahedra and triangles (in 2D, H(div) RT_p uses
 * the H(curl) prolongation and smoother: its Whitney functions are the
 * quarter turns of Ned_p's, so its flux dofs prolong like circulations);
 * first-kind spaces and pure Neumann problems only (RZ_ERR_UNSUPPORTED
 * otherwise); RZ_ERR_MESH when the hierarchy does not match the problem's
 * mesh or is not nested. */
typedef enum { RZ_COARSE_EXACT = 0, RZ_COARSE_MG = 1 } rz_coarse;

typedef struct {
  double alpha;           /* coefficient of (d u, d v), >= 0 */
  double beta;            /* coefficient of (u, v), > 0 */
  int32_t max_iter;       /* PCG iteration cap, per inner solve under refinement (<= 0: 1000) */
  int32_t precision;      /* rz_precision */
  double inner_rtol;      /* refinement: relative residual of each correction solve (<= 0: 3e-3,
                           * about the contraction one FP32-operator correction can give) */
  int32_t pc;             /* rz_pc */
  int32_t eager;          /* nonzero: rz_solve launches every kernel directly; 0: its PCG iteration
                             chunks are captured into HIP graphs (per solution vector and column
                             count) and replayed, on a stream of the handle ordered after and
                             before the caller's stream */
  int32_t decomposition;  /* rz_decomposition (0: RZ_DECOMP_PAPER) */
  const uint8_t *dirichlet_facet; /* NULL: pure Neumann.  Else host, n_cells x (dim+1): a nonzero entry
                             (c, j) puts the facet of cell c opposite its j-th vertex (in the order of
                             mesh->cells) on the Dirichlet boundary Gamma_D; it must be a boundary facet
                             (RZ_ERR_MESH otherwise).  The problem is then posed on X^k_{p,D}: as in
                             Sec. 5, every basis function tied to a subsimplex of Gamma_D (the facets, their
                             edges and vertices) is removed -- the remaining functions are those with zero
                             trace on Gamma_D.  The removed dofs keep their numbers (rz_dirichlet_dofs lists
                             them); rz_apply_A and rz_apply_P read their entries as zero and write zero
                             there, and rz_solve ignores b and returns x = 0 on them.  The preconditioner's
                             patches, potentials and coarse space are restricted the same way (columns that
                             touch a removed dof are dropped). */
  int32_t coarse;         /* rz_coarse: the solver on the Whitney space W^k (0: RZ_COARSE_EXACT) */
  int32_t mg_levels;      /* RZ_COARSE_MG: number of meshes in mg_meshes (>= 2) */
  const rz_mesh *mg_meshes; /* RZ_COARSE_MG: the nested hierarchy, finest first, host.  mg_meshes[0] has the
                             problem's vertices (same count and numbering) and cells (same list), with the
                             vertex positions at which the hierarchy is nested (the problem's own
                             coordinates may be a perturbation of them); every entity of mesh l lies in a
                             cell of mesh l + 1.  Only the coordinates of these meshes and the cells of the
                             coarser ones are read. */
} rz_options;

typedef struct {
  int32_t status;         /* RZ_OK / RZ_ERR_NO_CONVERGENCE / RZ_ERR_BREAKDOWN */
  int32_t iterations;     /* PCG iterations taken (summed over the correction solves) */
  double rel_residual;    /* FP64: ||r_k||_2 / ||b||_2 of the recursively updated residual;
                             refinement: ||b - A x||_2 / ||b||_2 with the FP64 operator */
  double cond_estimate;   /* Lanczos estimate of kappa(P^{-1} A) from the CG coefficients
                             (of the first correction solve under refinement) */
  double solve_ms;        /* wall time of the iteration loop (rz_batch_solve: from the start of the batch
                             to the host seeing this problem finish) */
  int32_t outer_iterations; /* refinement steps (0 for RZ_FP64) */
  double setup_ms;        /* wall time of the handle's rz_setup (reference build, numbering, patch and
                             coarse assembly and factorisation, hybrid weights) */
} rz_info;

typedef struct rz_problem rz_problem;

/* Builds the reference element (Sec. 3-4) on the host, the numbering and the
 * patches (Sec. 6), uploads them, and assembles and factors the patch and
 * coarse matrices on the device in FP64 (plus the reduced-precision copies
 * that opts->precision reads).  opts may be NULL (alpha = beta = 1, FP64).
 * On success *out receives a new handle. */
int rz_setup(const rz_mesh *mesh, int32_t degree, rz_space space, const rz_options *opts,
             void *hip_stream, rz_problem **out);

/* Sizes: global dofs, interior dofs (the trailing block), local dofs per cell,
 * number of stacked reference matrices.  Any output pointer may be NULL. */
int rz_sizes(const rz_problem *P, int64_t *n_dofs, int64_t *n_interior, int32_t *n_loc, int32_t *Q);

/* y = A x (the matrix-free operator of eq:weak-form: gather, stacked
 * reference-matrix contraction with per-cell geometric weights, scatter-add).
 * x, y: device, n_dofs x n_rhs, leading dimension ld; y is overwritten. */
int rz_apply_A(rz_problem *P, const double *x, double *y, int32_t n_rhs, int64_t ld, void *hip_stream);

/* z = P^{-1} r: point-Jacobi on the interior dofs, exact interface patch
 * solves and the exact coarse (Whitney) solve, combined as the handle's
 * rz_pc form (additive sum, or the symmetric multiplicative hybrid sweep).
 * r, z: device, n_dofs x n_rhs, leading dimension ld; z is overwritten. */
int rz_apply_P(rz_problem *P, const double *r, double *z, int32_t n_rhs, int64_t ld, void *hip_stream);

/* The FP32-copy applies, with the rz_apply_A / rz_apply_P argument
 * conventions (FP64 vectors in and out).  rz_apply_A_fp32 (RZ_FP32_IR and
 * RZ_BF16_PC handles): the reference tables, weights and x are rounded to FP32 and
 * contracted by FP32 MFMA (FP32 accumulation per cell); the cell results
 * are summed into each dof in FP64 in a fixed order.
 * rz_apply_P_fp32 (RZ_FP32_IR, RZ_FP32_PC and RZ_BF16_PC handles): the
 * preconditioner of rz_solve's iteration -- the reduced-precision patch
 * (FP32, or bfloat16 under RZ_BF16_PC) and FP32 coarse inverses with FP64
 * accumulation (FP32 within a bfloat16 patch), and under RZ_FP32_IR and
 * RZ_BF16_PC also the FP32 operator inside the hybrid sweep.  RZ_ERR_ARG for
 * a handle without the copies. */
int rz_apply_A_fp32(rz_problem *P, const double *x, double *y, int32_t n_rhs, int64_t ld, void *hip_stream);
int rz_apply_P_fp32(rz_problem *P, const double *r, double *z, int32_t n_rhs, int64_t ld, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): y = A x as
 * rz_apply_A computes it (same kernels, same result), with the operator's
 * cell-local work vectors in a static device array of 128 MiB that the
 * library holds on each GPU it runs on, instead of the handle's workspace
 * (which rz_apply_A grows on demand).  The call allocates nothing.  It needs
 * (KP + NP) * ncp * n_rhs * 8 bytes <= 128 MiB, where KP and NP are n_loc
 * rounded up to 4 and 16 and ncp the cell count rounded up to 256 (for
 * example Ned_6 on 24,576 cells: 86.5 MB per column); larger requests return
 * RZ_ERR_ARG with the sizes in rz_last_error().  x, y, n_rhs, ld and stream
 * as rz_apply_A.  Every call on one GPU shares that GPU's array and leaves
 * its last contents there: calls that overlap on one GPU (other streams,
 * threads or handles) race and must be ordered by the caller. */
int rz_apply_A_noalloc(rz_problem *P, const double *x, double *y, int32_t n_rhs, int64_t ld, void *hip_stream);

/* PCG on A X = B for n_rhs independent columns (each with its own CG
 * scalars and stopping test), from the initial guess in X, stopping column j
 * when its recursive residual satisfies ||r_j||_2 <= rtol ||b_j||_2 (under
 * RZ_FP32_IR: when its true FP64 residual does, checked after each
 * refinement step; a column with b_j = 0 is left unchanged).
 * B, X: device, n_dofs x n_rhs, leading dimension ld.  The columns share
 * every operator and preconditioner pass (the patch and coarse inverses are
 * streamed once for a group of columns).  info (host, n_rhs entries, may be
 * NULL) is filled on return; the return value is the first non-OK column
 * status. */
int rz_solve(rz_problem *P, const double *b, double *x, int32_t n_rhs, int64_t ld, double rtol, rz_info *info,
             void *hip_stream);

/* The preconditioner's patch families (the stream that dominates its
 * apply), one at a time.  rz_patch_set_info: the number of families of the
 * handle (*n_sets; H(curl) under RZ_DECOMP_PAPER: the edge stars, then the
 * vertex-star potentials), and for family `set` its patch count, largest
 * patch, the FP64 entries stored for its inverses (families of patches up
 * to 128 dofs: segmented upper rows, row i holding the columns from its
 * 16-byte segment on; larger ones: folded pair rows, ceil(m/2) + 1 rows of
 * 2 hP entries, hP = ceil(m/2) rounded up to 8) and the entries of the
 * packed upper triangles sum m (m + 1) / 2, and sum m.  Any output pointer
 * may be NULL; with only n_sets requested any `set` is accepted.
 * rz_patch_set_apply: z += sum over the patches m of the family of
 * R_m^T A_m^{-1} R_m r (the FP64 inverses; one pass of that family's solves
 * as inside rz_apply_P, Sec. 6).  r, z, n_rhs, ld, stream as rz_apply_P. */
int rz_patch_set_info(const rz_problem *P, int32_t set, int32_t *n_sets, int64_t *n_patches, int32_t *max_size,
                      int64_t *stored_entries, int64_t *packed_entries, int64_t *sum_size);
int rz_patch_set_apply(rz_problem *P, int32_t set, const double *r, double *z, int32_t n_rhs, int64_t ld,
                       void *hip_stream);

/* The dofs removed by the handle's Dirichlet boundary (rz_options.
 * dirichlet_facet), ascending.  Pass dofs = NULL to query *n first; n = 0
 * for a pure Neumann problem. */
int rz_dirichlet_dofs(const rz_problem *P, int64_t *n, int32_t *dofs);

/* The hybrid group weights rho (host, 3 entries: interior, interface,
 * coarse; the coarse weight is 1 for the exact coarse solve); all 1 for an
 * additive handle. */
int rz_pc_weights(const rz_problem *P, double *rho);

/* Host copies of the numbering for parity checks: cell_dofs (n_cells x n_loc
 * int32, local dofs in the element's order) and the interface patches as
 * CSR over their ascending dof lists: patch_ptr (n_patches + 1), patch_dofs.
 * Pass NULL pointers to query *n_patches and *n_patch_entries first.
 * For H(curl) only the edge patches are listed (vertex potentials act through
 * the discrete gradient). */
int rz_export_topology(const rz_problem *P, int32_t *cell_dofs, int64_t *n_patches,
                       int64_t *n_patch_entries, int64_t *patch_ptr, int32_t *patch_dofs);

/* Host copy of the stacked reference matrices R_q (Q x n_loc x n_loc,
 * row-major), ordered: the value family then the derivative family; a vector
 * family lists the component pairs 00, 11, 22, 01, 02, 12 (3D; 00, 11, 01 in
 * 2D) with off-diagonal pairs symmetrised (R_ab + R_ba), a scalar family one
 * matrix (the 2D rot and div are scalars: Q = 4 for 2D Ned_p and RT_p).
 * A_T = sum_q w_{T,q} R_q with w from the Piola maps of
 * eq:pullback-3d-def. */
int rz_export_reference(const rz_problem *P, double *Rq);

/* Host-only (no device work): the stacked reference matrices of
 * (dim, degree, space) in the rz_export_reference layout.  Pass Rq = NULL to
 * query *n_loc and *Q first. */
int rz_reference(int32_t dim, int32_t degree, rz_space space, int32_t *n_loc, int32_t *Q, double *Rq);

/* Host-only (no device work): the numbering and plain patch lists that
 * rz_setup would build for this mesh, in the rz_export_topology layout.
 * Pass NULL output arrays to query *n_dofs, *n_patches and *n_patch_entries
 * first; cell_dofs needs n_cells x n_loc entries. */
int rz_numbering(const rz_mesh *mesh, int32_t degree, rz_space space, int64_t *n_dofs, int32_t *cell_dofs,
                 int64_t *n_patches, int64_t *n_patch_entries, int64_t *patch_ptr, int32_t *patch_dofs);

/* Host-only (no device work): the patch lists of the first patch family
 * that rz_setup builds under the given rz_decomposition, in the
 * rz_export_topology layout (ascending dofs per patch; for H(curl) under
 * the potential-space decompositions the edge patches).  Pass NULL patch_ptr / patch_dofs to
 * query *n_patches and *n_patch_entries first.  Errors as rz_numbering,
 * RZ_ERR_ARG for an unknown decomposition, and RZ_ERR_UNSUPPORTED for a
 * decomposition not built for the space.  Under RZ_DECOMP_TYPEI for H(div)
 * the first family is the potentials: each patch lists the dofs its columns
 * combine, column by column. */
int rz_patch_lists(const rz_mesh *mesh, int32_t degree, rz_space space, int32_t decomposition, int64_t *n_patches,
                   int64_t *n_patch_entries, int64_t *patch_ptr, int32_t *patch_dofs);

void rz_destroy(rz_problem *P);

/* ---- Hodge Laplacians (Sec. 7.2, eq:hodge-laplace)
 * The mixed problem on X^{k-1} x X^k with natural boundary conditions,
 * k = 1 (CG_p x Ned_p), k = 2 (Ned_p x RT_p) or k = 3 (RT_p x DG_{p-1},
 * the mixed Poisson problem, K_3 = 0), in the two bases:
 *   [ -M_{k-1}   D^T M_k ] [sigma]   [b_0]
 *   [  M_k D     K_k     ] [  u  ] = [b_1],
 * M the mass matrices, K_k the matrix of (d u, d v) and D the exterior
 * derivative in the X^k basis (the discrete complex is exact).  Vectors are
 * [sigma (n0 entries); u (n1)], caller-owned device FP64 arrays.
 * rz_hodge_setup: builds two Riesz-map handles for the block-diagonal
 * weighted Riesz-map preconditioner of eq:augmented-lagrangian,
 * (sigma, tau) + gamma (d sigma, d tau) on X^{k-1} and gamma^{-1} (u, v) +
 * (d u, d v) on X^k, each applied as one application of the handle's
 * Schwarz preconditioner (opts: pc form, decomposition, coarse solver and
 * max_iter as for rz_setup; NULL: the hybrid form; RZ_FP64 only, no
 * Dirichlet facets -> RZ_ERR_UNSUPPORTED), and D on the device.  gamma > 0
 * (RZ_ERR_ARG otherwise); k outside 1..3 -> RZ_ERR_UNSUPPORTED.  For
 * k = 3 the DG_{p-1} dofs are numbered cell by cell (cell c owns n_dg = p
 * (p+1) (p+2) / 6 consecutive dofs, cells in input order) and carry the
 * L2-orthonormal basis of P_{p-1} on the reference cell pulled back as a
 * 3-form, so M_3 is diagonal (1 / |det J_c|) and B_1 = gamma |det J_c| is
 * the exact inverse of gamma^{-1} M_3 (the paper's exact solver on X^3).
 * rz_hodge_apply: y = A x.  rz_hodge_apply_P: z = blockdiag(B_0, B_1) r.
 * rz_hodge_solve: preconditioned MINRES from x = 0 until the preconditioned
 * residual norm falls to rtol times its initial value (the paper's MINRES
 * test), at most max_iter iterations (RZ_ERR_NO_CONVERGENCE, info still
 * filled); info: status, iterations, rel_residual (the preconditioned
 * residual ratio), solve_ms.  Calls on one handle must not overlap.
 * rz_derivative_reference (host only): the reference-cell derivative
 * matrix D_hat of the complex (k = 1: grad CG_p -> Ned_p, k = 2: curl
 * Ned_p -> RT_p, k = 3: div RT_p -> DG_{p-1} in that orthonormal basis),
 * n_to x n_from row-major, any pointer may be NULL. */
typedef struct rz_hodge rz_hodge;
int rz_hodge_setup(const rz_mesh *mesh, int32_t degree, int32_t k, double gamma, const rz_options *opts,
                   void *hip_stream, rz_hodge **out);
int rz_hodge_sizes(const rz_hodge *H, int64_t *n0, int64_t *n1);
int rz_hodge_apply(rz_hodge *H, const double *x, double *y, void *hip_stream);
int rz_hodge_apply_P(rz_hodge *H, const double *r, double *z, void *hip_stream);
int rz_hodge_solve(rz_hodge *H, const double *b, double *x, double rtol, rz_info *info, void *hip_stream);
void rz_hodge_destroy(rz_hodge *H);
int rz_derivative_reference(int32_t k, int32_t degree, int32_t *n_to, int32_t *n_from, double *D);

/* Tile shape of the operator apply's contraction: each wave multiplies the
 * reference stack into 16, 32 or 64 cells (more cells reuse each loaded
 * reference fragment more often, fewer keep more waves in flight).  The
 * default takes the largest that keeps >= 2048 waves in flight over the row
 * blocks an apply covers.  rz_set_apply_tiles(P, c, 0) fixes c cells per
 * wave for the single-column applies over all rows (the choice
 * rz_batch_create's autotuner makes; 0 restores the default);
 * rz_set_apply_tiles(P, c, 1) fixes it for every apply of the handle,
 * including the restricted applies of the hybrid sweep and multi-column
 * applies (0 restores the per-apply rule).  RZ_ERR_ARG unless c is 0, 16,
 * 32 or 64.  rz_get_apply_tiles returns the single-column choice (0: the
 * default rule). */
int rz_set_apply_tiles(rz_problem *P, int32_t cells_per_wave, int32_t every_apply);
int rz_get_apply_tiles(const rz_problem *P, int32_t *cells_per_wave);

/* Batches of problems of uneven size (different meshes, spaces, degrees,
 * precisions), solved together: each problem runs on a stream of the batch,
 * its PCG iterations in chunks of 8 that are captured into a HIP graph once
 * per problem and solution vector and then replayed (under RZ_FP32_IR the
 * outer residual checks run between the chunks of the correction solves);
 * the host starts a problem's next chunk as soon as its previous one has
 * completed.  At creation the operator apply of each problem without a
 * tile choice (rz_set_apply_tiles) is tuned: 16, 32 and 64 cells per wave
 * are timed and the fastest is kept if it beats the default rule by more
 * than 3%; the choice is reused for every later problem of the same (dim,
 * space, degree, cells, dofs, precision) in the process and, if the
 * environment variable RZ_TUNING_FILE names a writable file, read from and
 * appended to that file.  The problems stay owned by the caller, must
 * outlive the batch, and must not be used by other calls while the batch
 * solves.  Not thread-safe. */
typedef struct rz_batch rz_batch;
int rz_batch_create(rz_problem *const *problems, int32_t n, rz_batch **out);

/* Solves A_i x_i = b_i for every problem i (one right-hand side each) to
 * ||r_i|| <= rtol ||b_i||, from the initial guesses in x_i, each with its
 * handle's precision and preconditioner.  b, x: host arrays of n device
 * pointers (n_dofs_i doubles each).  Work starts after earlier work on
 * hip_stream and later work on hip_stream waits for it; returns when done.
 * info: host, n entries, may be NULL.  Returns the first non-OK status. */
int rz_batch_solve(rz_batch *B, const double *const *b, double *const *x, double rtol, rz_info *info,
                   void *hip_stream);
void rz_batch_destroy(rz_batch *B);

const char *rz_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RZ_H */
