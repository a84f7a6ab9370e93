// Device kernels of the Riesz-map solver (gfx950) and their host launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace rz {

// PCG state shared by the iteration kernels (device memory).
constexpr int kMaxIter = 4096;
struct PcgState {
  double rz, pAp, alpha, rr, bb, tol2, beta;
  int done, iter, status, maxit;
  double alphas[kMaxIter];
  double betas[kMaxIter];
};
enum { PCG_RUNNING = 0, PCG_CONVERGED = 1, PCG_MAXIT = 2, PCG_BREAKDOWN = 3 };

// ---- setup
void launch_weights(int d, int k, int64_t n_cells, const double *X, const double *Einv, double alpha, double beta,
                    double *w, int Q, hipStream_t s);
void launch_interior_diag(int64_t n_cells, int n, int Q, const double *R, const double *w, const int32_t *cell_dofs,
                          const int32_t *loc_interior, int n_int_loc, int64_t off_I, double *dinv, hipStream_t s);
void launch_pad_identity(int64_t B, int N, const int32_t *sizes, double *A, hipStream_t s);
void launch_patch_assemble(int64_t n_items, const int32_t *item_patch, const int32_t *item_cell,
                           const int64_t *item_trip, const int32_t *tr_col, const int32_t *tr_loc,
                           const double *tr_coef, int n, int Q, const double *R, const double *w, int N,
                           double *A, hipStream_t s);
// batched blocked Cholesky + inverse of B uniform N x N SPD matrices (N % 32 == 0)
void launch_chol_inverse(int64_t B, int N, double *A, double *Linv, int *status, hipStream_t s);
void launch_pack_upper(int64_t B, int N, const int32_t *sizes, const int64_t *off, const double *Ainv,
                       double *packed, hipStream_t s);
void launch_pack_tiles(int N, int n, const double *Ainv, double *tiles, hipStream_t s);

// ---- hot path
struct ApplyATables {
  int n, Q, NP, KP;         // local dofs, stacked matrices, padded rows, padded k
  const double *Afrag;      // fragment-ordered reference stack
  const double *w;          // n_cells x Q weights
  const int32_t *cell_dofs; // n_cells x n
  int64_t n_cells;
};
void launch_apply_A(const ApplyATables &t, const double *x, double *y, int n_rhs, int64_t ld,
                    const PcgState *st, hipStream_t s);
void launch_fill(double *y, int64_t n, double v, const PcgState *st, hipStream_t s);

struct PatchApply {
  int64_t n_patches, n_chunks;
  int max_size;
  const int64_t *chunk_patch;  // patch of each work chunk
  const int32_t *chunk_rows;   // [r0, r1) row range of each chunk
  const int64_t *patch_col, *col_ent, *inv_off;
  const int32_t *ent_dof;
  const double *ent_coef;
  const double *inv;        // packed upper rows per patch
};
void launch_patch_apply(const PatchApply &pa, const double *r, double *z, const PcgState *st, hipStream_t s);
void launch_jacobi(int64_t n_dofs, int64_t off_I, const double *dinv, const double *r, double *z,
                   const PcgState *st, hipStream_t s);
struct CoarseApply {
  int nW, NT;               // coarse size, tiles per side
  const int32_t *wdofs;
  const double *tiles;      // upper tiles (I <= J), 64 x 64 each, row-major
  double *rW, *zW;          // work vectors (NT * 64)
};
void launch_coarse_apply(const CoarseApply &ca, const double *r, double *z, const PcgState *st, hipStream_t s);

// The coarse correction kept in zW and added on the fly to the dofs
// off + t N (t < span / N): the Whitney dofs are every N-th dof of one
// entity-dimension block.
struct CoarseFold {
  const double *zW;
  int64_t off, span, N;
};

// ---- Krylov vector kernels
constexpr int kRedBlocks = 512;
void launch_dot_partial(int64_t n, const double *a, const double *b, double *part, const PcgState *st,
                        hipStream_t s);
void launch_pcg_init(PcgState *st, const double *part, const double *part2, double tol2, int maxit,
                     hipStream_t s);
void launch_set_rz(PcgState *st, const double *part, hipStream_t s);
void launch_finalize_alpha(PcgState *st, const double *part, hipStream_t s);
void launch_update_xr(int64_t n, double *x, double *r, const double *p, const double *Ap, double *part,
                      const PcgState *st, hipStream_t s);
void launch_finalize_rr(PcgState *st, const double *part, hipStream_t s);
void launch_finalize_beta(PcgState *st, const double *part, hipStream_t s);
void launch_update_p(int64_t n, double *p, const double *z, const PcgState *st, hipStream_t s);
void launch_residual(int64_t n, const double *b, const double *Ax, double *r, hipStream_t s);
void launch_copy(int64_t n, const double *a, double *b, hipStream_t s);
// fused iteration kernels: a reduction leaves per-block partials, the
// consuming kernel re-sums them in every block
void launch_dot2(int64_t n, const double *a, const double *b, const CoarseFold &cf, double *part,
                 const PcgState *st, hipStream_t s);
void launch_update_xr2(int64_t n, double *x, double *r, const double *p, const double *Ap, const double *partZ,
                       const double *partA, double *partR, PcgState *st, hipStream_t s);
void launch_check_jacobi(int64_t n, int64_t off_I, const double *dinv, const double *r, double *z,
                         const CoarseApply &ca, const double *partR, PcgState *st, hipStream_t s);
void launch_coarse_tiles(const CoarseApply &ca, const PcgState *st, hipStream_t s);
void launch_update_p2(int64_t n, double *p, const double *z, const CoarseFold &cf, double *Ap, const double *partZ,
                      PcgState *st, hipStream_t s);

}  // namespace rz
