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
// k: the pullback, 0 identity, 1 covariant Piola, 2 contravariant Piola
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
// A (B matrices N x N, N a multiple of 32) -> A^{-1} through Cholesky,
// L^{-1} (in Linv) and L^{-T} L^{-1}; work: chol_inverse_work(B, N) doubles
// for the split triangular-inverse sums (null: no splitting)
int64_t chol_inverse_work(int64_t B, int N);
void launch_chol_inverse(int64_t B, int N, double *A, double *Linv, int *status, double *work, hipStream_t s);
// patch inverses in the segmented upper layout (see seg_size)
void launch_pack_seg(int64_t B, int N, int E, const int32_t *sizes, const int64_t *off, const double *Ainv,
                     double *packed, hipStream_t s);
void launch_pack_tiles(int N, int n, const double *Ainv, double *tiles, hipStream_t s);

// ---- hot path (multi-column: column c of a vector at base + c * ld)
// position of row r of cell `cell` in the operator's cell-local result Yc
inline int64_t yc_index(int64_t ncp, int64_t cell, int r) {
  const int mb = r / 16, rr = r % 16;
  return (int64_t(mb) * ncp + (cell & ~int64_t(15))) * 16 + 64 * (rr / 4) + (cell & 15) + 16 * (rr % 4);
}
struct ApplyATables {
  int n, Q, NP, KP;         // local dofs, stacked matrices, padded rows, padded k
  const double *Afrag;      // fragment-ordered reference stack
  const double *w;          // n_cells x Q weights
  const int32_t *cell_dofs; // n_cells x n
  int64_t n_cells;
  const float *Afrag32;     // FP32 copies for the mixed-precision inner operator (or null)
  const float *w32;
  int nb1;                  // cells per wave (16 nb1) for single-column applies; 0: by occupancy
  int nb_all;               // cells per wave (16 nb_all) for every apply; 0: none
  // FP64 three-stage apply: cell-local work vectors (per column KP ncp and
  // NP ncp doubles, for up to ws_cols columns) and the dof -> (cell, row)
  // assembly lists (CSR over dofs, entries index Yc)
  int64_t ncp, n_dofs;
  double *Xc, *Yc;
  int ws_cols;
  const int64_t *asm_ptr;
  const int32_t *asm_ent;
  // Dirichlet boundary (or null): nonzero for the removed dofs, which the
  // gather reads as zero and the assembly leaves at zero (overwrite) or
  // untouched (accumulate)
  const uint8_t *dmask;
};
// y += A x for n_rhs columns (y zeroed by the caller), or y = A x with
// overwrite; st: per-column state (columns that are done are skipped) or
// null; lo: the FP32 copies.  [col0, col1): only these local columns of A_T
// take part (x is zero on the others: a restricted apply); y += alpha A x.
// row0 > 0: only the local rows from row0 and the global dofs
// from dof0 are updated (the trailing interior blocks of the local and
// global numberings).  clear_x: x is zeroed once the apply has read it (x
// must be writable; not with dof0 > 0).
void launch_apply_A(const ApplyATables &t, const double *x, int64_t ldx, double *y, int64_t ldy, int n_rhs,
                    const PcgState *st, hipStream_t s, bool lo = false, int col0 = 0, int col1 = -1,
                    double alpha = 1.0, int row0 = 0, int64_t dof0 = 0, bool overwrite = false,
                    bool clear_x = false);

// Patch inverse storage: row i of a patch of size m holds the columns
// [V floor(i/V), V ceil(m/V)) -- zero left of the diagonal and beyond m, the
// diagonal halved -- so every row is a whole number of aligned V-element
// (16-byte) segments: V = 2 for the FP64 inverses, V = 4 for their FP32 copies,
// V = 8 for bfloat16 copies.
constexpr int kMaxPatch = 2048;
int64_t seg_size(int m, int V);  // stored entries of one patch
// Patch sets whose largest patch exceeds kFoldMin dofs store their inverses
// in the folded layout instead: with h = ceil(m / 2) and hP = fold_hp (h
// rounded up, below), pair row k = 0 .. h holds 2 hP entries; position p < hP of its
// first half is A[k][p] for k <= p < h (row k of the leading h x h block)
// or A[h + p][h + k - 1] for p < k (column k - 1 of the trailing block's
// upper triangle), position p of its second half A[k][h + p] (row k of the
// off-diagonal block); the diagonal halved, entries beyond m zero.  Every
// upper-triangle entry is stored once, all pair rows have one length, and
// a lane's positions stand for fixed columns (p and h + p).
#ifndef RZ_FOLD_MIN
#define RZ_FOLD_MIN 128
#endif
constexpr int kFoldMin = RZ_FOLD_MIN;
// half-row length of the folded layout for entries of `esize` bytes --
// hP: h rounded up to a multiple of max(16 bytes, RZ_FOLD_ALIGN_EL
// entries): FP64 half rows start on 64-byte boundaries (measured 2-3%
// faster streams of the 625-855-dof star sets than 16-byte alignment),
// reduced-precision ones add at most 7 padding entries per half row
#ifndef RZ_FOLD_ALIGN_EL
#define RZ_FOLD_ALIGN_EL 8
#endif
__host__ __device__ inline int fold_hp(int m, int esize) {
  const int a = 16 / esize > RZ_FOLD_ALIGN_EL ? 16 / esize : RZ_FOLD_ALIGN_EL;
  return ((m + 1) / 2 + a - 1) / a * a;
}
int64_t fold_size(int m, int esize);  // stored entries of one patch, folded
void launch_pack_fold(int64_t B, int N, const int32_t *sizes, const int64_t *off, const double *Ainv,
                      double *packed, hipStream_t s);
// FP32 copy of the patch inverses (V = 4), from the FP64 layout (segmented,
// or folded when `fold`)
void launch_seg_to_float(int64_t n_patches, const int64_t *patch_col, const int64_t *off64, const int64_t *off32,
                         const double *A, float *B, bool fold, hipStream_t s);
// bfloat16 copy of the patch inverses (bits in uint16_t, round to nearest
// even) in the V = 8 layout
void launch_seg_to_bf16(int64_t n_patches, const int64_t *patch_col, const int64_t *off64, const int64_t *off16,
                        const double *A, uint16_t *B, bool fold, hipStream_t s);

struct PatchApply {
  int64_t n_patches, n_chunks;
  int64_t n_entries;        // stored entries of the set (FP64 copy)
  int max_size;
  int fold;                    // 1: the folded layout (max_size > kFoldMin), 0: segmented rows
  const int64_t *chunk_patch;  // patch of each work chunk
  const int32_t *chunk_rows;   // [r0, r1) row range (pair rows when folded) of each chunk
  const int64_t *patch_col, *col_ent, *inv_off;
  const int32_t *ent_dof;
  const double *ent_coef;
  const double *inv;        // segmented upper rows or folded pair rows per patch (V = 2)
  const float *inv32;       // FP32 copy (V = 4) for mixed precision, or null
  const int64_t *inv_off32; // its patch offsets
  const uint16_t *inv16;    // bfloat16 copy (V = 8), or null
  const int64_t *inv_off16;
  // multi-column solves of segmented sets on MFMA (see frag_size): the
  // inverses in fragment order (FP64 and/or bfloat16, or null), their patch
  // offsets, the result buffer (sum_size x columns; double or float), and
  // the set's dofs with their (patch column, coefficient) entries
  const double *frag64;
  const uint16_t *frag16;
  const float *frag32;
  const int64_t *frag_off64, *frag_off16, *frag_off32;
  void *zb;                    // results, dof-major: zb[pr * zb_cols + c]
  void *rt;                    // right-hand sides of the set's dofs, dof-major: rt[a * zb_cols + c]
  int zb_cols;                 // columns zb and rt hold (the MFMA path needs ncol <= zb_cols)
  int64_t sum_size, n_adof;
  const int32_t *ent_a;        // per map entry: the index a of its dof in adof
  const int32_t *adof, *apr;
  const int64_t *aptr;
  const double *acoef;
};
// entries of one patch inverse in MFMA fragment order (full MP x MP; MP = m
// rounded up to 16 for FP64 and FP32, 32 for bfloat16); kind 0 FP64, 1
// bfloat16, 2 FP32
int64_t frag_size(int m, int kind);
void launch_seg_to_frag(const PatchApply &pa, int kind, void *frag, const int64_t *frag_off, hipStream_t s);
// ---- Hodge Laplacians (Sec. 7.2): y = alpha A x (+ y), A in CSR with
// `lanes` (1, 4, 16 or 64) lanes per row; weights w[c, q] scaled by smass
// for q < qm (the mass family) and sderiv after; out = a x + b y + c z
// (null: zero); per-block partials of a . b
void launch_csr_spmv(int64_t n, const int64_t *ptr, const int32_t *col, const double *val, const double *x,
                     double *y, double alpha, bool accumulate, int lanes, hipStream_t s);
void launch_scale_weights(int64_t nc, int Q, int qm, const double *w, double smass, double sderiv, double *out,
                          hipStream_t s);
void launch_lincomb3(int64_t n, double a, const double *x, double b, const double *y, double c, const double *z,
                     double *out, hipStream_t s);
void launch_dot_part(int64_t n, const double *a, const double *b, double *part, int nparts, hipStream_t s);
// out = d .* x (elementwise; out may alias x)
void launch_diag_mul(int64_t n, const double *d, const double *x, double *out, hipStream_t s);

// Geometric multigrid V-cycle on W^k (device data; host-resident struct).
// Level l: operator A (CSR), prolongation P from level l+1 and R = P^T,
// relaxation data (k = 0: dinv; k = 1: dinv, vertex-hat gradients G and
// G^T, gdiag = 1 / (g^T A g); k = 2: edge stars with dense inverses), the
// damping omega, and work vectors (per column: n entries of b, x, t, z and
// nv of u).  The last level is solved with the dense inverse cinv.
struct MgDevLevel {
  int64_t n = 0;
  const int64_t *Ap = nullptr, *Pp = nullptr, *Rp = nullptr, *Gp = nullptr, *Gtp = nullptr, *sp = nullptr,
                *so = nullptr;
  const int32_t *Ac = nullptr, *Pc = nullptr, *Rc = nullptr, *Gc = nullptr, *Gtc = nullptr, *sf = nullptr;
  const double *Av = nullptr, *Pv = nullptr, *Rv = nullptr, *Gv = nullptr, *Gtv = nullptr, *sinv = nullptr;
  const double *dinv = nullptr, *gdiag = nullptr;
  int64_t nv = 0, nstar = 0;
  double omega = 1.0;
  double *b = nullptr, *x = nullptr, *t = nullptr, *z = nullptr, *u = nullptr;
};
struct MgDev {
  int k = 0, nu = 2;
  MgDevLevel lev[12];
  int L = 0;
  const double *cinv = nullptr;
};
// x0 = V-cycle(b0) for ncol columns (level-0 vectors at b0 + c ldb0, x0 + c ldx0)
void launch_mg_cycle(const MgDev &mg, const double *b0, int64_t ldb0, double *x0, int64_t ldx0, int ncol,
                     hipStream_t s);

struct CoarseApply {
  int nW, NT;               // coarse size, tiles per side
  const int32_t *wdofs;
  const double *tiles;      // upper tiles (I <= J), 64 x 64 each, row-major
  double *rW, *zW;          // work vectors (NT * 64 per column)
  const double *full;       // all NT x NT tiles in MFMA fragment order (many-column solves), or null
  const float *tiles32;     // FP32 copy of the upper tiles (mixed precision) or null
  const uint8_t *dmask;     // removed (Dirichlet) dofs read as zero by the coarse gather, or null
  const MgDev *mg = nullptr;  // the W^k solver is this V-cycle (null: the dense inverse in tiles)
  double wscale = 1.0;        // weight 1 / rho_W of the hybrid sweep's coarse correction (1: exact solve)
};
// builds CoarseApply::full from the packed upper tiles
void launch_coarse_expand(int NT, const double *tiles, double *full, hipStream_t s);
// The coarse correction kept in zW and added on the fly to the dofs
// off + t N (t < span / N): the Whitney dofs are every N-th dof of one
// entity-dimension block.
struct CoarseFold {
  const double *zW;
  int64_t off, span, N;
};

// z += sum_patches (scatter-add; z must hold the Jacobi part already)
void launch_patch_apply(const PatchApply &pa, const double *r, int64_t ldr, double *z, int64_t ldz, int ncol,
                        const PcgState *st, hipStream_t s, bool lo = false, double scale = 1.0);
void launch_coarse_tiles(const CoarseApply &ca, int ncol, const PcgState *st, hipStream_t s, bool lo = false);
void launch_to_float(int64_t n, const double *a, float *b, hipStream_t s);
void launch_axpy(int64_t n, const double *d, double *x, int64_t ldx, int ncol, hipStream_t s);
// the whole preconditioner, z = P^{-1} r (no state)
void launch_apply_P(const PatchApply *sets, int nsets, const CoarseApply &ca, int64_t n, int64_t off_I,
                    const double *dinv, const double *r, int64_t ldr, double *z, int64_t ldz, int ncol,
                    hipStream_t s, bool lo = false);

// ---- Krylov (RB block partials per column)
void launch_fill(double *y, int64_t n, int64_t ld, int ncol, const PcgState *st, hipStream_t s);
void launch_copy(int64_t n, const double *a, int64_t lda, double *b, int64_t ldb, int ncol, hipStream_t s);
void launch_residual(int64_t n, const double *b, int64_t ldb, const double *Ax, double *r, int ncol, hipStream_t s);
void launch_dot(int64_t n, const double *a, int64_t lda, const double *b, int64_t ldb, const CoarseFold &cf,
                int npad, double *part, int RB, int ncol, const PcgState *st, hipStream_t s);
// outer (or null): columns whose outer state is done start as converged
void launch_pcg_start(const double *partB, const double *partR, int RB, double tol2, int maxit, PcgState *st,
                      int ncol, hipStream_t s, const PcgState *outer = nullptr);
void launch_update_xr(int64_t n, double *x, int64_t ldx, double *r, const double *p, const double *Ap,
                      const double *partZ, const double *partA, double *partR, int RB, int ncol, PcgState *st,
                      hipStream_t s);
void launch_check_jacobi(int64_t n, int64_t off_I, const double *dinv, const double *r, double *z,
                         const CoarseApply &ca, const double *partR, int RB, int ncol, PcgState *st, hipStream_t s);
void launch_update_p(int64_t n, double *p, const double *z, const CoarseFold &cf, int npad, double *Ap,
                     const double *partZ, int RB, int ncol, PcgState *st, hipStream_t s);

// ---- symmetric multiplicative hybrid sweep (Sec. 7.1)
// z = w1 D_I^{-1} r (interior), s = r; with st, after the convergence test
// hybrid sweep start: z = w1 D^-1 r on the interior (0 elsewhere), s = r,
// d = 0 (d and s have leading dimension n)
void launch_hyb_init(int64_t n, int64_t off_I, const double *dinv, double w1, const double *r, int64_t ldr, double *z,
                     int64_t ldz, double *sres, double *d, const double *partR, int RB, int ncol, PcgState *st,
                     hipStream_t s);
void launch_add(int64_t n, const double *d, double *z, int64_t ldz, int ncol, const PcgState *st, hipStream_t s);
void launch_jacobi_add(int64_t n, int64_t off_I, const double *dinv, double w1, const double *sres, double *z,
                       int64_t ldz, int ncol, const PcgState *st, hipStream_t s);
// rW = R_W r, zW = 0
void launch_coarse_gather(const CoarseApply &ca, const double *r, int64_t ldr, int ncol, hipStream_t s);
// d = R_W^T zW (d zero elsewhere beforehand), z += d
void launch_coarse_scatter2(const CoarseApply &ca, int64_t n, double *d, double *z, int64_t ldz, int ncol,
                            const PcgState *st, hipStream_t s);
void launch_axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s);
// y[rows[i]] = 0 for every column (the removed dofs of a Dirichlet boundary)
void launch_zero_rows(const int32_t *rows, int64_t nrows, double *y, int64_t ld, int ncol, hipStream_t s);
// A[idx[i]][idx[i]] = 1 in an N x N matrix (decoupled coarse rows of removed dofs)
void launch_set_diag(int N, const int32_t *idx, int n, double *A, hipStream_t s);
void launch_mask(int64_t n, int64_t lo, int64_t hi, double *y, hipStream_t s);

}  // namespace rz
