// Geometric multigrid V-cycle on the Whitney space W^k (the W^k solver of
// the paper's experiments, Sec. 7.1): host-side set-up of the hierarchy and
// a host V-cycle used to estimate the hybrid weight of the coarse group.
#pragma once
#include <cstdint>
#include <functional>
#include <vector>

#include "topology.hpp"

namespace rz {

// Compressed sparse rows (FP64 values).
struct Csr {
  int64_t n_rows = 0, n_cols = 0;
  std::vector<int64_t> ptr;
  std::vector<int32_t> col;
  std::vector<double> val;
};
// duplicates summed, columns ascending within a row
Csr csr_from_triplets(int64_t n_rows, int64_t n_cols, const std::vector<int64_t> &r, const std::vector<int32_t> &c,
                      const std::vector<double> &v);
Csr csr_transpose(const Csr &A);
Csr csr_multiply(const Csr &A, const Csr &B);
void csr_apply(const Csr &A, const double *x, double *y);  // y = A x

// One level of the hierarchy (level 0 is the problem's mesh).
struct MgLevel {
  Csr A;                       // level operator (Galerkin below level 0)
  Csr P, R;                    // prolongation from the next coarser level and R = P^T (not on the coarsest)
  std::vector<double> dinv;    // 1 / diag(A)
  // k = 1 (Hiptmair-Jacobi): vertex-hat gradients G (edges x vertices, +-1),
  // G^T, and 1 / (g_v^T A g_v)
  Csr G, Gt;
  std::vector<double> gdiag;
  // k = 2 (edge stars of W^2): per edge its faces, and the inverse of the
  // star's principal submatrix (m x m, row-major, concatenated)
  std::vector<int64_t> star_ptr, inv_off;
  std::vector<int32_t> star_face;
  std::vector<double> inv;
  double omega = 1.0;          // smoothing damping 1 / rho
};

struct MgHierarchy {
  int k = 0, nu = 2;
  std::vector<MgLevel> lev;    // finest first; the last one is solved directly
  std::vector<double> coarse_inv;  // dense inverse of the coarsest operator (row-major)
  int64_t n_coarse = 0;
};

// The Whitney prolongation from the coarse mesh (topology tc, vertex
// coordinates Xc) to the fine mesh (tf, Xf; the fine entities must lie in
// coarse cells): the fine Whitney dofs of every coarse Whitney form -- point
// values (k = 0), line integrals along the fine edge (k = 1), fluxes through
// the fine face (k = 2), orientations from the sorted vertex tuples.
// Throws std::invalid_argument when a fine entity lies in no coarse cell.
Csr whitney_prolongation(int k, const Topology &tf, const double *Xf, const Topology &tc, const double *Xc);

// Builds the hierarchy from the Whitney block AW of the problem's operator,
// the level topologies (finest first; tops[0] the problem's) and the level
// vertex coordinates (for the prolongations).
MgHierarchy build_multigrid(int k, const Csr &AW, const std::vector<const Topology *> &tops,
                            const std::vector<const double *> &X, int nu);

// x = one V-cycle applied to b (level-0 vectors).
void mg_cycle_host(const MgHierarchy &H, const double *b, double *x);

// (lambda_min + 3 lambda_max) / 4 of B A from the Lanczos matrix of up to 10
// preconditioned CG steps on A with b = 2u - 1, u from SplitMix64(seed) per
// entry (stopping early once ||r|| <= 1e-12 ||b||), the subspace weight of
// Sec. 7.1.
double lanczos_weight(int64_t n, const std::function<void(const double *, double *)> &applyA,
                      const std::function<void(const double *, double *)> &applyB, uint64_t seed);

}  // namespace rz
