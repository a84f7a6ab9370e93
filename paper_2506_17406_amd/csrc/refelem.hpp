// Host-side construction of the paper's orthogonality-promoting reference
// elements (FP64).  See refelem.cpp for the method and its citations.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "linalg.hpp"

namespace rz {

enum Family { FAM_CG = 0, FAM_NED = 1, FAM_NEDTWO = 2, FAM_RT = 3, FAM_BDM = 4 };
enum DofKind { KIND_W = 0, KIND_I = 1, KIND_II = 2 };

struct LocalDof {
  int entity_dim;    // dimension of the subsimplex the dof belongs to
  int entity_index;  // index among the subsimplices of that dimension
  int kind;          // DofKind
  int j;             // index within (entity, kind)
};

struct RefElement {
  int d = 0, k = 0, p = 0;
  Family fam = FAM_CG;
  int n = 0;                    // local dofs
  int Q = 0;                    // stacked reference matrices
  std::vector<LocalDof> dofs;   // local dof order (entity-major)
  std::vector<int> per_entity;  // dofs per entity of dimension 0..d
  std::vector<int> kind_start;  // per dimension: first within-entity index of W / I / II (3 each)
  std::vector<double> R;        // Q x n x n, row-major
  double cond_probe = 1.0;      // worst conditioning of a canonicalisation probe matrix
  double min_cluster_gap = 1e300;  // smallest relative gap between distinct eigenvalues
};

// Builds the element for (dimension d, family, degree p): CG/NED/RT in 2D
// and 3D, the second-kind NEDTWO/BDM in 3D.
// Throws std::runtime_error when a numerical check of the construction fails.
RefElement build_reference(int d, Family fam, int p);

// The exterior derivative from the first-kind 3D family `from` to the next
// one (CG -> NED, NED -> RT) on the reference cell in the two elements'
// bases: n_to x n_from, row-major (Sec. 7.2; lem:d-preserves-basis-functions
// makes it the signed incidence on the Whitney functions).
std::vector<double> derivative_reference(int d, Family from, Family to, int p);

// The divergence RT_p -> DG_{p-1} on the reference cell: n_dg x n_rt
// row-major, the coefficients of div phi_j in the L2-orthonormal basis of
// P_{p-1} (the DG_{p-1} basis).
std::vector<double> divergence_reference_dg(int d, int p);

// Equilateral reference simplex of edge length 2 centred at the origin.
void eq_vertices(int d, double *out /* (d+1) x d */);

}  // namespace rz
