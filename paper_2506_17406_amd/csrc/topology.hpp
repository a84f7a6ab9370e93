// Host-side mesh topology, global numbering and patch (subspace) lists.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "refelem.hpp"

namespace rz {

struct Topology {
  int d = 0;
  int64_t n_vertices = 0, n_cells = 0;
  std::vector<int64_t> cells;                  // n_cells x (d+1), sorted per cell
  std::vector<std::vector<int64_t>> ent;       // per dim l: n_ent x (l+1) sorted tuples
  std::vector<int64_t> n_ent;                  // per dim
  std::vector<std::vector<int64_t>> cell_ent;  // per dim l: n_cells x C(d+1, l+1) entity ids
  std::vector<int64_t> offset;                 // d+2 dof offsets per dimension
  int64_t n_dofs = 0, n_interior = 0;
  std::vector<int32_t> cell_dofs;              // n_cells x n_loc
};

// Throws std::invalid_argument (bad indices / repeated vertex) on bad input.
Topology build_topology(int d, int64_t n_vertices, int64_t n_cells, const int64_t *cells, const RefElement &el);

// A family of subspaces ("patches"): each patch is a list of columns, each
// column a sparse combination of global dofs (one entry with coefficient 1
// for a plain dof; several for a discrete-gradient column).
struct PatchSet {
  std::vector<int64_t> patch_col;  // n_patches + 1, ranges into columns
  std::vector<int64_t> col_ent;    // n_cols + 1, ranges into entries
  std::vector<int32_t> ent_dof;    // global dof per entry
  std::vector<double> ent_coef;    // coefficient per entry
  // per patch: the cells of its support, and per (patch, cell) the triples
  // (patch column, local dof of the cell, coefficient) that couple them
  std::vector<int64_t> pc_ptr;     // n_patches + 1, ranges into pc_cell
  std::vector<int32_t> pc_cell;    // cell of each (patch, cell) item
  std::vector<int64_t> pc_trip;    // n_items + 1, ranges into triples
  std::vector<int32_t> tr_col, tr_loc;
  std::vector<double> tr_coef;
  int64_t n_patches() const { return int64_t(patch_col.size()) - 1; }
  int64_t max_size() const;
};

// Which space decomposition the patches follow (Sec. 6).
//  DECOMP_PAPER: the interface patches of the default solvers -- H(grad):
//  vertex stars of X^0_Gamma; H(curl): edge stars of X^{1,I}_Gamma (plain)
//  and vertex-star potentials through the discrete gradient; H(div): edge
//  stars of X^2_Gamma.
//  DECOMP_VERTEX: PAFW(0)(X^k_Gamma) (eq:approx-sc-pafw) for every space:
//  per vertex, the dofs of the vertex and of the edges and faces containing it.
//  DECOMP_VERTEX_FULL: PAFW(0)(X^k) (eq:pafw): those vertex stars together
//  with the interior dofs of the cells containing the vertex.
//  DECOMP_PAPER_FULL: DECOMP_PAPER without the split -- every star also
//  holds the dofs (of the kinds it keeps) of the cells containing its centre,
//  and the H(curl) potentials the CG cell interiors: H(grad) PAFW(0)(X^0),
//  H(curl) PH(X^0, X^{1,I}), H(div) PAFW(1)(X^2).
//  DECOMP_HIPTMAIR (H(curl) only): PH(X^0_Gamma, X^1_Gamma)
//  (eq:pavarino_hiptmair with the split): the DECOMP_PAPER potentials and
//  edge stars of every kind of interface dof; DECOMP_HIPTMAIR_FULL:
//  PH(X^0, X^1), the same with the cell interiors.
//  DECOMP_TYPEI / DECOMP_TYPEI_FULL (H(curl), H(div)): the type-I
//  Hiptmair-Toselli decomposition PH(X^{k-1,I}, X^{k,I})
//  (eq:pavarino_hiptmair-novel) with / without the split.  H(curl): the same
//  as DECOMP_PAPER / DECOMP_PAPER_FULL.  H(div): edge-star potentials
//  curl X^{1,I}|star E (eq:hdiv-ph-reduced), and, full, the cell type-I
//  curls in them and the face stars X^{2,I}|star F.
enum Decomposition {
  DECOMP_PAPER = 0,
  DECOMP_VERTEX = 1,
  DECOMP_VERTEX_FULL = 2,
  DECOMP_PAPER_FULL = 3,
  DECOMP_HIPTMAIR = 4,
  DECOMP_HIPTMAIR_FULL = 5,
  DECOMP_TYPEI = 6,
  DECOMP_TYPEI_FULL = 7
};
// whether the decomposition keeps no interior-interface split (no Jacobi group)
inline bool decomposition_full(int dec) {
  return dec == DECOMP_VERTEX_FULL || dec == DECOMP_PAPER_FULL || dec == DECOMP_HIPTMAIR_FULL ||
         dec == DECOMP_TYPEI_FULL;
}
std::vector<PatchSet> build_patches(const Topology &top, const RefElement &el, Decomposition dec = DECOMP_PAPER);

// The standard H(div) Hiptmair-Toselli decomposition (eq:pavarino_hiptmair,
// k = 2; full: without the split): the face stars X^2|star F and the
// edge-star potentials curl X^1|star E with X^1 = NedTwo (t2, el2: its
// topology on the same cells and its element, degree p for RT_p and p + 1 for
// BDM_p).  Returns the two sets; `second` receives, per set, the coupling of
// its columns to the NedTwo dofs (empty for the face stars), for the
// regularising mass of eq:local-potential-problem-added-mass.
std::vector<PatchSet> build_hdiv_hiptmair(const Topology &t, const RefElement &el, const Topology &t2,
                                          const RefElement &el2, bool full, std::vector<PatchSet> &second);

// Dirichlet boundary (Sec. 5): the dofs of every subsimplex of the marked
// facets (the facet, its edges and vertices), ascending.  flags: n_cells x
// (d+1), nonzero (c, j) marks the facet of input cell c (cells_in, the
// caller's vertex order) opposite its j-th vertex.  Throws
// std::invalid_argument when a marked facet belongs to two cells.
std::vector<int32_t> dirichlet_dofs(const Topology &top, const RefElement &el, const int64_t *cells_in,
                                    const uint8_t *flags);
// Restricts a patch family to X^k_{p,D}: drops every column with an entry on
// a removed dof (removed[g] != 0) and the patches left without columns.
void restrict_patches(PatchSet &ps, const std::vector<uint8_t> &removed);

// Whitney dofs (one per k-subsimplex, lem:basis-contains-whitney), ascending,
// and per cell the local Whitney dofs with their coarse indices.
void whitney_dofs(const Topology &top, const RefElement &el, std::vector<int32_t> &wdofs,
                  std::vector<int32_t> &cell_wloc, std::vector<int32_t> &cell_widx, int &n_wloc);

}  // namespace rz
