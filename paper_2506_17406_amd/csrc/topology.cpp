// Mesh topology, entity-major numbering and the interface patches of Sec. 6.
//
// Orientation (Sec. 5, the global basis of Rognes et al.): cell vertices are
// sorted by global number and each local subsimplex with ascending local
// vertex tuple is the global subsimplex with the same (sorted) global tuple,
// so neighbouring cells agree on every shared trace without permutations or
// signs.  Numbering: all vertex dofs, then edges, faces and cell interiors
// (last, contiguous); entities of one dimension in lexicographic order of
// their sorted vertex tuples; dof = offset(dim) + id * N_dim + j.
#include "topology.hpp"

#include <algorithm>
#include <map>
#include <numeric>
#include <stdexcept>

namespace rz {

namespace {

std::vector<std::vector<int>> combos(int npts, int k) {
  std::vector<std::vector<int>> out;
  std::vector<int> sel(k);
  std::iota(sel.begin(), sel.end(), 0);
  while (true) {
    out.push_back(sel);
    int i = k - 1;
    while (i >= 0 && sel[i] == npts - k + i) --i;
    if (i < 0) break;
    ++sel[i];
    for (int j = i + 1; j < k; ++j) sel[j] = sel[j - 1] + 1;
  }
  return out;
}

}  // namespace

Topology build_topology(int d, int64_t nv, int64_t nc, const int64_t *cells, const RefElement &el) {
  Topology t;
  t.d = d;
  t.n_vertices = nv;
  t.n_cells = nc;
  const int nvc = d + 1;
  t.cells.assign(cells, cells + nc * nvc);
  for (int64_t c = 0; c < nc; ++c) {
    int64_t *cv = t.cells.data() + (c * nvc);
    for (int a = 0; a < nvc; ++a)
      if (cv[a] < 0 || cv[a] >= nv) throw std::invalid_argument("cell vertex index out of range");
    std::sort(cv, cv + nvc);
    for (int a = 1; a < nvc; ++a)
      if (cv[a] == cv[a - 1]) throw std::invalid_argument("repeated vertex in a cell");
  }
  t.ent.resize(d + 1);
  t.cell_ent.resize(d + 1);
  t.n_ent.assign(d + 1, 0);
  for (int l = 0; l <= d; ++l) {
    auto loc = combos(nvc, l + 1);
    const int ns = int(loc.size());
    auto &ce = t.cell_ent[l];
    ce.resize(nc * ns);
    if (l == 0) {
      t.n_ent[0] = nv;
      t.ent[0].resize(nv);
      std::iota(t.ent[0].begin(), t.ent[0].end(), 0);
      for (int64_t i = 0; i < nc * ns; ++i) ce[i] = t.cells[i];
      continue;
    }
    if (l == d) {
      t.n_ent[d] = nc;
      t.ent[d] = t.cells;
      for (int64_t c = 0; c < nc; ++c) ce[c] = c;
      continue;
    }
    const int w = l + 1;
    std::vector<int64_t> tup(nc * ns * w);
    for (int64_t c = 0; c < nc; ++c)
      for (int s = 0; s < ns; ++s)
        for (int a = 0; a < w; ++a) tup[(c * ns + s) * w + a] = t.cells[c * nvc + loc[s][a]];
    std::vector<int64_t> order(nc * ns);
    std::iota(order.begin(), order.end(), 0);
    auto less = [&](int64_t x, int64_t y) {
      for (int a = 0; a < w; ++a) {
        if (tup[x * w + a] != tup[y * w + a]) return tup[x * w + a] < tup[y * w + a];
      }
      return false;
    };
    std::sort(order.begin(), order.end(), less);
    int64_t id = -1;
    for (size_t i = 0; i < order.size(); ++i) {
      if (i == 0 || less(order[i - 1], order[i])) {
        ++id;
        for (int a = 0; a < w; ++a) t.ent[l].push_back(tup[order[i] * w + a]);
      }
      ce[order[i]] = id;
    }
    t.n_ent[l] = id + 1;
  }
  t.offset.assign(d + 2, 0);
  for (int l = 0; l <= d; ++l) t.offset[l + 1] = t.offset[l] + t.n_ent[l] * el.per_entity[l];
  t.n_dofs = t.offset[d + 1];
  t.n_interior = t.n_ent[d] * el.per_entity[d];
  if (t.n_dofs >= (int64_t(1) << 31)) throw std::invalid_argument("more than 2^31 dofs");
  t.cell_dofs.resize(nc * el.n);
  std::vector<int> nsub(d + 1);
  for (int l = 0; l <= d; ++l) nsub[l] = int(combos(nvc, l + 1).size());
  for (int64_t c = 0; c < nc; ++c)
    for (int i = 0; i < el.n; ++i) {
      const LocalDof &ld = el.dofs[i];
      const int l = ld.entity_dim;
      const int64_t e = t.cell_ent[l][c * nsub[l] + ld.entity_index];
      t.cell_dofs[c * el.n + i] =
          int32_t(t.offset[l] + e * el.per_entity[l] + el.kind_start[3 * l + ld.kind] + ld.j);
    }
  return t;
}

int64_t PatchSet::max_size() const {
  int64_t m = 0;
  for (int64_t p = 0; p + 1 < int64_t(patch_col.size()); ++p) m = std::max(m, patch_col[p + 1] - patch_col[p]);
  return m;
}

namespace {

// dofs of entity (l, e) of the given kind (-1: all kinds)
void entity_dofs(const Topology &t, const RefElement &el, int l, int64_t e, int kind, std::vector<int32_t> &out) {
  const int N = el.per_entity[l];
  const int64_t base = t.offset[l] + e * N;
  for (int j = 0; j < N; ++j) {
    int kj = KIND_W;
    for (int kk = 0; kk < 3; ++kk)
      if (el.kind_start[3 * l + kk] >= 0 && j >= el.kind_start[3 * l + kk]) kj = kk;
    if (kind < 0 || kj == kind) out.push_back(int32_t(base + j));
  }
}

struct Incidence {
  std::vector<std::vector<int64_t>> v_edges, v_faces, v_cells, e_faces, e_cells, f_cells;
};

Incidence incidence(const Topology &t) {
  Incidence in;
  const int d = t.d;
  in.v_edges.resize(t.n_vertices);
  in.v_faces.resize(t.n_vertices);
  in.v_cells.resize(t.n_vertices);
  for (int64_t e = 0; e < t.n_ent[1]; ++e)
    for (int a = 0; a < 2; ++a) in.v_edges[t.ent[1][e * 2 + a]].push_back(e);
  for (int64_t c = 0; c < t.n_cells; ++c)
    for (int a = 0; a <= d; ++a) in.v_cells[t.cells[c * (d + 1) + a]].push_back(c);
  in.e_cells.resize(t.n_ent[1]);
  if (d == 2)
    for (int64_t c = 0; c < t.n_cells; ++c)
      for (int s = 0; s < 3; ++s) in.e_cells[t.cell_ent[1][c * 3 + s]].push_back(c);
  if (d == 3) {
    in.e_faces.resize(t.n_ent[1]);
    for (int64_t f = 0; f < t.n_ent[2]; ++f) {
      for (int a = 0; a < 3; ++a) in.v_faces[t.ent[2][f * 3 + a]].push_back(f);
      // the three edges of face f are cell-edge ids of any cell; find them via sorted lookup
    }
    auto edge_id = [&](int64_t a, int64_t b) {
      auto &lst = in.v_edges[a];
      for (int64_t e : lst)
        if (t.ent[1][e * 2] == std::min(a, b) && t.ent[1][e * 2 + 1] == std::max(a, b)) return e;
      throw std::logic_error("edge not found");
    };
    for (int64_t f = 0; f < t.n_ent[2]; ++f) {
      const int64_t *v = t.ent[2].data() + (f * 3);
      in.e_faces[edge_id(v[0], v[1])].push_back(f);
      in.e_faces[edge_id(v[0], v[2])].push_back(f);
      in.e_faces[edge_id(v[1], v[2])].push_back(f);
    }
    for (int64_t c = 0; c < t.n_cells; ++c)
      for (int s = 0; s < 6; ++s) in.e_cells[t.cell_ent[1][c * 6 + s]].push_back(c);
    in.f_cells.resize(t.n_ent[2]);
    for (int64_t c = 0; c < t.n_cells; ++c)
      for (int s = 0; s < 4; ++s) in.f_cells[t.cell_ent[2][c * 4 + s]].push_back(c);
  }
  return in;
}

// Adds one patch given its columns (each a list of (dof, coef)) and the
// cells of its support; builds the (patch, cell) coupling triples.
void add_patch(PatchSet &ps, const Topology &t, const RefElement &el,
               const std::vector<std::vector<std::pair<int32_t, double>>> &cols, const std::vector<int64_t> &cells,
               std::vector<int32_t> &mark_col, std::vector<double> &mark_coef) {
  for (size_t j = 0; j < cols.size(); ++j) {
    for (auto &pr : cols[j]) {
      ps.ent_dof.push_back(pr.first);
      ps.ent_coef.push_back(pr.second);
      mark_col[pr.first] = int32_t(j);
      mark_coef[pr.first] = pr.second;
    }
    ps.col_ent.push_back(int64_t(ps.ent_dof.size()));
  }
  ps.patch_col.push_back(int64_t(ps.col_ent.size()) - 1);
  for (int64_t c : cells) {
    const int64_t before = int64_t(ps.tr_col.size());
    for (int i = 0; i < el.n; ++i) {
      const int32_t g = t.cell_dofs[c * el.n + i];
      if (mark_col[g] >= 0) {
        ps.tr_col.push_back(mark_col[g]);
        ps.tr_loc.push_back(i);
        ps.tr_coef.push_back(mark_coef[g]);
      }
    }
    if (int64_t(ps.tr_col.size()) > before) {
      ps.pc_cell.push_back(int32_t(c));
      ps.pc_trip.push_back(int64_t(ps.tr_col.size()));
    }
  }
  ps.pc_ptr.push_back(int64_t(ps.pc_cell.size()));
  for (auto &col : cols)
    for (auto &pr : col) mark_col[pr.first] = -1;
}

PatchSet empty_set() {
  PatchSet ps;
  ps.patch_col = {0};
  ps.col_ent = {0};
  ps.pc_ptr = {0};
  ps.pc_trip = {0};
  return ps;
}

}  // namespace

std::vector<PatchSet> build_patches(const Topology &t, const RefElement &el, Decomposition dec) {
  const int d = t.d;
  Incidence in = incidence(t);
  std::vector<int32_t> mark_col(t.n_dofs, -1);
  std::vector<double> mark_coef(t.n_dofs, 0.0);
  std::vector<PatchSet> out;
  auto plain_cols = [](std::vector<int32_t> &dofs) {
    std::sort(dofs.begin(), dofs.end());
    std::vector<std::vector<std::pair<int32_t, double>>> cols;
    for (int32_t g : dofs) cols.push_back({{g, 1.0}});
    return cols;
  };
  const bool full = decomposition_full(dec);
  const bool hiptmair = dec == DECOMP_HIPTMAIR || dec == DECOMP_HIPTMAIR_FULL;
  const bool typeI = dec == DECOMP_TYPEI || dec == DECOMP_TYPEI_FULL;
  // 2D RT_p is the quarter turn of 2D Ned_p: the same dofs, and the curl of a
  // CG function has the coefficients of its gradient, so it takes the H(curl)
  // decompositions
  // the second-kind spaces take the decompositions of the first-kind space of
  // the same form degree (their potentials come from the next-lower space of
  // the second-kind sequence: CG_{p+1}, NedTwo_{p+1}; entity_dofs reads the
  // per-entity counts from the element)
  const Family fam = (d == 2 && el.fam == FAM_RT) || el.fam == FAM_NEDTWO ? FAM_NED
                     : el.fam == FAM_BDM                                  ? FAM_RT
                                                                          : el.fam;
  if (hiptmair && fam != FAM_NED)
    throw std::runtime_error("the H(div) Hiptmair-Toselli decompositions are built by build_hdiv_hiptmair");
  if (typeI && fam == FAM_CG)
    throw std::runtime_error("the type-I Hiptmair-Toselli decompositions need H(curl) or H(div)");
  if (typeI && fam == FAM_RT) {
    // PH(X^{1,I}, X^{2,I}) (eq:pavarino_hiptmair-novel; split: eq:hdiv-ph-reduced)
    if (full) {
      // face stars X^{2,I}|star F: the face's Whitney dof and the type-I
      // dofs of the cells containing it
      PatchSet pf = empty_set();
      for (int64_t f = 0; f < t.n_ent[2]; ++f) {
        std::vector<int32_t> dofs;
        entity_dofs(t, el, 2, f, KIND_W, dofs);
        for (int64_t c : in.f_cells[f]) entity_dofs(t, el, 3, c, KIND_I, dofs);
        add_patch(pf, t, el, plain_cols(dofs), in.f_cells[f], mark_col, mark_coef);
      }
      out.push_back(std::move(pf));
    }
    // edge-star potentials curl X^{1,I}|star E in RT coefficients: the curl of
    // the Whitney edge function is, by Stokes, the signed sum of the Whitney
    // functions of the faces containing the edge (-1 where the edge is (a, c)
    // of the face (a, b, c), vertices ascending); the curls of the NedTwo
    // type-I functions are the RT type-II functions of the same entity and
    // index (lem:d-preserves-basis-functions)
    PatchSet pv = empty_set();
    for (int64_t e = 0; e < t.n_ent[1]; ++e) {
      const int64_t a0 = t.ent[1][e * 2], b0 = t.ent[1][e * 2 + 1];
      std::vector<std::vector<std::pair<int32_t, double>>> cols(1);
      for (int64_t f : in.e_faces[e]) {
        std::vector<int32_t> w;
        entity_dofs(t, el, 2, f, KIND_W, w);
        const int64_t *v = t.ent[2].data() + (f * 3);
        cols[0].push_back({w[0], (a0 == v[0] && b0 == v[2]) ? -1.0 : 1.0});
      }
      auto add_typeII = [&](int l, int64_t ent) {
        std::vector<int32_t> ii;
        entity_dofs(t, el, l, ent, KIND_II, ii);
        for (int32_t g : ii) cols.push_back({{g, 1.0}});
      };
      for (int64_t f : in.e_faces[e]) add_typeII(2, f);
      if (full)
        for (int64_t c : in.e_cells[e]) add_typeII(3, c);
      add_patch(pv, t, el, cols, in.e_cells[e], mark_col, mark_coef);
    }
    out.push_back(std::move(pv));
    return out;
  }
  if (dec == DECOMP_VERTEX || dec == DECOMP_VERTEX_FULL || fam == FAM_CG) {
    // vertex stars (eq:approx-sc-pafw; with the cell interiors, eq:pafw):
    // the entities containing the vertex carry the dofs whose support lies
    // in its star; entity_dofs adds nothing where the space has no dofs
    PatchSet ps = empty_set();
    for (int64_t v = 0; v < t.n_vertices; ++v) {
      std::vector<int32_t> dofs;
      entity_dofs(t, el, 0, v, -1, dofs);
      for (int64_t e : in.v_edges[v]) entity_dofs(t, el, 1, e, -1, dofs);
      if (d == 3)
        for (int64_t f : in.v_faces[v]) entity_dofs(t, el, 2, f, -1, dofs);
      if (full)
        for (int64_t c : in.v_cells[v]) entity_dofs(t, el, d, c, -1, dofs);
      add_patch(ps, t, el, plain_cols(dofs), in.v_cells[v], mark_col, mark_coef);
    }
    out.push_back(std::move(ps));
    return out;
  }
  if (fam == FAM_NED) {
    // edge stars of the type-I interface space X^{1,I}_Gamma (eq:hcurl-decomp),
    // or of every kind of dof (eq:pavarino_hiptmair); the full forms add the
    // dofs of those kinds of the cells containing the edge.  In 2D the faces
    // are the cells: an edge star holds the edge's Whitney dof (Hiptmair:
    // every edge dof) and, full, the cells' type-I (every) dofs
    const int kw = hiptmair ? -1 : KIND_W, ki = hiptmair ? -1 : KIND_I;  // type-I forms: as DECOMP_PAPER
    PatchSet pe = empty_set();
    for (int64_t e = 0; e < t.n_ent[1]; ++e) {
      std::vector<int32_t> dofs;
      entity_dofs(t, el, 1, e, kw, dofs);
      if (d == 3)
        for (int64_t f : in.e_faces[e]) entity_dofs(t, el, 2, f, ki, dofs);
      if (full)
        for (int64_t c : in.e_cells[e]) entity_dofs(t, el, d, c, ki, dofs);
      add_patch(pe, t, el, plain_cols(dofs), in.e_cells[e], mark_col, mark_coef);
    }
    out.push_back(std::move(pe));
    // vertex-star potentials: d of X^0_Gamma|star V through the discrete
    // gradient (lem:d-preserves-basis-functions): the vertex function maps to
    // +-1 on the Whitney dofs of its edges (+1 when V is the larger vertex),
    // a CG type-I dof to the Ned type-II dof of the same entity and index.
    PatchSet pv = empty_set();
    for (int64_t v = 0; v < t.n_vertices; ++v) {
      std::vector<std::vector<std::pair<int32_t, double>>> cols(1);
      for (int64_t e : in.v_edges[v]) {
        std::vector<int32_t> w;
        entity_dofs(t, el, 1, e, KIND_W, w);
        cols[0].push_back({w[0], t.ent[1][e * 2 + 1] == v ? 1.0 : -1.0});
      }
      for (int64_t e : in.v_edges[v]) {
        std::vector<int32_t> ii;
        entity_dofs(t, el, 1, e, KIND_II, ii);
        for (int32_t g : ii) cols.push_back({{g, 1.0}});
      }
      for (int64_t f : in.v_faces[v]) {
        std::vector<int32_t> ii;
        entity_dofs(t, el, 2, f, KIND_II, ii);
        for (int32_t g : ii) cols.push_back({{g, 1.0}});
      }
      if (full)  // the CG cell interiors: the Ned type-II cell dofs
        for (int64_t c : in.v_cells[v]) {
          std::vector<int32_t> ii;
          entity_dofs(t, el, d, c, KIND_II, ii);
          for (int32_t g : ii) cols.push_back({{g, 1.0}});
        }
      add_patch(pv, t, el, cols, in.v_cells[v], mark_col, mark_coef);
    }
    out.push_back(std::move(pv));
  } else if (fam == FAM_RT) {
    // edge stars of X^2_Gamma (eq:hdiv-decomp); full: PAFW(1)(X^2)
    PatchSet ps = empty_set();
    for (int64_t e = 0; e < t.n_ent[1]; ++e) {
      std::vector<int32_t> dofs;
      for (int64_t f : in.e_faces[e]) entity_dofs(t, el, 2, f, -1, dofs);
      if (full)
        for (int64_t c : in.e_cells[e]) entity_dofs(t, el, 3, c, -1, dofs);
      add_patch(ps, t, el, plain_cols(dofs), in.e_cells[e], mark_col, mark_coef);
    }
    out.push_back(std::move(ps));
  }
  return out;
}

std::vector<PatchSet> build_hdiv_hiptmair(const Topology &t, const RefElement &el, const Topology &t2,
                                          const RefElement &el2, bool full, std::vector<PatchSet> &second) {
  Incidence in = incidence(t);
  std::vector<int32_t> mark_col(t.n_dofs, -1), mark2(t2.n_dofs, -1);
  std::vector<double> mark_coef(t.n_dofs, 0.0), mcoef2(t2.n_dofs, 0.0);
  std::vector<PatchSet> out;
  second.clear();
  auto plain = [](std::vector<int32_t> &dofs) {
    std::sort(dofs.begin(), dofs.end());
    std::vector<std::vector<std::pair<int32_t, double>>> cols;
    for (int32_t g : dofs) cols.push_back({{g, 1.0}});
    return cols;
  };
  // face stars X^2|star F: the dofs of the face, and (full) of its cells
  PatchSet pf = empty_set();
  for (int64_t f = 0; f < t.n_ent[2]; ++f) {
    std::vector<int32_t> dofs;
    entity_dofs(t, el, 2, f, -1, dofs);
    if (full)
      for (int64_t c : in.f_cells[f]) entity_dofs(t, el, 3, c, -1, dofs);
    add_patch(pf, t, el, plain(dofs), in.f_cells[f], mark_col, mark_coef);
  }
  out.push_back(std::move(pf));
  second.push_back(empty_set());
  // edge-star potentials: one column per NedTwo dof of the edge, of the faces
  // containing it and (full) of its cells, holding the curl of that function
  // in the H(div) basis -- the Whitney edge function to the signed Whitney
  // functions of the faces (Stokes; -1 where the edge is (a, c) of the face
  // (a, b, c)), a type-I function to the type-II function of the same entity
  // and index (lem:d-preserves-basis-functions), a gradient to nothing; the
  // second set couples the same columns to the NedTwo dofs themselves
  PatchSet pv = empty_set(), p2 = empty_set();
  auto kind_at = [&](int l, int j) {
    int kj = KIND_W;
    for (int kk = 0; kk < 3; ++kk)
      if (el2.kind_start[3 * l + kk] >= 0 && j >= el2.kind_start[3 * l + kk]) kj = kk;
    return kj;
  };
  for (int64_t e = 0; e < t.n_ent[1]; ++e) {
    const int64_t a0 = t.ent[1][e * 2], b0 = t.ent[1][e * 2 + 1];
    std::vector<std::pair<int, int64_t>> ents{{1, e}};
    for (int64_t f : in.e_faces[e]) ents.push_back({2, f});
    if (full)
      for (int64_t c : in.e_cells[e]) ents.push_back({3, c});
    std::vector<std::vector<std::pair<int32_t, double>>> cols, cols2;
    for (auto [l, ent] : ents) {
      const int N2 = el2.per_entity[l];
      const int64_t base2 = t2.offset[l] + ent * N2;
      std::vector<int32_t> two;
      if (l >= 2) entity_dofs(t, el, l, ent, KIND_II, two);
      size_t nI = 0;
      for (int j = 0; j < N2; ++j) {
        cols2.push_back({{int32_t(base2 + j), 1.0}});
        std::vector<std::pair<int32_t, double>> col;
        const int kj = kind_at(l, j);
        if (kj == KIND_W) {
          for (int64_t f : in.e_faces[e]) {
            std::vector<int32_t> w;
            entity_dofs(t, el, 2, f, KIND_W, w);
            const int64_t *v = t.ent[2].data() + (f * 3);
            col.push_back({w[0], (a0 == v[0] && b0 == v[2]) ? -1.0 : 1.0});
          }
        } else if (kj == KIND_I) {
          if (nI >= two.size()) throw std::logic_error("type-I potential without a type-II image");
          col.push_back({two[nI++], 1.0});
        }
        cols.push_back(std::move(col));
      }
    }
    add_patch(pv, t, el, cols, in.e_cells[e], mark_col, mark_coef);
    add_patch(p2, t2, el2, cols2, in.e_cells[e], mark2, mcoef2);
  }
  out.push_back(std::move(pv));
  second.push_back(std::move(p2));
  return out;
}

std::vector<int32_t> dirichlet_dofs(const Topology &t, const RefElement &el, const int64_t *cells_in,
                                    const uint8_t *flags) {
  const int d = t.d;
  // facet (sorted tuple) -> number of cells containing it, and its entity id
  std::map<std::vector<int64_t>, int> count;
  auto facet = [&](int64_t c, int j) {
    std::vector<int64_t> f;
    for (int a = 0; a <= d; ++a)
      if (a != j) f.push_back(cells_in[c * (d + 1) + a]);
    std::sort(f.begin(), f.end());
    return f;
  };
  for (int64_t c = 0; c < t.n_cells; ++c)
    for (int j = 0; j <= d; ++j) ++count[facet(c, j)];
  std::vector<std::map<std::vector<int64_t>, int64_t>> id(d);
  for (int l = 0; l < d; ++l)
    for (int64_t e = 0; e < t.n_ent[l]; ++e)
      id[l][std::vector<int64_t>(t.ent[l].begin() + e * (l + 1), t.ent[l].begin() + (e + 1) * (l + 1))] = e;
  std::vector<uint8_t> mark(t.n_dofs, 0);
  for (int64_t c = 0; c < t.n_cells; ++c)
    for (int j = 0; j <= d; ++j) {
      if (!flags[c * (d + 1) + j]) continue;
      const std::vector<int64_t> f = facet(c, j);
      if (count[f] != 1)
        throw std::invalid_argument("Dirichlet facet " + std::to_string(j) + " of cell " + std::to_string(c) +
                                    " is not on the boundary");
      // every subsimplex of the facet: vertex subsets of size 1 .. d
      for (int l = 0; l < d; ++l)
        for (const auto &sub : combos(d, l + 1)) {
          std::vector<int64_t> key;
          for (int a : sub) key.push_back(f[a]);
          std::vector<int32_t> dofs;
          entity_dofs(t, el, l, id[l].at(key), -1, dofs);
          for (int32_t g : dofs) mark[g] = 1;
        }
    }
  std::vector<int32_t> out;
  for (int64_t g = 0; g < t.n_dofs; ++g)
    if (mark[g]) out.push_back(int32_t(g));
  return out;
}

void restrict_patches(PatchSet &ps, const std::vector<uint8_t> &removed) {
  PatchSet out = empty_set();
  for (int64_t p = 0; p < ps.n_patches(); ++p) {
    // kept columns and their new numbers
    std::vector<int32_t> newcol(ps.patch_col[p + 1] - ps.patch_col[p], -1);
    int32_t nk = 0;
    for (int64_t j = ps.patch_col[p]; j < ps.patch_col[p + 1]; ++j) {
      bool ok = true;
      for (int64_t e = ps.col_ent[j]; e < ps.col_ent[j + 1]; ++e) ok = ok && !removed[ps.ent_dof[e]];
      if (!ok) continue;
      newcol[j - ps.patch_col[p]] = nk++;
      for (int64_t e = ps.col_ent[j]; e < ps.col_ent[j + 1]; ++e) {
        out.ent_dof.push_back(ps.ent_dof[e]);
        out.ent_coef.push_back(ps.ent_coef[e]);
      }
      out.col_ent.push_back(int64_t(out.ent_dof.size()));
    }
    if (nk == 0) continue;
    out.patch_col.push_back(int64_t(out.col_ent.size()) - 1);
    for (int64_t it = ps.pc_ptr[p]; it < ps.pc_ptr[p + 1]; ++it) {
      const int64_t before = int64_t(out.tr_col.size());
      for (int64_t q = ps.pc_trip[it]; q < ps.pc_trip[it + 1]; ++q) {
        const int32_t nc = newcol[ps.tr_col[q]];
        if (nc < 0) continue;
        out.tr_col.push_back(nc);
        out.tr_loc.push_back(ps.tr_loc[q]);
        out.tr_coef.push_back(ps.tr_coef[q]);
      }
      if (int64_t(out.tr_col.size()) > before) {
        out.pc_cell.push_back(ps.pc_cell[it]);
        out.pc_trip.push_back(int64_t(out.tr_col.size()));
      }
    }
    out.pc_ptr.push_back(int64_t(out.pc_cell.size()));
  }
  ps = std::move(out);
}

void whitney_dofs(const Topology &t, const RefElement &el, std::vector<int32_t> &wdofs,
                  std::vector<int32_t> &cell_wloc, std::vector<int32_t> &cell_widx, int &n_wloc) {
  const int k = el.k;
  wdofs.clear();
  for (int64_t e = 0; e < t.n_ent[k]; ++e)
    wdofs.push_back(int32_t(t.offset[k] + e * el.per_entity[k] + el.kind_start[3 * k + KIND_W]));
  std::vector<int> loc;
  for (int i = 0; i < el.n; ++i)
    if (el.dofs[i].kind == KIND_W) loc.push_back(i);
  n_wloc = int(loc.size());
  cell_wloc = std::vector<int32_t>(loc.begin(), loc.end());
  cell_widx.resize(t.n_cells * n_wloc);
  int nsub = int(combos(t.d + 1, k + 1).size());
  for (int64_t c = 0; c < t.n_cells; ++c)
    for (int a = 0; a < n_wloc; ++a) {
      const LocalDof &ld = el.dofs[loc[a]];
      cell_widx[c * n_wloc + a] = int32_t(t.cell_ent[k][c * nsub + ld.entity_index]);
    }
}

}  // namespace rz
