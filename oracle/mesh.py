"""Global topology and dof numbering (Sec. 5 of the paper).

The global basis is the pullback of the reference basis through maps F_T that
preserve a fixed global orientation of every subsimplex (the Rognes et al.
construction the paper adopts at the start of Sec. 5).  Reading R5: each
cell's vertices are sorted by global vertex number and F_T sends reference
vertex m to the m-th smallest; a local subentity with ascending local vertex
tuple is then the global subentity with the same (sorted) global tuple, and
neighbouring cells induce the same parametrisation of it, so traces conform
with no permutation or sign.

Reading R6 (numbering): entity-major -- all vertex dofs, then edges, faces,
and the cell interiors last; entities of one dimension are numbered by the
lexicographic order of their sorted global vertex tuples (cells keep their
input order); global dof = offset(dim) + entity_id * N_dim + j with j the
within-entity local index (Whitney, type-I, type-II).
"""
from itertools import combinations

import numpy as np


class Topology:
    def __init__(self, coords, cells, el):
        self.coords = np.asarray(coords, dtype=float)
        cells = np.asarray(cells, dtype=np.int64)
        self.d = d = cells.shape[1] - 1
        self.n_cells = cells.shape[0]
        self.cells = np.sort(cells, axis=1)
        self.n_vertices = self.coords.shape[0]
        self.el = el
        # entities of every dimension
        self.ent_tuples = []
        self.cell_ent = []
        for l in range(d + 1):
            loc = list(combinations(range(d + 1), l + 1))
            if l == 0:
                tup = np.arange(self.n_vertices)[:, None]
                ids = self.cells.copy()
            elif l == d:
                tup = self.cells.copy()
                ids = np.arange(self.n_cells)[:, None]
            else:
                allt = self.cells[:, np.array(loc)]          # (nc, nloc, l+1)
                flat = allt.reshape(-1, l + 1)
                tup, inv = np.unique(flat, axis=0, return_inverse=True)
                ids = inv.reshape(self.n_cells, len(loc))
            self.ent_tuples.append(tup)
            self.cell_ent.append(ids)
        self.n_ent = [t.shape[0] for t in self.ent_tuples]
        # dofs per entity of each dimension and the within-entity kinds
        self.N = [0] * (d + 1)
        self.kinds = [[] for _ in range(d + 1)]
        for di in el.dofs:
            if di.entity_index == 0:
                self.N[di.entity_dim] += 1
                self.kinds[di.entity_dim].append(di.kind)
        self.offset = [0] * (d + 2)
        for l in range(d + 1):
            self.offset[l + 1] = self.offset[l] + self.n_ent[l] * self.N[l]
        self.n_dofs = self.offset[d + 1]
        self.n_interior = self.n_ent[d] * self.N[d]
        # cell -> dof map
        cd = np.empty((self.n_cells, el.n), dtype=np.int64)
        for i, di in enumerate(el.dofs):
            l = di.entity_dim
            cd[:, i] = self.offset[l] + self.cell_ent[l][:, di.entity_index] * self.N[l] + di.j \
                + self.kinds[l].index(di.kind)
        self.cell_dofs = cd

    def entity_dofs(self, l, ent_id, kinds=None):
        """Global dofs of one entity, optionally only those of given kinds."""
        base = self.offset[l] + ent_id * self.N[l]
        return [base + j for j in range(self.N[l])
                if kinds is None or self.kinds[l][j] in kinds]

    def vertex_star(self):
        """For each vertex: the edges and faces containing it (the star,
        Sec. 6.1)."""
        d = self.d
        edges_of = [[] for _ in range(self.n_vertices)]
        for e, t in enumerate(self.ent_tuples[1]):
            for v in t:
                edges_of[v].append(e)
        faces_of = [[] for _ in range(self.n_vertices)]
        if d == 3:
            for f, t in enumerate(self.ent_tuples[2]):
                for v in t:
                    faces_of[v].append(f)
        return edges_of, faces_of

    def edge_faces(self):
        """For each edge of a 3D mesh: the faces containing it."""
        lookup = {tuple(t): e for e, t in enumerate(self.ent_tuples[1])}
        faces_of = [[] for _ in range(self.n_ent[1])]
        for f, t in enumerate(self.ent_tuples[2]):
            for a, b in combinations(t, 2):
                faces_of[lookup[(a, b)]].append(f)
        return faces_of


def dirichlet_dofs(top, cells_in, facet_flags):
    """Global dofs removed by a Dirichlet boundary Gamma_D (Sec. 5): every
    basis function tied to a subsimplex of Gamma_D -- the facets marked in
    facet_flags and their vertices, edges (and, in 3D, the faces themselves).
    The remaining functions span X^k_{p,D}: a function tied to an entity
    outside Gamma_D has zero trace (value, tangential or normal component)
    on every facet of Gamma_D, because the dofs of a facet's subentities are
    unisolvent for the trace space on that facet (Sec. 3.3).

    cells_in: the cells in the caller's vertex order; facet_flags (n_cells,
    d+1): a nonzero (c, j) marks the facet of cell c opposite its j-th vertex.
    A marked facet must lie on the boundary (belong to one cell).  Returns the
    ascending removed dofs."""
    d = top.d
    cells_in = np.asarray(cells_in, dtype=np.int64)
    flags = np.asarray(facet_flags).reshape(top.n_cells, d + 1)
    lookup = [{tuple(t): e for e, t in enumerate(top.ent_tuples[l])} for l in range(d)]
    count = {}
    for c in range(top.n_cells):
        for j in range(d + 1):
            f = tuple(sorted(np.delete(cells_in[c], j).tolist()))
            count[f] = count.get(f, 0) + 1
    out = set()
    for c, j in zip(*np.nonzero(flags)):
        f = tuple(sorted(np.delete(cells_in[c], j).tolist()))
        if count[f] != 1:
            raise ValueError(f"facet {f} of cell {c} is not on the boundary")
        for l in range(d):
            for sub in combinations(f, l + 1):
                out.update(top.entity_dofs(l, lookup[l][sub]))
    return np.array(sorted(out), dtype=np.int64)
