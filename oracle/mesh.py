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
