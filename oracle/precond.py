"""The interior-interface split Schwarz preconditioners of Sec. 6.

Additive form (reading R8: the theory of Sec. 6 is stated for the additive
Schwarz method; the experiments' symmetric multiplicative hybrid is a
separate variant):

    P^{-1} r = D_I^{-1} r_I + sum_m R_m^T A_m^{-1} R_m r + R_W^T A_W^{-1} R_W r

* D_I = diag(A) on the interior dofs: the point-Jacobi solver on X^k_I
  (Sec. 6, eq:abstract-space-decomp-split).
* Interface patches (exact solvers, dense Cholesky):
  - H(grad): vertex stars of X^0_Gamma, PAFW(0)(X^0_Gamma)+J (eq:approx-sc-pafw);
  - H(curl): vertex-star potentials d X^{0}_Gamma|star V (A_V = G_V^T A G_V)
    plus edge stars of the type-I interface space X^{1,I}_Gamma|star E
    (eq:hcurl-decomp);
  - H(div): edge stars of X^2_Gamma, PAFW(1)(X^2_Gamma)+J (eq:hdiv-decomp).
  A restriction to a star keeps the dofs of the entities that contain the
  star's centre (they vanish on the star's boundary).
* Coarse space W^k (Whitney forms; lem:basis-contains-whitney): reading R9,
  an exact solve with the principal submatrix A[W, W] in place of the
  paper's geometric multigrid V-cycle.

The discrete gradient G_V maps the CG_p vertex-star dofs into Ned_p:
grad of the vertex function lambda_V is sum_E (+1 if V is the larger vertex
of E else -1) times the Whitney function of E, and grad of a CG type-I
function is the Ned type-II function with the same entity and index
(lem:d-preserves-basis-functions, eq:d-preserves-basis-functions-global).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def interior_dofs(top):
    return np.arange(top.offset[top.d], top.n_dofs)


def whitney_dofs(top, k):
    return np.array([top.offset[k] + e * top.N[k] for e in range(top.n_ent[k])], dtype=np.int64)


def patch_lists(top, family):
    """Plain patches: list of ascending global dof arrays."""
    d = top.d
    out = []
    if family == "CG":
        edges_of, faces_of = top.vertex_star()
        for v in range(top.n_vertices):
            idx = [top.offset[0] + v]
            for e in edges_of[v]:
                idx += top.entity_dofs(1, e)
            for f in faces_of[v]:
                idx += top.entity_dofs(2, f)
            out.append(np.array(sorted(idx), dtype=np.int64))
    elif family == "Ned":
        faces_of = top.edge_faces()
        for e in range(top.n_ent[1]):
            idx = top.entity_dofs(1, e, kinds=("W",))
            for f in faces_of[e]:
                idx += top.entity_dofs(2, f, kinds=("I",))
            out.append(np.array(sorted(idx), dtype=np.int64))
    elif family == "RT":
        faces_of = top.edge_faces()
        for e in range(top.n_ent[1]):
            idx = []
            for f in faces_of[e]:
                idx += top.entity_dofs(2, f)
            out.append(np.array(sorted(idx), dtype=np.int64))
    else:
        raise ValueError(family)
    return out


def potential_patches(top, cg_N):
    """H(curl) vertex potentials: sparse G_V (n_dofs x n_V) per vertex.
    cg_N = dofs per entity of the CG_p potential space (vertex, edge, face).
    Columns: the vertex, then the CG dofs of its edges (ascending edge id,
    then index), then of its faces."""
    edges_of, faces_of = top.vertex_star()
    out = []
    for v in range(top.n_vertices):
        rows, cols, vals = [], [], []
        col = 0
        for e in edges_of[v]:
            a, b = top.ent_tuples[1][e]
            rows.append(top.entity_dofs(1, e, kinds=("W",))[0])
            cols.append(col)
            vals.append(1.0 if v == max(a, b) else -1.0)
        col += 1
        for e in edges_of[v]:
            ii = top.entity_dofs(1, e, kinds=("II",))
            assert len(ii) == cg_N[1]
            for j in ii:
                rows.append(j); cols.append(col); vals.append(1.0); col += 1
        for f in faces_of[v]:
            ii = top.entity_dofs(2, f, kinds=("II",))
            assert len(ii) == cg_N[2]
            for j in ii:
                rows.append(j); cols.append(col); vals.append(1.0); col += 1
        out.append(sp.csc_matrix((vals, (rows, cols)), shape=(top.n_dofs, col)))
    return out


class AdditiveSchwarz:
    def __init__(self, A, top, family):
        self.A = A
        self.top = top
        self.family = family
        k = {"CG": 0, "Ned": 1, "RT": 2}[family]
        diag = A.diagonal()
        self.I = interior_dofs(top)
        self.dI = diag[self.I]
        self.patches = []       # (index array, cho factor)
        for idx in patch_lists(top, family):
            Ap = A[idx][:, idx].toarray()
            self.patches.append((idx, sla.cho_factor(Ap, lower=True)))
        self.potentials = []    # (G_V, cho factor)
        if family == "Ned":
            p = top.el.p
            cg_N = (1, p - 1, (p - 1) * (p - 2) // 2)
            for G in potential_patches(top, cg_N):
                Ap = (G.T @ (A @ G)).toarray()
                self.potentials.append((G, sla.cho_factor(Ap, lower=True)))
        self.W = whitney_dofs(top, k)
        AW = A[self.W][:, self.W].toarray()
        self.coarse = sla.cho_factor(AW, lower=True)

    def apply(self, r):
        z = np.zeros_like(r)
        z[self.I] = r[self.I] / self.dI
        for idx, F in self.patches:
            z[idx] += sla.cho_solve(F, r[idx])
        for G, F in self.potentials:
            z += G @ sla.cho_solve(F, G.T @ r)
        z[self.W] += sla.cho_solve(self.coarse, r[self.W])
        return z

    def sizes(self):
        s = [len(i) for i, _ in self.patches] + [G.shape[1] for G, _ in self.potentials]
        return s
