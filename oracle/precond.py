"""The interior-interface split Schwarz preconditioners of Sec. 6, in the
additive form of the theory and in the symmetric multiplicative hybrid form
the experiments use (Sec. 7.1).

Additive form (AdditiveSchwarz):

    P^{-1} r = D_I^{-1} r_I + sum_m R_m^T A_m^{-1} R_m r + R_W^T A_W^{-1} R_W r

* D_I = diag(A) on the interior dofs: the point-Jacobi solver on X^k_I
  (Sec. 6, eq:abstract-space-decomp-split).
* Interface patches (exact solvers, dense Cholesky):
  - H(grad): vertex stars of X^0_Gamma, PAFW(0)(X^0_Gamma)+J (eq:approx-sc-pafw);
  - H(curl): vertex-star potentials d X^{0}_Gamma|star V (A_V = G_V^T A G_V)
    plus edge stars of the type-I interface space X^{1,I}_Gamma|star E
    (eq:hcurl-decomp);
  - H(div): edge stars of X^2_Gamma, PAFW(1)(X^2_Gamma)+J (eq:hdiv-decomp).
  - the second-kind spaces (eq:second-kind-def) take the decompositions of
    the first-kind space of the same form degree, with the potentials from
    the next-lower space of the second-kind sequence: NedTwo_p the H(curl)
    ones with CG_{p+1} vertex-star potentials (the NedTwo_p type-II dofs are
    gradients of CG_{p+1} type-I functions), BDM_p the H(div) ones, whose
    type-I Hiptmair-Toselli and standard Hiptmair-Toselli potentials are
    curls of NedTwo_{p+1} functions.
  - 2D H(curl) and 2D H(div) (both k = 1, and 2D RT_p is the quarter turn of
    2D Ned_p, so the two share every decomposition, the curl of a CG
    function having the coefficients of its gradient): the H(curl) form
    above with the dimensions shifted -- the edge stars of X^{1,I}_Gamma
    hold the edge's Whitney dof only (an edge of a triangle carries no
    type-I dofs and the faces are the cells), the vertex-star potentials
    the vertex function and the CG edge dofs; "full" adds the cells' type-I
    dofs to the edge stars and the CG cell interiors to the potentials.
  A restriction to a star keeps the dofs of the entities that contain the
  star's centre (they vanish on the star's boundary).
* Coarse space W^k (Whitney forms; lem:basis-contains-whitney): reading R9,
  an exact solve with the principal submatrix A[W, W] in place of the
  paper's geometric multigrid V-cycle.

The vertex-star comparators of Sec. 6.1 (decomposition="vertex" and
"vertex-full"), for every space:
  - "vertex": PAFW(0)(X^k_Gamma) + J(X^k_I) (eq:approx-sc-pafw): a patch per
    vertex holding the dofs of the vertex, edges and faces containing it;
    the same Jacobi and coarse parts as above;
  - "vertex-full": PAFW(0)(X^k) (eq:pafw): the vertex-star patches also hold
    the interior dofs of the cells containing the vertex, and there is no
    Jacobi part (the interior group is empty).
  For H(grad) "vertex" is the default decomposition.
The other comparators of the paper's tables:
  - "paper-full": the default decomposition without the split -- the
    stars also hold the cell interiors (of the kinds the patch keeps) and the
    Jacobi group is empty: H(grad) PAFW(0)(X^0) (= "vertex-full"), H(curl)
    PH(X^0, X^{1,I}) (eq:hcurl-decomp without the split), H(div) PAFW(1)(X^2);
  - "hiptmair" (H(curl) only): the standard Hiptmair-Toselli decomposition
    PH(X^0_Gamma, X^1_Gamma) + J(X^1_I) (eq:pavarino_hiptmair with the
    split): vertex-star potentials as above and edge stars of every kind
    of interface dof;
  - "hiptmair-full" (H(curl) only): PH(X^0, X^1) (eq:pavarino_hiptmair):
    the potentials also hold the CG cell interiors (mapped to the Ned type-II
    cell dofs) and the edge stars every dof of the cells containing the edge;
  - "typeI" / "typeI-full" (H(curl), H(div)): the type-I Hiptmair-Toselli
    decomposition PH(X^{k-1,I}, X^{k,I}) (eq:pavarino_hiptmair-novel) with
    and without the split.  For H(curl) these are "paper" / "paper-full".
    For H(div) the split form is eq:hdiv-ph-reduced: W^2 + J(X^2_I) + edge-
    star potentials curl X^{1,I}_Gamma|star E, with no face stars (the type-I
    interface space is W^2).  The full form adds to each potential the curls
    of the NedTwo type-I functions of the cells containing the edge, and the
    face stars X^{2,I}|star F (the Whitney dof of the face and the type-I
    dofs of its cells), and drops the Jacobi group.

Hybrid form (HybridSchwarz, Sec. 7.1, eq:generic-subspace-splitting-mult):
the three groups X_1 = X^k_I (point-Jacobi), X_2 = X^k_Gamma (the additive
interface patch solver above, coarse space excluded) and X_3 = W^k (exact)
are applied multiplicatively in the order X_1, X_2, X_3, X_2, X_1, each
correction z += rho_m^{-1} B_m (r - A z).  Under "vertex-full" X_1 is empty
and X_2 (the full vertex stars) spans every dof, so the sweep is X_2, X_3,
X_2.  The weight of a group is
rho_m = (lambda_min + 3 lambda_max) / 4 from the extreme Ritz values of 10
CG steps on A restricted to X_m, preconditioned by B_m, with a random
right-hand side.  Reading R17: the right-hand side is 2u - 1 per subspace
dof (ascending global order) with u from SplitMix64 seeded SEED_INTERIOR /
SEED_INTERFACE; the CG steps stop early once ||r|| <= 1e-12 ||b||; an empty
subspace has rho = 1; the exact coarse solver has rho_3 = 1.

The discrete gradient G_V maps the CG_p vertex-star dofs into Ned_p:
grad of the vertex function lambda_V is sum_E (+1 if V is the larger vertex
of E else -1) times the Whitney function of E, and grad of a CG type-I
function is the Ned type-II function with the same entity and index
(lem:d-preserves-basis-functions, eq:d-preserves-basis-functions-global).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .pcg import lanczos_extremes, pcg
from .simplex import splitmix64_stream

SEED_INTERIOR = 0x5EED1000
SEED_INTERFACE = 0x5EED2000
SEED_COARSE = 0x5EED4000


def interior_dofs(top):
    return np.arange(top.offset[top.d], top.n_dofs)


def whitney_dofs(top, k):
    return np.array([top.offset[k] + e * top.N[k] for e in range(top.n_ent[k])], dtype=np.int64)


def cells_containing(top, l):
    """For each entity of dimension l: the cells that contain it."""
    out = [[] for _ in range(top.n_ent[l])]
    for c in range(top.n_cells):
        for e in sorted(set(top.cell_ent[l][c].tolist())):
            out[e].append(c)
    return out


def face_stars_typeI(top):
    """Face stars of the type-I space X^{2,I}|star F: the Whitney dof of the
    face and the type-I dofs of the cells containing it (H(div))."""
    cells_of = cells_containing(top, 2)
    out = []
    for f in range(top.n_ent[2]):
        idx = top.entity_dofs(2, f, kinds=("W",))
        for c in cells_of[f]:
            idx += top.entity_dofs(3, c, kinds=("I",))
        out.append(np.array(sorted(idx), dtype=np.int64))
    return out


def face_stars(top, full):
    """The k-stars of the standard H(div) Hiptmair-Toselli decomposition
    (eq:pavarino_hiptmair, k = 2): per face, X^2_Gamma|star F -- the dofs of
    the face -- and, full (X^2|star F), also the dofs of its two cells."""
    cells_of = cells_containing(top, 2)
    out = []
    for f in range(top.n_ent[2]):
        idx = top.entity_dofs(2, f)
        if full:
            for c in cells_of[f]:
                idx += top.entity_dofs(3, c)
        out.append(np.array(sorted(idx), dtype=np.int64))
    return out


def nedtwo_curl_potentials(top, top2, full):
    """The potentials of the standard H(div) Hiptmair-Toselli decomposition
    d X^1|star E (eq:pavarino_hiptmair, k = 2) with X^1 = NedTwo_p, the space
    whose eigenfunctions define the RT_p type-II dofs (R4): per edge, the
    NedTwo dofs of the entities containing it (the edge and its faces; full:
    also its cells) as (S_E, G_E): S_E the NedTwo global dofs (numbering of
    top2) and G_E (n_RT x |S_E|) the curls of those functions in RT
    coefficients -- the Whitney edge function to the signed face Whitney
    functions (as in curl_potential_patches), a type-I function of a face or
    cell to the RT type-II function of the same entity and index
    (lem:d-preserves-basis-functions), a type-II (gradient) function to
    zero."""
    faces_of = top.edge_faces()
    cells_of = cells_containing(top, 1) if full else None
    out = []
    for e, (a0, b0) in enumerate(top.ent_tuples[1]):
        S, rows, cols, vals = [], [], [], []
        ents = [(1, e)] + [(2, f) for f in faces_of[e]] + ([(3, c) for c in cells_of[e]] if full else [])
        for l, ent in ents:
            base = top2.offset[l] + ent * top2.N[l]
            typeI = [top.entity_dofs(l, ent, kinds=("II",))] if l >= 2 else None
            nI = 0
            for j in range(top2.N[l]):
                col = len(S)
                S.append(base + j)
                kind = top2.kinds[l][j]
                if kind == "W":
                    for f in faces_of[e]:
                        a, b, c = top.ent_tuples[2][f]
                        rows.append(top.entity_dofs(2, f, kinds=("W",))[0])
                        cols.append(col)
                        vals.append(-1.0 if (a0, b0) == (a, c) else 1.0)
                elif kind == "I":
                    rows.append(typeI[0][nI])
                    cols.append(col)
                    vals.append(1.0)
                    nI += 1
        G = sp.csc_matrix((vals, (rows, cols)), shape=(top.n_dofs, len(S)))
        out.append((np.array(S, dtype=np.int64), G))
    return out


def curl_potential_patches(top, full=False):
    """H(div) edge-star potentials curl X^{1,I}|star E as sparse G_E
    (n_dofs x n_E) in RT coefficients.  Column 0 is the curl of the Whitney
    edge function: by Stokes' theorem the sum over the faces F containing E
    of s phi^W_F, with s = -1 if E is the edge (a, c) of F = (a, b, c)
    (ascending) and +1 otherwise (tangents and normals from sorted vertices;
    the basis holds the Whitney forms, lem:basis-contains-whitney).  Then the
    RT type-II dofs of the faces (and, full, of the cells) containing E: the
    curls of the NedTwo type-I functions of the same entity and index
    (lem:d-preserves-basis-functions)."""
    faces_of = top.edge_faces()
    cells_of = cells_containing(top, 1) if full else None
    out = []
    for e, (a0, b0) in enumerate(top.ent_tuples[1]):
        rows, cols, vals = [], [], []
        for f in faces_of[e]:
            a, b, c = top.ent_tuples[2][f]
            rows.append(top.entity_dofs(2, f, kinds=("W",))[0])
            cols.append(0)
            vals.append(-1.0 if (a0, b0) == (a, c) else 1.0)
        col = 1
        ents = [(2, f) for f in faces_of[e]] + ([(3, c) for c in cells_of[e]] if full else [])
        for l, ent in ents:
            for j in top.entity_dofs(l, ent, kinds=("II",)):
                rows.append(j); cols.append(col); vals.append(1.0); col += 1
        out.append(sp.csc_matrix((vals, (rows, cols)), shape=(top.n_dofs, col)))
    return out


def solver_family(top, family):
    """The family whose decompositions a space uses: 2D RT_p those of 2D
    Ned_p (its quarter turn); the second-kind spaces those of their first-
    kind counterparts (NedTwo_p: H(curl) with CG_{p+1} potentials, BDM_p:
    H(div) with NedTwo_{p+1} potentials)."""
    if family == "NedTwo" or (top.d == 2 and family == "RT"):
        return "Ned"
    if family == "BDM":
        return "RT"
    return family


def potential_degree(top, family):
    """Degree of the potential space: X^{k-1} is CG_{p+1} for NedTwo_p and
    NedTwo_{p+1} for BDM_p (exact second-kind sequence), degree p otherwise."""
    return top.el.p + (1 if family in ("NedTwo", "BDM") else 0)


def patch_lists(top, family, decomposition="paper"):
    """Plain patches of a decomposition: list of ascending global dof
    arrays (the potentials are separate: potential_patches,
    curl_potential_patches)."""
    family = solver_family(top, family)
    if decomposition in ("vertex", "vertex-full"):
        return vertex_star_lists(top, decomposition == "vertex-full")
    if decomposition not in DECOMPOSITIONS:
        raise ValueError(decomposition)
    if decomposition.startswith("typeI"):
        if family == "CG":
            raise ValueError("the type-I Hiptmair-Toselli decompositions need k >= 1")
        if family == "RT":
            return face_stars_typeI(top) if decomposition == "typeI-full" else []
        decomposition = decomposition.replace("typeI", "paper")
    if decomposition.startswith("hiptmair") and family == "CG":
        raise ValueError("the Hiptmair-Toselli decompositions need k >= 1")
    if decomposition.startswith("hiptmair") and family == "RT":
        return face_stars(top, decomposition == "hiptmair-full")
    full = decomposition.endswith("full")
    d = top.d
    out = []
    if family == "CG":
        return vertex_star_lists(top, full)
    elif family == "Ned":
        # type-I stars: the edge's Whitney dof and the type-I dofs of the faces
        # (and cells) containing it; Hiptmair stars: every dof of those
        typeI = decomposition.startswith("paper")
        faces_of = top.edge_faces() if d == 3 else [[] for _ in range(top.n_ent[1])]
        cells_of = cells_containing(top, 1)
        for e in range(top.n_ent[1]):
            idx = top.entity_dofs(1, e, kinds=("W",) if typeI else None)
            for f in faces_of[e]:
                idx += top.entity_dofs(2, f, kinds=("I",) if typeI else None)
            if full:
                for c in cells_of[e]:
                    idx += top.entity_dofs(d, c, kinds=("I",) if typeI else None)
            out.append(np.array(sorted(idx), dtype=np.int64))
    elif family == "RT":
        faces_of = top.edge_faces()
        cells_of = cells_containing(top, 1)
        for e in range(top.n_ent[1]):
            idx = []
            for f in faces_of[e]:
                idx += top.entity_dofs(2, f)
            if full:
                for c in cells_of[e]:
                    idx += top.entity_dofs(3, c)
            out.append(np.array(sorted(idx), dtype=np.int64))
    else:
        raise ValueError(family)
    return out


def vertex_star_lists(top, full):
    """PAFW(0) patches (eq:pafw, eq:approx-sc-pafw): per vertex, the global
    dofs (ascending) of the entities that contain it -- the vertex, its edges
    and faces -- and, for the full star X^k|star V, also its cells.  A space
    with no dofs on some entity dimension simply contributes none there."""
    d = top.d
    edges_of, faces_of = top.vertex_star()
    cells_of = [[] for _ in range(top.n_vertices)]
    for c, t in enumerate(top.cells):
        for v in t:
            cells_of[v].append(c)
    out = []
    for v in range(top.n_vertices):
        idx = list(top.entity_dofs(0, v))
        for e in edges_of[v]:
            idx += top.entity_dofs(1, e)
        for f in faces_of[v]:
            idx += top.entity_dofs(2, f)
        if full:
            for c in cells_of[v]:
                idx += top.entity_dofs(d, c)
        out.append(np.array(sorted(idx), dtype=np.int64))
    return out


DECOMPOSITIONS = ("paper", "vertex", "vertex-full", "paper-full", "hiptmair", "hiptmair-full", "typeI", "typeI-full")


def potential_patches(top, cg_N, full=False):
    """H(curl) vertex potentials: sparse G_V (n_dofs x n_V) per vertex.
    cg_N = dofs per entity dimension of the CG_p potential space.  Columns:
    the vertex, then the CG dofs of its edges (ascending edge id, then
    index), then of its faces (3D), then (full) of its cells."""
    d = top.d
    edges_of, faces_of = top.vertex_star()
    cells_of = cells_containing(top, 0) if full else None
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
        if full:
            for c in cells_of[v]:
                ii = top.entity_dofs(d, c, kinds=("II",))
                assert len(ii) == cg_N[d]
                for j in ii:
                    rows.append(j); cols.append(col); vals.append(1.0); col += 1
        out.append(sp.csc_matrix((vals, (rows, cols)), shape=(top.n_dofs, col)))
    return out


def restrict_columns(G, removed):
    """The columns of a sparse potential basis G that lie in X^k_{p,D}: those
    with no entry on a removed (Dirichlet) dof.  A potential whose function
    has a nonzero trace on Gamma_D (the gradient of a vertex function of a
    vertex on Gamma_D, the image of a CG dof on Gamma_D) touches one."""
    if removed is None or len(removed) == 0:
        return G
    hit = np.asarray(abs(G[removed, :]).sum(axis=0)).ravel() > 0
    return G[:, np.flatnonzero(~hit)]


class AdditiveSchwarz:
    """P^{-1} = D_I^{-1} + sum R^T A_m^{-1} R + R_W^T A_W^{-1} R_W on X^k_{p,D}.

    dirichlet (ascending removed dofs, see mesh.dirichlet_dofs) restricts
    every subspace to the functions that remain (Sec. 5): the patches lose
    their removed dofs, the potentials their columns that touch one, the
    coarse space its removed Whitney dofs; the cell interiors are never on
    the boundary.  The result is zero on the removed dofs."""

    def __init__(self, A, top, family, decomposition="paper", dirichlet=None, coarse_mg=None, beta=1.0):
        """coarse_mg: None for the exact coarse solve (reading R9), or the
        cells per edge n of the Kuhn mesh for the geometric multigrid V-cycle
        on W^k of the experiments (oracle.multigrid).  beta: the mass
        coefficient of A (it scales the regularisation of the H(div)
        Hiptmair-Toselli potentials)."""
        if decomposition not in DECOMPOSITIONS:
            raise ValueError(decomposition)
        self.A = A
        self.top = top
        self.family = family
        pdeg = potential_degree(top, family)
        family = solver_family(top, family)
        self.decomposition = decomposition
        self.removed = np.zeros(0, dtype=np.int64) if dirichlet is None else np.asarray(dirichlet, dtype=np.int64)
        keep = np.ones(top.n_dofs, dtype=bool)
        keep[self.removed] = False
        k = top.el.k
        diag = A.diagonal()
        full = decomposition.endswith("full")
        self.I = np.zeros(0, dtype=np.int64) if full else interior_dofs(top)
        self.dI = diag[self.I]
        self.patches = []       # (index array, cho factor)
        for idx in patch_lists(top, family, decomposition):
            idx = idx[keep[idx]]
            if len(idx) == 0:
                continue
            Ap = A[idx][:, idx].toarray()
            self.patches.append((idx, sla.cho_factor(Ap, lower=True)))
        self.potentials = []    # (G_V, cho factor)
        pots = []
        if family == "Ned" and not decomposition.startswith("vertex"):
            from .element import element
            pots = potential_patches(top, element(top.d, "CG", pdeg).counts(), full)
        if family == "RT" and decomposition.startswith("typeI"):
            pots = curl_potential_patches(top, full)
        for G in pots:
            G = restrict_columns(G, self.removed)
            if G.shape[1] == 0:
                continue
            Ap = (G.T @ (A @ G)).toarray()
            self.potentials.append((G, sla.cho_factor(Ap, lower=True)))
        if family == "RT" and decomposition.startswith("hiptmair"):
            # NedTwo_p edge-star potentials with the regularised local problem
            # eq:local-potential-problem-added-mass: (phi, eps psi) +
            # a(d phi, d psi), eps = 1e-8 beta (curl grad = 0 makes the
            # unregularised problem singular)
            if len(self.removed):
                raise ValueError("the H(div) Hiptmair-Toselli potentials are built for pure Neumann problems")
            from .element import element
            from .mesh import Topology
            from .operator import all_cell_matrices, assemble
            el2 = element(top.d, "NedTwo", pdeg)
            top2 = Topology(top.coords, top.cells, el2)
            M2 = assemble(top2, all_cell_matrices(el2, top2, alpha=0.0, beta=1.0))
            eps = 1e-8 * beta
            for S, G in nedtwo_curl_potentials(top, top2, full):
                Ap = eps * M2[S][:, S].toarray() + (G.T @ (A @ G)).toarray()
                self.potentials.append((G, sla.cho_factor(Ap, lower=True)))
        W = whitney_dofs(top, k)
        self.W = W[keep[W]]
        self.mg = None
        if coarse_mg is not None:
            if len(self.removed):
                raise ValueError("the multigrid coarse solver is built for pure Neumann problems")
            from .multigrid import WhitneyMultigrid
            self.mg = WhitneyMultigrid(A[self.W][:, self.W], coarse_mg, k, d=top.el.d)
            self.coarse = None
        else:
            AW = A[self.W][:, self.W].toarray()
            self.coarse = sla.cho_factor(AW, lower=True)

    def coarse_solve(self, rW):
        """The W^k solver: exact Cholesky, or one V-cycle."""
        return self.mg.cycle(rW) if self.mg is not None else sla.cho_solve(self.coarse, rW)

    def apply(self, r):
        z = np.zeros_like(r)
        z[self.I] = r[self.I] / self.dI
        for idx, F in self.patches:
            z[idx] += sla.cho_solve(F, r[idx])
        for G, F in self.potentials:
            z += G @ sla.cho_solve(F, G.T @ r)
        z[self.W] += self.coarse_solve(r[self.W])
        return z

    def sizes(self):
        s = [len(i) for i, _ in self.patches] + [G.shape[1] for G, _ in self.potentials]
        return s


def subspace_extremes(A, idx, solve, seed, steps=10):
    """Estimates (lambda_min, lambda_max) of the generalized eigenproblem
    a(u, v) = lambda a_m(u, v) on the subspace spanned by the dofs idx: the
    extreme Ritz values of `steps` CG iterations on A[idx, idx]
    preconditioned by `solve` (acting on full-length vectors supported on
    idx) with a SplitMix64 right-hand side (Sec. 7.1)."""
    if len(idx) == 0:
        return 1.0, 1.0
    n = A.shape[0]
    gen = splitmix64_stream(seed)
    b = np.array([2.0 * next(gen) - 1.0 for _ in range(len(idx))])
    Am = A[idx][:, idx]

    def Bm(r):
        f = np.zeros(n)
        f[idx] = r
        return solve(f)[idx]

    _, info = pcg(lambda v: Am @ v, Bm, b, rtol=1e-12, maxit=steps)
    return lanczos_extremes(info["alphas"], info["betas"])


def subspace_weight(A, idx, solve, seed, steps=10):
    """rho = (lambda_min + 3 lambda_max) / 4 from subspace_extremes."""
    lo, hi = subspace_extremes(A, idx, solve, seed, steps)
    return (lo + 3.0 * hi) / 4.0


class HybridSchwarz:
    """Symmetric multiplicative hybrid of the three groups of the
    interior-interface split (Sec. 7.1): z = 0, then for m in 1, 2, 3, 2, 1:
    z += rho_m^{-1} B_m (r - A z)."""

    def __init__(self, A, top, family, additive=None, decomposition="paper", dirichlet=None, coarse_mg=None):
        self.A = A
        self.add = additive if additive is not None else AdditiveSchwarz(A, top, family, decomposition, dirichlet,
                                                                         coarse_mg)
        n = top.n_dofs
        mask = np.zeros(n, dtype=bool)
        mask[self.add.I] = True
        mask[self.add.removed] = True       # X_Gamma of X^k_{p,D}: no removed dofs
        self.Gamma = np.flatnonzero(~mask)
        self.rho_I = subspace_weight(A, self.add.I, self.B_interior, SEED_INTERIOR)
        self.rho_Gamma = subspace_weight(A, self.Gamma, self.B_interface, SEED_INTERFACE)
        # the exact coarse solver has weight 1; the V-cycle is an inexact
        # solver and gets the same estimated weight as the other groups
        self.rho_W = 1.0 if self.add.mg is None else subspace_weight(A, self.add.W, self.B_coarse, SEED_COARSE)

    def B_interior(self, r):
        z = np.zeros_like(r)
        z[self.add.I] = r[self.add.I] / self.add.dI
        return z

    def B_interface(self, r):
        z = np.zeros_like(r)
        for idx, F in self.add.patches:
            z[idx] += sla.cho_solve(F, r[idx])
        for G, F in self.add.potentials:
            z += G @ sla.cho_solve(F, G.T @ r)
        return z

    def B_coarse(self, r):
        z = np.zeros_like(r)
        z[self.add.W] = self.add.coarse_solve(r[self.add.W])
        return z

    def groups(self):
        return [(self.B_interior, self.rho_I), (self.B_interface, self.rho_Gamma), (self.B_coarse, self.rho_W)]

    def apply(self, r):
        (b1, w1), (b2, w2), (b3, w3) = self.groups()
        z = np.zeros_like(r)
        for B, w in ((b1, w1), (b2, w2), (b3, w3), (b2, w2), (b1, w1)):
            z = z + B(r - self.A @ z) / w
        return z

