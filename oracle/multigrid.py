"""Geometric multigrid V-cycle on the Whitney space W^k: the inexact W^k
solver of the paper's experiments (Sec. 7.1; fig:solver-diagram-PAFW,
fig:solver-diagram-PH), in place of the exact coarse solve.

* Hierarchy: the Freudenthal (Kuhn) meshes with n, n/2, n/4, ... cells per
  edge, halving while n is even (the paper's coarsest mesh has 3 cells per
  edge, its finer levels are refinements of it).  The finest level is the
  problem's mesh (possibly jittered); the coarser meshes exist only
  combinatorially: the prolongation is computed on the unperturbed
  vertex positions, where the meshes are nested.
* Prolongation W^k(H) -> W^k(h): the Whitney forms are nested under
  refinement, and the basis contains them (lem:basis-contains-whitney), so a
  coarse Whitney form is exactly a combination of fine ones whose
  coefficients are the fine Whitney dofs of the coarse form: point values
  (k = 0), line integrals along the fine edge (k = 1), fluxes through the
  fine face (k = 2), with the orientations of the sorted vertex tuples.
* Level operators: A_0 = A[W, W] of the degree-p operator, A_{l+1} =
  P_l^T A_l P_l (Galerkin); Cholesky on the coarsest level.
* Relaxation (the additive Schwarz smoothers named in the solver diagrams):
  k = 0 vertex patches of W^0, i.e. point-Jacobi; k = 1 Hiptmair-Jacobi, the
  additive Schwarz method of eq:hiptmair-smoothing at lowest order (the
  gradients of the vertex hat functions and the Whitney edge functions,
  each with an exact one-dimensional solve); k = 2 patches on edge stars of
  W^2 (the Whitney face functions of the faces containing an edge), the
  PAFW(1) relaxation at lowest order.  Reading R22 (the paper gives no
  damping or step count): each smoothing step is z += omega_l S_l (b - A_l
  z) with omega_l = 1 / rho_l, rho_l = (lambda_min + 3 lambda_max) / 4 of
  S_l A_l estimated from 10 CG steps (the paper's subspace-weight rule,
  SplitMix64 right-hand side seeded SEED_LEVEL + l), NU steps before and
  after the coarse correction; the cycle is symmetric, so it is a valid
  PCG preconditioner.
"""
from itertools import combinations, permutations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .element import element
from .mesh import Topology
from .precond import subspace_extremes

SEED_LEVEL = 0x5EED3000
NU = 2


def kuhn_hierarchy(n):
    """Cells per edge of the levels, finest first: halve while even."""
    out = [n]
    while out[-1] % 2 == 0 and out[-1] > 1:
        out.append(out[-1] // 2)
    return out


def _kuhn_unit(n, d=3):
    # the unperturbed Kuhn mesh with the vertex numbering of the workloads
    h = 1.0 / n
    g = np.arange(n + 1)
    if d == 2:
        J, I = np.meshgrid(g, g, indexing="ij")
        X = np.stack([I.ravel(), J.ravel()], axis=1) * h
        vid = lambda i, j: i + (n + 1) * j
        cells = []
        for j in range(n):
            for i in range(n):
                corner = lambda b: vid(i + (b & 1), j + ((b >> 1) & 1))
                cells.append([corner(0), corner(1), corner(3)])
                cells.append([corner(0), corner(2), corner(3)])
        return X.astype(float), np.asarray(cells, dtype=np.int64)
    K, J, I = np.meshgrid(g, g, g, indexing="ij")
    X = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1) * h
    vid = lambda i, j, k: i + (n + 1) * (j + (n + 1) * k)
    cells = []
    for k in range(n):
        for j in range(n):
            for i in range(n):
                corner = lambda b: vid(i + (b & 1), j + ((b >> 1) & 1), k + ((b >> 2) & 1))
                for a, b, _ in permutations(range(3)):
                    ea, eb = 1 << a, 1 << b
                    cells.append([corner(0), corner(ea), corner(ea | eb), corner(7)])
    return X.astype(float), np.asarray(cells, dtype=np.int64)


def _barycentric(Xc):
    """Barycentric coordinates lam(x) = L @ [x, 1] of a simplex (d + 1
    vertices in d dimensions) and their (constant) gradients (rows of
    L[:, :d])."""
    M = np.vstack([Xc.T, np.ones(len(Xc))])
    L = np.linalg.inv(M)
    return L


def _whitney_value(k, L, verts, x):
    """The Whitney k-form of the local vertex tuple `verts` (ascending coarse
    ids) of a cell with barycentric matrix L, at the point x."""
    d = L.shape[0] - 1
    lam = L[:, :d] @ x + L[:, d]
    g = L[:, :d]
    if k == 0:
        return lam[verts[0]]
    if k == 1:
        a, b = verts
        return lam[a] * g[b] - lam[b] * g[a]
    a, b, c = verts
    cr = np.cross
    return 2.0 * (lam[a] * cr(g[b], g[c]) + lam[b] * cr(g[c], g[a]) + lam[c] * cr(g[a], g[b]))


def whitney_prolongation(nc, k, d=3):
    """Sparse P (n_W(fine) x n_W(coarse)) from W^k on the Kuhn mesh of
    [0,1]^d with nc cells per edge to W^k on the mesh with 2 nc, both in the
    entity order of their topologies (lowest-order elements: their dofs are
    the Whitney dofs).  In 2D, k = 1 is the H(curl) form; the 2D H(div)
    Whitney functions are its quarter turns, with the same coefficients."""
    fam = {0: "CG", 1: "Ned", 2: "RT"}[k]
    el = element(d, fam, 1)
    Xc, Cc = _kuhn_unit(nc, d)
    Xf, Cf = _kuhn_unit(2 * nc, d)
    tc, tf = Topology(Xc, Cc, el), Topology(Xf, Cf, el)
    cid = [{tuple(t): e for e, t in enumerate(tc.ent_tuples[l])} for l in range(d + 1)]
    Lall = np.array([_barycentric(Xc[tc.cells[c]]) for c in range(tc.n_cells)])
    per = 6 if d == 3 else 2                       # Kuhn cells per cube (square)
    rows, cols, vals = [], [], []
    for e, tup in enumerate(tf.ent_tuples[k]):
        xe = Xf[list(tup)]
        xb = xe.mean(axis=0)
        cube = np.minimum((xb * nc).astype(int), nc - 1)
        base = per * (cube[0] + nc * (cube[1] + (nc * cube[2] if d == 3 else 0)))
        # the coarse cell of the cube in which x_b has the largest smallest
        # barycentric coordinate (the one containing it)
        lam = np.einsum("cij,j->ci", Lall[base:base + per, :, :d], xb) + Lall[base:base + per, :, d]
        cp = int(np.argmax(lam.min(axis=1)))
        best, L, cell = lam[cp].min(), Lall[base + cp], base + cp
        assert best > -1e-12, "fine entity outside its coarse cube"
        gv = tc.cells[cell]                        # ascending coarse vertex ids of the cell
        for loc in combinations(range(d + 1), k + 1):
            glob = tuple(int(gv[a]) for a in loc)
            if k == 0:
                v = _whitney_value(0, L, loc, xe[0])
            elif k == 1:
                v = _whitney_value(1, L, loc, xb) @ (xe[1] - xe[0])
            else:
                v = _whitney_value(2, L, loc, xb) @ np.cross(xe[1] - xe[0], xe[2] - xe[0]) / 2.0
            if abs(v) > 1e-14:
                rows.append(e)
                cols.append(cid[k][glob])
                vals.append(v)
    P = sp.csr_matrix((vals, (rows, cols)), shape=(tf.n_ent[k], tc.n_ent[k]))
    return P, tc, tf


def incidence(top):
    """Gradients of the vertex hat functions in Whitney edge coefficients:
    G[e, v] = +1 if v is the larger vertex of edge e, -1 if the smaller."""
    E = top.ent_tuples[1]
    ne = len(E)
    rows = np.repeat(np.arange(ne), 2)
    cols = E.ravel()
    vals = np.tile([-1.0, 1.0], ne)
    return sp.csr_matrix((vals, (rows, cols)), shape=(ne, top.n_vertices))


def edge_face_stars(top):
    """For every edge, the (ascending) faces containing it."""
    return [np.array(sorted(f), dtype=np.int64) for f in top.edge_faces()]


class Smoother:
    """The additive Schwarz relaxation S_l of one level (see the module
    docstring), S_l r for a level vector r."""

    def __init__(self, A, k, top):
        self.k = k
        self.dinv = 1.0 / A.diagonal()
        if k == 1:
            G = incidence(top)
            self.G = G
            self.gdiag = 1.0 / (G.T @ (A @ G)).diagonal()
        if k == 2:
            # the additive edge-star relaxation sum_s R_s^T A_s^{-1} R_s,
            # assembled once as a sparse matrix (each star's principal
            # submatrix inverted through its Cholesky factor)
            rows, cols, vals = [], [], []
            for idx in edge_face_stars(top):
                F = sla.cho_factor(A[idx][:, idx].toarray(), lower=True)
                inv = sla.cho_solve(F, np.eye(len(idx)))
                rows.append(np.repeat(idx, len(idx)))
                cols.append(np.tile(idx, len(idx)))
                vals.append(inv.ravel())
            n = A.shape[0]
            self.S = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))

    def apply(self, r):
        if self.k == 0:
            return self.dinv * r
        if self.k == 1:
            return self.dinv * r + self.G @ (self.gdiag * (self.G.T @ r))
        return self.S @ r


class WhitneyMultigrid:
    """Symmetric V-cycle on W^k for the Whitney block AW of a problem on the
    Kuhn mesh of [0,1]^d with n cells per edge (its dofs in the entity order
    of the k-entities; k = 1 in 2D serves H(curl) and H(div) alike)."""

    def __init__(self, AW, n, k, nu=NU, d=3):
        self.k, self.nu = k, nu
        self.ns = kuhn_hierarchy(n)
        self.A, self.P, self.S, self.omega = [sp.csr_matrix(AW)], [], [], []
        tops = []
        for l, nl in enumerate(self.ns[:-1]):
            P, tc, tf = whitney_prolongation(nl // 2, k, d)
            assert P.shape[0] == self.A[l].shape[0]
            self.P.append(P)
            tops.append(tf)
            self.A.append((P.T @ self.A[l] @ P).tocsr())
        for l in range(len(self.ns) - 1):
            S = Smoother(self.A[l], k, tops[l])
            lo, hi = subspace_extremes(self.A[l], np.arange(self.A[l].shape[0]), S.apply, SEED_LEVEL + l)
            self.S.append(S)
            self.omega.append(4.0 / (lo + 3.0 * hi))
        self.coarse = sla.cho_factor(self.A[-1].toarray(), lower=True)

    def cycle(self, b, l=0):
        if l == len(self.ns) - 1:
            return sla.cho_solve(self.coarse, b)
        A, S, w = self.A[l], self.S[l], self.omega[l]
        x = np.zeros_like(b)
        for _ in range(self.nu):
            x = x + w * S.apply(b - A @ x)
        x = x + self.P[l] @ self.cycle(self.P[l].T @ (b - A @ x), l + 1)
        for _ in range(self.nu):
            x = x + w * S.apply(b - A @ x)
        return x
