"""The orthogonality-promoting finite elements of Sec. 3 of the paper.

For a first-kind space X^k_p(T_hat) (CG_p, Ned_p or RT_p; eq:first-kind-def)
this module builds, on the equilateral reference simplex:

1. the space as a subspace of P_p^c (coefficients in the orthonormal
   Dubiner basis), eq:first-kind-def / eq:second-kind-def;
2. for every subsimplex dimension l the bubble space X_ring^k(S) (the
   definition at the start of Sec. 3.1) as the null space of its boundary
   traces (eq:tr-k);
3. the eigenbasis of eq:ref-eval-problem-x, obtained through the augmented
   problem eq:ref-eval-problem-x-aug: keep the eigenpairs with mu != 0,
   psi = psi_hat / sqrt(mu), lambda = 1 / mu;
4. the degrees of freedom eq:abstract-dofs (Whitney moments, type-I moments
   of d_S, type-II moments against d_S of the (k-1)-form eigenbasis), in the
   concrete forms eq:hgrad-dofs, eq:hcurl-dofs, eq:hdiv-dofs;
5. the dual (Ciarlet) basis, l_i(phi_j) = delta_ij (Sec. 4, eq:reference-basis).

Readings where the paper is silent (each is listed in the design notes):

* R1 reference simplex: edge length 2, centroid at the origin.
* R2 eigenvector choice: eigenvalues of the symmetric reference simplex are
  exactly degenerate, and the paper does not say which orthonormal basis of
  a degenerate eigenspace is used.  Eigenpairs are ordered by ascending mu;
  consecutive mu within relative distance TAU form a cluster; within a
  cluster of m functions W (L2-orthonormal) the basis is rotated to
  W R, R = Y^T (Y Y^T)^{-1/2}, where Y_ij = pi_i(W_j) for the first m probe
  functionals pi_i of a fixed sequence (point values, projected on a fixed
  direction for vector fields, at points drawn from SplitMix64; for the 2D
  H(div) family the direction is turned by R, so that 2D RT_p is exactly the
  quarter turn R of 2D Ned_p, as the remark after eq:hdiv-dofs describes).
  The result
  does not depend on which orthonormal basis of the cluster the
  eigensolver returned, and it fixes signs.
* R3 "mu != 0": the number of discarded eigenpairs is the kernel dimension
  N^{k-1}_S from eq:bubble-trace-dim-counts, not a magnitude threshold.
* R4 RT_p uses NedTwo_p as its X^1 for the type-II eigenfunctions (Sec. 3.4.3:
  the implementation always takes the second kind).
* R5/R6 subentities are listed by ascending local vertex tuple and mapped
  from the lower-dimensional reference simplex by sending reference vertex m
  to the subentity's m-th vertex; local dofs are entity-major (vertices,
  edges, faces, cell) and, within an entity, Whitney, type-I (ascending mu),
  type-II (ascending mu).
"""
import functools
from itertools import combinations

import numpy as np
import scipy.linalg as sla

from .simplex import EQ_VERTICES, PolyBasis, quadrature, splitmix64_stream

TAU = 1e-7           # relative eigenvalue gap that defines a cluster (R2)
FORM = {"CG": 0, "Ned": 1, "NedTwo": 1, "RT": 2, "BDM": 2}
DIV_FAMILIES = ("RT", "BDM")


def form_degree(l, family):
    """k of a family on an l-simplex: H(div) is the (l-1)-forms (k = 1 in 2D:
    the remark after eq:hdiv-dofs)."""
    return l - 1 if family in DIV_FAMILIES else FORM[family]


def rot90(v):
    """R v = (v_1, -v_0) on the component axis 1: the quarter turn that carries
    2D H(curl) to 2D H(div) (n = R t on an edge, curl = R grad, and
    div R w = rot w)."""
    return np.stack([v[:, 1], -v[:, 0]], axis=1)


# --------------------------------------------------------------------------
# spaces as coefficient subspaces of P_p^c
# --------------------------------------------------------------------------
class Space:
    """A polynomial space on the equilateral l-simplex, given by an
    orthonormal coefficient matrix B over the vector Dubiner basis
    e_c (x) q_n (component-major)."""

    def __init__(self, l, c, poly, B, family, p):
        self.l, self.c, self.poly, self.B = l, c, poly, B
        self.family, self.p = family, p
        self.m = B.shape[1]

    def field(self, x, B=None):
        """values (N, c, m) and Jacobians (N, c, l, m) of the columns of B."""
        B = self.B if B is None else B
        n = self.poly.n
        Bc = B.reshape(self.c, n, B.shape[1])
        V = self.poly.values(x)
        G = self.poly.gradients(x)
        vals = np.tensordot(V, Bc, axes=([1], [1]))                          # (q, c, m)
        jac = np.tensordot(G, Bc, axes=([2], [1])).transpose(0, 2, 1, 3)    # (q, c, a, m)
        return vals, jac


def d_op(k, l, vals, jac):
    """Exterior derivative d^k on an l-dimensional simplex in its own
    coordinates (grad, rot / curl, div), shape (N, c', m)."""
    if k == 0:
        return jac[:, 0, :, :]
    if k == 1 and l == 2:
        return (jac[:, 1, 0, :] - jac[:, 0, 1, :])[:, None, :]
    if k == 1 and l == 3:
        return np.stack([jac[:, 2, 1] - jac[:, 1, 2],
                         jac[:, 0, 2] - jac[:, 2, 0],
                         jac[:, 1, 0] - jac[:, 0, 1]], axis=1)
    if k == 2 and l == 3:
        return (jac[:, 0, 0] + jac[:, 1, 1] + jac[:, 2, 2])[:, None, :]
    raise ValueError((k, l))


def d_family(family, l, vals, jac):
    """The exterior derivative of a family's fields on an l-simplex: div for
    the H(div) families in any dimension, otherwise d^k."""
    if family in DIV_FAMILIES:
        return sum(jac[:, a, a] for a in range(l))[:, None, :]
    return d_op(FORM[family], l, vals, jac)


def trace_family(family, A, vals):
    """tr of a family's field on a subsimplex with tangent frame A: the normal
    component n.v for H(div) on a facet (n = a_1 x a_2 in 3D, n = R a_1 in
    2D), otherwise tr^k (eq:tr-k)."""
    d, l = A.shape
    if family in DIV_FAMILIES and l == d - 1 and d == 2:
        n = np.array([A[1, 0], -A[0, 0]])
        return np.einsum("a,qam->qm", n, vals)[:, None, :]
    return trace(form_degree(d, family), A, vals)


def _orth_range(S, expected):
    U, s, _ = np.linalg.svd(S, full_matrices=False)
    rank = int(np.sum(s > 1e-10 * s[0]))
    if rank != expected:
        raise AssertionError(f"rank {rank} != expected dimension {expected}")
    if rank < len(s) and s[rank] > 1e-12 * s[0]:
        raise AssertionError("no clear rank gap")
    return U[:, :rank]


def space_dim(l, family, p):
    """Dimensions of the first/second kind spaces (Arnold, Falk & Winther
    2006, Sec. 5), used to check the numerically computed ranges."""
    from math import comb
    P = lambda q: comb(q + l, l) if q >= 0 else 0
    if family == "CG":
        return P(p)
    if family in ("NedTwo", "BDM"):
        return l * P(p)
    if family == "Ned":
        if l == 2:
            return p * (p + 2)
        return p * (p + 2) * (p + 3) // 2
    if family == "RT":
        if l == 2:
            return p * (p + 2)
        return p * (p + 1) * (p + 3) // 2
    raise ValueError(family)


@functools.lru_cache(maxsize=None)
def make_space(l, family, p):
    """X^k_p on the equilateral l-simplex (eq:first-kind-def,
    eq:second-kind-def; in 2D the first-kind H(curl) space is
    P_{p-1}^2 + P_{p-1} x_perp)."""
    poly = PolyBasis(l, p)
    n = poly.n
    if family == "CG":
        return Space(l, 1, poly, np.eye(n), family, p)
    if family in ("NedTwo", "BDM"):
        # second kind (eq:second-kind-def): all of P_p^l
        return Space(l, l, poly, np.eye(l * n), family, p)
    c = l
    low = np.flatnonzero(poly.degree <= p - 1)
    cols = []
    for comp in range(c):
        for m in low:
            e = np.zeros(c * n)
            e[comp * n + m] = 1.0
            cols.append(e)
    x, w = quadrature(l, p + 2)
    V = poly.values(x)
    extra = []
    if family == "Ned" and l == 3:
        for m in low:
            for comp in range(3):
                f = np.zeros((x.shape[0], 3))
                f[:, comp] = V[:, m]
                extra.append(np.cross(f, x))
    elif family == "Ned" and l == 2:
        for m in low:
            extra.append(np.stack([-x[:, 1] * V[:, m], x[:, 0] * V[:, m]], axis=1))
    elif family == "RT":
        for m in low:
            extra.append(x * V[:, m][:, None])
    else:
        raise ValueError((l, family))
    for f in extra:
        # L2 projection onto P_p^c (exact: f is a polynomial of degree <= p)
        cols.append(np.einsum("q,qc,qn->cn", w, f, V).ravel())
    S = np.stack(cols, axis=1)
    B = _orth_range(S, space_dim(l, family, p))
    return Space(l, c, poly, B, family, p)


# --------------------------------------------------------------------------
# subentity maps
# --------------------------------------------------------------------------
def entity_map(d, verts):
    """Affine map from the equilateral (len(verts)-1)-simplex onto the
    subsimplex of T_hat (dim d) with the given local vertices, sending
    reference vertex m to verts[m] (R5).  Returns (origin, A) with
    x = origin + A (y - yhat_0)."""
    l = len(verts) - 1
    V = EQ_VERTICES[d]
    if l == 0:
        return V[verts[0]], np.zeros((d, 0)), EQ_VERTICES[0][0]
    S = EQ_VERTICES[l]
    A = (V[list(verts[1:])] - V[verts[0]]).T @ np.linalg.inv((S[1:] - S[0]).T)
    return V[verts[0]], A, S[0]


def entities(d):
    """Subsimplices of the reference d-simplex: ascending local vertex tuples,
    grouped by dimension (R5)."""
    return [list(combinations(range(d + 1), l + 1)) for l in range(d + 1)]


def trace(k, A, vals):
    """tr^k of a field on a subsimplex with tangent frame A (eq:tr-k):
    value, tangential components A^T v, or normal component n.v with
    n = a_1 x a_2 (a (d-1)-subsimplex in 3D)."""
    l = A.shape[1]
    d = A.shape[0]
    if k == 0:
        return vals
    if l == d:
        return vals
    if k == 1:
        return np.einsum("al,qam->qlm", A, vals)
    if k == 2 and l == 2 and d == 3:
        nrm = np.cross(A[:, 0], A[:, 1])
        return np.einsum("a,qam->qm", nrm, vals)[:, None, :]
    raise ValueError((k, l, d))


# --------------------------------------------------------------------------
# bubble spaces and eigenbases (eq:ref-eval-problem-x, -aug)
# --------------------------------------------------------------------------
def bubble_space(l, family, p):
    """Orthonormal coefficient basis of X_ring^k(S_hat): the fields of the
    l-dimensional space whose trace vanishes on every facet."""
    sp = make_space(l, family, p)
    k = form_degree(l, family)
    rows = []
    for F in combinations(range(l + 1), l):
        o, A, y0 = entity_map(l, F)
        if l - 1 == 0:
            z = o[None, :]
            tw = np.ones(1)
            test = np.ones((1, 1))
        else:
            zq, tw = quadrature(l - 1, p + 2)
            z = o + (zq - y0) @ A.T
            test = PolyBasis(l - 1, p).values(zq)
        vals, _ = sp.field(z)
        tr = trace_family(family, A, vals) if l - 1 > 0 or k == 0 else None
        if tr is None:
            raise ValueError("no trace of a k>0 form on a vertex")
        # moments of each trace component against P_p on the facet
        rows.append(np.einsum("q,qcm,qn->cnm", tw, tr, test).reshape(-1, sp.m))
    C = np.concatenate(rows, axis=0)
    _, s, Vt = np.linalg.svd(C, full_matrices=True)
    rank = int(np.sum(s > 1e-10 * s[0]))
    null = Vt[rank:].T
    return sp, sp.B @ null


class EigenBasis:
    """psi_{S,j} (type-I bubble eigenfunctions) on the equilateral
    l-simplex, in primal coefficients, with mu_j and lambda_j = 1/mu_j."""

    def __init__(self, l, family, p, space, Psi, mu, mu_all, n_ker, cond_probe):
        self.l, self.family, self.p, self.space = l, family, p, space
        self.Psi, self.mu, self.lam = Psi, mu, 1.0 / mu
        self.mu_all, self.n_ker, self.cond_probe = mu_all, n_ker, cond_probe
        self.clusters = []
        self.k = form_degree(l, family)
        self.N = Psi.shape[1]

    def values(self, x):
        vals, jac = self.space.field(x, self.Psi)
        return vals

    def dvalues(self, x):
        vals, jac = self.space.field(x, self.Psi)
        return d_family(self.family, self.l, vals, jac)


def kernel_family(family, p, l=3):
    """The (k-1)-form family whose bubble derivatives span ker d_S on the
    k-form bubbles of an l-simplex (exact bubble complex,
    eq:bubble-subcomplex); for RT_p in 2D it is CG_p (the remark after
    eq:hdiv-dofs)."""
    if family == "CG":
        return None
    if family == "Ned":
        return ("CG", p)
    if family == "NedTwo":
        return ("CG", p + 1)
    if family == "RT":
        return ("CG", p) if l == 2 else ("NedTwo", p)
    if family == "BDM":
        # the remark after eq:hdiv-dofs: X^0 = CG_{p+1} in 2D; in 3D the
        # eigenfunctions are those of NedTwo_{p+1} (second kind, as for RT)
        return ("CG", p + 1) if l == 2 else ("NedTwo", p + 1)
    raise ValueError(family)


def probes(l, c, m):
    """The first m probe functionals of the canonicalisation rule (R2):
    points z_i in the l-simplex and directions e_i (c components)."""
    g = splitmix64_stream(0x5EED0000 + 256 * l + c)
    V = EQ_VERTICES[l]
    pts, dirs = [], []
    for _ in range(m):
        u = np.array([next(g) for _ in range(l + 1)])
        bary = (0.25 + u) / np.sum(0.25 + u)
        pts.append(bary @ V)
        dirs.append(np.array([2.0 * next(g) - 1.0 for _ in range(c)]) if c > 1 else np.ones(1))
    return np.array(pts), np.array(dirs)


def bubble_eigenproblem(l, family, p):
    """The generalized eigenproblem K c = mu M c of eq:ref-eval-problem-x-aug on
    the bubble space (M the L2 Gram matrix, K that of d_S), solved by
    scipy's eigh (M-orthonormal eigenvectors, ascending mu).  Returns the
    space, the bubble basis Bb, K, mu, the eigenvectors and the number of
    kernel eigenpairs to discard (R3: the dimension N^{k-1}_S of
    eq:bubble-trace-dim-counts, not a threshold)."""
    sp, Bb = bubble_space(l, family, p)
    if Bb.shape[1] == 0:
        return sp, Bb, None, np.zeros(0), None, 0
    x, w = quadrature(l, p + 2)
    vals, jac = sp.field(x, Bb)
    dv = d_family(family, l, vals, jac)
    M = np.einsum("q,qcm,qcn->mn", w, vals, vals)
    K = np.einsum("q,qcm,qcn->mn", w, dv, dv)
    mu, Vec = sla.eigh(K, M)
    kf = kernel_family(family, p, l)
    n_ker = 0 if kf is None else eigenbasis(l, *kf).N
    if n_ker:
        assert np.all(np.abs(mu[:n_ker]) < 1e-10 * mu[-1]), "kernel not null"
        assert mu[n_ker] > 1e-8 * mu[-1], "kernel dimension mismatch"
    return sp, Bb, K, mu, Vec, n_ker


@functools.lru_cache(maxsize=None)
def eigenbasis(l, family, p):
    """Type-I eigenbasis of eq:ref-eval-problem-x on the equilateral
    l-simplex, via the augmented problem eq:ref-eval-problem-x-aug."""
    sp, Bb, K, mu, Vec, n_ker = bubble_eigenproblem(l, family, p)
    if Bb.shape[1] == 0:
        return EigenBasis(l, family, p, sp, Bb, np.zeros(0), np.zeros(0), 0, 1.0)
    mu_keep = mu[n_ker:]
    W, mu_k, clusters = canonical_clusters(l, sp, Bb, K, mu_keep, Vec[:, n_ker:])
    Psi = Bb @ (W / np.sqrt(mu_k)) if len(mu_k) else Bb @ W
    eb = EigenBasis(l, family, p, sp, Psi, mu_k, mu, n_ker,
                    max(c[2] for c in clusters) if clusters else 1.0)
    eb.clusters = clusters
    return eb


def cluster_bounds(mu):
    """R2 clusters of a non-decreasing mu: maximal runs in which each mu is
    within relative distance TAU of its predecessor, as (start, stop)."""
    out, i = [], 0
    while i < len(mu):
        j = i + 1
        while j < len(mu) and (mu[j] - mu[j - 1]) < TAU * mu[j]:
            j += 1
        out.append((i, j))
        i = j
    return out


def canonical_clusters(l, sp, Bb, K, mu, W):
    """R2: the canonical basis of each cluster of equal eigenvalues.

    W holds M-orthonormal eigenvectors (coefficients over the bubble basis
    Bb) for the ascending eigenvalues mu.  Inside a cluster of m columns the
    basis is rotated to W R with R = Y^T (Y Y^T)^{-1/2}, Y_ij = pi_i(W_j) for
    the first m probe functionals.  For any orthogonal Q, (W Q) R' = W R, so
    the result does not depend on which orthonormal basis of the cluster
    the eigensolver returned.  Returns the rotated W, the Rayleigh quotients
    of its columns, and per cluster (start, size, cond(Y))."""
    out_cols, out_mu, clusters = [], [], []
    for i, j in cluster_bounds(mu):
        Wc = W[:, i:j]
        m = j - i
        pts, dirs = probes(l, sp.c, m)
        if sp.family in DIV_FAMILIES and l == 2:
            dirs = np.stack([dirs[:, 1], -dirs[:, 0]], axis=1)   # R e: 2D H(div) = R (2D H(curl))
        pv, _ = sp.field(pts, Bb @ Wc)          # (m, c, m)
        Y = np.einsum("ic,icj->ij", dirs, pv)   # Y_ij = pi_i(W_j)
        ev, evec = np.linalg.eigh(Y @ Y.T)
        R = Y.T @ (evec @ np.diag(ev ** -0.5) @ evec.T)
        Wc = Wc @ R
        clusters.append((i, m, float(np.sqrt(ev.max() / ev.min()))))
        for c_ in range(m):
            out_mu.append(Wc[:, c_] @ K @ Wc[:, c_])
            out_cols.append(Wc[:, c_])
    Wout = np.stack(out_cols, axis=1) if out_cols else np.zeros((W.shape[0], 0))
    return Wout, np.array(out_mu), clusters


def cluster_census(eb):
    """Gap statistics of an eigenbasis under the R2 cluster rule: the smallest
    relative gap between consecutive clusters, the largest relative spread
    inside a cluster, the largest cond(Y) and the largest cluster size."""
    mu = eb.mu_all[eb.n_ker:]
    bounds = cluster_bounds(mu)
    gaps = [(mu[j] - mu[j - 1]) / mu[j] for (_, j) in bounds[:-1]]
    spread = [(mu[j - 1] - mu[i]) / mu[j - 1] for (i, j) in bounds]
    return {"min_gap": min(gaps) if gaps else np.inf,
            "max_spread": max(spread) if spread else 0.0,
            "max_cond": max((c[2] for c in eb.clusters), default=1.0),
            "max_size": max((c[1] for c in eb.clusters), default=0)}


# --------------------------------------------------------------------------
# degrees of freedom and the dual basis (eq:abstract-dofs, Sec. 3.4)
# --------------------------------------------------------------------------
class DofInfo:
    __slots__ = ("entity_dim", "entity_index", "verts", "kind", "j")

    def __init__(self, entity_dim, entity_index, verts, kind, j):
        self.entity_dim, self.entity_index = entity_dim, entity_index
        self.verts, self.kind, self.j = verts, kind, j


class Element:
    """The Ciarlet element (T_hat, X^k_p, L) of Sec. 3.3 and its dual basis."""

    def __init__(self, d, family, p):
        if family not in ("CG", "Ned", "RT", "NedTwo", "BDM"):
            raise ValueError(family)
        self.d, self.family, self.p, self.k = d, family, p, form_degree(d, family)
        self.space = make_space(d, family, p)
        self.dofs = []
        rows = []
        k = self.k
        # functionals act on the whole primal space P_p^c (identity basis)
        full = np.eye(self.space.B.shape[0])
        # the (k-1)-form family whose bubble derivatives give the type-II dofs:
        # CG_p for Ned_p, NedTwo_p for RT_p (R4; CG_p in 2D), CG_{p+1} for
        # NedTwo_p, NedTwo_{p+1} for BDM_p
        typeII = kernel_family(family, p, d)
        for l, ents in enumerate(entities(d)):
            for ei, verts in enumerate(ents):
                o, A, y0 = entity_map(d, verts)
                if l == 0:
                    xq = o[None, :]
                    wq = np.ones(1)
                    yq = np.zeros((1, 0))
                else:
                    yq, wq = quadrature(l, p + 2)
                    xq = o + (yq - y0) @ A.T
                vals, jac = self.space.field(xq, full)
                if l == k:
                    # Whitney moment (1, tr v)_S  (point value for k = 0)
                    tr = trace_family(family, A, vals)
                    rows.append(np.einsum("q,qm->m", wq, tr[:, 0, :]))
                    self.dofs.append(DofInfo(l, ei, verts, "W", 0))
                if l > k:
                    # type-I: (d_S psi_j, d_S tr v)_S, via tr^{k+1} d v
                    eb = eigenbasis(l, family, p)
                    dpsi = eb.dvalues(yq)
                    dv = d_family(family, d, vals, jac)
                    trdv = trace(k + 1, A, dv)
                    for j in range(eb.N):
                        rows.append(np.einsum("q,qc,qcm->m", wq, dpsi[:, :, j], trdv))
                        self.dofs.append(DofInfo(l, ei, verts, "I", j))
                if l >= k and k >= 1 and l >= 1:
                    # type-II: (d_S psi^{k-1}_j, tr v)_S
                    eb = eigenbasis(l, *typeII)
                    dpsi = eb.dvalues(yq)
                    if family in DIV_FAMILIES and d == 2 and l == 2:
                        dpsi = rot90(dpsi)      # curl = R grad in 2D
                    tr = trace_family(family, A, vals)
                    for j in range(eb.N):
                        rows.append(np.einsum("q,qc,qcm->m", wq, dpsi[:, :, j], tr))
                        self.dofs.append(DofInfo(l, ei, verts, "II", j))
        self.L = np.array(rows)            # dofs as functionals on P_p^c
        self.D = self.L @ self.space.B     # D_ij = l_i(p_j), p_j basis of X
        self.n = self.D.shape[0]
        if self.n != self.space.m:
            raise AssertionError("dof count != dim X (unisolvence count)")
        self.C = np.linalg.solve(self.D, np.eye(self.n))
        self.coef = self.space.B @ self.C   # basis functions in primal coefficients
        self.cond_D = np.linalg.cond(self.D)

    # ---- tabulation --------------------------------------------------------
    def tabulate(self, x):
        """values (N, c, n) and exterior derivative (N, c', n) at points x."""
        vals, jac = self.space.field(x, self.coef)
        if self.k == 0:
            dv = jac[:, 0, :, :]
        else:
            dv = d_family(self.family, self.d, vals, jac)
        return vals, dv

    def counts(self):
        """number of dofs per entity dimension (uniform by construction)."""
        out = []
        for l, ents in enumerate(entities(self.d)):
            out.append(sum(1 for di in self.dofs if di.entity_dim == l and di.entity_index == 0))
        return out

    def interior(self):
        return np.array([di.entity_dim == self.d for di in self.dofs])


@functools.lru_cache(maxsize=None)
def element(d, family, p):
    return Element(d, family, p)


def reference_matrices(el):
    """Mass and stiffness on T_hat, M_ij = (phi_i, phi_j), K_ij = (d phi_i,
    d phi_j) (Sec. 4.2)."""
    x, w = quadrature(el.d, el.p + 2)
    vals, dv = el.tabulate(x)
    M = np.einsum("q,qci,qcj->ij", w, vals, vals)
    K = np.einsum("q,qci,qcj->ij", w, dv, dv)
    return M, K
