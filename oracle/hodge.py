"""Hodge Laplacians of the first-kind de Rham complex with the block-diagonal
(weighted) Riesz-map preconditioner and MINRES (Sec. 7.2,
sec:results-hodge-laplace; the appendix on augmented Lagrangian
preconditioning for Hodge Laplacians).  Test infrastructure: a plain FP64
restatement, used only by the tests and the benchmark's CPU baseline.

For k = 1 (X^0 x X^1 = CG_p x Ned_p), k = 2 (X^1 x X^2 = Ned_p x RT_p) and
k = 3 (X^2 x X^3 = RT_p x DG_{p-1}, the mixed scalar Poisson problem; d^3 =
0, so K_3 = 0), eq:hodge-laplace with natural boundary conditions reads, in
the bases of the two spaces,
    [ -M_{k-1}    D^T M_k ] [sigma]   [0]
    [  M_k D      K_k     ] [  u  ] = [b]
with M the mass matrices, K_k the matrix of (d u, d v) and D the exterior
derivative X^{k-1} -> X^k in the X^k basis (d X^{k-1}_p lies in X^k_p: the
discrete complex is exact, so (d sigma, v) = v^T M_k D sigma and the
stiffness of X^{k-1} is D^T M_k D).

The preconditioner is eq:augmented-lagrangian: the Riesz maps
(sigma, tau) + gamma (d sigma, d tau) on X^{k-1} and gamma^{-1} (u, v) +
(d u, d v) on X^k, each replaced by one application of the hybrid Schwarz
method of the Riesz experiments (the weak form a = beta (u, v) + alpha
(d u, d v): (alpha, beta) = (gamma, 1) and (1, 1 / gamma)), or inverted
exactly.  DG_{p-1} has the L2-orthonormal Dubiner basis of P_{p-1} pulled
back as a 3-form (psi = psi_hat o F^{-1} / det J), so its mass matrix is
diagonal, 1 / |det J_T| per cell, and its Riesz map gamma^{-1} M_3 is
inverted exactly (the paper's J(X^3), exact because the basis is
orthogonal).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .element import element
from .mesh import Topology
from .operator import all_cell_matrices, assemble
from .precond import HybridSchwarz
from .simplex import EQ_VERTICES, PolyBasis, quadrature

PAIRS_K = {1: ("CG", "Ned"), 2: ("Ned", "RT"), 3: ("RT", "DG")}


def divergence_reference_dg(p, d=3):
    """(n_dg x n_rt): the coefficients of div phi_j (RT_p reference basis) in
    the L2-orthonormal Dubiner basis of P_{p-1} on the reference cell, which
    is the DG_{p-1} basis (div RT_p = P_{p-1})."""
    el = element(d, "RT", p)
    xq, wq = quadrature(d, p + 2)
    _, dv = el.tabulate(xq)                               # (N, 1, n_rt)
    V = PolyBasis(d, p - 1).values(xq)                    # (N, n_dg)
    return np.einsum("q,qi,qj->ij", wq, V, dv[:, 0, :])


def cell_volume_ratio(X, C):
    """|det J_T| of the map from the equilateral reference cell, per cell."""
    E = EQ_VERTICES[3]
    Ei = np.linalg.inv((E[1:] - E[0]).T)
    out = np.empty(len(C))
    for c, cell in enumerate(np.sort(C, axis=1)):
        Xc = X[cell]
        out[c] = abs(np.linalg.det((Xc[1:] - Xc[0]).T @ Ei))
    return out


def derivative_reference(k, p, d=3):
    """D_hat (n_k x n_{k-1}): coefficients of d phi^{k-1}_j in the X^k basis
    on the reference cell -- the X^k dofs applied to the exterior
    derivative of each X^{k-1} basis function, after an exact L2 projection
    onto P_p^c (d X^{k-1}_p lies in P_p^c)."""
    fa, fb = PAIRS_K[k]
    ea, eb = element(d, fa, p), element(d, fb, p)
    xq, wq = quadrature(d, p + 2)
    _, dv = ea.tabulate(xq)                               # (N, c, n_{k-1})
    V = eb.space.poly.values(xq)                          # (N, n_poly), orthonormal
    proj = np.einsum("q,qcm,qn->cnm", wq, dv, V)
    return eb.L @ proj.reshape(-1, dv.shape[2])


def derivative_matrix(top0, top1, Dhat):
    """Global D (n1 x n0).  The pullbacks commute with d, and both bases
    are pulled back from the sorted-vertex reference cell, so D restricted
    to every cell is D_hat; entries shared by cells coincide (checked)."""
    n1, n0 = Dhat.shape
    rows = np.repeat(top1.cell_dofs, n0, axis=1).ravel()
    cols = np.tile(top0.cell_dofs, (1, n1)).ravel()
    vals = np.tile(Dhat.ravel(), top0.n_cells)
    nz = vals != 0.0
    rows, cols, vals = rows[nz], cols[nz], vals[nz]
    key = rows * top0.n_dofs + cols
    order = np.argsort(key, kind="stable")
    key, vals = key[order], vals[order]
    first = np.r_[True, key[1:] != key[:-1]]
    uk, uv = key[first], vals[first]
    # every cell that touches an entry gives the same value
    grp = np.cumsum(first) - 1
    spread = np.abs(vals - uv[grp]).max() if len(vals) else 0.0
    if spread > 1e-12 * max(1.0, np.abs(vals).max()):
        raise AssertionError("derivative entries differ between cells: %g" % spread)
    return sp.csr_matrix((uv, (uk // top0.n_dofs, uk % top0.n_dofs)), shape=(top1.n_dofs, top0.n_dofs))


class HodgeLaplacian:
    """The mixed system and its block preconditioner on one mesh."""

    def __init__(self, X, C, k, p, gamma=1.0, exact=False, decomposition="paper", preconditioner=True):
        """preconditioner=False builds the mixed operator only (no Riesz maps
        or Schwarz set-up): for checking residuals of solutions computed
        elsewhere."""
        fa, fb = PAIRS_K[k]
        self.k, self.p, self.gamma = k, p, gamma
        if k == 3:
            self._init_dg(X, C, p, gamma, exact, decomposition, preconditioner)
            return
        self.el0, self.el1 = element(3, fa, p), element(3, fb, p)
        self.top0, self.top1 = Topology(X, C, self.el0), Topology(X, C, self.el1)
        self.n0, self.n1 = self.top0.n_dofs, self.top1.n_dofs
        self.D = derivative_matrix(self.top0, self.top1, derivative_reference(k, p))
        self.M0 = assemble(self.top0, all_cell_matrices(self.el0, self.top0, alpha=0.0, beta=1.0))
        self.M1 = assemble(self.top1, all_cell_matrices(self.el1, self.top1, alpha=0.0, beta=1.0))
        self.K1 = assemble(self.top1, all_cell_matrices(self.el1, self.top1, alpha=1.0, beta=0.0))
        M1D = (self.M1 @ self.D).tocsr()
        self.A = sp.bmat([[-self.M0, M1D.T], [M1D, self.K1]]).tocsr()
        if not preconditioner:
            return
        # the weighted Riesz maps of eq:augmented-lagrangian
        self.R0 = assemble(self.top0, all_cell_matrices(self.el0, self.top0, alpha=gamma, beta=1.0))
        self.R1 = assemble(self.top1, all_cell_matrices(self.el1, self.top1, alpha=1.0, beta=1.0 / gamma))
        if exact:
            self.P0 = spla.splu(self.R0.tocsc()).solve
            self.P1 = spla.splu(self.R1.tocsc()).solve
        else:
            self.P0 = HybridSchwarz(self.R0, self.top0, fa, decomposition=decomposition).apply
            self.P1 = HybridSchwarz(self.R1, self.top1, fb, decomposition=decomposition).apply

    def _init_dg(self, X, C, p, gamma, exact, decomposition, preconditioner=True):
        self.el0 = element(3, "RT", p)
        self.top0 = Topology(X, C, self.el0)
        self.n0 = self.top0.n_dofs
        Dh = divergence_reference_dg(p)
        self.ndg = Dh.shape[0]
        nc = self.top0.n_cells
        self.n1 = nc * self.ndg
        rows = (np.arange(nc)[:, None, None] * self.ndg + np.arange(self.ndg)[None, :, None]) \
            * np.ones((1, 1, Dh.shape[1]), dtype=np.int64)
        cols = np.broadcast_to(self.top0.cell_dofs[:, None, :], rows.shape)
        vals = np.broadcast_to(Dh[None], rows.shape)
        self.D = sp.csr_matrix((vals.ravel(), (rows.ravel(), cols.ravel())), shape=(self.n1, self.n0))
        self.detJ = cell_volume_ratio(self.top0.coords, C)
        m3 = np.repeat(1.0 / self.detJ, self.ndg)
        self.M0 = assemble(self.top0, all_cell_matrices(self.el0, self.top0, alpha=0.0, beta=1.0))
        self.M1 = sp.diags(m3).tocsr()
        self.K1 = sp.csr_matrix((self.n1, self.n1))
        M1D = (self.M1 @ self.D).tocsr()
        self.A = sp.bmat([[-self.M0, M1D.T], [M1D, None]], format="csr")
        if not preconditioner:
            return
        self.R0 = assemble(self.top0, all_cell_matrices(self.el0, self.top0, alpha=gamma, beta=1.0))
        self.R1 = sp.diags(m3 / gamma).tocsr()
        if exact:
            self.P0 = spla.splu(self.R0.tocsc()).solve
        else:
            self.P0 = HybridSchwarz(self.R0, self.top0, "RT", decomposition=decomposition).apply
        inv1 = gamma / m3
        self.P1 = lambda r: inv1 * r

    def apply_P(self, r):
        return np.concatenate([self.P0(r[:self.n0]), self.P1(r[self.n0:])])

    def rhs(self, b1):
        """[0; b1]: the load acts on the X^k equation."""
        return np.concatenate([np.zeros(self.n0), b1])


def minres(apply_A, apply_P, b, rtol=1e-8, maxit=1000):
    """Preconditioned MINRES (Paige & Saunders, SIAM J. Numer. Anal. 12,
    1975) for symmetric A and symmetric positive definite P: the Lanczos
    process in the P^{-1} inner product and the Givens QR of its tridiagonal
    matrix, x_0 = 0.  Stops when the preconditioned residual norm
    ||r_j||_P = |phibar_j| <= rtol ||b||_P.  Returns (x, info) with info =
    dict(iterations, rel_residual (preconditioned, recursive), history,
    converged)."""
    n = b.shape[0]
    x = np.zeros(n)
    r1 = b.copy()
    y = apply_P(r1)
    beta1 = np.sqrt(r1 @ y)
    if beta1 == 0.0:
        return x, dict(iterations=0, rel_residual=0.0, history=[0.0], converged=True)
    oldb, beta, dbar, epsln = 0.0, beta1, 0.0, 0.0
    phibar, cs, sn = beta1, -1.0, 0.0
    w = np.zeros(n)
    w2 = np.zeros(n)
    r2 = r1.copy()
    hist = [1.0]
    it = 0
    for it in range(1, maxit + 1):
        v = y / beta
        y = apply_A(v)
        if it >= 2:
            y = y - (beta / oldb) * r1
        alfa = v @ y
        y = y - (alfa / beta) * r2
        r1, r2 = r2, y
        y = apply_P(r2)
        oldb, beta = beta, np.sqrt(r2 @ y)
        oldeps = epsln
        delta = cs * dbar + sn * alfa
        gbar = sn * dbar - cs * alfa
        epsln = sn * beta
        dbar = -cs * beta
        gamma = max(np.hypot(gbar, beta), np.finfo(float).eps)
        cs, sn = gbar / gamma, beta / gamma
        phi = cs * phibar
        phibar = sn * phibar
        w1, w2 = w2, w
        w = (v - oldeps * w1 - delta * w2) / gamma
        x = x + phi * w
        hist.append(abs(phibar) / beta1)
        if abs(phibar) <= rtol * beta1:
            break
    return x, dict(iterations=it, rel_residual=hist[-1], history=hist, converged=hist[-1] <= rtol)


def theorem_spectrum(H):
    """The generalized eigenvalues of (A, B_gamma) that
    thm:augmented-lagrangian-hl predicts when B_gamma is the exact weighted
    Riesz map and the domain has no harmonic k-forms: -1 with multiplicity
    n_{k-1}, mu gamma / (mu gamma + 1) for the nonzero eigenvalues mu of
    K_k u = mu M_k u, and nu gamma / (nu gamma + 1) for the nonzero
    eigenvalues nu of K_{k-1} s = nu M_{k-1} s (K_{k-1} = D^T M_k D)."""
    g = H.gamma
    K0 = (H.D.T @ H.M1 @ H.D).toarray()
    mu = sla.eigh(H.K1.toarray(), H.M1.toarray(), eigvals_only=True)
    nu = sla.eigh(K0, H.M0.toarray(), eigvals_only=True)
    tol_mu, tol_nu = 1e-9 * mu.max(), 1e-9 * nu.max()
    lam = [-1.0] * H.n0
    lam += [m * g / (m * g + 1) for m in mu if m > tol_mu]
    lam += [v * g / (v * g + 1) for v in nu if v > tol_nu]
    return np.sort(np.array(lam))
