"""Cell matrices of the Riesz-map weak form and their assembly.

eq:weak-form: a^k(u, v) = (u, beta v) + (d^k u, alpha d^k v).  A global basis
function on T is the pullback eq:pullback-3d-def of a reference basis
function: identity (H(grad)), covariant Piola J^{-T} (H(curl)), contravariant
Piola J / det J (H(div), also in 2D where it is k = 1).  The derivatives map
as J^{-T} grad, J curl / det J (3D), rot / det J (2D) and div / det J.  ``cell_matrix`` evaluates the definition by quadrature on
the physical cell; ``reference_stack`` / ``cell_weights`` give the same
matrix as a weighted sum of reference integrals (used only to check the
library's exported tables and as an identity pin).
"""
import numpy as np
import scipy.sparse as sp

from .simplex import EQ_VERTICES, quadrature

PAIRS = {2: [(0, 0), (1, 1), (0, 1)], 3: [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]}


def piola(el):
    """0 identity, 1 covariant, 2 contravariant."""
    if el.k == 0:
        return 0
    return 2 if el.family in ("RT", "BDM") else 1


def physical_fields(el, J, vals, dv):
    """Pulled-back values and derivatives on a cell with Jacobian J."""
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    kind = piola(el)
    if kind == 0:
        return vals, np.einsum("ba,qbn->qan", Jinv, dv)                 # J^{-T} grad
    if kind == 1:
        v = np.einsum("ba,qbn->qan", Jinv, vals)                        # J^{-T} v
        if el.d == 2:
            return v, dv / det                                          # rot / det J
        return v, np.einsum("ab,qbn->qan", J, dv) / det                 # J curl / det J
    return np.einsum("ab,qbn->qan", J, vals) / det, dv / det           # J v / det J, div / det J


def jacobian(el, X):
    """J_T of F_T(x_hat) = x_0 + J (x_hat - e_0), reference vertex m -> X[m]."""
    E = EQ_VERTICES[el.d]
    return (X[1:] - X[0]).T @ np.linalg.inv((E[1:] - E[0]).T)


def cell_matrix(el, X, alpha=1.0, beta=1.0, tab=None):
    """A_T[i, j] = a^k(phi_j, phi_i) restricted to the cell with sorted vertex
    coordinates X ((d+1, d)), by quadrature of the pulled-back basis."""
    if tab is None:
        xq, wq = quadrature(el.d, el.p + 2)
        tab = (wq,) + el.tabulate(xq)
    wq, vals, dv = tab
    J = jacobian(el, X)
    v, dphys = physical_fields(el, J, vals, dv)
    s = abs(np.linalg.det(J))
    # sum over quadrature points and components as one matrix product
    nq, n = v.shape[0], v.shape[2]
    V2 = v.reshape(-1, n)
    D2 = dphys.reshape(-1, n)
    M = V2.T @ (V2 * np.repeat(wq, v.shape[1])[:, None]) * s
    K = D2.T @ (D2 * np.repeat(wq, dphys.shape[1])[:, None]) * s
    return beta * M + alpha * K


def all_cell_matrices(el, top, alpha=1.0, beta=1.0):
    xq, wq = quadrature(el.d, el.p + 2)
    tab = (wq,) + el.tabulate(xq)
    out = np.empty((top.n_cells, el.n, el.n))
    for c in range(top.n_cells):
        out[c] = cell_matrix(el, top.coords[top.cells[c]], alpha, beta, tab)
    return out


def assemble(top, Acell):
    """Global sparse A = sum_T P_T^T A_T P_T."""
    nc, n, _ = Acell.shape
    rows = np.repeat(top.cell_dofs, n, axis=1).ravel()
    cols = np.tile(top.cell_dofs, (1, n)).ravel()
    A = sp.coo_matrix((Acell.ravel(), (rows, cols)), shape=(top.n_dofs, top.n_dofs))
    return A.tocsr()


def element_apply(top, Acell, x):
    """Matrix-free y = sum_T P_T^T A_T P_T x (x: (n_dofs,) or (n_dofs, r))."""
    xs = x[top.cell_dofs]                                  # (nc, n[, r])
    ys = np.einsum("cij,cj...->ci...", Acell, xs)
    y = np.zeros_like(x)
    np.add.at(y, top.cell_dofs, ys)
    return y


# ---- stacked reference form ------------------------------------------------
def reference_stack(el):
    """R_hat_q: the symmetric reference integrals whose weighted sum is A_T.
    Order: the mass family, then the derivative family; a vector family is
    listed by component pairs (00, 11, 22, 01, 02, 12) with the off-diagonal
    pairs symmetrised (R_ab + R_ba), a scalar family is one matrix."""
    xq, wq = quadrature(el.d, el.p + 2)
    vals, dv = el.tabulate(xq)
    out = []
    for fam in (vals, dv):
        c = fam.shape[1]
        if c == 1:
            out.append(np.einsum("q,qi,qj->ij", wq, fam[:, 0], fam[:, 0]))
        else:
            for a, b in PAIRS[c]:
                R = np.einsum("q,qi,qj->ij", wq, fam[:, a], fam[:, b])
                out.append(R if a == b else R + R.T)
    return np.array(out)


def cell_weights(el, X, alpha=1.0, beta=1.0):
    """Weights w_{T,q} with A_T = sum_q w_{T,q} R_hat_q (from the Piola maps
    of eq:pullback-3d-def)."""
    J = jacobian(el, X)
    det = np.linalg.det(J)
    s = abs(det)
    Ji = np.linalg.inv(J)
    G = Ji @ Ji.T          # J^{-1} J^{-T}
    H = J.T @ J
    pr = lambda Mx: [Mx[a, b] for a, b in PAIRS[el.d]]
    kind = piola(el)
    if kind == 0:
        return np.array([beta * s] + pr(alpha * s * G))
    if kind == 1:
        return np.array(pr(beta * s * G) + (pr(alpha * H / s) if el.d == 3 else [alpha / s]))
    return np.array(pr(beta * H / s) + [alpha / s])


def functional_load(el, top, u, du, alpha=1.0, beta=1.0, nq=None):
    """b_i = a^k(u*, phi_i) for a smooth field u* given by callables u(x) and
    du(x) (values (N, c) and d^k u* (N, c')), and the energy a^k(u*, u*);
    used for manufactured-solution convergence checks."""
    nq = nq or el.p + 4
    xq, wq = quadrature(el.d, nq)
    vals_r, dv_r = el.tabulate(xq)
    E = EQ_VERTICES[el.d]
    b = np.zeros(top.n_dofs)
    energy = 0.0
    for c in range(top.n_cells):
        X = top.coords[top.cells[c]]
        J = jacobian(el, X)
        det = np.linalg.det(J)
        xp = X[0] + (xq - E[0]) @ J.T
        v, dphys = physical_fields(el, J, vals_r, dv_r)
        U, DU = u(xp), du(xp)
        s = abs(det)
        b[top.cell_dofs[c]] += s * (beta * np.einsum("q,qc,qcn->n", wq, U, v)
                                    + alpha * np.einsum("q,qc,qcn->n", wq, DU, dphys))
        energy += s * (beta * np.einsum("q,qc,qc->", wq, U, U) + alpha * np.einsum("q,qc,qc->", wq, DU, DU))
    return b, energy
