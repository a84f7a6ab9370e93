"""Preconditioned conjugate gradients (the Krylov solver of Sec. 7.1) with a
Lanczos condition estimate from the CG coefficients.

Reading R10: the stopping test is on the unpreconditioned, recursively
updated residual, ||r_k||_2 <= rtol ||b||_2, checked after each update of r;
the true residual b - A x is reported beside it.
"""
import numpy as np


def pcg(apply_A, apply_P, b, rtol=1e-10, maxit=1000, x0=None, norm="residual"):
    """Hestenes-Stiefel PCG.  Returns (x, info) with info = dict(iterations,
    rel_residual (recursive), history, alphas, betas, converged).

    norm = "residual": stop when ||r_k|| <= rtol ||b|| (the library's test);
    norm = "preconditioned": stop when ||P^{-1} r_k|| <= rtol ||P^{-1} r_0||,
    the default test of the PETSc CG the paper's experiments ran with
    (reading R18)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_A(x) if x0 is not None else b.copy()
    bnorm = np.linalg.norm(b)
    hist = [np.linalg.norm(r) / bnorm]
    alphas, betas = [], []
    it = 0
    z = apply_P(r)
    z0norm = np.linalg.norm(z)

    def done(r, z):
        if norm == "preconditioned":
            return np.linalg.norm(z) <= rtol * z0norm
        return np.linalg.norm(r) <= rtol * bnorm

    converged = done(r, z)
    if not converged:
        p = z.copy()
        rz = r @ z
        while it < maxit:
            Ap = apply_A(p)
            pAp = p @ Ap
            if not pAp > 0:
                raise FloatingPointError("CG breakdown: p^T A p <= 0")
            alpha = rz / pAp
            x += alpha * p
            r -= alpha * Ap
            it += 1
            alphas.append(alpha)
            hist.append(np.linalg.norm(r) / bnorm)
            z = apply_P(r) if norm == "preconditioned" else None
            if done(r, z):
                converged = True
                break
            if z is None:
                z = apply_P(r)
            rz_new = r @ z
            beta = rz_new / rz
            rz = rz_new
            betas.append(beta)
            p = z + beta * p
    return x, dict(iterations=it, rel_residual=hist[-1], history=hist,
                   alphas=alphas, betas=betas, converged=converged)


def lanczos_extremes(alphas, betas):
    """Smallest and largest eigenvalue of the Lanczos tridiagonal matrix that
    k CG steps build implicitly (Golub & Van Loan, Sec. 11.3): diagonal
    1/alpha_j + beta_{j-1}/alpha_{j-1}, off-diagonal sqrt(beta_{j-1})/alpha_{j-1};
    only the first k - 1 betas enter."""
    k = len(alphas)
    if k == 0:
        return 1.0, 1.0
    T = np.zeros((k, k))
    for j in range(k):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j > 0:
            T[j, j - 1] = T[j - 1, j] = np.sqrt(betas[j - 1]) / alphas[j - 1]
    ev = np.linalg.eigvalsh(T)
    return ev[0], ev[-1]


def lanczos_condest(alphas, betas):
    """Extreme-eigenvalue ratio of the Lanczos tridiagonal matrix of CG."""
    lo, hi = lanczos_extremes(alphas, betas)
    return hi / lo
