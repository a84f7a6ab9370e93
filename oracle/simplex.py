"""Reference simplices, quadrature and an orthonormal polynomial basis.

The paper builds every basis on an *equilateral* reference simplex so that one
eigen-computation per subsimplex type serves every subentity (Sec. 3.3, the
paragraph after eq:ref-eval-problem-x).  Its size and placement are not
stated; the reading taken here is edge length 2 with the centroid at the
origin, so every edge and face of the reference tetrahedron is congruent to
the lower-dimensional reference simplex and the maps between them are
isometries.

Polynomials are represented in the orthonormal Dubiner (Proriol-Koornwinder)
basis, evaluated with the scaled three-term Jacobi recurrences in collapsed
coordinates (Dubiner 1991; Karniadakis & Sherwin, "Spectral/hp element
methods", Sec. 3.2).  Derivatives are taken by the complex-step method: for a
real polynomial f, Im f(x + i h e)/h = e . grad f(x) up to O(h^2) with no
subtractive cancellation, which is exact in FP64 for h = 1e-30.

Quadrature is the collapsed-coordinate (Stroud conical product) Gauss-Jacobi
rule, exact for polynomials of degree 2n - 1 with n points per direction.
"""
import functools

import numpy as np
from scipy.special import roots_jacobi

SQ3 = np.sqrt(3.0)
SQ6 = np.sqrt(6.0)

#: equilateral reference simplices, edge length 2, centroid at the origin
EQ_VERTICES = {
    0: np.zeros((1, 0)),
    1: np.array([[-1.0], [1.0]]),
    2: np.array([[-1.0, -1.0 / SQ3], [1.0, -1.0 / SQ3], [0.0, 2.0 / SQ3]]),
    3: np.array([[-1.0, -1.0 / SQ3, -1.0 / SQ6],
                 [1.0, -1.0 / SQ3, -1.0 / SQ6],
                 [0.0, 2.0 / SQ3, -1.0 / SQ6],
                 [0.0, 0.0, 3.0 / SQ6]]),
}

CSTEP = 1e-30


def poly_dim(d, p):
    """dim P_p in d variables."""
    if p < 0:
        return 0
    out = 1
    for i in range(1, d + 1):
        out = out * (p + i) // i
    return out


def _edge_matrix(d):
    v = EQ_VERTICES[d]
    return (v[1:] - v[0]).T  # d x d, columns e_m - e_0


def eq_to_collapsed_ref(x, d):
    """Map equilateral-simplex points to the collapsed-coordinate reference
    simplex with vertices -1 (all), and -1 + 2 e_m; vertex m maps to vertex m."""
    E = _edge_matrix(d)
    v0 = EQ_VERTICES[d][0]
    lam = np.linalg.solve(E, (x - v0).T).T  # barycentric coordinates 1..d
    return 2.0 * lam - 1.0


def collapsed_ref_to_eq(r, d):
    E = _edge_matrix(d)
    v0 = EQ_VERTICES[d][0]
    return v0 + ((r + 1.0) / 2.0) @ E.T


def quadrature(d, n):
    """Collapsed Gauss-Jacobi rule with n points per direction on the
    equilateral d-simplex; returns (points (N, d), weights (N,))."""
    if d == 0:
        return np.zeros((1, 0)), np.ones(1)
    xa, wa = roots_jacobi(n, 0.0, 0.0)
    if d == 1:
        r = xa[:, None]
        w = wa
    elif d == 2:
        xb, wb = roots_jacobi(n, 1.0, 0.0)
        A, B = np.meshgrid(xa, xb, indexing="ij")
        WA, WB = np.meshgrid(wa, wb, indexing="ij")
        r = np.stack([(1 + A) * (1 - B) / 2 - 1, B], axis=-1).reshape(-1, 2)
        w = (WA * WB / 2).ravel()
    elif d == 3:
        xb, wb = roots_jacobi(n, 1.0, 0.0)
        xc, wc = roots_jacobi(n, 2.0, 0.0)
        A, B, C = np.meshgrid(xa, xb, xc, indexing="ij")
        WA, WB, WC = np.meshgrid(wa, wb, wc, indexing="ij")
        r = np.stack([(1 + A) * (1 - B) * (1 - C) / 4 - 1,
                      (1 + B) * (1 - C) / 2 - 1, C], axis=-1).reshape(-1, 3)
        w = (WA * WB * WC / 8).ravel()
    else:
        raise ValueError(d)
    scale = abs(np.linalg.det(_edge_matrix(d))) / 2.0 ** d
    return collapsed_ref_to_eq(r, d), w * scale


def simplex_volume(d):
    return abs(np.linalg.det(_edge_matrix(d))) / np.prod(np.arange(1, d + 1)) if d else 1.0


def _scaled_jacobi(nmax, alpha, xv, v, v2):
    """R_n = v^n P_n^{(alpha,0)}(x) for n = 0..nmax, given xv = x v, v, v^2."""
    out = [np.ones_like(xv)]
    if nmax >= 1:
        out.append(((alpha + 2.0) * xv + alpha * v) / 2.0)
    for n in range(1, nmax):
        a = 2.0 * n + alpha
        num = (a + 1.0) * ((a + 2.0) * a * xv + alpha * alpha * v) * out[n] \
            - 2.0 * (n + alpha) * n * (a + 2.0) * v2 * out[n - 1]
        out.append(num / (2.0 * (n + 1.0) * (n + alpha + 1.0) * a))
    return out


def dubiner_indices(d, p):
    """Multi-indices of the Dubiner basis, graded by total degree."""
    idx = []
    for deg in range(p + 1):
        if d == 1:
            idx.append((deg,))
        elif d == 2:
            for i in range(deg, -1, -1):
                idx.append((i, deg - i))
        elif d == 3:
            for i in range(deg, -1, -1):
                for j in range(deg - i, -1, -1):
                    idx.append((i, j, deg - i - j))
    return idx


def _dubiner_raw(d, p, r):
    """Unnormalised Dubiner polynomials at collapsed-reference points r
    (real or complex), shape (N, dim P_p)."""
    idx = dubiner_indices(d, p)
    one = np.ones(r.shape[0], dtype=r.dtype)
    if d == 1:
        P = _scaled_jacobi(p, 0.0, r[:, 0], one, one)
        return np.stack([P[i] for (i,) in idx], axis=1)
    if d == 2:
        x, y = r[:, 0], r[:, 1]
        f1 = (1.0 + 2.0 * x + y) / 2.0
        u2 = ((1.0 - y) / 2.0) ** 2
        Q = _scaled_jacobi(p, 0.0, f1, one, u2)
        cols = []
        for (i, j) in idx:
            Pj = _scaled_jacobi(j, 2.0 * i + 1.0, y, one, one)[j]
            cols.append(Q[i] * Pj)
        return np.stack(cols, axis=1)
    if d == 3:
        x, y, z = r[:, 0], r[:, 1], r[:, 2]
        f1 = (2.0 + 2.0 * x + y + z) / 2.0
        U2 = ((y + z) / 2.0) ** 2
        Q = _scaled_jacobi(p, 0.0, f1, one, U2)
        xv = (1.0 + 2.0 * y + z) / 2.0
        V = (1.0 - z) / 2.0
        cols = []
        for (i, j, k) in idx:
            Rj = _scaled_jacobi(j, 2.0 * i + 1.0, xv, V, V * V)[j]
            Pk = _scaled_jacobi(k, 2.0 * i + 2.0 * j + 2.0, z, one, one)[k]
            cols.append(Q[i] * Rj * Pk)
        return np.stack(cols, axis=1)
    raise ValueError(d)


@functools.lru_cache(maxsize=None)
def _norms(d, p):
    x, w = quadrature(d, p + 2)
    vals = _dubiner_raw(d, p, eq_to_collapsed_ref(x, d))
    return np.sqrt(np.einsum("q,qn->n", w, vals * vals))


class PolyBasis:
    """L2(T_hat)-orthonormal basis of P_p on the equilateral d-simplex."""

    def __init__(self, d, p):
        self.d, self.p = d, p
        self.n = poly_dim(d, p)
        self.degree = np.array([sum(m) for m in dubiner_indices(d, p)])
        self._nrm = _norms(d, p) if d > 0 else np.ones(1)

    def _eval_complex(self, x):
        if self.d == 0:
            return np.ones((x.shape[0], 1), dtype=x.dtype)
        E = _edge_matrix(self.d)
        v0 = EQ_VERTICES[self.d][0]
        lam = np.linalg.solve(E, (x - v0).T).T
        return _dubiner_raw(self.d, self.p, 2.0 * lam - 1.0) / self._nrm

    def values(self, x):
        """(N, n) basis values at points x (N, d)."""
        return np.real(self._eval_complex(np.asarray(x, dtype=float)))

    def gradients(self, x):
        """(N, d, n) basis gradients (complex step, exact for polynomials)."""
        x = np.asarray(x, dtype=float)
        out = np.empty((x.shape[0], self.d, self.n))
        for a in range(self.d):
            xc = x.astype(complex)
            xc[:, a] += 1j * CSTEP
            out[:, a, :] = np.imag(self._eval_complex(xc)) / CSTEP
        return out


def splitmix64_stream(seed):
    """SplitMix64 (Steele, Lea & Flood 2014) as an infinite generator of
    uniform doubles in [0, 1): 53 high bits of each 64-bit output."""
    mask = (1 << 64) - 1
    state = seed & mask
    while True:
        state = (state + 0x9E3779B97F4A7C15) & mask
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & mask
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & mask
        z = z ^ (z >> 31)
        yield (z >> 11) * (1.0 / 9007199254740992.0)
