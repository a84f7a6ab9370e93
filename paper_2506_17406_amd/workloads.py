"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle
checks: Freudenthal (Kuhn) meshes of the unit square/cube with optional
interior-vertex jitter, and uniform[-1, 1] load vectors.

This module holds no part of the method's arithmetic: it only produces the
mesh (vertex coordinates and cell-vertex lists, in no particular vertex
order) and right-hand sides that both the library and the oracle receive.

Mesh: the paper's experiments use the Freudenthal subdivision of cubes into
six tetrahedra along the main diagonal (Sec. 7.1, fig:freudenthal).  Each unit
cube (corner bits: bit0 = x, bit1 = y, bit2 = z) is split into the six
tetrahedra v0 -> v0+e_a -> v0+e_a+e_b -> v7 for the permutations (a, b, c) of
the axes; in 2D each square is split along its (0,0)-(1,1) diagonal.
Jitter: each coordinate of each interior vertex is perturbed by
U(-jitter*h, jitter*h), h = 1/n; boundary vertices stay fixed.
"""
from itertools import permutations

import numpy as np


def kuhn_mesh(n, dim=3, jitter=0.0, seed=0):
    """Vertices (n_v, dim) float64 and cells (n_c, dim+1) int64 of the
    Freudenthal mesh of [0,1]^dim with n cells per edge."""
    h = 1.0 / n
    if dim == 3:
        g = np.arange(n + 1)
        K, J, I = np.meshgrid(g, g, g, indexing="ij")
        coords = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1) * h
        vid = lambda i, j, k: i + (n + 1) * (j + (n + 1) * k)
        cells = []
        for k in range(n):
            for j in range(n):
                for i in range(n):
                    corner = lambda b: vid(i + (b & 1), j + ((b >> 1) & 1), k + ((b >> 2) & 1))
                    for a, b, _ in permutations(range(3)):
                        ea, eb = 1 << a, 1 << b
                        cells.append([corner(0), corner(ea), corner(ea | eb), corner(7)])
    elif dim == 2:
        g = np.arange(n + 1)
        J, I = np.meshgrid(g, g, indexing="ij")
        coords = np.stack([I.ravel(), J.ravel()], axis=1) * h
        vid = lambda i, j: i + (n + 1) * j
        cells = []
        for j in range(n):
            for i in range(n):
                corner = lambda b: vid(i + (b & 1), j + ((b >> 1) & 1))
                cells.append([corner(0), corner(1), corner(3)])
                cells.append([corner(0), corner(2), corner(3)])
    else:
        raise ValueError(dim)
    coords = coords.astype(np.float64)
    if jitter:
        rng = np.random.default_rng(seed)
        delta = rng.uniform(-jitter * h, jitter * h, size=coords.shape)
        interior = np.all((coords > 0.5 * h) & (coords < 1.0 - 0.5 * h), axis=1)
        coords = coords + delta * interior[:, None]
    return coords, np.asarray(cells, dtype=np.int64)


def fichera_mesh(n, jitter=0.0, seed=0):
    """Vertices and cells of the Freudenthal mesh of the Fichera corner
    (0, 1)^3 minus [1/2, 1)^3 with n cells per edge (n even): the Kuhn cubes
    (i, j, k) of the unit-cube mesh except those with i, j, k >= n / 2,
    vertices renumbered in the unit-cube order.  jitter: interior vertices
    (all eight surrounding cubes present) moved by U(-jitter h, jitter h)
    per coordinate."""
    if n % 2:
        raise ValueError("the Fichera mesh needs an even n")
    X, C = kuhn_mesh(n, 3)
    h, m = 1.0 / n, n // 2
    cube = np.repeat(np.arange(n ** 3), 6)                      # cells come 6 per cube, cube index i + n (j + n k)
    ci, cj, ck = cube % n, (cube // n) % n, cube // (n * n)
    keep = ~((ci >= m) & (cj >= m) & (ck >= m))
    C = C[keep]
    used = np.zeros(len(X), dtype=bool)
    used[C.ravel()] = True
    new = -np.ones(len(X), dtype=np.int64)
    new[used] = np.arange(used.sum())
    X, C = X[used], new[C]
    if jitter:
        g = np.rint(X / h).astype(np.int64)
        present = lambda i, j, k: (0 <= i < n and 0 <= j < n and 0 <= k < n and not (i >= m and j >= m and k >= m))
        interior = np.array([all(present(i + a, j + b, k + c) for a in (-1, 0) for b in (-1, 0) for c in (-1, 0))
                             for i, j, k in g])
        rng = np.random.default_rng(seed)
        X = X + rng.uniform(-jitter * h, jitter * h, size=X.shape) * interior[:, None]
    return X, C


def load_vectors(n_dofs, seed, n_rhs=1):
    """Column-major (n_dofs, n_rhs) uniform[-1, 1] load vectors; column j is
    the j-th block of n_dofs consecutive draws of default_rng(seed)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.uniform(-1.0, 1.0, size=(n_rhs, n_dofs)).T)


def kuhn_counts(n, dim=3):
    """(vertices, edges, faces, cells) of the Kuhn mesh, closed forms."""
    if dim == 3:
        return ((n + 1) ** 3, 7 * n ** 3 + 9 * n ** 2 + 3 * n, 12 * n ** 3 + 6 * n ** 2, 6 * n ** 3)
    return ((n + 1) ** 2, 3 * n ** 2 + 2 * n, 2 * n ** 2)


def uneven_batch(seed=8, count=32, spaces=("CG", "Ned"), n_range=(4, 16), p_range=(2, 10)):
    """Draws of the uneven batch: `count` problems, each (space, n, p,
    mesh_seed, rhs_seed) with space, n and p uniform from default_rng(seed)
    in that order per problem, mesh seed 100 + i and load-vector seed
    200 + i.  Further draws continue the same generator (for re-drawing a
    problem that does not fit)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        sp = spaces[int(rng.integers(len(spaces)))]
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        p = int(rng.integers(p_range[0], p_range[1] + 1))
        out.append((sp, n, p, 100 + i, 200 + i))
    return out, rng

