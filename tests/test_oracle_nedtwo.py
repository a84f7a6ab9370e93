"""Pins of the oracle's second-kind Nedelec element NedTwo_p and of the
discrete curl NedTwo_p -> RT_p behind the standard H(div) Hiptmair-Toselli
potentials (no GPU).

* dim NedTwo_p = 3 dim P_p; per-entity counts: edges 1 + p (Whitney and the
  CG_{p+1} edge bubbles), faces and cells the type-I NedTwo bubbles plus the
  CG_{p+1} type-II bubbles (eq:bubble-trace-dim-counts);
* lem:ref-element-matrix-properties for NedTwo_p (curl-curl identity on the
  type-I block, zero on type-II rows, mass diag(Lambda, I) on the interior);
* lem:d-preserves-basis-functions for both maps of the complex
  CG_{p+1} -> NedTwo_p -> RT_p on the reference element: the gradient of a
  CG_{p+1} function is the incidence (vertex functions) or the NedTwo type-II
  function of the same entity and index; the curl of a NedTwo function is
  the signed face-edge incidence (Whitney edge functions), the RT type-II
  function of the same entity and index (type-I), or zero (type-II).
"""
from math import comb

import numpy as np
import pytest

from oracle.element import eigenbasis, element, entities, reference_matrices
from oracle.simplex import quadrature


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_nedtwo_dimensions(p):
    el = element(3, "NedTwo", p)
    assert el.n == 3 * comb(p + 3, 3)
    nI_f = eigenbasis(2, "NedTwo", p).N
    nI_c = eigenbasis(3, "NedTwo", p).N
    assert el.counts() == [0, 1 + p, nI_f + p * (p - 1) // 2, nI_c + p * (p - 1) * (p - 2) // 6]


@pytest.mark.parametrize("p", [3, 4, pytest.param(5, marks=pytest.mark.slow)])
def test_nedtwo_reference_matrix_structure(p):
    el = element(3, "NedTwo", p)
    M, K = reference_matrices(el)
    interior = el.interior()
    kinds = np.array([di.kind for di in el.dofs])
    I1 = np.flatnonzero(interior & (kinds == "I"))
    I2 = np.flatnonzero(interior & (kinds == "II"))
    G = np.flatnonzero(~interior)
    assert len(I1) and len(I2)
    assert np.abs(K[np.ix_(I1, I1)] - np.eye(len(I1))).max() < 1e-10
    assert np.abs(K[I2]).max() < 1e-10 * np.abs(K).max()
    assert np.abs(K[np.ix_(I1, G)]).max() < 1e-10 * np.abs(K).max()
    assert np.abs(M[np.ix_(I2, I2)] - np.eye(len(I2))).max() < 1e-10
    assert np.abs(M[np.ix_(I2, G)]).max() < 1e-10 * np.abs(M).max()


def _coeffs_in(el_to, field_vals, xq, wq):
    """Coefficients of a field (values at quadrature points xq, (N, c, m))
    in the basis of el_to: L2-project onto P_p^c, then apply el_to's dofs
    (its basis is dual to them)."""
    V = el_to.space.poly.values(xq)                       # (N, n_poly), orthonormal
    proj = np.einsum("q,qcm,qn->cnm", wq, field_vals, V)   # exact for degree <= p
    return el_to.L @ proj.reshape(-1, field_vals.shape[2])


@pytest.mark.parametrize("p", [1, 2, 3])
def test_curl_maps_nedtwo_to_rt_basis(p):
    n2, rt = element(3, "NedTwo", p), element(3, "RT", p)
    xq, wq = quadrature(3, p + 2)
    _, curl = n2.tabulate(xq)
    C = _coeffs_in(rt, curl, xq, wq)                       # (n_RT, n_N2)
    rt_idx = {(di.entity_dim, di.entity_index, di.kind, di.j): i for i, di in enumerate(rt.dofs)}
    faces = entities(3)[2]
    ref = np.zeros_like(C)
    for s, di in enumerate(n2.dofs):
        if di.kind == "W":
            a0, b0 = di.verts
            for fi, (a, b, c) in enumerate(faces):
                if {a0, b0} <= {a, b, c}:
                    ref[rt_idx[(2, fi, "W", 0)], s] = -1.0 if (a0, b0) == (a, c) else 1.0
        elif di.kind == "I":
            ref[rt_idx[(di.entity_dim, di.entity_index, "II", di.j)], s] = 1.0
    assert np.abs(C - ref).max() < 1e-10


@pytest.mark.parametrize("p", [1, 2, 3])
def test_grad_maps_cg_to_nedtwo_basis(p):
    cg, n2 = element(3, "CG", p + 1), element(3, "NedTwo", p)
    xq, wq = quadrature(3, p + 3)
    _, grad = cg.tabulate(xq)
    Gm = _coeffs_in(n2, grad, xq, wq)
    n2_idx = {(di.entity_dim, di.entity_index, di.kind, di.j): i for i, di in enumerate(n2.dofs)}
    edges = entities(3)[1]
    ref = np.zeros_like(Gm)
    for s, di in enumerate(cg.dofs):
        if di.entity_dim == 0:
            v = di.verts[0]
            for ei, (a, b) in enumerate(edges):
                if v in (a, b):
                    ref[n2_idx[(1, ei, "W", 0)], s] = 1.0 if v == b else -1.0
        else:
            ref[n2_idx[(di.entity_dim, di.entity_index, "II", di.j)], s] = 1.0
    assert np.abs(Gm - ref).max() < 1e-10
