"""Exact P1/P2 element matrices on simplices and vectorised assembly.

Integrals of products of barycentric coordinates are evaluated exactly with
    int_T prod_k lambda_k^{a_k} = d! |T| prod_k a_k! / (sum_k a_k + d)!,
so every element matrix is exact up to rounding.  Basis functions (Section 2.1):
  P1 vertex i: lambda_i
  P2 vertex i: lambda_i (2 lambda_i - 1);  P2 edge (i,j): 4 lambda_i lambda_j
The bilinear forms are those of the Stokes weak form (Section 2):
  a(u,v) = int grad u : grad v,   b(p,v) = - int p div v.
"""
from __future__ import annotations

from functools import lru_cache
from math import factorial

import numpy as np
import scipy.sparse as sp

from .mesh import EDGES_2D, EDGES_3D, Mesh, cell_measures

# ---------------------------------------------------------------------------
# polynomials in barycentric coordinates: dict {exponent tuple: coefficient}


def _mono(d1: int, k: int, p: int = 1) -> dict:
    e = [0] * d1
    e[k] = p
    return {tuple(e): 1.0}


def _add(a: dict, b: dict, s: float = 1.0) -> dict:
    out = dict(a)
    for k, v in b.items():
        out[k] = out.get(k, 0.0) + s * v
    return out


def _mul(a: dict, b: dict) -> dict:
    out: dict = {}
    for ka, va in a.items():
        for kb, vb in b.items():
            k = tuple(x + y for x, y in zip(ka, kb))
            out[k] = out.get(k, 0.0) + va * vb
    return out


def _scale(a: dict, s: float) -> dict:
    return {k: s * v for k, v in a.items()}


def _diff(a: dict, k: int) -> dict:
    out: dict = {}
    for e, v in a.items():
        if e[k] > 0:
            f = list(e)
            f[k] -= 1
            out[tuple(f)] = out.get(tuple(f), 0.0) + v * e[k]
    return out


def _integral_per_measure(a: dict, d: int) -> float:
    """int_T poly / |T|."""
    s = 0.0
    for e, v in a.items():
        num = factorial(d)
        for x in e:
            num *= factorial(x)
        s += v * num / factorial(sum(e) + d)
    return s


def _basis(d: int, order: int) -> list[dict]:
    d1 = d + 1
    if order == 1:
        return [_mono(d1, i) for i in range(d1)]
    edges = EDGES_2D if d == 2 else EDGES_3D
    out = []
    for i in range(d1):
        li = _mono(d1, i)
        out.append(_add(_scale(_mul(li, li), 2.0), li, -1.0))
    for i, j in edges:
        out.append(_scale(_mul(_mono(d1, i), _mono(d1, j)), 4.0))
    return out


@lru_cache(maxsize=None)
def ref_tensors(d: int, vel_order: int, pres_order: int):
    """Geometry-free reference tensors (all per unit measure):
    mass[a,b]      = int phi_a phi_b
    stiff[a,k,b,l] = int d_k phi_a d_l phi_b        (d_k = d/d lambda_k)
    div[q,a,k]     = int psi_q d_k phi_a            (psi: pressure basis)
    pmass[q,r]     = int psi_q psi_r
    """
    phi = _basis(d, vel_order)
    psi = _basis(d, pres_order)
    d1 = d + 1
    nb, nq = len(phi), len(psi)
    dphi = [[_diff(f, k) for k in range(d1)] for f in phi]
    mass = np.array([[_integral_per_measure(_mul(a, b), d) for b in phi] for a in phi])
    stiff = np.zeros((nb, d1, nb, d1))
    for a in range(nb):
        for k in range(d1):
            for b in range(nb):
                for l in range(d1):
                    stiff[a, k, b, l] = _integral_per_measure(_mul(dphi[a][k], dphi[b][l]), d)
    div = np.zeros((nq, nb, d1))
    for q in range(nq):
        for a in range(nb):
            for k in range(d1):
                div[q, a, k] = _integral_per_measure(_mul(psi[q], dphi[a][k]), d)
    pmass = np.array([[_integral_per_measure(_mul(a, b), d) for b in psi] for a in psi])
    return mass, stiff, div, pmass


def bary_grads(m: Mesh) -> tuple[np.ndarray, np.ndarray]:
    """grad lambda_k per cell, shape (ne, d+1, d), and cell measures."""
    x = m.verts[m.cells]
    J = (x[:, 1:, :] - x[:, :1, :]).transpose(0, 2, 1)  # (ne, d, d)
    Jinv = np.linalg.inv(J)  # rows = grad xi_k
    g = np.empty((m.ne, m.dim + 1, m.dim))
    g[:, 1:, :] = Jinv
    g[:, 0, :] = -Jinv.sum(axis=1)
    return g, cell_measures(m)


def _coo(rows, cols, vals, shape) -> sp.csr_matrix:
    A = sp.coo_matrix((vals.ravel(), (rows.ravel(), cols.ravel())), shape=shape).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A


def stiffness(m: Mesh, c2n: np.ndarray, order: int, n_nodes: int, nu: float = 1.0) -> sp.csr_matrix:
    """Scalar stiffness nu int grad phi_a . grad phi_b (P1 or P2)."""
    _, st, _, _ = ref_tensors(m.dim, order, 1)
    g, vol = bary_grads(m)
    G = np.einsum("ekx,elx->ekl", g, g)  # grad lambda_k . grad lambda_l
    Ke = nu * vol[:, None, None] * np.einsum("akbl,ekl->eab", st, G)
    nb = c2n.shape[1]
    rows = np.repeat(c2n[:, :, None], nb, 2)
    cols = np.repeat(c2n[:, None, :], nb, 1)
    return _coo(rows, cols, Ke, (n_nodes, n_nodes))


def mass(m: Mesh, c2n: np.ndarray, order: int, n_nodes: int) -> sp.csr_matrix:
    ms, _, _, _ = ref_tensors(m.dim, order, 1)
    _, vol = bary_grads(m)
    Me = vol[:, None, None] * ms[None]
    nb = c2n.shape[1]
    rows = np.repeat(c2n[:, :, None], nb, 2)
    cols = np.repeat(c2n[:, None, :], nb, 1)
    return _coo(rows, cols, Me, (n_nodes, n_nodes))


def divergence(m: Mesh, c2n: np.ndarray, vel_order: int, p_c2n: np.ndarray,
               n_nodes: int, n_p: int) -> sp.csr_matrix:
    """B[q, c*n_nodes + a] = - int psi_q d phi_a / d x_c  (field-blocked velocity)."""
    d = m.dim
    _, _, dv, _ = ref_tensors(d, vel_order, 1)
    g, vol = bary_grads(m)
    # Be[e, q, a, c] = -vol * sum_k div[q,a,k] g[e,k,c]
    Be = -vol[:, None, None, None] * np.einsum("qak,ekc->eqac", dv, g)
    nq, nb = p_c2n.shape[1], c2n.shape[1]
    rows = np.broadcast_to(p_c2n[:, :, None, None], (m.ne, nq, nb, d))
    cols = np.stack([c * n_nodes + c2n for c in range(d)], -1)  # (ne, nb, d)
    cols = np.broadcast_to(cols[:, None, :, :], (m.ne, nq, nb, d))
    return _coo(rows, cols, Be, (n_p, d * n_nodes))


def iso_divergence(fine: Mesh, coarse: Mesh, n_nodes: int) -> sp.csr_matrix:
    """B for P1isoP2/P1: B[q, c*n_nodes + j] = - sum_t int_t phi_q d psi_j/d x_c,
    psi_j the P1 basis of the refined mesh, phi_q the P1 basis of ``coarse``.
    Children are stored consecutively per parent (quadrisect order); phi_q is
    linear on each child and d psi_j is constant there, so the child integral is
    |t| phi_q(centroid_t) d psi_j / d x_c exactly."""
    d = fine.dim
    nch = 4 if d == 2 else 8
    g, vol = bary_grads(fine)  # (nf, d+1, d)
    parent = np.repeat(np.arange(coarse.ne), nch)
    # barycentric coordinates of child centroids w.r.t. the parent
    cen = fine.verts[fine.cells].mean(axis=1)  # (nf, d)
    px = coarse.verts[coarse.cells[parent]]  # (nf, d+1, d)
    J = (px[:, 1:, :] - px[:, :1, :]).transpose(0, 2, 1)
    xi = np.linalg.solve(J, (cen - px[:, 0, :])[..., None])[..., 0]  # (nf, d)
    lam = np.concatenate([1.0 - xi.sum(1, keepdims=True), xi], 1)  # (nf, d+1)
    Be = -vol[:, None, None, None] * lam[:, :, None, None] * g[:, None, :, :]  # (nf, q, j, c)
    rows = np.broadcast_to(coarse.cells[parent][:, :, None, None], Be.shape)
    cols = np.stack([c * n_nodes + fine.cells for c in range(d)], -1)
    cols = np.broadcast_to(cols[:, None, :, :], Be.shape)
    return _coo(rows, cols, Be, (coarse.nv, d * n_nodes))


def p1_integrals(m: Mesh) -> np.ndarray:
    """w_i = int phi_i for the continuous P1 basis."""
    _, vol = bary_grads(m)
    w = np.zeros(m.nv)
    np.add.at(w, m.cells.ravel(), np.repeat(vol / (m.dim + 1), m.dim + 1))
    return w
