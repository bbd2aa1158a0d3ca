"""Simplicial meshes and the refinements the method needs (Section 2.1, Figure 1).

* structured triangle meshes of a rectangle, every square split along the same
  diagonal, with optional seeded jitter of interior vertices;
* structured tetrahedral meshes of a box, every cube split into the six
  path simplices (Kuhn / Freudenthal split);
* quadrisection R_U (2D: 4 children; 3D: 8 children, Bey's rule, which keeps a
  Kuhn mesh Kuhn), whose vertices are exactly the P2 nodes of the parent mesh;
* barycentric (Alfeld) refinement R_B (2D).

Vertex numbering is row-major (x fastest).  Edges are numbered in lexicographic
order of their sorted vertex pair; P2 node k >= n_vertices is the midpoint of
edge k - n_vertices.  This module holds no solver arithmetic.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass

import numpy as np

EDGES_2D = ((0, 1), (0, 2), (1, 2))
EDGES_3D = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


@dataclass
class Mesh:
    verts: np.ndarray  # (nv, d) float64
    cells: np.ndarray  # (ne, d+1) int64

    @property
    def dim(self) -> int:
        return self.verts.shape[1]

    @property
    def nv(self) -> int:
        return self.verts.shape[0]

    @property
    def ne(self) -> int:
        return self.cells.shape[0]


def rect_mesh(n: int, lx: float = 1.0, ly: float = 1.0, jitter: float = 0.0,
              rng: np.random.Generator | None = None) -> Mesh:
    """n x n squares on [0,lx]x[0,ly], each split along its (i,j)->(i+1,j+1) diagonal.

    Interior vertices are moved by U(-jitter*h, jitter*h) per coordinate (h the
    cell size in that coordinate), drawn from ``rng`` in vertex order."""
    xs = np.linspace(0.0, lx, n + 1)
    ys = np.linspace(0.0, ly, n + 1)
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    verts = np.stack([X.ravel(), Y.ravel()], axis=1)
    if jitter > 0.0:
        assert rng is not None
        ii = np.arange(n + 1)
        I, J = np.meshgrid(ii, ii, indexing="xy")
        interior = ((I > 0) & (I < n) & (J > 0) & (J < n)).ravel()
        idx = np.nonzero(interior)[0]
        h = np.array([lx / n, ly / n])
        d = rng.uniform(-jitter, jitter, size=(idx.size, 2)) * h
        verts[idx] += d
    j, i = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    v00 = (j * (n + 1) + i).ravel()
    v10 = v00 + 1
    v01 = v00 + (n + 1)
    v11 = v01 + 1
    t1 = np.stack([v00, v10, v11], 1)
    t2 = np.stack([v00, v11, v01], 1)
    cells = np.stack([t1, t2], 1).reshape(-1, 3).astype(np.int64)
    m = Mesh(verts, cells)
    assert np.all(cell_measures(m, signed=True) > 0), "inverted triangle"
    return m


def box_mesh(n: int, lx: float = 1.0, ly: float = 1.0, lz: float = 1.0) -> Mesh:
    """n^3 cubes, each split into the 6 path simplices 0 -> e_s1 -> e_s1+e_s2 -> (1,1,1)."""
    xs = np.linspace(0.0, lx, n + 1)
    ys = np.linspace(0.0, ly, n + 1)
    zs = np.linspace(0.0, lz, n + 1)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")
    verts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    base = ((k * (n + 1) + j) * (n + 1) + i).ravel()
    step = (1, n + 1, (n + 1) ** 2)
    tets = []
    for perm in itertools.permutations(range(3)):
        v0 = base
        v1 = v0 + step[perm[0]]
        v2 = v1 + step[perm[1]]
        v3 = v2 + step[perm[2]]
        tets.append(np.stack([v0, v1, v2, v3], 1))
    cells = np.stack(tets, 1).reshape(-1, 4).astype(np.int64)
    return Mesh(verts, cells)


def cell_measures(m: Mesh, signed: bool = False) -> np.ndarray:
    x = m.verts[m.cells]  # (ne, d+1, d)
    J = (x[:, 1:, :] - x[:, :1, :]).transpose(0, 2, 1)  # columns = edge vectors
    det = np.linalg.det(J)
    fact = 2.0 if m.dim == 2 else 6.0
    return det / fact if signed else np.abs(det) / fact


def edges(m: Mesh) -> tuple[np.ndarray, np.ndarray]:
    """Unique edges (sorted vertex pairs, lexicographic) and the cell->edge map
    in the local edge order EDGES_2D / EDGES_3D."""
    loc = EDGES_2D if m.dim == 2 else EDGES_3D
    a = np.stack([m.cells[:, i] for i, _ in loc], 1)
    b = np.stack([m.cells[:, j] for _, j in loc], 1)
    lo = np.minimum(a, b).ravel()
    hi = np.maximum(a, b).ravel()
    key = lo * m.nv + hi
    uniq, inv = np.unique(key, return_inverse=True)
    e = np.stack([uniq // m.nv, uniq % m.nv], 1)
    return e, inv.reshape(m.ne, len(loc))


def p2_nodes(m: Mesh) -> tuple[np.ndarray, np.ndarray]:
    """P2 node coordinates (vertices then edge midpoints) and the cell->node map
    (local order: vertices, then edges in EDGES_2D / EDGES_3D order)."""
    e, c2e = edges(m)
    mid = 0.5 * (m.verts[e[:, 0]] + m.verts[e[:, 1]])
    coords = np.concatenate([m.verts, mid], 0)
    c2n = np.concatenate([m.cells, m.nv + c2e], 1)
    return coords, c2n


def quadrisect(m: Mesh) -> Mesh:
    """R_U: uniform refinement whose vertices are the P2 nodes of ``m``."""
    coords, c2n = p2_nodes(m)
    if m.dim == 2:
        v0, v1, v2 = c2n[:, 0], c2n[:, 1], c2n[:, 2]
        m01, m02, m12 = c2n[:, 3], c2n[:, 4], c2n[:, 5]
        ch = [
            (v0, m01, m02),
            (m01, v1, m12),
            (m02, m12, v2),
            (m01, m12, m02),
        ]
    else:
        x0, x1, x2, x3 = (c2n[:, i] for i in range(4))
        x01, x02, x03, x12, x13, x23 = (c2n[:, 4 + i] for i in range(6))
        # Bey's rule: corner simplices plus the octahedron cut along x02-x13.
        ch = [
            (x0, x01, x02, x03),
            (x01, x1, x12, x13),
            (x02, x12, x2, x23),
            (x03, x13, x23, x3),
            (x01, x02, x03, x13),
            (x01, x02, x12, x13),
            (x02, x03, x13, x23),
            (x02, x12, x13, x23),
        ]
    cells = np.stack([np.stack(c, 1) for c in ch], 1).reshape(-1, m.dim + 1)
    return Mesh(coords, cells.astype(np.int64))


def children_of(m: Mesh) -> int:
    return 4 if m.dim == 2 else 8


def alfeld(m: Mesh) -> Mesh:
    """R_B in 2D: add each triangle's barycentre and split it into 3."""
    assert m.dim == 2
    c = m.verts[m.cells].mean(axis=1)
    verts = np.concatenate([m.verts, c], 0)
    b = m.nv + np.arange(m.ne)
    v0, v1, v2 = m.cells[:, 0], m.cells[:, 1], m.cells[:, 2]
    cells = np.stack([np.stack([v0, v1, b], 1), np.stack([v1, v2, b], 1),
                      np.stack([v2, v0, b], 1)], 1).reshape(-1, 3)
    out = Mesh(verts, cells.astype(np.int64))
    assert np.all(cell_measures(out, signed=True) > 0)
    return out


def boundary_vertices(m: Mesh, lo: np.ndarray, hi: np.ndarray, tol: float = 1e-12) -> np.ndarray:
    x = m.verts
    return np.any((np.abs(x - lo) < tol) | (np.abs(x - hi) < tol), axis=1)
