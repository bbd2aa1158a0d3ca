"""Algebraic Vanka patches and additive Vanka relaxation (Section 3.3.1).
Test infrastructure (oracle).

Patch i on a level is the seed pressure DoF(s) plus every velocity DoF stored
in the seed rows of B (the structural pattern of the level operator).  One
seed per pressure row for Taylor-Hood and P1isoP2/P1 levels; for P2/P1disc the
three pressures of one element are seeded together.  Inside a patch the
velocities come first, ordered by (component, global index), then the seeds.
One additive sweep is
    x <- x + omega * sum_i V_i^T W_i K_i^{-1} V_i (b - K x),   K_i = V_i K V_i^T,
with W the partition of unity 1 / (number of patches holding the DoF).
K_i^{-1} is applied by a dense LU solve of the full patch matrix.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .sparse import csr, dense_blocks


@dataclass
class Patches:
    dofs: list[np.ndarray]  # global (level) DoF ids per patch
    n_seed: list[int]
    weight: np.ndarray  # W per DoF (0 for DoFs in no patch)


def patches_single_seed(K: sp.csr_matrix, field: np.ndarray, dim: int) -> Patches:
    K = csr(K)
    isvel = field < dim
    dofs = []
    for i in np.nonzero(field == dim)[0]:
        cols = K.indices[K.indptr[i]:K.indptr[i + 1]]
        v = np.sort(cols[isvel[cols]])
        dofs.append(np.concatenate([v, [i]]).astype(np.int64))
    return _finish(dofs, [1] * len(dofs), K.shape[0])


def patches_element_seeds(K: sp.csr_matrix, field: np.ndarray, dim: int,
                          seeds: np.ndarray) -> Patches:
    """seeds: (n_elem, s) level-numbered pressure DoFs seeded together."""
    K = csr(K)
    isvel = field < dim
    dofs = []
    for row in seeds:
        cols = np.concatenate([K.indices[K.indptr[i]:K.indptr[i + 1]] for i in row])
        v = np.unique(cols[isvel[cols]])
        dofs.append(np.concatenate([v, row]).astype(np.int64))
    return _finish(dofs, [seeds.shape[1]] * len(dofs), K.shape[0])


def _finish(dofs, n_seed, n) -> Patches:
    cnt = np.bincount(np.concatenate(dofs), minlength=n).astype(np.float64)
    w = np.zeros(n)
    w[cnt > 0] = 1.0 / cnt[cnt > 0]
    return Patches(dofs=dofs, n_seed=n_seed, weight=w)


CACHE_ENTRIES = 2 * 10 ** 8  # keep dense patch matrices between sweeps below this size
PROGRESS = False  # print a line per group of patches solved (long full-size runs)


def _buckets(K: sp.csr_matrix, P: Patches, chunk: int):
    """(index array, dense patch matrices or None) per group of equal-size patches."""
    if getattr(P, "_cache", None) is not None:
        return P._cache
    sizes = np.array([d.size for d in P.dofs])
    keep = int((sizes.astype(np.int64) ** 2).sum()) <= CACHE_ENTRIES
    out = []
    for m in np.unique(sizes):
        ids = np.nonzero(sizes == m)[0]
        for s in range(0, ids.size, chunk):
            idx = np.stack([P.dofs[i] for i in ids[s:s + chunk]])
            out.append((idx, dense_blocks(K, idx) if keep else None))
    if keep:
        P._cache = out
    return out


def sweep(K: sp.csr_matrix, P: Patches, b: np.ndarray, x: np.ndarray, omega: float,
          chunk: int = 8192) -> np.ndarray:
    """One additive Vanka sweep; returns the updated x (x may be all zeros)."""
    r = b - K @ x
    upd = np.zeros_like(x)
    groups = _buckets(K, P, chunk)
    for g, (idx, Ki) in enumerate(groups):
        if Ki is None:
            Ki = dense_blocks(K, idx)
        yi = np.linalg.solve(Ki, r[idx][..., None])[..., 0]  # dense LU per patch
        np.add.at(upd, idx.ravel(), (P.weight[idx] * yi).ravel())
        if PROGRESS and (g + 1) % 32 == 0 or (PROGRESS and g + 1 == len(groups)):
            print(f"    [oracle] sweep over {K.shape[0]} DoFs: group {g + 1}/{len(groups)} "
                  f"({idx.shape[0]} patches of {idx.shape[1]} DoFs)", flush=True)
    return x + omega * upd


def krylov_relax(K: sp.csr_matrix, P: Patches, b: np.ndarray, x: np.ndarray, its: int) -> np.ndarray:
    """Relaxation accelerated by FGMRES (Section 3.3.1, the relaxation wrapper
    that replaces the damping parameter): `its` iterations of flexible,
    right-preconditioned GMRES on K e = b - K x from e = 0, the preconditioner
    being one undamped additive Vanka sweep; returns x + e.  Arnoldi with
    modified Gram-Schmidt; the small least-squares problem is solved directly."""
    r = b - K @ x
    beta = np.linalg.norm(r)
    if beta == 0.0:
        return x.copy()
    V = [r / beta]
    Z = []
    H = np.zeros((its + 1, its))
    k = 0
    for j in range(its):
        z = sweep(K, P, V[j], np.zeros_like(x), 1.0)
        Z.append(z)
        w = K @ z
        for i in range(j + 1):
            H[i, j] = V[i] @ w
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        k = j + 1
        if H[j + 1, j] == 0.0:  # the correction lies in the space built so far
            break
        V.append(w / H[j + 1, j])
    g = np.zeros(k + 1)
    g[0] = beta
    y = np.linalg.lstsq(H[:k + 1, :k], g, rcond=None)[0]
    return x + np.column_stack(Z[:k]) @ y
