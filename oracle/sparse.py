"""Sparse helpers for the oracle (test infrastructure).

Every sparse product here keeps the *structural* pattern: an entry exists
wherever some path of stored entries reaches it, even if its value cancels to
zero.  Patch membership and W weights (Section 3.3.1) are read from patterns,
so patterns must not depend on rounding.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


def splitmix64(counter: np.ndarray, seed: int) -> np.ndarray:
    """SplitMix64 output for state seed + (counter+1)*golden (Steele, Lea and
    Flood, OOPSLA 2014), as uint64."""
    with np.errstate(over="ignore"):
        z = (np.uint64(seed) + (counter.astype(np.uint64) + np.uint64(1)) * np.uint64(GOLDEN))
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_pm1(n: int, seed: int) -> np.ndarray:
    """n values in [-1, 1): top 53 bits of SplitMix64 scaled."""
    z = splitmix64(np.arange(n, dtype=np.uint64), seed)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) * 2.0 - 1.0


def csr(A) -> sp.csr_matrix:
    A = sp.csr_matrix(A)
    A.sort_indices()
    return A


def pattern_product(A: sp.csr_matrix, B: sp.csr_matrix) -> sp.csr_matrix:
    """C = A @ B with the full structural pattern of the product."""
    Pa = sp.csr_matrix((np.ones(A.nnz), A.indices, A.indptr), shape=A.shape)
    Pb = sp.csr_matrix((np.ones(B.nnz), B.indices, B.indptr), shape=B.shape)
    S = csr(Pa @ Pb)  # strictly positive sums: nothing cancels, nothing dropped
    C = csr(A @ B)
    C.sum_duplicates()
    out = S.copy()
    out.data = np.zeros(S.nnz)
    if C.nnz:
        n = S.shape[1]
        srow = np.repeat(np.arange(S.shape[0]), np.diff(S.indptr)).astype(np.int64)
        skey = srow * n + S.indices
        crow = np.repeat(np.arange(C.shape[0]), np.diff(C.indptr)).astype(np.int64)
        ckey = crow * n + C.indices
        pos = np.searchsorted(skey, ckey)
        assert np.all(skey[pos] == ckey)
        out.data[pos] = C.data
    return out


def galerkin(P: sp.csr_matrix, A: sp.csr_matrix) -> sp.csr_matrix:
    """P^T A P with structural pattern."""
    return pattern_product(csr(P.T), pattern_product(A, P))


def submatrix(A: sp.csr_matrix, rows: np.ndarray, cols: np.ndarray) -> sp.csr_matrix:
    """A[rows][:, cols] keeping explicit zeros."""
    A = csr(A)
    C = A[rows].tocoo()
    cmap = -np.ones(A.shape[1], dtype=np.int64)
    cmap[cols] = np.arange(len(cols))
    keep = cmap[C.col] >= 0
    out = sp.coo_matrix((C.data[keep], (C.row[keep], cmap[C.col[keep]])),
                        shape=(len(rows), len(cols))).tocsr()
    out.sort_indices()
    return out


def dense_blocks(A: sp.csr_matrix, idx: np.ndarray) -> np.ndarray:
    """Stack of dense principal submatrices A[idx[k]][:, idx[k]] for an (N, m)
    index array: for each patch, its rows of A are read and every stored entry
    whose column lies in the patch is placed at (local row, local column)."""
    A = csr(A)
    N, m = idx.shape
    out = np.zeros((N, m, m))
    pos = -np.ones(A.shape[1], dtype=np.int64)  # global column -> local position (current patch)
    local = np.arange(m)
    for k in range(N):
        d = idx[k]
        pos[d] = local
        lo = A.indptr[d]
        cnt = A.indptr[d + 1] - lo
        ent = np.repeat(lo - np.cumsum(cnt) + cnt, cnt) + np.arange(int(cnt.sum()))  # entries of rows d
        rows = np.repeat(local, cnt)
        cols = pos[A.indices[ent]]
        keep = cols >= 0
        out[k, rows[keep], cols[keep]] = A.data[ent[keep]]
        pos[d] = -1
    return out
