"""Algorithm 1 (Section 3.2): smoothed-aggregation interpolation built
independently for each velocity component and for the pressure (auxiliary
operator A_p), combined block-diagonally, and Galerkin coarse saddle operators
K_{l+1} = P_l^T K_l P_l.  Test infrastructure (oracle).

Scalar SA, per field (readings of what the paper leaves open):
  * strength: the evolution measure Section 3.2 names (Olson, Schroder and
    Tuminaro, "A new perspective on strength measures in algebraic
    multigrid", NLAA 2010) with k = 2 relaxation steps, filter epsilon = 4
    and the l2 projection onto the near-null vector B; see
    `evolution_strength`.  The classical symmetric test
    a_ij^2 >= theta^2 a_ii a_jj (the measure Section 3.2 says needed tuning)
    stays available as soc = "symmetric";
  * aggregation: the standard three passes, nodes visited in increasing index;
    pass 1 seeds an aggregate at a node whose strong neighbours are all free
    (a node without strong neighbours becomes a singleton), pass 2 attaches a
    leftover node to the aggregate of its lowest-numbered strong neighbour
    aggregated in pass 1, pass 3 seeds new aggregates from what is left;
  * tentative interpolation from the near-null vector (constant on the finest
    level, eq. (3.5)): T[i, agg(i)] = B_i / ||B_agg||, coarse vector ||B_agg||;
  * prolongator smoothing P = (I - omega D^{-1} A) T with
    omega = (4/3) / rho and rho bounded by max_i sum_j |a_ij| / a_ii;
  * stop when n <= max_coarse or after max_levels levels, or when a level
    does not coarsen.
The hierarchy depth is the minimum over the fields (Algorithm 1).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp

from .sparse import csr, galerkin, pattern_product, submatrix


def gershgorin_rho(A: sp.csr_matrix) -> float:
    """Upper bound max_i sum_j |a_ij| / a_ii of the spectral radius of D^-1 A.
    Used as rho(D^-1 A) wherever the method needs it (evolution time step,
    prolongator smoothing): deterministic, and exact for constant-coefficient
    stencils whose off-diagonal entries are non-positive with zero row sums."""
    A = csr(A)
    n = A.shape[0]
    d = A.diagonal()
    row = np.repeat(np.arange(n), np.diff(A.indptr))
    return float(np.max(np.bincount(row, weights=np.abs(A.data), minlength=n) / d))


def evolution_measure(A: sp.csr_matrix, B: np.ndarray, k: int = 2, floor: float = 1e-4):
    """Evolution measure of every stored off-diagonal pair of A (Section 3.2
    uses this measure; Olson, Schroder and Tuminaro, "A new perspective on
    strength measures in algebraic multigrid", NLAA 2010).

    For each point i the unit vector e_i is evolved by k steps of Jacobi
    relaxation, z_i = (I - dt D^-1 A)^k e_i, dt = 1 / rho(D^-1 A) (the
    Gershgorin bound).  Near i, a smooth error is expected to look like the
    near-null vector B, so z_i is compared with its best l2 approximation
    from span{B} among those that agree with z_i at i itself: zt = z_i[i] B / B_i.
    For every stored neighbour j of row i (j != i) the relative misfit
        s_ij = |zt_j - z_i[j]| / |z_i[j]|
    measures the connection (small = strong); it is infinite where
    z_i[j] = 0 or where zt_j and z_i[j] have opposite signs (the two differ by
    more than 90 degrees), and it is floored at `floor`, so that a (near)
    perfect connection does not turn every other connection of its row weak
    at rounding level.  Returns (rows, cols, s) over the stored off-diagonal
    entries in CSR order."""
    A = csr(A)
    n = A.shape[0]
    d = A.diagonal()
    dt = 1.0 / gershgorin_rho(A)
    J = (sp.identity(n, format="csr") - dt * (sp.diags(1.0 / d) @ A)).tocsr()
    Z = J
    for _ in range(k - 1):
        Z = (Z @ J).tocsr()
    ZT = csr(Z.T)  # row i of ZT is z_i = Z e_i
    row = np.repeat(np.arange(n), np.diff(A.indptr))
    col = A.indices
    off = row != col
    row, col = row[off], col[off]
    z_ij = np.asarray(ZT[row, col]).ravel()  # z_i at the stored neighbours j of i
    z_ii = ZT.diagonal()[row]
    zt_j = z_ii * B[col] / B[row]  # the approximation from span{B}, equal to z_i at i
    ok = (z_ij != 0.0) & (zt_j * z_ij > 0.0)
    s = np.full(row.size, np.inf)
    s[ok] = np.maximum(np.abs(zt_j[ok] - z_ij[ok]) / np.abs(z_ij[ok]), floor)
    return row, col, s


def evolution_strength(A: sp.csr_matrix, B: np.ndarray, eps: float = 4.0, k: int = 2) -> sp.csr_matrix:
    """Strength graph of the evolution measure: j is strong for i when
    s_ij <= eps * min_{m != i} s_im (finite measures only), and the graph is
    made symmetric (j strong for i, or i strong for j).  Returns the pattern
    of strong off-diagonal pairs."""
    n = A.shape[0]
    row, col, s = evolution_measure(A, B, k)
    fin = np.isfinite(s)
    smin = np.full(n, np.inf)
    np.minimum.at(smin, row[fin], s[fin])
    strong = fin & (s <= eps * smin[row])
    S = sp.csr_matrix((np.ones(int(strong.sum())), (row[strong], col[strong])), shape=(n, n))
    S = (S + S.T).tocsr()
    S.data[:] = 1.0
    S.sort_indices()
    return S


def strength(A: sp.csr_matrix, theta: float) -> sp.csr_matrix:
    """Classical symmetric strength: j != i is strong for i when
    a_ij^2 >= theta^2 a_ii a_jj."""
    A = csr(A)
    n = A.shape[0]
    d = A.diagonal()
    row = np.repeat(np.arange(n), np.diff(A.indptr))
    v = A.data
    th2 = theta * theta
    strong = (row != A.indices) & (v * v >= th2 * (d[row] * d[A.indices]))
    S = sp.csr_matrix((np.ones(int(strong.sum())), (row[strong], A.indices[strong])), shape=A.shape)
    S.sort_indices()
    return S


def aggregate(S: sp.csr_matrix) -> np.ndarray:
    """Aggregate id per node (standard three-pass aggregation)."""
    n = S.shape[0]
    ptr, ind = S.indptr, S.indices
    agg = -np.ones(n, dtype=np.int64)
    pass1 = np.zeros(n, dtype=bool)
    na = 0
    for i in range(n):
        if agg[i] >= 0:
            continue
        nb = ind[ptr[i]:ptr[i + 1]]
        if np.all(agg[nb] < 0):
            agg[i] = na
            agg[nb] = na
            pass1[i] = True
            pass1[nb] = True
            na += 1
    for i in range(n):
        if agg[i] >= 0:
            continue
        for j in ind[ptr[i]:ptr[i + 1]]:
            if pass1[j]:
                agg[i] = agg[j]
                break
    for i in range(n):
        if agg[i] >= 0:
            continue
        nb = ind[ptr[i]:ptr[i + 1]]
        agg[i] = na
        for j in nb:
            if agg[j] < 0:
                agg[j] = na
        na += 1
    return agg


def tentative(agg: np.ndarray, B: np.ndarray) -> tuple[sp.csr_matrix, np.ndarray]:
    n = agg.size
    nc = int(agg.max()) + 1
    norms = np.sqrt(np.bincount(agg, weights=B * B, minlength=nc))
    T = sp.csr_matrix((B / norms[agg], (np.arange(n), agg)), shape=(n, nc))
    T.sort_indices()
    return T, norms


def smooth(A: sp.csr_matrix, T: sp.csr_matrix) -> sp.csr_matrix:
    """P = (I - omega D^-1 A) T, omega = (4/3) / rho(D^-1 A) (Gershgorin bound)."""
    A = csr(A)
    d = A.diagonal()
    n = A.shape[0]
    row = np.repeat(np.arange(n), np.diff(A.indptr))
    omega = (4.0 / 3.0) / gershgorin_rho(A)
    DA = sp.csr_matrix((A.data / d[row], A.indices, A.indptr), shape=A.shape)
    AT = pattern_product(DA, T)  # pattern of A T contains that of T (A has its diagonal)
    P = AT.copy()
    P.data = -omega * AT.data
    # add T (its entries are in the pattern of A T)
    Tc = T.tocoo()
    key = np.repeat(np.arange(P.shape[0]), np.diff(P.indptr)).astype(np.int64) * P.shape[1] + P.indices
    tkey = Tc.row.astype(np.int64) * P.shape[1] + Tc.col
    pos = np.searchsorted(key, tkey)
    assert np.all(key[pos] == tkey)
    P.data[pos] += Tc.data
    return P


def strength_graph(A: sp.csr_matrix, B: np.ndarray, soc: str, theta: float) -> sp.csr_matrix:
    if soc == "evolution":
        return evolution_strength(A, B)
    if soc == "symmetric":
        return strength(A, theta)
    raise ValueError(soc)


def field_hierarchy(A: sp.csr_matrix, theta: float, max_coarse: int, max_levels: int,
                    soc: str = "evolution"):
    """Interpolation operators P_1, P_2, ... for one scalar field, and the
    near-null vector on every level (ones on the finest).  `theta` is read by
    the symmetric strength measure only."""
    Ps = []
    B = np.ones(A.shape[0])
    Bs = [B]
    Al = csr(A)
    while Al.shape[0] > max_coarse and len(Ps) + 1 < max_levels:
        agg = aggregate(strength_graph(Al, B, soc, theta))
        T, Bc = tentative(agg, B)
        if T.shape[1] >= Al.shape[0]:
            break
        P = smooth(Al, T)
        Ps.append(P)
        Al = galerkin(P, Al)
        B = Bc
        Bs.append(B)
    return Ps, Bs


@dataclass
class Level:
    K: sp.csr_matrix  # saddle operator on this level (free DoFs)
    field: np.ndarray  # 0..d-1 velocity component, d pressure
    P: sp.csr_matrix | None = None  # interpolation to this level from the next
    null_p: np.ndarray | None = None  # pressure near-null vector on this level


def stokes_hierarchy(K1: sp.csr_matrix, field1: np.ndarray, Ap: sp.csr_matrix, dim: int,
                     theta: float = 0.02, max_coarse: int = 300, max_levels: int = 10,
                     soc: str = "evolution") -> list[Level]:
    """Algorithm 1: levels K_1 .. K_lmax on free DoFs (field-blocked order)."""
    K1 = csr(K1)
    blocks = [np.nonzero(field1 == f)[0] for f in range(dim + 1)]
    ops = []
    for f in range(dim):
        idx = blocks[f]
        Af = submatrix(K1, idx, idx)
        ops.append(Af)
    ops.append(csr(Ap))
    hier = [field_hierarchy(A, theta, max_coarse, max_levels, soc) for A in ops]
    lmax = min(len(h[0]) for h in hier) + 1
    levels = [Level(K=K1, field=field1.copy(), null_p=hier[dim][1][0])]
    for l in range(lmax - 1):
        Pl = sp.block_diag([hier[f][0][l] for f in range(dim + 1)], format="csr")
        Pl.sort_indices()
        levels[-1].P = Pl
        Kc = galerkin(Pl, levels[-1].K)
        fc = np.concatenate([np.full(hier[f][0][l].shape[1], f) for f in range(dim + 1)]).astype(np.int8)
        levels.append(Level(K=Kc, field=fc, null_p=hier[dim][1][l + 1]))
    return levels
