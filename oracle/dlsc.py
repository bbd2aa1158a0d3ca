"""Chebyshev polynomial relaxation and the DLSC sweep (Algorithm 2,
Section 3.3.2, Table 2).  Test infrastructure (oracle).

Readings:
  * Chebyshev "degree k" on [a, b] = [0.5^d lambda, 1.1 lambda] is k steps of
    the textbook Chebyshev semi-iteration for X y = r from y = 0, i.e. the
    residual polynomial T_k((b+a-2t)/(b-a)) / T_k((b+a)/(b-a)), using k-1
    products with X.
  * lambda is the largest Ritz value of 20 Lanczos steps (full
    reorthogonalisation) from a SplitMix64 start vector.
  * The sign of the pressure correction is the one of Algorithm 2:
    delta p solves S delta p = -(B M^-1 A M^-1 B^T) q, S = B M^-1 B^T.
  * AMG stages (Section 5, the application problems): the continuity and
    pressure-correction stages may instead take one smoothed-aggregation
    V-cycle on S (Algorithm 1's scalar SA, constants as near-null vector)
    with `sweeps` weighted-Jacobi sweeps before and after the coarse
    correction, weight (4/3) / rho, rho = max_i sum_j |s_ij| / s_ii on each
    level (the bound used for prolongator smoothing), and an exact coarsest
    solve, bordered with the coarse near-null vector when S is singular.
"""
from __future__ import annotations

import numpy as np

import scipy.sparse as sp

from .sa import field_hierarchy
from .sparse import csr, galerkin, pattern_product, uniform_pm1

LANCZOS_STEPS = 20


def lanczos_max(matvec, n: int, seed: int, steps: int = LANCZOS_STEPS) -> float:
    v = uniform_pm1(n, seed)
    v /= np.linalg.norm(v)
    V = [v]
    alpha, beta = [], []
    k = min(steps, n)
    for j in range(k):
        w = matvec(V[j])
        a = float(V[j] @ w)
        alpha.append(a)
        for u in V:  # full reorthogonalisation (two passes of classical GS)
            w = w - (u @ w) * u
        for u in V:
            w = w - (u @ w) * u
        bnorm = float(np.linalg.norm(w))
        if j == k - 1 or bnorm == 0.0:
            break
        beta.append(bnorm)
        V.append(w / bnorm)
    T = np.diag(alpha) + np.diag(beta[:len(alpha) - 1], 1) + np.diag(beta[:len(alpha) - 1], -1)
    return float(np.linalg.eigvalsh(T)[-1])


def chebyshev(matvec, r: np.ndarray, lo: float, hi: float, degree: int) -> np.ndarray:
    """Approximate X^{-1} r by ``degree`` Chebyshev steps from zero (Saad, Iterative
    Methods for Sparse Linear Systems, Alg. 12.1)."""
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    sigma = theta / delta
    rho = 1.0 / sigma
    d = r / theta
    y = np.zeros_like(r)
    res = r.copy()
    for k in range(degree):
        y = y + d
        if k == degree - 1:
            break
        res = res - matvec(d)
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * res
        rho = rho_new
    return y


class SAVcycle:
    """One V-cycle of smoothed aggregation with weighted Jacobi for S y = r."""

    def __init__(self, S, theta: float, max_coarse: int, max_levels: int, sweeps: int, singular: bool,
                 soc: str = "evolution"):
        S = csr(S)
        Ps, Bs = field_hierarchy(S, theta, max_coarse, max_levels, soc)
        self.ops = [S]
        for P in Ps:
            self.ops.append(galerkin(P, self.ops[-1]))
        self.Ps = Ps
        self.sweeps = sweeps
        self.wdinv = []
        for A in self.ops[:-1]:
            d = A.diagonal()
            rho = np.max(np.abs(A).sum(axis=1).A1 / d)
            self.wdinv.append((4.0 / 3.0) / rho / d)
        C = self.ops[-1].toarray()
        self.singular = singular
        if singular:
            nvec = Bs[-1] / np.linalg.norm(Bs[-1])
            m = C.shape[0]
            Cb = np.zeros((m + 1, m + 1))
            Cb[:m, :m] = C
            Cb[:m, m] = nvec
            Cb[m, :m] = nvec
            C = Cb
        self.C = C

    def _coarse(self, b):
        if self.singular:
            return np.linalg.solve(self.C, np.concatenate([b, [0.0]]))[:-1]
        return np.linalg.solve(self.C, b)

    def _cycle(self, k: int, b: np.ndarray) -> np.ndarray:
        if k == len(self.ops) - 1:
            return self._coarse(b)
        A, w = self.ops[k], self.wdinv[k]
        x = np.zeros_like(b)
        for _ in range(self.sweeps):
            x = x + w * (b - A @ x)
        P = self.Ps[k]
        x = x + P @ self._cycle(k + 1, P.T @ (b - A @ x))
        for _ in range(self.sweeps):
            x = x + w * (b - A @ x)
        return x

    def apply(self, r: np.ndarray) -> np.ndarray:
        return self._cycle(0, r)


class DLSCLevel:
    """Operators of one level for Algorithm 2: A (velocity block), B, M_u (diagonal)."""

    def __init__(self, K, field, dim, mu_diag, degrees, seed, amg=None):
        isv = field < dim
        self.iv = np.nonzero(isv)[0]
        self.ip = np.nonzero(~isv)[0]
        K = K.tocsr()
        self.A = K[self.iv][:, self.iv]
        self.B = K[self.ip][:, self.iv]
        self.minv = 1.0 / mu_diag
        self.deg = degrees
        self.dim = dim
        self.lam_A = lanczos_max(lambda v: self.A @ v, self.iv.size, seed)
        self.lam_S = lanczos_max(self.S, self.ip.size, seed + 1)
        self.svc = None
        if amg is not None:  # (theta, max_coarse, max_levels, sweeps, singular, soc)
            Bt = csr(self.B.T)
            S = pattern_product(self.B, csr(sp.diags(self.minv) @ Bt))
            self.svc = SAVcycle(S, *amg)

    def S(self, q):
        return self.B @ (self.minv * (self.B.T @ q))

    def sweep(self, f: np.ndarray, g: np.ndarray, u: np.ndarray, p: np.ndarray):
        c = 0.5 ** self.dim
        A, B, minv = self.A, self.B, self.minv
        ru = f - A @ u - B.T @ p
        vs = chebyshev(lambda v: A @ v, ru, c * self.lam_A, 1.1 * self.lam_A, self.deg[0])
        rp = g - B @ (u + vs)
        if self.svc is not None:
            q = self.svc.apply(rp)
        else:
            q = chebyshev(self.S, rp, c * self.lam_S, 1.1 * self.lam_S, self.deg[1])
        rhs = -(B @ (minv * (A @ (minv * (B.T @ q)))))
        if self.svc is not None:
            dp = self.svc.apply(rhs)
        else:
            dp = chebyshev(self.S, rhs, c * self.lam_S, 1.1 * self.lam_S, self.deg[2])
        du = vs + minv * (B.T @ q)
        return u + du, p + dp

    def relax(self, b: np.ndarray, x: np.ndarray, sweeps: int) -> np.ndarray:
        u, p = x[self.iv].copy(), x[self.ip].copy()
        f, g = b[self.iv], b[self.ip]
        for _ in range(sweeps):
            u, p = self.sweep(f, g, u, p)
        out = np.empty_like(x)
        out[self.iv] = u
        out[self.ip] = p
        return out
