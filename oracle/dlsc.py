"""Chebyshev polynomial relaxation and the DLSC sweep (Algorithm 2,
Section 3.3.2, Table 3).  Test infrastructure (oracle).

Readings:
  * Chebyshev "degree k" on [a, b] = [0.5^d lambda, 1.1 lambda] is k steps of
    the textbook Chebyshev semi-iteration for X y = r from y = 0, i.e. the
    residual polynomial T_k((b+a-2t)/(b-a)) / T_k((b+a)/(b-a)), using k-1
    products with X.
  * lambda is the largest Ritz value of 20 Lanczos steps (full
    reorthogonalisation) from a SplitMix64 start vector.
  * The sign of the pressure correction is the one of Algorithm 2:
    delta p solves S delta p = -(B M^-1 A M^-1 B^T) q, S = B M^-1 B^T.
"""
from __future__ import annotations

import numpy as np

from .sparse import uniform_pm1

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


class DLSCLevel:
    """Operators of one level for Algorithm 2: A (velocity block), B, M_u (diagonal)."""

    def __init__(self, K, field, dim, mu_diag, degrees, seed):
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

    def S(self, q):
        return self.B @ (self.minv * (self.B.T @ q))

    def sweep(self, f: np.ndarray, g: np.ndarray, u: np.ndarray, p: np.ndarray):
        c = 0.5 ** self.dim
        A, B, minv = self.A, self.B, self.minv
        ru = f - A @ u - B.T @ p
        vs = chebyshev(lambda v: A @ v, ru, c * self.lam_A, 1.1 * self.lam_A, self.deg[0])
        rp = g - B @ (u + vs)
        q = chebyshev(self.S, rp, c * self.lam_S, 1.1 * self.lam_S, self.deg[1])
        rhs = -(B @ (minv * (A @ (minv * (B.T @ q)))))
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
