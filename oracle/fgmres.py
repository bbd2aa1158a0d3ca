"""Restarted, right-preconditioned FGMRES (Section 3.3.1 footnote; Section 4:
restart 20, relative l2 residual criterion).  Test infrastructure (oracle).

Readings: x0 = 0; modified Gram-Schmidt; Givens rotations on the Hessenberg
matrix; the cycle stops when the rotated residual estimate drops to
rtol * ||b||, then the true residual is checked and the method restarts from
the current iterate if it is not yet met.  The convergence factor reported is
the geometric mean of the residual reductions over the last 10 iterations
(Section 4).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class FGMRESResult:
    x: np.ndarray
    iters: int
    converged: bool
    relres: float
    history: list = field(default_factory=list)  # residual estimate after each iteration

    @property
    def conv_factor(self) -> float:
        h = self.history
        if len(h) < 11:
            return float("nan")
        return float((h[-1] / h[-11]) ** 0.1)


def fgmres(matvec, precond, b: np.ndarray, rtol: float = 1e-8, restart: int = 20,
           max_it: int = 1000) -> FGMRESResult:
    n = b.size
    bnorm = float(np.linalg.norm(b))
    x = np.zeros(n)
    if bnorm == 0.0:
        return FGMRESResult(x, 0, True, 0.0)
    target = rtol * bnorm
    r = b.copy()
    beta = bnorm
    it = 0
    hist = [beta]
    while True:
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(restart):
            Z[j] = precond(V[j])
            w = matvec(Z[j])
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            k = j + 1
            hist.append(abs(g[j + 1]))
            if abs(g[j + 1]) <= target or it >= max_it:
                break
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        x = x + Z[:k].T @ y
        r = b - matvec(x)
        beta = float(np.linalg.norm(r))
        if beta <= target:
            return FGMRESResult(x, it, True, beta / bnorm, hist)
        if it >= max_it:
            return FGMRESResult(x, it, False, beta / bnorm, hist)


def solve(prob, pre, rtol: float = 1e-8, max_it: int = 1000, rhs: np.ndarray | None = None):
    """FGMRES on K0 x = b with the DC preconditioner; the pressure of the result
    is shifted to zero mean (weights int psi_i) when it is only defined up to a
    constant."""
    b = prob.b if rhs is None else rhs
    res = fgmres(lambda v: prob.K0 @ v, pre.apply, b, rtol, 20, max_it)
    if prob.p_nullspace:
        nu = prob.meta["n_u"]
        w = prob.p_weight0
        res.x[nu:] -= (w @ res.x[nu:]) / w.sum()
    return res
