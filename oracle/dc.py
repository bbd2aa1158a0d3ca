"""The defect-correction preconditioner (Section 3.1, eqs. (3.1)-(3.4)).
Test infrastructure (oracle).

One application to a residual r (the error propagator of eq. (3.1)):
  level 0 (K0):   x0 = 0;  nu1 pre-relaxation sweeps on K0 x0 = r
                  r0 = r - K0 x0;  b1 = eta R0 r0            (eq. (3.2))
  levels 1..L-1:  the multilevel cycle of eq. (3.4) on the P1isoP2/P1
                  hierarchy of Algorithm 1 (pre-relax, residual, restrict with
                  P_l^T, recurse, prolong with P_l, post-relax)
  level L:        exact solve (dense LU of K_L bordered with the coarse
                  pressure null vector when the pressure is only defined up
                  to a constant)
  back on K0:     x0 += P0 x1;  nu2 post-relaxation sweeps.
Transfers (Section 3.1): Taylor-Hood P0 = R0 = I.  Scott-Vogelius: velocity
identity, P0^p duplicates a continuous P1 pressure onto the discontinuous
DoFs, R0^p = M_cg^{-1} (P0^p)^T M_dg (an L2 projection, solved exactly here).
Schedules (Section 4): "all" relaxes on every level but the coarsest,
"skip1" skips level 1, "skip0" skips level 0.  "ho" is HO-AMG (the remark
after Algorithm 1, compared in Section 4): Algorithm 1 is applied to K0
itself, so the hierarchy's finest entry is K0 and the defect-correction
level 0 is left out (no relaxation there and no eta weights): one monolithic
AMG V-cycle on K0.  Taylor-Hood only (the remark reports that algebraic
coarsening of the discontinuous SV pressure does not give a usable method).
Relaxation kinds: "vanka" (Section 3.3.1) and "dlsc" (Section 3.3.2) on every
relaxed level, and "vanka-dlsc", the hybrid of the Scott-Vogelius parameter
study (Section 4, Table 4): Vanka on K0 (nu1/nu2 sweeps, omega0) and nu_dlsc
DLSC sweeps on the levels of the K1 hierarchy.
Dirichlet rows are identity rows: the preconditioner returns r there.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.sparse.linalg as spla

from . import vanka
from .dlsc import DLSCLevel
from .sa import stokes_hierarchy
from .sparse import submatrix


@dataclass
class Params:
    relax: str = "vanka"  # "vanka", "dlsc" or "vanka-dlsc" (Vanka on K0, DLSC below)
    schedule: str = "all"  # "all", "skip1", "skip0", "ho"
    nu1: int = 1
    nu2: int = 1
    omega0: float = 0.5
    omega: float = 0.5
    eta_u: float = 1.0
    eta_p: float = 1.0
    cheb: tuple | None = None  # DLSC Chebyshev degrees (momentum, continuity, pressure)
    soc: str = "evolution"  # strength of connection: "evolution" (Section 3.2) or "symmetric"
    theta: float = 0.02  # threshold of the symmetric measure (not read by the evolution measure)
    max_coarse: int = 300
    max_levels: int = 10
    seed: int = 0x5EED
    dlsc_amg: int = 0  # >0: the DLSC continuity and pressure stages take one SA V-cycle on S with this many
                       # weighted-Jacobi sweeps before and after the coarse correction (Section 4)
    nu_dlsc: int = 2  # "vanka-dlsc": DLSC sweeps pre and post on the K1 hierarchy (two, Section 4)
    krylov_its: int = 0  # >0: FGMRES(krylov_its)-wrapped Vanka instead of damped sweeps (Section 3.3.1);
                         # Scott-Vogelius keeps the stationary sweep on K0


class DCPreconditioner:
    def __init__(self, prob, par: Params):
        self.par = par
        d = self.dim = prob.dim
        self.disc = prob.disc
        self.n0 = prob.n0
        self.free0 = np.nonzero(~prob.dir0)[0]
        self.dir0 = np.nonzero(prob.dir0)[0]
        self.K0 = submatrix(prob.K0, self.free0, self.free0)
        self.f0 = prob.field0[self.free0]
        self.ho = par.schedule == "ho"
        if self.ho:
            if prob.disc != "TH":
                raise ValueError("HO-AMG (Algorithm 1 on K0) is defined for Taylor-Hood only")
            K1, f1 = self.K0, self.f0  # Algorithm 1's input is K0 itself
        else:
            free1 = np.nonzero(~prob.dir1)[0]
            K1 = submatrix(prob.K1, free1, free1)
            f1 = prob.field1[free1]
        self.levels = stokes_hierarchy(K1, f1, prob.Ap, d, par.theta, par.max_coarse, par.max_levels,
                                       par.soc)
        self.nvel = int((self.f0 < d).sum())
        assert self.nvel == int((f1 < d).sum())
        L = len(self.levels)
        relax_l = [True] * (L + 1)  # index 0 = K0, 1.. = hierarchy entries; the coarsest is solved
        if par.schedule == "skip1":
            relax_l[1] = False
        elif par.schedule in ("skip0", "ho"):
            relax_l[0] = False
        self.relax_on = relax_l
        cheb = par.cheb or ((3, 3, 6) if d == 2 else (4, 4, 16))
        # relaxation data, level 0 and levels 1..L-1 (hierarchy entries 0..L-2)
        self.relax = []
        ops = [(self.K0, self.f0)] + [(lv.K, lv.field) for lv in self.levels[:-1]]
        for l, (K, f) in enumerate(ops):
            if par.relax == "vanka" or (par.relax == "vanka-dlsc" and l == 0):
                if l == 0 and self.disc == "SV":
                    pos = -np.ones(self.n0, dtype=np.int64)
                    pos[self.free0] = np.arange(self.free0.size)
                    seeds = pos[prob.elem_p0]
                    self.relax.append(vanka.patches_element_seeds(K, f, d, seeds))
                else:
                    self.relax.append(vanka.patches_single_seed(K, f, d))
            else:
                nv = int((f < d).sum())
                on_k0 = l == 0 or (self.ho and l == 1)  # M_u = diag(P2 mass) wherever the operator is K0
                mu = prob.mu_diag0[self.free0[:nv]] if on_k0 else np.ones(nv)
                amg = None
                if par.dlsc_amg > 0:
                    amg = (par.theta, par.max_coarse, par.max_levels, par.dlsc_amg, bool(prob.p_nullspace),
                           par.soc)
                self.relax.append(DLSCLevel(K, f, d, mu, cheb, par.seed + 2 * l, amg))
        # coarsest level: dense LU of the (bordered) operator
        last = self.levels[-1]
        Kc = last.K.toarray()
        self.singular = bool(prob.p_nullspace)
        if self.singular:
            nvec = np.zeros(Kc.shape[0])
            nvec[last.field == d] = last.null_p
            nvec /= np.linalg.norm(nvec)
            Kb = np.zeros((Kc.shape[0] + 1,) * 2)
            Kb[:-1, :-1] = Kc
            Kb[:-1, -1] = nvec
            Kb[-1, :-1] = nvec
            self.Kc = Kb
        else:
            self.Kc = Kc
        if self.disc == "SV":
            fp0 = self.free0[self.nvel:] - prob.meta["n_u"]
            self.Pp = prob.Pp0.tocsr()[fp0]
            self.Mdg = submatrix(prob.Mdg, fp0, fp0)
            self.Mcg_lu = spla.splu(prob.Mcg.tocsc())

    # -- pieces -------------------------------------------------------------
    def _relax(self, l: int, K, b, x, sweeps: int, omega: float):
        R = self.relax[l]
        if isinstance(R, vanka.Patches):
            if self.par.krylov_its > 0 and not (self.disc == "SV" and l == 0):
                for _ in range(sweeps):  # nu wrapped relaxations (one each in V(1,1))
                    x = vanka.krylov_relax(K, R, b, x, self.par.krylov_its)
                return x
            for _ in range(sweeps):
                x = vanka.sweep(K, R, b, x, omega)
            return x
        return R.relax(b, x, sweeps)

    def _coarse(self, b):
        if self.singular:
            y = np.linalg.solve(self.Kc, np.concatenate([b, [0.0]]))
            return y[:-1]
        return np.linalg.solve(self.Kc, b)

    def _vcycle(self, j: int, b: np.ndarray) -> np.ndarray:
        """Cycle on hierarchy entry j (paper level l = j + 1)."""
        lv = self.levels[j]
        if j == len(self.levels) - 1:
            return self._coarse(b)
        p = self.par
        x = np.zeros_like(b)
        relax = self.relax_on[j + 1]
        nu1, nu2 = (p.nu_dlsc, p.nu_dlsc) if p.relax == "vanka-dlsc" else (p.nu1, p.nu2)
        if relax:
            x = self._relax(j + 1, lv.K, b, x, nu1, p.omega)
        r = b - lv.K @ x
        xc = self._vcycle(j + 1, lv.P.T @ r)
        x = x + lv.P @ xc
        if relax:
            x = self._relax(j + 1, lv.K, b, x, nu2, p.omega)
        return x

    def restrict0(self, r0: np.ndarray) -> np.ndarray:
        p, nv = self.par, self.nvel
        eta_u, eta_p = (1.0, 1.0) if self.ho else (p.eta_u, p.eta_p)
        out = np.empty(self.levels[0].K.shape[0])
        out[:nv] = eta_u * r0[:nv]
        if self.disc == "TH":
            out[nv:] = eta_p * r0[nv:]
        else:
            out[nv:] = eta_p * self.Mcg_lu.solve(self.Pp.T @ (self.Mdg @ r0[nv:]))
        return out

    def prolong0(self, x1: np.ndarray) -> np.ndarray:
        nv = self.nvel
        if self.disc == "TH":
            return x1.copy()
        return np.concatenate([x1[:nv], self.Pp @ x1[nv:]])

    def apply(self, r: np.ndarray) -> np.ndarray:
        p = self.par
        b = r[self.free0]
        x = np.zeros_like(b)
        if self.relax_on[0]:
            x = self._relax(0, self.K0, b, x, p.nu1, p.omega0)
        r0 = b - self.K0 @ x
        x1 = self._vcycle(0, self.restrict0(r0))
        x = x + self.prolong0(x1)
        if self.relax_on[0]:
            x = self._relax(0, self.K0, b, x, p.nu2, p.omega0)
        z = np.empty(self.n0)
        z[self.free0] = x
        z[self.dir0] = r[self.dir0]
        return z


def default_params(prob, relax: str = "vanka", **over) -> Params:
    """Section 4 defaults.  Strength of connection: the evolution measure of
    Section 3.2 for Taylor-Hood.  Scott-Vogelius keeps the symmetric measure:
    on the Alfeld meshes the evolution measure coarsens the continuous
    pressure of K1 at about half the velocity rate, and the stationary
    omega = 0.5 Vanka sweeps then diverge on the coarse saddle levels (the
    paper's own coarse-level relaxation is wrapped in FGMRES, which
    converges with either measure)."""
    if prob.disc == "SV" and relax == "vanka-dlsc":  # Table 4, structured, Vanka-DLSC row
        p = Params(relax=relax, omega0=0.87, omega=0.5, eta_u=1.0, eta_p=2.96, soc="symmetric")
    elif prob.disc == "SV":
        p = Params(relax=relax, omega0=0.78, omega=0.5, eta_u=1.0, eta_p=2.68, soc="symmetric")
    else:
        p = Params(relax=relax)
    if relax == "dlsc":
        p.nu1 = p.nu2 = 2
    for k, v in over.items():
        setattr(p, k, v)
    return p
