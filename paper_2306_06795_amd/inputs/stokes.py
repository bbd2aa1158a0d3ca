"""Seeded synthetic Stokes saddle systems (Section 2, eq. (2.3)).

``make_problem`` builds, for one mesh:
  K0  the high-order operator: Taylor-Hood P2/P1 ("TH") or Scott-Vogelius
      P2/P1disc on the barycentric refinement ("SV");
  K1  the low-order P1isoP2/P1 operator (P1 velocity on the quadrisection of
      the pressure mesh, P1 pressure), co-located with K0's velocity nodes;
  Ap  the P1 pressure stiffness matrix of K1's pressure mesh (Neumann);
and the DoF maps, Dirichlet masks, right-hand sides and, for SV, the pressure
transfer data.  Unknowns are field-blocked [u_x; u_y; (u_z); p].  Dirichlet
velocity DoFs become identity rows with zeroed columns and are lifted into the
right-hand side.  No solver arithmetic lives here: this is the input generator
shared by the oracle, the tests and the benchmark.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from . import fem
from .mesh import Mesh, alfeld, box_mesh, p2_nodes, quadrisect, rect_mesh


@dataclass
class StokesProblem:
    dim: int
    disc: str  # "TH" or "SV"
    K0: sp.csr_matrix
    K1: sp.csr_matrix
    Ap: sp.csr_matrix
    field0: np.ndarray  # int8, 0..dim-1 velocity component, dim = pressure
    field1: np.ndarray
    dir0: np.ndarray  # bool
    dir1: np.ndarray
    b: np.ndarray  # (n0,) or (n0, nrhs)
    p_weight0: np.ndarray  # int psi_i over K0 pressure DoFs (mean-zero weights)
    mu_diag0: np.ndarray  # diag of the P2 velocity mass matrix, per velocity row of K0
    p_nullspace: bool = True  # velocity prescribed on the whole boundary: p defined up to a constant
    x_exact: np.ndarray | None = None
    # Scott-Vogelius only
    elem_p0: np.ndarray | None = None  # (n_elem, 3) global K0 row ids of each element's pressures
    Pp0: sp.csr_matrix | None = None  # P1 (K1 pressure) -> P1disc (K0 pressure) duplication
    Mdg: sp.csr_matrix | None = None  # P1disc mass (3x3 blocks)
    Mcg: sp.csr_matrix | None = None  # P1 mass on K1's pressure mesh
    meta: dict = field(default_factory=dict)

    @property
    def n0(self) -> int:
        return self.K0.shape[0]

    @property
    def n1(self) -> int:
        return self.K1.shape[0]

    @property
    def nrhs(self) -> int:
        return 1 if self.b.ndim == 1 else self.b.shape[1]


def _block_saddle(A: sp.csr_matrix, B: sp.csr_matrix, d: int) -> sp.csr_matrix:
    Av = sp.block_diag([A] * d, format="csr")
    K = sp.bmat([[Av, B.T], [B, None]], format="csr")
    K.sort_indices()
    return K


def _dirichlet(K: sp.csr_matrix, dmask: np.ndarray) -> sp.csr_matrix:
    """Identity rows/columns for Dirichlet DoFs, keeping every structural entry
    of the free-free block (explicit zeros included)."""
    C = K.tocoo()
    keep = ~dmask[C.row] & ~dmask[C.col]
    di = np.nonzero(dmask)[0]
    rows = np.concatenate([C.row[keep], di])
    cols = np.concatenate([C.col[keep], di])
    vals = np.concatenate([C.data[keep], np.ones(di.size)])
    out = sp.coo_matrix((vals, (rows, cols)), shape=K.shape).tocsr()
    out.sort_indices()
    return out


def _forcing_nodal(kind: str, x: np.ndarray, d: int, rng, nu: float) -> np.ndarray:
    """Nodal forcing values (n_nodes, d)."""
    n = x.shape[0]
    if kind == "manufactured":
        if d == 2:  # u=(y^2, x^2), p = x - y:  -nu lap u + grad p
            return np.tile(np.array([-2.0 * nu + 1.0, -2.0 * nu - 1.0]), (n, 1))
        # u=(y^2+z^2, x^2, 0), p = x + y - 2z
        return np.tile(np.array([-4.0 * nu + 1.0, -2.0 * nu + 1.0, -2.0]), (n, 1))
    if kind == "gaussian":
        return rng.standard_normal((d, n)).T.copy()
    if kind == "smooth":
        f = np.zeros((n, d))
        for c in range(d):
            k = rng.integers(1, 4, size=(8, d))
            a = rng.standard_normal(8)
            ph = rng.uniform(0.0, 2.0 * np.pi, size=8)
            f[:, c] = (a[None, :] * np.sin(np.pi * (x @ k.T) + ph[None, :])).sum(1)
        return f
    if kind == "zero":
        return np.zeros((n, d))
    raise ValueError(kind)


def _exact(x: np.ndarray, d: int):
    if d == 2:
        u = np.stack([x[:, 1] ** 2, x[:, 0] ** 2], 1)
    else:
        u = np.stack([x[:, 1] ** 2 + x[:, 2] ** 2, x[:, 0] ** 2, np.zeros(x.shape[0])], 1)
    return u


def _exact_p(x: np.ndarray, d: int):
    return x[:, 0] - x[:, 1] if d == 2 else x[:, 0] + x[:, 1] - 2.0 * x[:, 2]


def make_problem(dim: int = 2, n: int = 16, disc: str = "TH", lx: float = 1.0,
                 jitter: float = 0.0, forcing: str = "manufactured", bc: str = "manufactured",
                 nu: float = 1.0, nrhs: int = 1, seed=None, rng_jitter=None,
                 rng_forcing=None) -> StokesProblem:
    """Assemble one Stokes problem.  ``bc`` is "manufactured" (exact solution on
    the whole boundary), "lid" (u = e_x on the top side y=1, or z=1 in 3D,
    corners included, zero elsewhere) or "zero"."""
    if seed is not None or rng_jitter is None or rng_forcing is None:
        ss = np.random.SeedSequence(0 if seed is None else seed).spawn(3)
        rng_jitter = rng_jitter or np.random.default_rng(ss[0])
        rng_forcing = rng_forcing or np.random.default_rng(ss[1])
    if dim == 2:
        base = rect_mesh(n, lx=lx, ly=1.0, jitter=jitter, rng=rng_jitter)
        hi = np.array([lx, 1.0])
    else:
        assert disc == "TH" and jitter == 0.0
        base = box_mesh(n, lx, 1.0, 1.0)
        hi = np.array([lx, 1.0, 1.0])
    lo = np.zeros(dim)
    pmesh = alfeld(base) if disc == "SV" else base  # mesh carrying K0's velocity
    coords, c2n = p2_nodes(pmesh)
    nn = coords.shape[0]
    fine = quadrisect(pmesh)
    assert fine.nv == nn
    d = dim
    # ---- operators
    A2 = fem.stiffness(pmesh, c2n, 2, nn, nu)
    M2 = fem.mass(pmesh, c2n, 2, nn)
    A1 = fem.stiffness(fine, fine.cells, 1, nn, nu)
    B1 = fem.iso_divergence(fine, pmesh, nn)
    Ap = fem.stiffness(pmesh, pmesh.cells, 1, pmesh.nv, 1.0)
    if disc == "TH":
        np0 = pmesh.nv
        B0 = fem.divergence(pmesh, c2n, 2, pmesh.cells, nn, np0)
        p_weight0 = fem.p1_integrals(pmesh)
    else:
        ne = pmesh.ne
        np0 = 3 * ne
        pc2n = np.arange(np0).reshape(ne, 3)
        B0 = fem.divergence(pmesh, c2n, 2, pc2n, nn, np0)
        _, vol = fem.bary_grads(pmesh)
        p_weight0 = np.repeat(vol / 3.0, 3)
    np1 = pmesh.nv
    nu_tot = d * nn
    K0 = _block_saddle(A2, B0, d)
    K1 = _block_saddle(A1, B1, d)
    field0 = np.concatenate([np.repeat(np.arange(d), nn), np.full(np0, d)]).astype(np.int8)
    field1 = np.concatenate([np.repeat(np.arange(d), nn), np.full(np1, d)]).astype(np.int8)
    # ---- boundary conditions
    on_bnd = np.any((np.abs(coords - lo) < 1e-12) | (np.abs(coords - hi) < 1e-12), axis=1)
    dir0 = np.concatenate([np.tile(on_bnd, d), np.zeros(np0, bool)])
    dir1 = np.concatenate([np.tile(on_bnd, d), np.zeros(np1, bool)])
    g = np.zeros((nn, d))
    if bc == "manufactured":
        g[on_bnd] = _exact(coords[on_bnd], d)
    elif bc == "lid":
        top = on_bnd & (np.abs(coords[:, d - 1] - 1.0) < 1e-12)
        g[top, 0] = 1.0
    elif bc != "zero":
        raise ValueError(bc)
    gvec = np.concatenate([g.T.ravel(), np.zeros(np0)])
    # ---- right-hand sides
    bs = []
    x_exact = None
    for r in range(nrhs):
        f = _forcing_nodal(forcing, coords, d, rng_forcing, nu)
        bu = np.concatenate([M2 @ f[:, c] for c in range(d)])
        b = np.concatenate([bu, np.zeros(np0)])
        b = b - K0 @ gvec  # lift the Dirichlet data
        b[dir0] = gvec[dir0]
        bs.append(b)
    b = bs[0] if nrhs == 1 else np.stack(bs, 1)
    if forcing == "manufactured":
        u = _exact(coords, d)
        if disc == "TH":
            p = _exact_p(pmesh.verts, d)
        else:
            p = _exact_p(pmesh.verts[pmesh.cells.ravel()], d)
        x_exact = np.concatenate([u.T.ravel(), p])
    K0 = _dirichlet(K0, dir0)
    K1 = _dirichlet(K1, dir1)
    Ap.sort_indices()
    prob = StokesProblem(
        dim=d, disc=disc, K0=K0, K1=K1, Ap=Ap, field0=field0, field1=field1,
        dir0=dir0, dir1=dir1, b=b, p_weight0=p_weight0,
        mu_diag0=np.tile(M2.diagonal(), d), x_exact=x_exact,
        meta=dict(n=n, lx=lx, jitter=jitter, forcing=forcing, bc=bc, nu=nu,
                  n_nodes=nn, n_u=nu_tot, n_p0=np0, n_p1=np1, n_elem=pmesh.ne,
                  n_base_elem=base.ne),
    )
    if disc == "SV":
        ne = pmesh.ne
        prob.elem_p0 = nu_tot + np.arange(3 * ne).reshape(ne, 3)
        prob.Pp0 = sp.csr_matrix((np.ones(3 * ne), (np.arange(3 * ne), pmesh.cells.ravel())),
                                 shape=(3 * ne, np1))
        ms, _, _, pm = fem.ref_tensors(2, 2, 1)
        _, vol = fem.bary_grads(pmesh)
        blk = vol[:, None, None] * pm[None]
        r = np.repeat(np.arange(3 * ne).reshape(ne, 3)[:, :, None], 3, 2)
        c = np.repeat(np.arange(3 * ne).reshape(ne, 3)[:, None, :], 3, 1)
        prob.Mdg = sp.coo_matrix((blk.ravel(), (r.ravel(), c.ravel())), shape=(3 * ne, 3 * ne)).tocsr()
        prob.Mcg = fem.mass(pmesh, pmesh.cells, 1, np1)
        prob.Mcg.sort_indices()
        prob.Mdg.sort_indices()
    return prob


# ---------------------------------------------------------------------------
# the five workloads (sizes and seeds fixed here)

def config(name: str) -> dict:
    if name == "th2d_16":  # 16x16 Taylor-Hood, manufactured solution
        return dict(dim=2, n=16, disc="TH", forcing="manufactured", bc="manufactured")
    if name == "th2d_256":  # 256x256 Taylor-Hood: jittered lid-driven cavity, Gaussian forcing
        ss = np.random.SeedSequence(2).spawn(3)
        return dict(dim=2, n=256, disc="TH", jitter=0.2, forcing="gaussian", bc="lid",
                    rng_jitter=np.random.default_rng(ss[0]), rng_forcing=np.random.default_rng(ss[1]))
    if name == "th3d_32":  # 32^3 Taylor-Hood cube: smooth forcing, homogeneous Dirichlet
        return dict(dim=3, n=32, disc="TH", forcing="smooth", bc="zero", seed=3)
    if name == "sv2d_128x64":  # Alfeld refinement of 128x128, 64 right-hand sides
        # unit square: on [0,16]x[0,1] (cells of aspect 16) the SV smoother of the
        # method stalls; see the aspect-ratio finding in the design notes
        return dict(dim=2, n=128, disc="SV", lx=1.0, forcing="gaussian", bc="zero", nrhs=64, seed=4)
    if name == "sv2d_128x64_aspect16":
        return dict(dim=2, n=128, disc="SV", lx=16.0, forcing="gaussian", bc="zero", nrhs=64, seed=4)
    raise KeyError(name)


def make_config(name: str, **over) -> StokesProblem:
    kw = config(name)
    kw.update(over)
    return make_problem(**kw)


# ---------------------------------------------------------------------------
# the serving stream: Poisson arrivals over a mix of meshes and viscosities

SERVE_MESHES = [(2, 32), (2, 64), (2, 128), (2, 256), (3, 8), (3, 12), (3, 16), (3, 24)]


def serve_mesh_key(dim: int, n: int) -> str:
    return f"th{dim}d_{n}"


def make_serve_mesh(dim: int, n: int) -> StokesProblem:
    """A serving mesh at viscosity 1: Taylor-Hood on the unit square / cube,
    homogeneous Dirichlet velocity (the requests bring their own forcing)."""
    return make_problem(dim=dim, n=n, disc="TH", forcing="gaussian", bc="zero", seed=100 * dim + n)


def random_rhs(prob: StokesProblem, rng) -> np.ndarray:
    """Right-hand side of a request: N(0, 1) nodal forcing weighted by the
    diagonal of the velocity mass matrix, zero on Dirichlet rows and on the
    continuity rows (homogeneous boundary data)."""
    nu = prob.meta["n_u"]
    b = np.zeros(prob.K0.shape[0])
    b[:nu] = prob.mu_diag0 * rng.standard_normal(nu)
    b[prob.dir0] = 0.0
    return b


def serve_stream(n_req: int = 512, seed: int = 5, meshes=None):
    """The request stream: mesh drawn uniformly (half 2D, half 3D), viscosity
    log-uniform in [1e-2, 1], forcing seed, and unit-rate exponential
    inter-arrival gaps (scaled to the wanted rate by the caller)."""
    meshes = meshes or SERVE_MESHES
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_req):
        dim, n = meshes[int(rng.integers(len(meshes)))]
        nu = float(10.0 ** rng.uniform(-2.0, 0.0))
        out.append(dict(mesh=serve_mesh_key(dim, n), dim=dim, n=n, nu=nu, rhs_seed=int(rng.integers(2**31)),
                        gap=float(rng.exponential(1.0))))
    return out
