"""Pins for the input generator's assembly and the transfer operators.

* A quadratic velocity / linear pressure Stokes solution lies in the discrete
  spaces, so the discrete solution must equal its interpolant (Section 2:
  TH P2/P1, SV P2/P1disc; the pressure is fixed by its zero mean).
* The P1isoP2/P1 divergence equals the P1/P1 divergence on the refined mesh
  followed by geometric restriction of the pressure (how the paper forms K1,
  Section 4).
* SV transfers (Section 3.1): M_cg = (P0^p)^T M_dg P0^p and R0^p P0^p = I.
* SV velocities are pointwise divergence-free, TH ones weakly (Section 2.1).
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from paper_2306_06795_amd.inputs import fem, make_problem
from paper_2306_06795_amd.inputs.mesh import quadrisect, rect_mesh


def bordered_direct(prob):
    """Sparse direct solve of K0 x = b with the pressure mean fixed to zero."""
    nu = prob.meta["n_u"]
    w = np.zeros(prob.n0)
    w[nu:] = prob.p_weight0
    Kb = sp.bmat([[prob.K0, sp.csr_matrix(w[:, None])], [sp.csr_matrix(w[None, :]), None]], format="csc")
    y = spla.spsolve(Kb, np.concatenate([prob.b, [0.0]]))
    return y[:-1]


CASES = [dict(dim=2, n=4), dict(dim=2, n=8), dict(dim=2, n=6, jitter=0.2, seed=7),
         dict(dim=3, n=2), dict(dim=3, n=3), dict(dim=2, n=4, disc="SV"),
         dict(dim=2, n=5, disc="SV", jitter=0.2, seed=8)]


@pytest.mark.parametrize("kw", CASES)
def test_manufactured_solution_is_reproduced(kw):
    P = make_problem(forcing="manufactured", bc="manufactured", **kw)
    r = P.b - P.K0 @ P.x_exact
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(P.b)
    x = bordered_direct(P)
    assert np.linalg.norm(x - P.x_exact) <= 1e-10 * np.linalg.norm(P.x_exact)


def test_config_sizes_th2d_16():
    P = make_problem(dim=2, n=16)
    assert P.meta["n_u"] == 2178 and P.meta["n_p0"] == 289
    f = ~P.dir0
    assert P.K0[f][:, f].nnz == 38662


@pytest.mark.parametrize("dim,n", [(2, 4), (2, 7), (3, 2)])
def test_iso_divergence_equals_restricted_fine_p1p1(dim, n):
    from paper_2306_06795_amd.inputs.mesh import box_mesh
    base = rect_mesh(n, jitter=0.2, rng=np.random.default_rng(1)) if dim == 2 else box_mesh(n)
    fine = quadrisect(base)
    nn = fine.nv
    B1 = fem.iso_divergence(fine, base, nn)
    Bf = fem.divergence(fine, fine.cells, 1, fine.cells, nn, nn)  # P1/P1 on the refined mesh
    # geometric interpolation of base-mesh P1 pressure onto the refined vertices
    from paper_2306_06795_amd.inputs.mesh import edges
    e, _ = edges(base)
    rows = np.concatenate([np.arange(base.nv), base.nv + np.arange(len(e)), base.nv + np.arange(len(e))])
    cols = np.concatenate([np.arange(base.nv), e[:, 0], e[:, 1]])
    vals = np.concatenate([np.ones(base.nv), 0.5 * np.ones(2 * len(e))])
    Igeo = sp.csr_matrix((vals, (rows, cols)), shape=(nn, base.nv))
    D = (Igeo.T @ Bf - B1).toarray()
    assert np.abs(D).max() <= 1e-13 * np.abs(B1).max()


def test_sv_transfers():
    P = make_problem(dim=2, n=6, disc="SV", jitter=0.2, seed=3)
    Mcg2 = (P.Pp0.T @ P.Mdg @ P.Pp0).toarray()
    assert np.abs(Mcg2 - P.Mcg.toarray()).max() <= 1e-15
    R0 = spla.spsolve(P.Mcg.tocsc(), (P.Pp0.T @ P.Mdg).tocsc()).toarray()
    assert np.abs(R0 @ P.Pp0.toarray() - np.eye(P.Mcg.shape[0])).max() <= 1e-12


def _div_l2(P, x):
    """|| div u_h ||_L2 through the P1disc representation (exact for SV).  K0
    has its Dirichlet columns zeroed and lifted into b, so the divergence of
    the full velocity is -(B_F u_F - b_p)."""
    nu = P.meta["n_u"]
    Bu = P.K0[nu:, :nu] @ x[:nu] - P.b[nu:]
    c = spla.spsolve(P.Mdg.tocsc(), -Bu)
    return float(np.sqrt(c @ (P.Mdg @ c)))


def test_sv_velocity_pointwise_divergence_free():
    P = make_problem(dim=2, n=6, disc="SV", jitter=0.2, seed=5, forcing="gaussian", bc="lid")
    x = bordered_direct(P)
    nu = P.meta["n_u"]
    A = P.K0[:nu, :nu]
    energy = float(np.sqrt(x[:nu] @ (A @ x[:nu])))
    assert _div_l2(P, x) <= 1e-11 * energy
    # mean-zero pressure
    assert abs(P.p_weight0 @ x[nu:]) <= 1e-13 * np.abs(x[nu:]).max()


def test_th_velocity_weakly_divergence_free():
    P = make_problem(dim=2, n=6, jitter=0.2, seed=5, forcing="gaussian", bc="lid")
    x = bordered_direct(P)
    nu = P.meta["n_u"]
    Bu = P.K0[nu:, :nu] @ x[:nu] - P.b[nu:]
    assert np.linalg.norm(Bu) <= 1e-11 * np.linalg.norm(x[:nu])


def test_lid_data_is_compatible():
    """Enclosed flow: the pressure right-hand side is orthogonal to constants."""
    P = make_problem(dim=2, n=16, jitter=0.2, seed=2, forcing="gaussian", bc="lid")
    nu = P.meta["n_u"]
    assert abs(P.b[nu:].sum()) <= 1e-12 * np.abs(P.b).max()


def test_jacobi_scaled_p1_mass_spectrum():
    """Wathen's bounds: for linear triangles the eigenvalues of diag(M)^-1 M lie in
    [1/2, 2] (the interval the library's Chebyshev mass solve relies on)."""
    P = make_problem(dim=2, n=5, disc="SV", jitter=0.2, seed=6)
    M = P.Mcg.toarray()
    d = np.sqrt(np.diag(M))
    ev = np.linalg.eigvalsh(M / d[:, None] / d[None, :])
    assert ev.min() >= 0.5 - 1e-12 and ev.max() <= 2.0 + 1e-12
