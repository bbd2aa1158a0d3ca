"""Pins of the oracle's smoothed aggregation (Algorithm 1, Section 3.2), of the
Scott-Vogelius transfers (Section 3.1) and of the algebraic Vanka patches
(Section 3.3.1), against closed forms derived by hand from the definitions:
path counting for the evolution measure on stencils with known entries, the
1D Laplacian for prolongator smoothing, the mesh geometry for patch
membership, and the P1 -> P1disc duplication read off the mesh for the SV
transfers.  None of them calls the function it pins to make its expectation.
"""
from __future__ import annotations

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import dc, sa
from paper_2306_06795_amd.inputs.mesh import alfeld, p2_nodes, rect_mesh
from paper_2306_06795_amd.inputs.stokes import make_problem


def _grid_aniso(m: int, a: float) -> sp.csr_matrix:
    """-a u_xx - u_yy, 5-point stencil on an m x m interior grid (Dirichlet rows
    eliminated): diagonal 2a + 2, x-neighbours -a, y-neighbours -1; node
    (ix, iy) has index ix + m iy."""
    n = m * m
    rows, cols, vals = [], [], []
    for iy in range(m):
        for ix in range(m):
            i = ix + m * iy
            rows.append(i), cols.append(i), vals.append(2 * a + 2)
            for dx, dy, v in ((1, 0, -a), (-1, 0, -a), (0, 1, -1.0), (0, -1, -1.0)):
                jx, jy = ix + dx, iy + dy
                if 0 <= jx < m and 0 <= jy < m:
                    rows.append(i), cols.append(jx + m * jy), vals.append(v)
    A = sp.csr_matrix((vals, (rows, cols)), shape=(n, n))
    A.sort_indices()
    return A


@pytest.mark.parametrize("a", [0.01, 1.0])
def test_evolution_measure_closed_form_on_the_anisotropic_stencil(a):
    """Every row with four neighbours has sum |a_ij| / a_ii = 2, so dt = 1/2 and
    J = I - D^-1 A / 2 has 1/2 on the diagonal and c_x = a / (4 (a + 1)),
    c_y = 1 / (4 (a + 1)) towards the x / y neighbours.  Two neighbours of the
    5-point stencil share no neighbour, so the only two-step paths are
    i->i->j and i->j->j: z_i[j] = 2 (1/2) c = c; the paths back to i give
    z_i[i] = 1/4 + n_x c_x^2 + n_y c_y^2 (n_x, n_y: neighbours present).  With
    B = 1: s_ij = z_i[i] / z_i[j] - 1."""
    m = 7
    A = _grid_aniso(m, a)
    cx, cy = a / (4 * (a + 1)), 1 / (4 * (a + 1))
    row, col, s = sa.evolution_measure(A, np.ones(m * m))
    ix, iy = row % m, row // m
    nx = (ix > 0).astype(int) + (ix < m - 1)
    ny = (iy > 0).astype(int) + (iy < m - 1)
    zii = 0.25 + nx * cx ** 2 + ny * cy ** 2
    horiz = (col - row) ** 2 == 1
    zij = np.where(horiz, cx, cy)
    expect = np.maximum(zii / zij - 1, 1e-4)
    np.testing.assert_allclose(s, expect, rtol=1e-13, atol=0)
    S = sa.evolution_strength(A, np.ones(m * m)).tocoo()
    pairs = set(zip(S.row.tolist(), S.col.tolist()))
    vert = {(i, j) for i, j in zip(row.tolist(), col.tolist()) if abs(i - j) == m}
    if a < 0.1:  # strong anisotropy: only the y links survive the filter
        assert pairs == vert
    else:  # isotropic: every link is within a factor 4 of the row minimum
        assert pairs == set(zip(row.tolist(), col.tolist()))


def _chain(d: np.ndarray) -> sp.csr_matrix:
    n = d.size
    A = sp.diags([-np.ones(n - 1), d, -np.ones(n - 1)], [-1, 0, 1]).tocsr()
    A.sort_indices()
    return A


def _chain_expect(d, B):
    """Closed form of the evolution measure on a chain a_ii = d_i, a_{i,i+-1} = -1:
    J_ii = 1 - dt, J_{i,i+-1} = dt / d_i with dt = 1 / max_i (d_i + #nbrs_i) / d_i;
    z_i[j] = J_jj J_ji + J_ji J_ii = 2 dt (1 - dt) / d_j (the row of the
    destination j, not of i), z_i[i] = (1 - dt)^2 + sum_m (dt / d_i)(dt / d_m)."""
    n = d.size
    nb = np.full(n, 2)
    nb[0] = nb[-1] = 1
    dt = 1.0 / np.max((d + nb) / d)
    out = {}
    for i in range(n):
        zii = (1 - dt) ** 2 + sum((dt / d[i]) * (dt / d[m]) for m in (i - 1, i + 1) if 0 <= m < n)
        for j in (i - 1, i + 1):
            if not 0 <= j < n:
                continue
            zij = 2 * dt * (1 - dt) / d[j]
            zt = zii * B[j] / B[i]
            out[(i, j)] = max(abs(zt - zij) / abs(zij), 1e-4) if zt * zij > 0 else np.inf
    return out


def test_evolution_measure_chain_with_variable_diagonal_and_near_null_vector():
    """A varying diagonal makes D^-1 A unsymmetric (a transposed evolution
    gives dt (1 - dt) / d_i instead of / d_j), and a varying B (the coarse-level
    near-null vector) enters through the constrained approximation; a sign
    change of B makes the approximation point the other way (angle > 90
    degrees): that connection is weak (infinite measure)."""
    n = 12
    i = np.arange(n)
    d = 2.2 + 1.5 * (np.sin(1.7 * i) + 1)
    B = 1.0 + 0.4 * np.cos(0.9 * i)
    B[7] = -B[7]
    row, col, s = sa.evolution_measure(_chain(d), B)
    exp = _chain_expect(d, B)
    assert np.isinf(exp[(6, 7)]) and np.isinf(exp[(8, 7)])
    for r, c, v in zip(row.tolist(), col.tolist(), s):
        e = exp[(r, c)]
        if np.isinf(e):
            assert np.isinf(v)
        else:
            assert v == pytest.approx(e, rel=1e-13)


def test_evolution_filter_and_symmetrisation():
    """Chain 0 - 1 - 2 with d_2 >> d_0: from row 1 the link to 2 measures more
    than 4x the link to 0 (weak for 1), but it is node 2's only link (strong for
    2); the symmetric strength graph keeps it.  Node 3 hangs off 2 only."""
    d = np.array([2.5, 2.5, 40.0, 2.5])
    exp = _chain_expect(d, np.ones(4))
    assert exp[(1, 2)] > 4 * exp[(1, 0)]  # one-sided: 2 is weak for 1
    S = sa.evolution_strength(_chain(d), np.ones(4)).toarray()
    assert np.array_equal(S, S.T)
    assert S[1, 2] == 1 and S[2, 1] == 1 and S[0, 1] == 1
    assert np.count_nonzero(S) == 6  # all three links, both ways


def test_symmetric_strength_compares_squares():
    """a_ij^2 >= theta^2 a_ii a_jj.  On -a u_xx - u_yy the x link has
    |a_ij| / sqrt(a_ii a_jj) = a / (2a + 2): 0.1 at a = 0.25 (strong at theta =
    0.02; a test of a_ij^2 against theta instead of theta^2 would drop it) and
    0.00495 at a = 0.01 (weak)."""
    m = 5
    for a, x_strong in ((0.25, True), (0.01, False)):
        A = _grid_aniso(m, a)
        S = sa.strength(A, 0.02).tocoo()
        pairs = set(zip(S.row.tolist(), S.col.tolist()))
        C = A.tocoo()
        for r, c in zip(C.row.tolist(), C.col.tolist()):
            if r == c:
                continue
            expected = x_strong if abs(r - c) == 1 else True
            assert ((r, c) in pairs) == expected


def test_prolongator_smoothing_on_the_1d_laplacian():
    """1D Laplacian tridiag(-1, 2, -1) with Dirichlet ends: the largest
    sum |a_ij| / a_ii is 2, so omega = (4/3) / 2 = 2/3 and
    P = (I - omega D^-1 A) T = (I - A / 3) T, i.e. P[i, :] = (T[i-1] + T[i] + T[i+1]) / 3
    (T = 0 outside the chain).  Aggregates of three with T = 1/sqrt(3)."""
    n = 9
    A = _chain(np.full(n, 2.0))
    agg = np.repeat(np.arange(3), 3)
    T, Bc = sa.tentative(agg, np.ones(n))
    np.testing.assert_allclose(Bc, np.sqrt(3.0), rtol=1e-15)
    P = sa.smooth(A, T).toarray()
    t = 1 / np.sqrt(3)
    E = np.zeros((n, 3))
    for i in range(n):
        for j in (i - 1, i, i + 1):
            if 0 <= j < n:
                E[i, agg[j]] += t / 3
    np.testing.assert_allclose(P, E, rtol=1e-14, atol=1e-16)
    assert sa.gershgorin_rho(A) == 2.0


def _sv_dup(n: int, prob) -> np.ndarray:
    """P1 -> P1disc duplication read off the Alfeld mesh: element e's three
    pressure values are the continuous pressure at its vertices."""
    m = alfeld(rect_mesh(n))
    return m.cells  # (n_elem, 3) vertex ids, in the order of the element's pressure DoFs


def test_sv_restriction_inverts_the_duplication():
    """R0^p = M_cg^-1 (P0^p)^T M_dg with M_cg = (P0^p)^T M_dg P0^p, so the
    restriction of a duplicated continuous pressure is the pressure itself:
    restrict0 returns eta_p q exactly (up to rounding) and prolong0 duplicates q."""
    n = 4
    P = make_problem(dim=2, n=n, disc="SV", seed=4, forcing="gaussian", bc="zero")
    par = dc.default_params(P, max_coarse=10 ** 6)
    pre = dc.DCPreconditioner(P, par)
    cells = _sv_dup(n, P)
    q = np.random.default_rng(1).standard_normal(P.meta["n_p1"])
    nv = pre.nvel
    dup = q[cells].ravel()  # K0 pressure DoF 3e + k sits at vertex cells[e, k]
    r0 = np.concatenate([np.zeros(nv), dup])
    out = pre.restrict0(r0)
    np.testing.assert_allclose(out[nv:], par.eta_p * q, rtol=1e-12, atol=1e-12 * np.abs(q).max())
    assert np.all(out[:nv] == 0.0)
    x1 = np.concatenate([np.zeros(nv), q])
    np.testing.assert_array_equal(pre.prolong0(x1)[nv:], dup)


def test_sv_two_level_cycle_equals_dense_formula():
    """Scott-Vogelius with the K1 hierarchy reduced to one exactly solved level:
    apply(r) = x3 with x1 = w0 M0 r, x2 = x1 + P0 K1^+ eta R0 (r - K0 x1),
    x3 = x2 + w0 M0 (r - K0 x2), where M0 = sum_e V_e^T W_e K_e^-1 V_e over
    the element patches, P0 = diag(I, Dup), R0 = diag(I, M_cg^-1 Dup^T M_dg),
    and Dup is read off the mesh, all written with dense matrices."""
    n = 3
    P = make_problem(dim=2, n=n, disc="SV", seed=4, forcing="gaussian", bc="zero")
    par = dc.default_params(P, max_coarse=10 ** 6)
    pre = dc.DCPreconditioner(P, par)
    assert len(pre.levels) == 1
    nv = pre.nvel
    n1 = pre.levels[0].K.shape[0]
    np1 = n1 - nv
    cells = _sv_dup(n, P)
    np0 = cells.size
    Dup = np.zeros((np0, np1))
    Dup[np.arange(np0), cells.ravel()] = 1.0
    Mdg = P.Mdg.toarray()
    Mcg = Dup.T @ Mdg @ Dup  # the P1 mass on the macro mesh (checked against the input below)
    np.testing.assert_allclose(Mcg, P.Mcg.toarray(), rtol=1e-12, atol=1e-16)
    R0 = np.zeros((n1, nv + np0))
    R0[:nv, :nv] = np.eye(nv)
    R0[nv:, nv:] = np.linalg.solve(Mcg, Dup.T @ Mdg)
    P0 = np.zeros((nv + np0, n1))
    P0[:nv, :nv] = np.eye(nv)
    P0[nv:, nv:] = Dup
    eta = np.diag(np.r_[np.full(nv, par.eta_u), np.full(np1, par.eta_p)])
    K0 = pre.K0.toarray()
    M0 = np.zeros_like(K0)
    for dofs in pre.relax[0].dofs:
        Ki = K0[np.ix_(dofs, dofs)]
        M0[np.ix_(dofs, dofs)] += np.diag(pre.relax[0].weight[dofs]) @ np.linalg.inv(Ki)
    K1p = np.linalg.pinv(pre.levels[0].K.toarray())
    r = np.random.default_rng(7).standard_normal(P.n0)
    rf = r[pre.free0]
    w = par.omega0
    x1 = w * M0 @ rf
    x2 = x1 + P0 @ (K1p @ (eta @ (R0 @ (rf - K0 @ x1))))
    x3 = x2 + w * M0 @ (rf - K0 @ x2)
    z = pre.apply(r)[pre.free0]
    # the bordered coarse solve and the pseudo-inverse differ by a constant
    # continuous pressure, which P0 duplicates and the K0 sweep then carries on
    # linearly: compare after removing the component along the pressure null
    # vector of K0
    c = np.zeros(nv + np0)
    c[nv:] = 1.0
    Mc = c - w * M0 @ (K0 @ c)  # what the post-sweep makes of a constant pressure shift
    dz = z - x3
    alpha = (Mc @ dz) / (Mc @ Mc)
    assert np.linalg.norm(dz - alpha * Mc) <= 1e-9 * np.linalg.norm(x3)


def _star_offsets():
    """The 19 P2 nodes of the closed star of a vertex in a mesh of squares split
    along (i,j)->(i+1,j+1), in units of h: the vertex, its six neighbours, the
    six spoke midpoints and the six rim-edge midpoints."""
    nbr = [(1, 0), (1, 1), (0, 1), (-1, 0), (-1, -1), (0, -1)]  # counter-clockwise
    pts = {(0.0, 0.0)}
    pts |= {(float(a), float(b)) for a, b in nbr}
    pts |= {(a / 2, b / 2) for a, b in nbr}
    for k in range(6):
        (a, b), (c, e) = nbr[k], nbr[(k + 1) % 6]
        pts.add(((a + c) / 2, (b + e) / 2))
    assert len(pts) == 19
    return pts


@pytest.mark.parametrize("n", [6, 9])
def test_vertex_star_patches_closed_form(n):
    """Taylor-Hood, Dirichlet velocity on the whole boundary: the patch of the
    pressure at vertex (i, j) holds the velocity DoFs of B's row, i.e. both
    components at the 19 P2 nodes of the vertex's closed star, and is free of
    Dirichlet DoFs exactly when 2 <= i, j <= n - 2: (n - 3)^2 patches of 39 DoFs.
    The same sets on K1 (P1 on the quadrisected mesh has the same B pattern)."""
    P = make_problem(dim=2, n=n, disc="TH", forcing="gaussian", bc="zero", seed=1)
    par = dc.default_params(P, max_coarse=10)
    pre = dc.DCPreconditioner(P, par)
    assert len(pre.levels) >= 2  # K1 is relaxed, not solved
    base = rect_mesh(n)
    coords, _ = p2_nodes(base)
    nn = coords.shape[0]
    h = 1.0 / n
    star = _star_offsets()
    free0 = pre.free0
    nv = pre.nvel
    for level, pt in ((0, pre.relax[0]), (1, pre.relax[1])):
        full = [d for d in pt.dofs if d.size == 39]
        assert len(full) == (n - 3) ** 2
        for dofs in pt.dofs:
            g = free0[dofs]  # K0 and K1 share the free numbering on TH
            vel, pres = g[g < 2 * nn], g[g >= 2 * nn]
            assert pres.size == 1
            v = pres[0] - 2 * nn
            vi, vj = np.rint(base.verts[v] / h).astype(int)
            interior = 2 <= vi <= n - 2 and 2 <= vj <= n - 2
            assert (dofs.size == 39) == interior
            for comp in (0, 1):
                nodes = vel[(vel // nn) == comp] % nn
                offs = {tuple(x) for x in np.round((coords[nodes] - base.verts[v]) / h * 2) / 2}
                assert offs <= star  # never outside the closed star
                if interior:
                    assert offs == star
        assert len(pt.dofs) == P.meta["n_p1"]
    assert nv == int((~P.dir0[: 2 * nn]).sum())


def test_dense_patch_blocks_are_the_principal_submatrices():
    """The oracle's dense patch matrices equal scipy's fancy-indexed submatrix
    A[idx][:, idx] (explicit zeros included as zeros)."""
    from oracle.sparse import dense_blocks
    rng = np.random.default_rng(0)
    A = sp.random(120, 120, density=0.08, random_state=3, format="csr")
    A = sp.csr_matrix(A + A.T + sp.identity(120))
    A.sort_indices()
    idx = np.stack([np.sort(rng.choice(120, 13, replace=False)) for _ in range(25)])
    D = dense_blocks(A, idx)
    assert np.array_equal(D, np.stack([A[i][:, i].toarray() for i in idx]))
