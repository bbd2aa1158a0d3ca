"""Pins for the oracle's solver pieces, each against something other than itself:
closed forms, special cases that reduce to an exact solve, invariants the
paper states, dense linear algebra and a sparse direct solve."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import dc, dlsc, fgmres, sa, vanka
from oracle.sparse import galerkin, pattern_product, submatrix, uniform_pm1
from paper_2306_06795_amd.inputs import make_problem

from test_oracle_assembly import bordered_direct


# --------------------------------------------------------------------------
# block factorisation of a Vanka patch (eqs. (3.6)-(3.8), U = A^-1 B^T)

def block_apply(K, nv, ncomp_sizes, b):
    """x = [I Uhat; 0 I][A^-1 0; Bhat S^-1] b with A block-diagonal per component."""
    A = K[:nv, :nv]
    B = K[nv:, :nv]
    Ainv = np.zeros_like(A)
    o = 0
    for m in ncomp_sizes:
        Ainv[o:o + m, o:o + m] = np.linalg.inv(A[o:o + m, o:o + m])
        o += m
    U = Ainv @ B.T
    S = -B @ U
    Sinv = np.linalg.inv(S)
    Bhat = -Sinv @ B @ Ainv
    Uhat = -U
    yu = Ainv @ b[:nv]
    yp = Bhat @ b[:nv] + Sinv @ b[nv:]
    return np.concatenate([yu + Uhat @ yp, yp])


@pytest.mark.parametrize("kw", [dict(dim=2, n=8, jitter=0.2, seed=1), dict(dim=3, n=3),
                                dict(dim=2, n=4, disc="SV")])
def test_block_lu_equals_dense_solve_on_every_patch(kw):
    P = make_problem(forcing="gaussian", bc="zero", **kw)
    f = np.nonzero(~P.dir0)[0]
    K = submatrix(P.K0, f, f)
    fld = P.field0[f]
    d = P.dim
    if P.disc == "SV":
        pos = -np.ones(P.n0, dtype=np.int64)
        pos[f] = np.arange(f.size)
        pt = vanka.patches_element_seeds(K, fld, d, pos[P.elem_p0])
    else:
        pt = vanka.patches_single_seed(K, fld, d)
    rng = np.random.default_rng(0)
    dense_entries = block_entries = 0
    for dofs, ns in zip(pt.dofs, pt.n_seed):
        Ki = K[dofs][:, dofs].toarray()
        nv = dofs.size - ns
        sizes = np.bincount(fld[dofs[:nv]], minlength=d)
        b = rng.standard_normal(dofs.size)
        x = block_apply(Ki, nv, sizes, b)
        ref = np.linalg.solve(Ki, b)
        assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)
        dense_entries += dofs.size ** 2
        block_entries += int((sizes ** 2).sum()) + 2 * nv * ns + ns * ns
    ratio = dense_entries / block_entries
    # Section 3.3.1: the block form saves up to 2x (2D) and 3x (3D) storage
    assert 1.0 < ratio <= d


# --------------------------------------------------------------------------
# additive Vanka

def test_partition_of_unity():
    P = make_problem(dim=2, n=8, jitter=0.2, seed=3, forcing="gaussian", bc="zero")
    f = np.nonzero(~P.dir0)[0]
    K = submatrix(P.K0, f, f)
    pt = vanka.patches_single_seed(K, P.field0[f], 2)
    s = np.zeros(f.size)
    for dofs in pt.dofs:
        s[dofs] += pt.weight[dofs]
    assert np.allclose(s, 1.0, rtol=0, atol=1e-15)


def test_single_patch_vanka_is_exact():
    """One patch holding every DoF, W = 1: one sweep with omega = 1 is a direct solve."""
    rng = np.random.default_rng(4)
    nv = 9
    G = rng.standard_normal((nv, nv))
    A = G @ G.T + nv * np.eye(nv)
    bt = rng.standard_normal((1, nv))
    K = sp.csr_matrix(np.block([[A, bt.T], [bt, np.zeros((1, 1))]]))
    fld = np.array([0] * 5 + [1] * 4 + [2], dtype=np.int8)
    pt = vanka.patches_single_seed(K, fld, 2)
    assert len(pt.dofs) == 1 and np.all(pt.weight == 1.0)
    b = rng.standard_normal(nv + 1)
    x = vanka.sweep(K, pt, b, np.zeros(nv + 1), 1.0)
    assert np.linalg.norm(K @ x - b) <= 1e-12 * np.linalg.norm(b)


# --------------------------------------------------------------------------
# FGMRES-wrapped relaxation (Section 3.3.1)

def small_saddle(seed, nv=9):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((nv, nv))
    A = G @ G.T + nv * np.eye(nv)
    bt = rng.standard_normal((1, nv))
    return rng, sp.csr_matrix(np.block([[A, bt.T], [bt, np.zeros((1, 1))]]))


def test_wrapped_relaxation_exact_with_one_patch():
    """With a single patch the preconditioner is K^-1: one iteration solves."""
    rng, K = small_saddle(7)
    fld = np.array([0] * 5 + [1] * 4 + [2], dtype=np.int8)
    pt = vanka.patches_single_seed(K, fld, 2)
    b = rng.standard_normal(10)
    x0 = rng.standard_normal(10)
    x = vanka.krylov_relax(K, pt, b, x0, 1)
    assert np.linalg.norm(K @ x - b) <= 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("its", [1, 2, 3])
def test_wrapped_relaxation_beats_every_damping(its):
    """FGMRES minimises the residual over a space holding omega M r for every
    omega, so its residual is at most that of the best damped sweep (scanned
    here), and the first iteration equals the best damping exactly."""
    P = make_problem(dim=2, n=6, jitter=0.2, seed=3, forcing="gaussian", bc="lid")
    pre = dc.DCPreconditioner(P, dc.default_params(P, max_coarse=30))
    K, pt = pre.K0, pre.relax[0]
    rng = np.random.default_rng(1)
    b = rng.standard_normal(K.shape[0])
    x0 = 0.1 * rng.standard_normal(K.shape[0])
    x = vanka.krylov_relax(K, pt, b, x0, its)
    res = np.linalg.norm(b - K @ x)
    r0 = b - K @ x0
    d = vanka.sweep(K, pt, r0, np.zeros_like(x0), 1.0)
    Kd = K @ d
    best = min(np.linalg.norm(r0 - w * Kd) for w in np.linspace(0.0, 2.0, 2001))
    assert res <= best * (1 + 1e-12)
    if its == 1:  # one iteration: the residual-minimising damping in closed form
        w_opt = (Kd @ r0) / (Kd @ Kd)
        assert np.linalg.norm(x - (x0 + w_opt * d)) <= 1e-10 * np.linalg.norm(x)


def test_wrapped_relaxation_zero_residual_and_scaling():
    """A zero residual leaves x unchanged (exactly when it is exactly zero);
    scaling b and x scales the result."""
    P = make_problem(dim=2, n=4, seed=2, forcing="gaussian", bc="zero")
    pre = dc.DCPreconditioner(P, dc.default_params(P, max_coarse=30))
    K, pt = pre.K0, pre.relax[0]
    rng = np.random.default_rng(2)
    x0 = rng.standard_normal(K.shape[0])
    assert np.array_equal(vanka.krylov_relax(K, pt, np.zeros_like(x0), np.zeros_like(x0), 2), np.zeros_like(x0))
    assert np.linalg.norm(vanka.krylov_relax(K, pt, K @ x0, x0, 2) - x0) <= 1e-13 * np.linalg.norm(x0)
    b = rng.standard_normal(K.shape[0])
    x1 = vanka.krylov_relax(K, pt, b, x0, 2)
    x2 = vanka.krylov_relax(K, pt, 3.0 * b, 3.0 * x0, 2)
    assert np.linalg.norm(x2 - 3.0 * x1) <= 1e-12 * np.linalg.norm(x2)


def test_wrapped_cycle_converges_and_sv_keeps_stationary_k0():
    for kw in (dict(dim=2, n=8, jitter=0.2, seed=5, forcing="gaussian", bc="lid"),
               dict(dim=2, n=4, disc="SV", seed=4, forcing="gaussian", bc="zero")):
        P = make_problem(**kw)
        par = dc.default_params(P, max_coarse=30, krylov_its=2)
        pre = dc.DCPreconditioner(P, par)
        out = fgmres.solve(P, pre, rtol=1e-10)
        assert out.converged
        assert np.linalg.norm(P.b - P.K0 @ out.x) <= 1e-10 * np.linalg.norm(P.b)
        if P.disc == "SV":  # K0 relaxation is the damped sweep: linear in r there
            r = np.random.default_rng(0).standard_normal(P.n0)
            b = r[pre.free0]
            a = pre._relax(0, pre.K0, b, np.zeros_like(b), 1, par.omega0)
            c = pre._relax(0, pre.K0, 2.0 * b, np.zeros_like(b), 1, par.omega0)
            assert np.linalg.norm(c - 2.0 * a) <= 1e-12 * np.linalg.norm(c)


# --------------------------------------------------------------------------
# Chebyshev and DLSC (Algorithm 2, Table 2)

def cheb_T(k, x):
    return np.cos(k * np.arccos(x)) if abs(x) <= 1 else np.cosh(k * np.arccosh(abs(x))) * (np.sign(x) ** k)


@pytest.mark.parametrize("k", [1, 2, 3, 6, 16])
def test_chebyshev_residual_polynomial(k):
    lam = np.linspace(0.3, 2.0, 40)
    lo, hi = 0.25, 2.2
    r = np.ones_like(lam)
    y = dlsc.chebyshev(lambda v: lam * v, r, lo, hi, k)
    res = 1.0 - lam * y  # residual factor per eigenvalue
    ref = np.array([cheb_T(k, (hi + lo - 2 * t) / (hi - lo)) for t in lam]) / cheb_T(k, (hi + lo) / (hi - lo))
    assert np.abs(res - ref).max() <= 1e-13


def _rand_saddle(rng, nv, npr):
    G = rng.standard_normal((nv, nv))
    A = G @ G.T / nv + np.eye(nv)
    B = rng.standard_normal((npr, nv))
    return A, B


def test_dlsc_exact_when_commutator_exact():
    """A = M_u (diagonal) and exact inner solves: one DLSC sweep solves K x = b."""
    rng = np.random.default_rng(5)
    nv, npr = 12, 5
    m = rng.uniform(0.5, 2.0, nv)
    A = np.diag(m)
    B = rng.standard_normal((npr, nv))
    K = np.block([[A, B.T], [B, np.zeros((npr, npr))]])
    lv = dlsc.DLSCLevel(sp.csr_matrix(K), np.array([0] * nv + [2] * npr), 2, m, (1, 1, 1), 1)
    # replace the polynomial inner solves by exact ones
    orig = dlsc.chebyshev
    try:
        def exact(matvec, r, lo, hi, deg):
            n = r.size
            X = np.column_stack([matvec(e) for e in np.eye(n)])
            return np.linalg.solve(X, r)
        dlsc.chebyshev = exact
        b = rng.standard_normal(nv + npr)
        x = lv.relax(b, np.zeros(nv + npr), 1)
    finally:
        dlsc.chebyshev = orig
    assert np.linalg.norm(K @ x - b) <= 1e-10 * np.linalg.norm(b)


def test_dlsc_sweep_matches_dense_formula():
    """One sweep from zero equals [I, M^-1 B^T; 0, -Ahat_p] [A 0; B S]^-1 r with
    every inverse replaced by its Chebyshev polynomial (dense eigen-decomposition)."""
    rng = np.random.default_rng(6)
    nv, npr = 14, 6
    A, B = _rand_saddle(rng, nv, npr)
    m = rng.uniform(0.5, 2.0, nv)
    K = np.block([[A, B.T], [B, np.zeros((npr, npr))]])
    deg = (3, 3, 6)
    lv = dlsc.DLSCLevel(sp.csr_matrix(K), np.array([0] * nv + [2] * npr), 2, m, deg, 3)
    Mi = np.diag(1 / m)
    S = B @ Mi @ B.T

    def poly_inv(X, lam, k):
        w, V = np.linalg.eigh(X)
        lo, hi = 0.25 * lam, 1.1 * lam
        R = np.array([cheb_T(k, (hi + lo - 2 * t) / (hi - lo)) for t in w]) / cheb_T(k, (hi + lo) / (hi - lo))
        return V @ np.diag((1 - R) / w) @ V.T

    QA = poly_inv(A, lv.lam_A, deg[0])
    QS1 = poly_inv(S, lv.lam_S, deg[1])
    QS2 = poly_inv(S, lv.lam_S, deg[2])
    b = rng.standard_normal(nv + npr)
    f, g = b[:nv], b[nv:]
    vs = QA @ f
    q = QS1 @ (g - B @ vs)
    ref = np.concatenate([vs + Mi @ B.T @ q, -QS2 @ (B @ Mi @ A @ Mi @ B.T @ q)])
    x = lv.relax(b, np.zeros(nv + npr), 1)
    assert np.linalg.norm(x - ref) <= 1e-11 * np.linalg.norm(ref)


def test_lanczos_estimate_close_to_top_eigenvalue():
    rng = np.random.default_rng(7)
    G = rng.standard_normal((60, 60))
    X = G @ G.T
    lam = dlsc.lanczos_max(lambda v: X @ v, 60, 11)
    top = np.linalg.eigvalsh(X)[-1]
    assert lam <= top * (1 + 1e-12) and lam >= 0.9 * top


def test_splitmix64_reference_values():
    """First outputs of SplitMix64 seeded with 0 (Vigna's reference generator)."""
    from oracle.sparse import splitmix64
    z = splitmix64(np.arange(3, dtype=np.uint64), 0)
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    u = uniform_pm1(1000, 5)
    assert u.min() >= -1.0 and u.max() < 1.0 and abs(u.mean()) < 0.1


# --------------------------------------------------------------------------
# smoothed aggregation (Algorithm 1)

def test_sa_invariants():
    P = make_problem(dim=2, n=12, jitter=0.2, seed=9, forcing="gaussian", bc="zero")
    f1 = np.nonzero(~P.dir1)[0]
    K1 = submatrix(P.K1, f1, f1)
    levels = sa.stokes_hierarchy(K1, P.field1[f1], P.Ap, 2, max_coarse=20)
    assert len(levels) >= 3
    for l, lv in enumerate(levels):
        K = lv.K
        assert abs(K - K.T).max() <= 1e-13 * abs(K).max()
        z = np.zeros(K.shape[0])
        z[lv.field == 2] = lv.null_p
        assert np.linalg.norm(K @ z) <= 1e-12 * abs(K).max() * np.linalg.norm(z)
        # zero pressure-pressure block
        pp = lv.field == 2
        assert abs(submatrix(K, np.nonzero(pp)[0], np.nonzero(pp)[0])).max() == 0.0
        if lv.P is not None:
            # interpolating the coarse pressure null vector gives the fine one
            zc = np.zeros(lv.P.shape[1])
            zc[levels[l + 1].field == 2] = levels[l + 1].null_p
            assert np.allclose((lv.P @ zc)[pp], lv.null_p, rtol=1e-13, atol=0)
            # block-diagonal interpolation: fields never mix
            C = lv.P.tocoo()
            assert np.all(lv.field[C.row] == levels[l + 1].field[C.col])
    # the velocity-to-pressure ratio stays of the same order (Section 3.2)
    ratios = [np.sum(lv.field == 0) / np.sum(lv.field == 2) for lv in levels]
    assert max(ratios) / min(ratios) < 3.0


def test_structural_product_keeps_cancelled_entries():
    A = sp.csr_matrix(np.array([[1.0, 1.0], [0.0, 1.0]]))
    B = sp.csr_matrix(np.array([[1.0], [-1.0]]))
    C = pattern_product(A, B)
    assert C.nnz == 2 and C.toarray()[0, 0] == 0.0
    G = galerkin(sp.csr_matrix(np.array([[1.0], [1.0]])), sp.csr_matrix(np.array([[1.0, -1.0], [-1.0, 1.0]])))
    assert G.nnz == 1 and G.toarray()[0, 0] == 0.0


def test_aggregation_small_graph():
    # path graph 0-1-2-3-4-5, every link strong
    n = 6
    rows = [i for i in range(n - 1)] + [i + 1 for i in range(n - 1)]
    cols = [i + 1 for i in range(n - 1)] + [i for i in range(n - 1)]
    S = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(n, n))
    agg = sa.aggregate(S)
    # pass 1: node 0 seeds {0,1}; node 2 sees 1 taken and waits; node 3 seeds {2,3,4};
    # node 5 sees 4 taken and waits.  Pass 2: node 5 joins the aggregate of node 4.
    assert list(agg) == [0, 0, 1, 1, 1, 1]


# --------------------------------------------------------------------------
# the defect-correction cycle and FGMRES

def _dense_vanka(K, pt):
    n = K.shape[0]
    M = np.zeros((n, n))
    for dofs in pt.dofs:
        Ki = K[dofs][:, dofs].toarray()
        M[np.ix_(dofs, dofs)] += np.diag(pt.weight[dofs]) @ np.linalg.inv(Ki)
    return M


def test_two_level_cycle_equals_dense_formula():
    """With the K1 hierarchy reduced to one exactly solved level (gamma = inf in
    eq. (3.1)), apply(r) = x3 where x1 = w M0^-1 r, x2 = x1 + P0 K1^+ eta R0 (r - K0 x1),
    x3 = x2 + w M0^-1 (r - K0 x2), written with dense matrices."""
    P = make_problem(dim=2, n=4, jitter=0.2, seed=2, forcing="gaussian", bc="lid")
    par = dc.default_params(P, max_coarse=10 ** 6, eta_u=0.8, eta_p=0.9)
    pre = dc.DCPreconditioner(P, par)
    assert len(pre.levels) == 1
    K0 = pre.K0.toarray()
    M0 = _dense_vanka(pre.K0, pre.relax[0])
    K1 = pre.levels[0].K.toarray()
    n1 = K1.shape[0]
    nv = pre.nvel
    eta = np.diag(np.r_[np.full(nv, 0.8), np.full(n1 - nv, 0.9)])
    K1p = np.linalg.pinv(K1)  # consistent right-hand sides: pseudo-inverse = bordered solve
    r = np.random.default_rng(3).standard_normal(P.n0)
    rf = r[pre.free0]
    w = par.omega0
    x1 = w * M0 @ rf
    x2 = x1 + K1p @ (eta @ (rf - K0 @ x1))
    x3 = x2 + w * M0 @ (rf - K0 @ x2)
    z = pre.apply(r)
    # the bordered solve and the pseudo-inverse differ by a constant pressure
    d = z[pre.free0] - x3
    d[nv:] -= d[nv:].mean()
    assert np.linalg.norm(d) <= 1e-9 * np.linalg.norm(x3)
    assert np.all(z[pre.dir0] == r[pre.dir0])


def test_ho_amg_one_level_is_the_exact_solve_of_k0():
    """HO-AMG (Algorithm 1 applied to K0): with the coarsening limit above the
    problem size the hierarchy is K0 alone, solved exactly (bordered with the
    constant pressure), so K0 z = r up to a constant in the pressure rows, the
    null vector of the enclosed-flow K0.  Built from K1 it would solve K1."""
    P = make_problem(dim=2, n=4, jitter=0.2, seed=2, forcing="gaussian", bc="lid")
    pre = dc.DCPreconditioner(P, dc.default_params(P, schedule="ho", max_coarse=10 ** 6))
    assert len(pre.levels) == 1 and not pre.relax_on[0]
    r = np.random.default_rng(4).standard_normal(P.n0)
    z = pre.apply(r)
    f = pre.free0
    nv = pre.nvel

    def off_null(v):
        v = v.copy()
        v[nv:] -= v[nv:].mean()
        return v

    assert np.linalg.norm(off_null(r[f] - pre.K0 @ z[f])) <= 1e-10 * np.linalg.norm(r)
    K1f = P.K1.tocsr()[f][:, f]
    assert np.linalg.norm(off_null(r[f] - K1f @ z[f])) > 1e-3 * np.linalg.norm(r)  # K1 is another operator


@pytest.mark.parametrize("relax_its", [0, 2])
def test_ho_amg_two_level_cycle_equals_dense_formula(relax_its):
    """Two-level HO-AMG with Vanka, written with dense matrices: x1 = w M r,
    x2 = x1 + P Kc^+ P^T (r - K0 x1) with Kc = P^T K0 P, x3 = x2 + w M (r - K0 x2).
    No eta weights and no extra relaxation on a defect-correction level.  With
    the wrapped relaxation (relax_its = 2) only the coarse-correction identity
    P^T (r - K0 x2) in span{Kc's null vector} is checked."""
    P = make_problem(dim=2, n=4, jitter=0.2, seed=2, forcing="gaussian", bc="lid")
    par = dc.default_params(P, schedule="ho", max_coarse=5, max_levels=2, eta_u=0.3, eta_p=3.0,
                            krylov_its=relax_its, nu2=1 if relax_its == 0 else 0)
    pre = dc.DCPreconditioner(P, par)
    assert len(pre.levels) == 2
    K0 = pre.K0.toarray()
    assert (pre.levels[0].K != pre.K0).nnz == 0
    Pm = pre.levels[0].P.toarray()
    Kc = Pm.T @ K0 @ Pm
    r = np.random.default_rng(3).standard_normal(P.n0)
    rf = r[pre.free0]
    nv = pre.nvel
    z = pre.apply(r)[pre.free0]
    if relax_its == 0:
        M = _dense_vanka(pre.K0, pre.relax[1])
        w = par.omega
        x1 = w * M @ rf
        x2 = x1 + Pm @ (np.linalg.pinv(Kc) @ (Pm.T @ (rf - K0 @ x1)))
        x3 = x2 + w * M @ (rf - K0 @ x2)
        d = z - x3
        d[nv:] -= d[nv:].mean()  # bordered solve vs pseudo-inverse: a constant pressure
        assert np.linalg.norm(d) <= 1e-9 * np.linalg.norm(x3)
    else:
        g = Pm.T @ (rf - K0 @ z)  # no post-relaxation: z is the coarse-corrected iterate
        nc = np.zeros(Kc.shape[0])
        nc[pre.levels[1].field == P.dim] = pre.levels[1].null_p
        nc /= np.linalg.norm(nc)
        assert np.linalg.norm(g - (nc @ g) * nc) <= 1e-10 * np.linalg.norm(rf)


def test_ho_amg_is_a_working_preconditioner_and_refuses_sv():
    """The remark after Algorithm 1: HO-AMG is a usable preconditioner for
    Taylor-Hood; it is not defined here for the discontinuous SV pressure."""
    P = make_problem(dim=2, n=8, jitter=0.2, seed=2, forcing="gaussian", bc="lid")
    for relax in ("vanka", "dlsc"):
        pre = dc.DCPreconditioner(P, dc.default_params(P, relax=relax, schedule="ho", max_coarse=20))
        res = fgmres.solve(P, pre, rtol=1e-10, max_it=200)
        assert res.converged and res.iters <= 40, (relax, res.iters)
        ref = bordered_direct(P)
        assert np.linalg.norm(res.x - ref) <= 1e-7 * np.linalg.norm(ref)
    S = make_problem(dim=2, n=4, disc="SV", seed=4, forcing="gaussian", bc="zero")
    with pytest.raises(ValueError):
        dc.DCPreconditioner(S, dc.default_params(S, schedule="ho"))


def _dense_sweep_map(level, n):
    """D with x_new = x + D (b - K x) for one DLSC sweep, read off the sweep
    from x = 0 (a DLSC sweep is affine in b and x: each stage is a fixed
    polynomial in its operator applied to a residual)."""
    D = np.zeros((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        D[:, i] = level.relax(e, np.zeros(n), 1)
    return D


@pytest.mark.parametrize("kw", [dict(dim=2, n=4, disc="SV", seed=4, forcing="gaussian", bc="zero"),
                                dict(dim=2, n=6, jitter=0.2, seed=2, forcing="gaussian", bc="lid")])
def test_vanka_dlsc_hybrid_is_vanka_on_k0_and_dlsc_below(kw):
    """The Vanka-DLSC hybrid (Section 4, Table 4): with the K1 hierarchy cut to
    K1 and one exactly solved coarse level, apply(r) = x3 with
    x1 = w0 M0 r, x2 = x1 + P0 y(eta R0 (r - K0 x1)), x3 = x2 + w0 M0 (r - K0 x2),
    where y(b1) runs nu_dlsc = 2 DLSC sweeps on K1 from zero, the Galerkin
    coarse correction, and 2 more DLSC sweeps (dense matrices throughout)."""
    P = make_problem(**kw)
    par = dc.default_params(P, relax="vanka-dlsc", max_coarse=5, max_levels=2)
    if P.disc == "SV":
        assert (par.omega0, par.eta_u, par.eta_p) == (0.87, 1.0, 2.96)  # Table 4, structured
    pre = dc.DCPreconditioner(P, par)
    assert len(pre.levels) == 2
    assert isinstance(pre.relax[0], vanka.Patches) and isinstance(pre.relax[1], dlsc.DLSCLevel)
    K0 = pre.K0.toarray()
    K1 = pre.levels[0].K.toarray()
    n1 = K1.shape[0]
    Pm = pre.levels[0].P.toarray()
    Kc = Pm.T @ K1 @ Pm
    D = _dense_sweep_map(pre.relax[1], n1)
    M0 = _dense_vanka(pre.K0, pre.relax[0])
    r = np.random.default_rng(5).standard_normal(P.n0)
    rf = r[pre.free0]
    w = par.omega0

    def y_of(b1):
        y = np.zeros(n1)
        for _ in range(2):
            y = y + D @ (b1 - K1 @ y)
        y = y + Pm @ (np.linalg.pinv(Kc) @ (Pm.T @ (b1 - K1 @ y)))
        for _ in range(2):
            y = y + D @ (b1 - K1 @ y)
        return y

    x1 = w * M0 @ rf
    x2 = x1 + pre.prolong0(y_of(pre.restrict0(rf - K0 @ x1)))
    x3 = x2 + w * M0 @ (rf - K0 @ x2)
    d = pre.apply(r)[pre.free0] - x3
    nv = pre.nvel
    d[nv:] -= d[nv:].mean()  # bordered coarse solve vs pseudo-inverse: a constant pressure
    assert np.linalg.norm(d) <= 1e-9 * np.linalg.norm(x3)


@pytest.mark.parametrize("kw", [dict(dim=2, n=6, disc="SV", seed=4, forcing="gaussian", bc="zero"),
                                dict(dim=2, n=8, jitter=0.2, seed=2, forcing="gaussian", bc="lid"),
                                dict(dim=3, n=3, seed=3, forcing="smooth", bc="zero")])
def test_vanka_dlsc_hybrid_solves(kw):
    P = make_problem(**kw)
    pre = dc.DCPreconditioner(P, dc.default_params(P, relax="vanka-dlsc", max_coarse=20))
    res = fgmres.solve(P, pre, rtol=1e-11, max_it=400)
    assert res.converged
    ref = bordered_direct(P)
    assert np.linalg.norm(res.x - ref) <= 1e-7 * np.linalg.norm(ref)


def _poisson2d(m, neumann=False):
    """5-point Laplacian on an m x m grid (Dirichlet: diagonal 4; Neumann: the
    graph Laplacian, singular with the constants as null space)."""
    T = sp.diags([-np.ones(m - 1), 2 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1])
    if neumann:
        T = T.tolil()
        T[0, 0] = T[m - 1, m - 1] = 1.0
    I = sp.identity(m)
    return sp.csr_matrix(sp.kron(T, I) + sp.kron(I, T))


def test_sa_vcycle_jacobi_weight_closed_form_and_two_level_formula():
    """SA V-cycle with weighted Jacobi (the DLSC AMG stages, Section 4).  On the
    Dirichlet 5-point Laplacian every row has s_ii = 4 and the largest absolute
    row sum is 8, so the weight is (4/3)/2 and w D^-1 = 1/6 on every row.  The
    two-level cycle equals x1 = 2 Jacobi sweeps from 0, x2 = x1 + P Sc^-1 P^T (b - S x1),
    x3 = 2 Jacobi sweeps from x2, with Sc = P^T S P (dense)."""
    S = _poisson2d(12)
    v = dlsc.SAVcycle(S, 0.02, 20, 2, 2, False)
    assert len(v.ops) == 2
    assert np.allclose(v.wdinv[0], 1.0 / 6.0, rtol=0, atol=1e-15)
    Sd = S.toarray()
    P = v.Ps[0].toarray()
    Sc = P.T @ Sd @ P
    b = np.random.default_rng(0).standard_normal(S.shape[0])
    x = np.zeros_like(b)
    for _ in range(2):
        x = x + (b - Sd @ x) / 6.0
    x = x + P @ np.linalg.solve(Sc, P.T @ (b - Sd @ x))
    for _ in range(2):
        x = x + (b - Sd @ x) / 6.0
    assert np.linalg.norm(v.apply(b) - x) <= 1e-12 * np.linalg.norm(x)


def test_sa_vcycle_one_level_exact_symmetric_and_convergent():
    # one level: the bordered exact solve of the singular Neumann Laplacian
    S = _poisson2d(8, neumann=True)
    n = S.shape[0]
    b = np.random.default_rng(1).standard_normal(n)
    b -= b.mean()  # consistent right-hand side
    v1 = dlsc.SAVcycle(S, 0.02, 10 ** 6, 10, 2, True)
    assert len(v1.ops) == 1
    y = v1.apply(b)
    assert np.linalg.norm(S @ y - b) <= 1e-10 * np.linalg.norm(b) and abs(y.sum()) <= 1e-10
    # several levels: the cycle is a symmetric operator and a convergent iteration on range(S)
    S = _poisson2d(16, neumann=True)
    n = S.shape[0]
    v = dlsc.SAVcycle(S, 0.02, 10, 10, 2, True)
    assert len(v.ops) >= 3
    V = np.column_stack([v.apply(e) for e in np.eye(n)])
    assert np.linalg.norm(V - V.T) <= 1e-10 * np.linalg.norm(V)
    Q = np.eye(n) - np.ones((n, n)) / n  # projector onto range(S)
    E = Q @ (np.eye(n) - V @ S.toarray()) @ Q
    # ~0.55 here; four Jacobi sweeps without the coarse correction would give ~0.99
    assert np.max(np.abs(np.linalg.eigvals(E))) < 0.8


@pytest.mark.parametrize("kw", [dict(dim=2, n=8, jitter=0.2, seed=2, forcing="gaussian", bc="lid"),
                                dict(dim=3, n=3, seed=3, forcing="smooth", bc="zero"),
                                dict(dim=2, n=6, disc="SV", seed=4, forcing="gaussian", bc="zero")])
def test_dlsc_with_amg_stages_solves(kw):
    P = make_problem(**kw)
    relax = "vanka-dlsc" if P.disc == "SV" else "dlsc"
    pre = dc.DCPreconditioner(P, dc.default_params(P, relax=relax, max_coarse=20, dlsc_amg=2))
    assert all(R.svc is not None for R in pre.relax if isinstance(R, dlsc.DLSCLevel))
    res = fgmres.solve(P, pre, rtol=1e-11, max_it=400)
    assert res.converged
    ref = bordered_direct(P)
    assert np.linalg.norm(res.x - ref) <= 1e-7 * np.linalg.norm(ref)


def test_apply_is_linear():
    P = make_problem(dim=2, n=8, jitter=0.2, seed=2, forcing="gaussian", bc="lid")
    pre = dc.DCPreconditioner(P, dc.default_params(P, max_coarse=20))
    rng = np.random.default_rng(1)
    r, s = rng.standard_normal(P.n0), rng.standard_normal(P.n0)
    lhs = pre.apply(2.0 * r - 0.5 * s)
    rhs = 2.0 * pre.apply(r) - 0.5 * pre.apply(s)
    assert np.linalg.norm(lhs - rhs) <= 1e-12 * np.linalg.norm(rhs)


@pytest.mark.parametrize("kw,relax,nu", [
    (dict(dim=2, n=8, jitter=0.2, seed=2, bc="lid"), "vanka", 0.05),
    (dict(dim=2, n=8, jitter=0.2, seed=2, bc="lid"), "dlsc", 0.05),
    (dict(dim=2, n=8, jitter=0.2, seed=2, bc="lid"), "vanka-dlsc", 20.0),
    (dict(dim=2, n=6, disc="SV", seed=4, bc="zero"), "vanka", 0.05),
    (dict(dim=3, n=3, seed=3, bc="lid"), "vanka", 20.0),
])
def test_viscosity_scaling_of_the_preconditioner(kw, relax, nu):
    """K_nu = S K_1 S on the free block, S = diag(sqrt(nu) I_u, I_p / sqrt(nu)):
    every piece of the cycle (Galerkin products, strength of connection,
    Gershgorin and Chebyshev bounds, patch solves, the bordered coarse solve)
    is built from the nu = 1 one by the same diagonal scaling, so the whole
    preconditioner satisfies B_nu = S^-1 B_1 S^-1.  Dirichlet rows are identity
    rows in both operators and pass through unchanged."""
    P1 = make_problem(nu=1.0, forcing="gaussian", **kw)
    Pn = make_problem(nu=nu, forcing="gaussian", **kw)
    B1 = dc.DCPreconditioner(P1, dc.default_params(P1, relax, max_coarse=20))
    Bn = dc.DCPreconditioner(Pn, dc.default_params(Pn, relax, max_coarse=20))
    n_u = P1.meta["n_u"]
    s = np.r_[np.full(n_u, np.sqrt(nu)), np.full(P1.n0 - n_u, 1.0 / np.sqrt(nu))]
    s[P1.dir0] = 1.0
    r = np.random.default_rng(1).standard_normal(P1.n0)
    zn = Bn.apply(r)
    assert np.linalg.norm(zn - B1.apply(r / s) / s) <= 1e-13 * np.linalg.norm(zn)
    assert np.array_equal(zn[P1.dir0], r[P1.dir0])


def test_skip0_iterations_invariant_to_eta():
    """Section 4.1: with no relaxation on K0, eta only scales the preconditioner."""
    P = make_problem(dim=2, n=8, jitter=0.2, seed=2, forcing="gaussian", bc="lid")
    its = []
    for eta in (0.5, 1.0, 1.7):
        pre = dc.DCPreconditioner(P, dc.default_params(P, schedule="skip0", eta_u=eta, eta_p=eta, max_coarse=20))
        its.append(fgmres.solve(P, pre, rtol=1e-8).iters)
    assert its[0] == its[1] == its[2]


def test_gmres_is_krylov_least_squares():
    """FGMRES with the identity preconditioner, no restart: the k-th iterate
    minimises ||b - K x|| over span{b, Kb, ..., K^{k-1} b}."""
    rng = np.random.default_rng(8)
    n = 30
    K = rng.standard_normal((n, n)) + 6 * np.eye(n)
    b = rng.standard_normal(n)
    for k in (3, 7, 12):
        res = fgmres.fgmres(lambda v: K @ v, lambda v: v, b, rtol=0.0, restart=50, max_it=k)
        Kr = np.column_stack([np.linalg.matrix_power(K, j) @ b for j in range(k)])
        Q, _ = np.linalg.qr(Kr)
        y, *_ = np.linalg.lstsq(K @ Q, b, rcond=None)
        assert np.linalg.norm(res.x - Q @ y) <= 1e-9 * np.linalg.norm(Q @ y)
        assert res.iters == k


@pytest.mark.parametrize("kw,relax", [
    (dict(dim=2, n=8, jitter=0.2, seed=2, forcing="gaussian", bc="lid"), "vanka"),
    (dict(dim=2, n=8, jitter=0.2, seed=2, forcing="gaussian", bc="lid"), "dlsc"),
    (dict(dim=2, n=6, disc="SV", seed=4, forcing="gaussian", bc="zero"), "vanka"),
    (dict(dim=3, n=3, seed=3, forcing="smooth", bc="zero"), "vanka"),
    (dict(dim=3, n=3, seed=3, forcing="smooth", bc="zero"), "dlsc"),
])
def test_fgmres_solution_matches_sparse_direct(kw, relax):
    P = make_problem(**kw)
    pre = dc.DCPreconditioner(P, dc.default_params(P, relax=relax, max_coarse=20))
    res = fgmres.solve(P, pre, rtol=1e-11, max_it=400)
    assert res.converged
    ref = bordered_direct(P)
    assert np.linalg.norm(res.x - ref) <= 1e-7 * np.linalg.norm(ref)
    nu = P.meta["n_u"]
    assert abs(P.p_weight0 @ res.x[nu:]) <= 1e-13 * np.abs(res.x).max()


def test_manufactured_solve_th2d_16():
    """16x16 Taylor-Hood, u = (y^2, x^2), p = x - y: the solve returns the interpolant."""
    P = make_problem(dim=2, n=16)
    pre = dc.DCPreconditioner(P, dc.default_params(P))
    res = fgmres.solve(P, pre, rtol=1e-12)
    assert res.converged
    assert np.linalg.norm(res.x - P.x_exact) <= 1e-9 * np.linalg.norm(P.x_exact)
