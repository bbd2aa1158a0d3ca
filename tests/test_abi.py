"""The C-ABI library on the CPU: it loads, exports every function include/mas.h
declares, its ctypes structures match the C layout, and its host-only analysis
(Algorithm 1 hierarchy, patches) agrees with the oracle's."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

from paper_2306_06795_amd import mas
from paper_2306_06795_amd.inputs import make_problem
from oracle import dc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mas.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mas_[a-z_]+)\s*\(", src)))


def test_every_declared_function_is_exported():
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(mas.lib, n), n
    assert set(names) == set(mas.EXPORTED)


def test_struct_layout_matches_c():
    prog = r'''
#include <stdio.h>
#include <stddef.h>
#include "mas.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\n", sizeof(mas_csr), sizeof(mas_problem), sizeof(mas_params),
         sizeof(mas_solve_info), sizeof(mas_hier_info));
  printf("%zu %zu %zu %zu %zu %zu\n", offsetof(mas_problem, p_nullspace), offsetof(mas_problem, Mcg),
         offsetof(mas_params, cheb_deg), offsetof(mas_params, mass_rtol), offsetof(mas_params, soc_eps),
         offsetof(mas_params, device_galerkin));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(prog)
        exe = os.path.join(d, "t")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.check_output([exe], text=True).split()
    sizes = [int(v) for v in out]
    assert sizes[:5] == [C.sizeof(mas.mas_csr), C.sizeof(mas.mas_problem), C.sizeof(mas.mas_params),
                         C.sizeof(mas.mas_solve_info), C.sizeof(mas.mas_hier_info)]
    assert sizes[5:] == [mas.mas_problem.p_nullspace.offset, mas.mas_problem.Mcg.offset,
                         mas.mas_params.cheb_deg.offset, mas.mas_params.mass_rtol.offset,
                         mas.mas_params.soc_eps.offset, mas.mas_params.device_galerkin.offset]


def test_default_params_follow_the_paper():
    p = mas.default_params(2, mas.MAS_SV)
    assert (p.omega0, p.eta_p, p.eta_u, p.restart) == (0.78, 2.68, 1.0, 20)
    # the setup of mas_setup runs on the device by default (the same hierarchy as mas_analyze)
    assert (p.device_sa, p.device_galerkin, p.spgemm_cap) == (1, 1, 0)
    p3 = mas.default_params(3, mas.MAS_TH, mas.MAS_RELAX_DLSC)
    assert list(p3.cheb_deg) == [4, 4, 16] and p3.nu1 == 2
    ph = mas.default_params(2, mas.MAS_SV, mas.MAS_RELAX_VANKA_DLSC)  # Table 4, Vanka-DLSC row
    assert (ph.omega0, ph.eta_p, ph.eta_u, ph.nu1, ph.nu_dlsc) == (0.87, 2.96, 1.0, 1, 2)
    # evolution strength (Section 3.2) for Taylor-Hood; SV keeps the symmetric measure
    assert mas.default_params(3).soc == mas.MAS_SOC_EVOLUTION and mas.default_params(2).soc_eps == 4.0
    assert p.soc == ph.soc == mas.MAS_SOC_SYMMETRIC
    for prob in (make_problem(dim=2, n=4), make_problem(dim=2, n=2, disc="SV", seed=1)):
        par = dc.default_params(prob)
        assert SOC[par.soc] == mas.default_params(2, mas.MAS_SV if prob.disc == "SV" else mas.MAS_TH).soc


SCHED = {"all": mas.MAS_DC_ALL, "ho": mas.MAS_HO_AMG}
SOC = {"evolution": mas.MAS_SOC_EVOLUTION, "symmetric": mas.MAS_SOC_SYMMETRIC}


def _same_params(prob, **over):
    par = dc.default_params(prob, **over)
    mp = mas.default_params(prob.dim, mas.MAS_SV if prob.disc == "SV" else mas.MAS_TH, theta=par.theta,
                            max_coarse=par.max_coarse, max_levels=par.max_levels, schedule=SCHED[par.schedule],
                            soc=SOC[par.soc])
    return par, mp


@pytest.mark.parametrize("kw,mc,sched,soc", [
    (dict(dim=2, n=16), 300, "all", "evolution"),
    (dict(dim=2, n=16), 30, "all", "evolution"),
    (dict(dim=2, n=24, jitter=0.2, seed=2, forcing="gaussian", bc="lid"), 40, "all", "evolution"),
    (dict(dim=2, n=24, jitter=0.2, seed=2, forcing="gaussian", bc="lid"), 40, "all", "symmetric"),
    (dict(dim=3, n=4, forcing="smooth", bc="zero", seed=3), 40, "all", "evolution"),
    (dict(dim=3, n=5, forcing="smooth", bc="zero", seed=3), 20, "all", "evolution"),
    (dict(dim=3, n=4, forcing="smooth", bc="zero", seed=3), 40, "all", "symmetric"),
    (dict(dim=2, n=12, disc="SV", seed=4, forcing="gaussian", bc="zero"), 30, "all", "evolution"),
    # HO-AMG: the hierarchy below K0 is Algorithm 1 applied to K0 itself
    (dict(dim=2, n=24, jitter=0.2, seed=2, forcing="gaussian", bc="lid"), 40, "ho", "evolution"),
    (dict(dim=3, n=4, forcing="smooth", bc="zero", seed=3), 40, "ho", "evolution"),
])
def test_host_hierarchy_matches_oracle(kw, mc, sched, soc):
    P = make_problem(**kw)
    par, mp = _same_params(P, max_coarse=mc, schedule=sched, soc=soc)
    pre = dc.DCPreconditioner(P, par)
    h = mas.Handle(P, mp, analyze_only=True)
    info = h.info()
    assert info["n_levels"] == 1 + len(pre.levels)
    levels = [pre.K0] + [lv.K for lv in pre.levels]
    for l, K in enumerate(levels):
        Kl = h.export_level(l)
        assert Kl.shape == K.shape
        assert np.array_equal(Kl.indptr, K.indptr) and np.array_equal(Kl.indices, K.indices), f"level {l} pattern"
        scale = np.abs(K.data).max()
        assert np.abs(Kl.data - K.data).max() <= 1e-13 * scale, f"level {l} values"
    # patch counts on relaxed levels (HO-AMG relaxes no defect-correction level 0)
    for l, R in enumerate(pre.relax):
        if not pre.relax_on[l]:
            assert info["n_patches"][l] == 0
            continue
        assert info["n_patches"][l] == len(R.dofs)
        assert info["patch_dofs"][l] == sum(d.size for d in R.dofs)
    h.close()


def test_analyze_rejects_bad_input():
    P = make_problem(dim=2, n=4)
    mp = mas.default_params(2)
    bad = make_problem(dim=2, n=4)
    bad.field0 = bad.field0[::-1].copy()  # not field-blocked
    with pytest.raises(mas.MasError) as e:
        mas.Handle(bad, mp, analyze_only=True)
    assert e.value.code == mas.MAS_EINVAL
    bad2 = make_problem(dim=2, n=4)
    bad2.K0 = bad2.K0.copy()
    bad2.K0.data[3] = np.nan
    with pytest.raises(mas.MasError) as e:
        mas.Handle(bad2, mp, analyze_only=True)
    assert e.value.code == mas.MAS_EINVAL and "non-finite" in str(e.value)
    sv = make_problem(dim=2, n=4, disc="SV", seed=4, forcing="gaussian", bc="zero")
    with pytest.raises(mas.MasError) as e:  # HO-AMG is defined for Taylor-Hood only
        mas.Handle(sv, mas.default_params(2, mas.MAS_SV, schedule=mas.MAS_HO_AMG), analyze_only=True)
    assert e.value.code == mas.MAS_EINVAL and "Taylor-Hood" in str(e.value)
    with pytest.raises(mas.MasError) as e:
        mas.Handle(P, mas.default_params(2, schedule=7), analyze_only=True)
    assert e.value.code == mas.MAS_EINVAL and "schedule" in str(e.value)
    with pytest.raises(mas.MasError) as e:
        mas.Handle(P, mas.default_params(2, patch_kernel=6), analyze_only=True)
    assert e.value.code == mas.MAS_EINVAL and "patch_kernel" in str(e.value)
    for bad, word in ((dict(device_sa=2), "device_sa"), (dict(spgemm_cap=-1), "spgemm_cap")):
        with pytest.raises(mas.MasError) as e:
            mas.Handle(P, mas.default_params(2, **bad), analyze_only=True)
        assert e.value.code == mas.MAS_EINVAL and word in str(e.value)
    h = mas.Handle(P, mp, analyze_only=True)
    with pytest.raises(mas.MasError):
        import torch
        t = torch.zeros(P.n0, dtype=torch.float64)
        h.apply(t, t, stream=0)
    h.close()


_THREADS_SCRIPT = r"""
import sys
import numpy as np
from paper_2306_06795_amd import mas
from paper_2306_06795_amd.inputs import make_problem
P = make_problem(dim=2, n=64, jitter=0.2, seed=2, forcing="gaussian", bc="lid")  # ~33k rows: 7 threads split
h = mas.Handle(P, mas.default_params(2, max_coarse=30), analyze_only=True)
out = {}
for l in range(h.info()["n_levels"]):
    K = h.export_level(l)
    out[f"p{l}"], out[f"i{l}"], out[f"v{l}"] = K.indptr, K.indices, K.data
np.savez(sys.argv[1], **out)
"""


def test_host_analysis_is_independent_of_the_thread_count(tmp_path):
    """The row-parallel host setup gives the same hierarchy, bit for bit, with
    one thread and with several (each run is its own process: the thread
    count is read once per process)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    res = {}
    for t in ("1", "7"):
        f = tmp_path / f"h{t}.npz"
        env = dict(os.environ, MAS_SETUP_THREADS=t, PYTHONPATH=root)
        subprocess.run([sys.executable, "-c", _THREADS_SCRIPT, str(f)], check=True, env=env, cwd=root, timeout=300)
        res[t] = np.load(f)
    a, b = res["1"], res["7"]
    assert sorted(a.files) == sorted(b.files) and len(a.files) >= 9
    for k in a.files:
        assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), k


def test_documented_refusals_need_no_gpu():
    """The argument checks of the C-ABI return their documented status before
    any device call: NULL handles and arrays, levels out of range, and the
    device calls of an analysed-only handle."""
    import ctypes as C
    lib = mas.lib
    P = make_problem(dim=2, n=4)
    h = mas.Handle(P, mas.default_params(2), analyze_only=True)
    hi = mas.mas_hier_info()
    assert lib.mas_get_info(None, C.byref(hi)) == mas.MAS_EINVAL
    assert lib.mas_get_info(h.h, None) == mas.MAS_EINVAL
    assert lib.mas_release(None) == mas.MAS_EINVAL
    assert lib.mas_upload(None, None) == mas.MAS_EINVAL
    sz = C.c_size_t()
    assert lib.mas_workspace_size(None, C.byref(sz)) == mas.MAS_EINVAL
    assert lib.mas_workspace_size(h.h, None) == mas.MAS_EINVAL
    assert lib.mas_upload_ws(None, C.c_void_p(256), 1024, None) == mas.MAS_EINVAL
    assert lib.mas_upload_ws(h.h, None, 1024, None) == mas.MAS_EINVAL
    assert lib.mas_upload_ws(h.h, C.c_void_p(0x1004), 1 << 20, None) == mas.MAS_EINVAL  # misaligned
    assert lib.mas_set_timing(None, 1) == mas.MAS_EINVAL
    out = (C.c_double * 18)()
    assert lib.mas_get_timing(None, out, 18) == mas.MAS_EINVAL
    assert lib.mas_destroy(None) == mas.MAS_OK
    # export: sizes first (arrays NULL), then a level out of range
    L = h.info()["n_levels"]
    nr, nnz = C.c_int64(), C.c_int64()
    assert lib.mas_export_level(h.h, 0, C.byref(nr), C.byref(nnz), None, None, None) == mas.MAS_OK
    assert nr.value == int((~P.dir0).sum()) and nnz.value > 0
    assert lib.mas_export_level(h.h, L, C.byref(nr), C.byref(nnz), None, None, None) == mas.MAS_EINVAL
    assert lib.mas_export_level(h.h, -1, C.byref(nr), C.byref(nnz), None, None, None) == mas.MAS_EINVAL
    # device calls on an analysed-only handle (host buffers: never dereferenced)
    buf = np.zeros(P.n0, np.float64)
    p = C.c_void_p(buf.ctypes.data)
    info = (mas.mas_solve_info * 1)()
    assert lib.mas_solve(h.h, p, p, 1, 1e-8, 10, info, None) == mas.MAS_EINVAL
    tol = (C.c_double * 1)(1e-8)
    assert lib.mas_solve_rtols(h.h, p, p, 1, tol, 10, info, None) == mas.MAS_EINVAL
    one = (C.c_double * 1)(1.0)
    assert lib.mas_scale_rows(h.h, p, 1, one, one, 0, None) == mas.MAS_EINVAL
    assert lib.mas_apply(h.h, p, p, 1, None) == mas.MAS_EINVAL
    assert b"analysed only" in lib.mas_last_error()
    assert lib.mas_release(h.h) == mas.MAS_OK  # nothing on the device: a no-op
    h.close()


@pytest.mark.parametrize("kw", [dict(dim=2, n=1), dict(dim=3, n=1), dict(dim=2, n=1, disc="SV", seed=1)])
def test_single_cell_meshes_analyse_under_every_variant(kw):
    """Degenerate inputs: one square or cube (2 / 11 free unknowns for
    Taylor-Hood).  Every relaxation and schedule either builds a two-level
    hierarchy whose coarsest level is K1 itself (solved exactly) or refuses
    with its documented error (HO-AMG on Scott-Vogelius)."""
    bc = "zero" if kw.get("disc") == "SV" else "lid"
    P = make_problem(forcing="gaussian", bc=bc, **kw)
    disc = mas.MAS_SV if P.disc == "SV" else mas.MAS_TH
    nfree = int((~P.dir0).sum())
    for relax in (mas.MAS_RELAX_VANKA, mas.MAS_RELAX_DLSC, mas.MAS_RELAX_VANKA_DLSC):
        for sched in (mas.MAS_DC_ALL, mas.MAS_DC_SKIP1, mas.MAS_DC_SKIP0, mas.MAS_HO_AMG):
            par = mas.default_params(P.dim, disc, relax, schedule=sched)
            if disc == mas.MAS_SV and sched == mas.MAS_HO_AMG:
                with pytest.raises(mas.MasError) as e:
                    mas.Handle(P, par, analyze_only=True)
                assert e.value.code == mas.MAS_EINVAL
                continue
            h = mas.Handle(P, par, analyze_only=True)
            i = h.info()
            h.close()
            assert i["n_levels"] == 2 and i["n"][0] == nfree
            assert i["n_patches"][1] == 0  # the coarsest level is not relaxed
            vanka_on_k0 = relax != mas.MAS_RELAX_DLSC and sched not in (mas.MAS_DC_SKIP0, mas.MAS_HO_AMG)
            assert (i["n_patches"][0] > 0) == vanka_on_k0


def test_stalled_coarsening_is_refused_before_a_huge_dense_solve():
    """The coarsest level is inverted densely: a threshold that leaves (almost)
    no strong connections stops the coarsening at the fine size, and the
    analysis refuses it (EINVAL, naming the cause) unless max_coarse accepts a
    coarsest level that large."""
    P = make_problem(dim=2, n=48, jitter=0.2, seed=2, forcing="gaussian", bc="lid")
    sym = dict(theta=0.9, soc=mas.MAS_SOC_SYMMETRIC)
    with pytest.raises(mas.MasError) as e:
        mas.Handle(P, mas.default_params(2, **sym), analyze_only=True)
    assert e.value.code == mas.MAS_EINVAL and "coarsest" in str(e.value)
    h = mas.Handle(P, mas.default_params(2, max_coarse=10 ** 6, **sym), analyze_only=True)
    assert h.info()["n_levels"] == 2
    h.close()


def test_coarsest_size_is_checked_where_the_fields_are_cut():
    """The hierarchy depth is the minimum over the fields (Algorithm 1), so a
    field that stops early cuts the others short.  With max_coarse = 2500 the
    2401 pressures of the 48 x 48 mesh are not coarsened at all, while each
    velocity component (9025 free nodes) coarsens below the limit on its own:
    the level actually inverted is K1 itself (20,451 rows with the border),
    which the analysis refuses even though every field's own coarsest level is
    below the limit."""
    P = make_problem(dim=2, n=48, jitter=0.2, seed=2, forcing="gaussian", bc="lid")
    assert P.meta["n_p1"] == 2401
    with pytest.raises(mas.MasError) as e:
        mas.Handle(P, mas.default_params(2, max_coarse=2500), analyze_only=True)
    assert e.value.code == mas.MAS_EINVAL and "coarsest" in str(e.value)
    h = mas.Handle(P, mas.default_params(2, max_coarse=300), analyze_only=True)
    i = h.info()
    assert i["coarse_n"] <= 8192 and i["n_levels"] >= 3
    h.close()


def oracle_prebuilt(pre):
    """Per-field interpolations of the oracle's hierarchy (Ps[l][f]) and the
    coarsest pressure near-null vector, in the form mas_problem.prebuilt_P takes."""
    from oracle.sparse import submatrix
    d = pre.dim
    Ps = []
    for l, lv in enumerate(pre.levels[:-1]):
        fine, coarse = lv.field, pre.levels[l + 1].field
        Ps.append([submatrix(lv.P, np.nonzero(fine == f)[0], np.nonzero(coarse == f)[0]) for f in range(d + 1)])
    return Ps, pre.levels[-1].null_p


@pytest.mark.parametrize("kw,soc", [
    (dict(dim=2, n=24, jitter=0.2, seed=2, forcing="gaussian", bc="lid"), "symmetric"),
    (dict(dim=2, n=24, jitter=0.2, seed=2, forcing="gaussian", bc="lid"), "evolution"),
    (dict(dim=3, n=5, forcing="smooth", bc="zero", seed=3), "symmetric"),
    (dict(dim=2, n=10, disc="SV", seed=4, forcing="gaussian", bc="zero"), "evolution"),
])
def test_prebuilt_hierarchy_gives_the_oracle_levels(kw, soc):
    """A hierarchy injected through prebuilt_P / prebuilt_null_p replaces
    Algorithm 1: the library's levels are the oracle's (patterns equal, values
    to rounding), whatever strength measure the library's own parameters name."""
    P = make_problem(**kw)
    par = dc.default_params(P, max_coarse=30, soc=soc)
    pre = dc.DCPreconditioner(P, par)
    other = "evolution" if soc == "symmetric" else "symmetric"
    _, mp = _same_params(P, max_coarse=30, soc=other)
    h = mas.Handle(P, mp, analyze_only=True, prebuilt=oracle_prebuilt(pre))
    info = h.info()
    assert info["n_levels"] == 1 + len(pre.levels)
    for l, K in enumerate([pre.K0] + [lv.K for lv in pre.levels]):
        Kl = h.export_level(l)
        assert np.array_equal(Kl.indptr, K.indptr) and np.array_equal(Kl.indices, K.indices), l
        assert np.abs(Kl.data - K.data).max() <= 1e-13 * np.abs(K.data).max(), l
    h.close()


def test_prebuilt_hierarchy_is_validated():
    P = make_problem(dim=2, n=12, jitter=0.2, seed=2, forcing="gaussian", bc="lid")
    pre = dc.DCPreconditioner(P, dc.default_params(P, max_coarse=30))
    Ps, null_p = oracle_prebuilt(pre)
    mp = mas.default_params(2, max_coarse=30)
    bad = [list(level) for level in Ps]
    bad[0][1] = bad[0][1][1:]  # one row short
    for prebuilt in ((bad, null_p), (Ps, None)):
        with pytest.raises(mas.MasError) as e:
            mas.Handle(P, mp, analyze_only=True, prebuilt=prebuilt)
        assert e.value.code == mas.MAS_EINVAL


@pytest.mark.parametrize("kw", [
    dict(dim=2, n=24, jitter=0.2, seed=2, forcing="gaussian", bc="lid"),
    dict(dim=3, n=4, forcing="smooth", bc="zero", seed=3),
    dict(dim=2, n=8, disc="SV", jitter=0.2, seed=4, forcing="gaussian", bc="lid"),
])
def test_identical_component_blocks_are_found_on_the_host(kw):
    """Every patch of these problems has identical velocity blocks in all
    components (vector Laplacian, the same Dirichlet data on each component):
    the analysis marks each relaxed level shared and counts one packed block
    per patch; with share_blocks = 0, or once the y-velocity unknowns are
    rescaled (blocks differ by a factor 4), one block per component.  Counts
    from the oracle's patches and the level fields."""
    import dataclasses
    import scipy.sparse as sp
    P = make_problem(**kw)
    par, mp = _same_params(P, max_coarse=40)
    pre = dc.DCPreconditioner(P, par)
    fields = [pre.f0] + [lv.field for lv in pre.levels]

    def expected(shared):
        out = []
        for l, R in enumerate(pre.relax):
            f = fields[l]
            tot = 0
            for dofs, ns in zip(R.dofs, R.n_seed):
                nc = [int(np.sum(f[dofs] == c)) for c in range(P.dim)]
                nv = sum(nc)
                blocks = nc[:1] if shared else nc
                tot += sum(n * (n + 1) // 2 for n in blocks) + nv * ns + ns * (ns + 1) // 2
            out.append(tot)
        return out

    for share, want_layout in ((1, 2), (0, 0)):
        mp.share_blocks = share
        h = mas.Handle(P, mp, analyze_only=True)
        info = h.info()
        n = len(pre.relax)
        assert info["patch_layout"][:n] == [want_layout] * n
        assert info["factor_entries"][:n] == expected(share == 1)
        h.close()
    d0 = np.where((P.field0 == 1) & ~P.dir0, 2.0, 1.0)
    d1 = np.where((P.field1 == 1) & ~P.dir1, 2.0, 1.0)
    Q = dataclasses.replace(P, K0=(sp.diags(d0) @ P.K0 @ sp.diags(d0)).tocsr(),
                            K1=(sp.diags(d1) @ P.K1 @ sp.diags(d1)).tocsr())
    mp.share_blocks = 1
    h = mas.Handle(Q, mp, analyze_only=True)
    assert not any(v & 2 for v in h.info()["patch_layout"])
    h.close()


def test_workspace_size_is_computed_on_the_host():
    """mas_workspace_size sizes mas_upload_ws from the analysis alone: no device
    is touched (this runs without one), the handle stays analysed-only, the
    answer is reproducible and grows with the right-hand sides a call may carry."""
    P = make_problem(dim=3, n=4, forcing="smooth", bc="zero", seed=3)
    sizes = []
    for nr in (1, 4):
        h = mas.Handle(P, mas.default_params(3, max_coarse=40, nrhs_max=nr), analyze_only=True)
        a, b = h.workspace_size(), h.workspace_size()
        assert a == b and a > 0 and a % 256 == 0
        assert h.info()["device_bytes"] == 0
        sizes.append(a)
        h.close()
    assert sizes[1] > sizes[0]
    h = mas.Handle(P, mas.default_params(3, max_coarse=40, precision=mas.MAS_FP32), analyze_only=True)
    assert 0 < h.workspace_size() < sizes[0]
    h.close()
