"""Setup on the device (Algorithm 1, the default of mas_setup): the Galerkin products of the
level operators (device_galerkin = 1), and the per-field smoothed aggregation
with its operators resident on the device (device_sa = 1: Gershgorin bound,
symmetric and evolution strength of Section 3.2, smoothed prolongator, the
field's Galerkin products).  The hierarchy a handle builds through mas_setup
must equal, bit for bit, the one mas_analyze builds on the host -- also when
rows overflow the product kernel's LDS table (spgemm_cap) and take the
global-memory product kernel."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2306_06795_amd import mas  # noqa: E402
from paper_2306_06795_amd.inputs import make_problem  # noqa: E402

pytestmark = pytest.mark.gpu

CASES = {
    "th24_lid": (dict(dim=2, n=24, jitter=0.2, seed=2, forcing="gaussian", bc="lid"), {}),
    "th3d6": (dict(dim=3, n=6, forcing="smooth", bc="zero", seed=3), {}),
    "sv8": (dict(dim=2, n=8, disc="SV", seed=4, forcing="gaussian", bc="zero"), {}),
    "th24_ho": (dict(dim=2, n=24, jitter=0.2, seed=2, forcing="gaussian", bc="lid"), dict(schedule=mas.MAS_HO_AMG)),
}


def levels(h):
    return [h.export_level(l) for l in range(h.info()["n_levels"])]


def assert_same_hierarchy(hd, hh):
    Ld, Lh = levels(hd), levels(hh)
    assert len(Ld) == len(Lh) >= 3
    for l, (A, B) in enumerate(zip(Ld, Lh)):
        assert A.shape == B.shape, l
        assert np.array_equal(A.indptr, B.indptr) and np.array_equal(A.indices, B.indices), l
        assert np.array_equal(A.data.view(np.int64), B.data.view(np.int64)), f"level {l} values differ"
    assert hd.info()["p_nnz"] == hh.info()["p_nnz"]


@pytest.mark.parametrize("cap", [0, 4])
@pytest.mark.parametrize("name", list(CASES))
def test_device_galerkin_equals_host_bitwise(name, cap):
    kw, over = CASES[name]
    P = make_problem(**kw)
    mp = mas.default_params(P.dim, mas.MAS_SV if P.disc == "SV" else mas.MAS_TH, max_coarse=20, **over)
    mp.device_galerkin, mp.device_sa = 1, 0
    mp.spgemm_cap = cap  # 4: rows with more than 4 distinct columns take the global-memory product
    print(f"[setup {name}] cap={cap}", flush=True)
    hd = mas.Handle(P, mp)
    hh = mas.Handle(P, mp, analyze_only=True)
    assert_same_hierarchy(hd, hh)
    hd.close()
    hh.close()


SA_CASES = dict(CASES, **{
    "th3d8": (dict(dim=3, n=8, forcing="smooth", bc="zero", seed=3), dict(max_levels=4)),
    "th24_sym": (dict(dim=2, n=24, jitter=0.2, seed=2, forcing="gaussian", bc="lid"), dict(soc=mas.MAS_SOC_SYMMETRIC)),
    "sv8_evol": (dict(dim=2, n=8, disc="SV", seed=4, forcing="gaussian", bc="zero"),
                 dict(soc=mas.MAS_SOC_EVOLUTION, max_coarse=60)),
})


@pytest.mark.parametrize("cap", [0, 4])
@pytest.mark.parametrize("name", list(SA_CASES))
def test_device_smoothed_aggregation_equals_host_bitwise(name, cap):
    kw, over = SA_CASES[name]
    P = make_problem(**kw)
    over = dict(dict(max_coarse=20), **over)
    mp = mas.default_params(P.dim, mas.MAS_SV if P.disc == "SV" else mas.MAS_TH, **over)
    mp.device_sa, mp.device_galerkin = 1, 0
    mp.spgemm_cap = cap  # 4: rows with more than 4 distinct columns take the global-memory product
    print(f"[device sa {name}] cap={cap} soc={mp.soc}", flush=True)
    hd = mas.Handle(P, mp)
    hh = mas.Handle(P, mp, analyze_only=True)
    assert_same_hierarchy(hd, hh)
    # the two together: device aggregation, device Galerkin products of the system
    mp.device_galerkin = 1
    hb = mas.Handle(P, mp)
    assert_same_hierarchy(hb, hh)
    for h in (hd, hh, hb):
        h.close()


@pytest.mark.parametrize("config", [
    "th2d_256",
    "sv2d_128x64",
    pytest.param("th3d_32", marks=pytest.mark.slow),
])
def test_device_setup_equals_host_at_benchmark_size(config):
    """The default mas_setup (smoothed aggregation and Galerkin products on the
    device) and the host analysis build the same hierarchy, bit for bit, on
    the benchmark workloads."""
    from paper_2306_06795_amd.inputs import make_config
    P = make_config(config)
    mp = mas.default_params(P.dim, mas.MAS_SV if P.disc == "SV" else mas.MAS_TH)
    assert mp.device_sa == 1 and mp.device_galerkin == 1
    print(f"[device setup {config}]", flush=True)
    hd = mas.Handle(P, mp)
    hh = mas.Handle(P, mp, analyze_only=True)
    assert_same_hierarchy(hd, hh)
    hd.close()
    hh.close()
