"""Galerkin products of the setup on the device (Algorithm 1, opt-in with
device_galerkin = 1): the hierarchy a handle builds through mas_setup with
device products must equal, bit for bit, the one mas_analyze builds on the
host -- also when rows overflow the kernel's LDS table and are finished on the
host."""
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


@pytest.mark.parametrize("cap", [None, "4"])
@pytest.mark.parametrize("name", list(CASES))
def test_device_galerkin_equals_host_bitwise(name, cap, monkeypatch):
    kw, over = CASES[name]
    P = make_problem(**kw)
    mp = mas.default_params(P.dim, mas.MAS_SV if P.disc == "SV" else mas.MAS_TH, max_coarse=20, **over)
    mp.device_galerkin = 1
    if cap:  # rows with more than 4 distinct columns are finished on the host
        monkeypatch.setenv("MAS_SPGEMM_CAP", cap)
    print(f"[setup {name}] cap={cap}", flush=True)
    hd = mas.Handle(P, mp)
    hh = mas.Handle(P, mp, analyze_only=True)
    Ld, Lh = levels(hd), levels(hh)
    assert len(Ld) == len(Lh) >= 3
    for l, (A, B) in enumerate(zip(Ld, Lh)):
        assert A.shape == B.shape, l
        assert np.array_equal(A.indptr, B.indptr) and np.array_equal(A.indices, B.indices), l
        assert np.array_equal(A.data.view(np.int64), B.data.view(np.int64)), f"level {l} values differ"
    hd.close()
    hh.close()
