"""The boundary's caller-owned workspace and prebuilt-hierarchy inputs on the
GPU: a handle uploaded into a caller's device buffer of exactly
mas_workspace_size bytes computes what a library-owned handle computes, bit for
bit; a buffer one byte short is refused without harm; and a hierarchy injected
from the oracle gives apply parity with the oracle's cycle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import dc  # noqa: E402
from paper_2306_06795_amd import mas  # noqa: E402
from paper_2306_06795_amd.inputs import make_problem  # noqa: E402
from parity import assert_parity  # noqa: E402
from test_abi import oracle_prebuilt  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.mark.parametrize("kw,prec,nr", [
    (dict(dim=2, n=24, jitter=0.2, seed=2, forcing="gaussian", bc="lid"), mas.MAS_FP64, 1),
    (dict(dim=3, n=6, forcing="smooth", bc="zero", seed=3), mas.MAS_FP32, 3),
    (dict(dim=2, n=8, disc="SV", seed=4, forcing="gaussian", bc="zero"), mas.MAS_FP32, 2),
])
def test_caller_workspace_equals_library_memory(kw, prec, nr):
    P = make_problem(nrhs=nr, **kw)
    disc = mas.MAS_SV if P.disc == "SV" else mas.MAS_TH
    # autotune off: both handles take the same kernels, so results are bitwise comparable
    mp = mas.default_params(P.dim, disc, max_coarse=30, precision=prec, nrhs_max=nr, autotune=0)
    ref = mas.Handle(P, mp)
    h = mas.Handle(P, mp, analyze_only=True)
    need = h.workspace_size()
    print(f"[workspace] n0={P.n0} precision={prec} nrhs={nr}: {need} bytes "
          f"(library-owned handle holds {ref.info()['device_bytes']})", flush=True)
    short = torch.empty(need - 256, dtype=torch.uint8, device=DEV)
    with pytest.raises(mas.MasError) as e:
        h.upload_ws(short)
    assert e.value.code == mas.MAS_ENOMEM
    assert h.info()["device_bytes"] == 0  # left analysed-only
    del short
    ws = torch.empty(need, dtype=torch.uint8, device=DEV)
    h.upload_ws(ws)
    R = torch.tensor(np.random.default_rng(3).standard_normal((P.n0, nr)), device=DEV)
    Z0, Z1 = torch.empty_like(R), torch.empty_like(R)
    ref.apply(R, Z0, nrhs=nr)
    h.apply(R, Z1, nrhs=nr)
    torch.cuda.synchronize()
    assert torch.equal(Z0, Z1)
    B = torch.tensor(P.b.reshape(P.n0, nr), device=DEV)
    X0, X1 = torch.empty_like(B), torch.empty_like(B)
    rc0, i0 = ref.solve(B, X0, rtol=1e-8, nrhs=nr)
    rc1, i1 = h.solve(B, X1, rtol=1e-8, nrhs=nr)
    assert rc0 == rc1 == mas.MAS_OK and [a["iters"] for a in i0] == [b["iters"] for b in i1]
    assert torch.equal(X0, X1)
    h.release()  # the buffer may be reused once release returns
    ws.zero_()
    h.upload_ws(ws)
    h.apply(R, Z1, nrhs=nr)
    torch.cuda.synchronize()
    assert torch.equal(Z0, Z1)
    h.close()
    ref.close()


@pytest.mark.parametrize("kw", [dict(dim=2, n=24, jitter=0.2, seed=2, forcing="gaussian", bc="lid"),
                                dict(dim=3, n=5, forcing="smooth", bc="zero", seed=3)])
def test_prebuilt_oracle_hierarchy_apply_parity(kw):
    """The oracle built with the symmetric strength measure, the library told to
    use the evolution measure: with the oracle's hierarchy injected, the FP64
    cycle applications agree to 1e-11."""
    P = make_problem(**kw)
    par = dc.default_params(P, max_coarse=30, soc="symmetric")
    pre = dc.DCPreconditioner(P, par)
    mp = mas.default_params(P.dim, max_coarse=30, soc=mas.MAS_SOC_EVOLUTION)
    h = mas.Handle(P, mp, prebuilt=oracle_prebuilt(pre))
    rng = np.random.default_rng(5)
    for trial in range(2):
        r = rng.standard_normal(P.n0)
        z = torch.empty(P.n0, dtype=torch.float64, device=DEV)
        h.apply(torch.tensor(r, device=DEV), z)
        torch.cuda.synchronize()
        assert_parity(z.cpu().numpy(), pre.apply(r), P.field0, 1e-11, f"prebuilt trial {trial}")
    h.close()
