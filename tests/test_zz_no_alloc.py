"""mas_apply_static (cycle scratch in the library's static device array)
against mas_apply through the C-ABI: the same result bit for bit on two calls
in a row, the second with a smaller input (fewer right-hand sides on a smaller
mesh, so it runs on the first call's leftover scratch contents), and a clear
refusal when a handle's scratch exceeds the array."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2306_06795_amd import mas  # noqa: E402
from paper_2306_06795_amd.inputs import make_problem  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _both(h, R, nr):
    Z0, Z1 = torch.empty_like(R), torch.empty_like(R)
    rc0 = mas.lib.mas_apply(h.h, C.c_void_p(R.data_ptr()), C.c_void_p(Z0.data_ptr()), nr, None)
    rc1 = mas.lib.mas_apply_static(h.h, C.c_void_p(R.data_ptr()), C.c_void_p(Z1.data_ptr()), nr, None)
    torch.cuda.synchronize()
    assert rc0 == rc1 == mas.MAS_OK, (rc0, rc1, mas.lib.mas_last_error())
    return Z0, Z1


def test_static_scratch_apply_equals_apply_on_two_calls():
    torch.zeros(1, device=DEV)  # the default stream's context
    cases = [  # first call: 3D, 3 right-hand sides; second: a smaller 2D mesh, 1 right-hand side
        (make_problem(dim=3, n=5, forcing="smooth", bc="zero", seed=3), 3, mas.MAS_FP64, mas.MAS_RELAX_VANKA),
        (make_problem(dim=2, n=8, jitter=0.2, seed=2, forcing="gaussian", bc="lid"), 1, mas.MAS_FP32,
         mas.MAS_RELAX_DLSC),
    ]
    for k, (P, nr, prec, relax) in enumerate(cases):
        h = mas.Handle(P, mas.default_params(P.dim, mas.MAS_TH, relax, max_coarse=30, nrhs_max=nr, precision=prec))
        R = torch.tensor(np.random.default_rng(k).standard_normal((P.n0, nr)), device=DEV)
        Z0, Z1 = _both(h, R, nr)
        print(f"[static scratch] call {k}: n0={P.n0} nrhs={nr} equal={torch.equal(Z0, Z1)}", flush=True)
        assert torch.equal(Z0, Z1)
        # the handle's own path is unaffected afterwards
        Z2 = torch.empty_like(R)
        h.apply(R, Z2, nrhs=nr)
        torch.cuda.synchronize()
        assert torch.equal(Z0, Z2)
        h.close()


def test_static_scratch_refuses_handles_beyond_its_size():
    P = make_problem(dim=2, n=96, forcing="gaussian", bc="lid", jitter=0.2, seed=2, nrhs=64)
    h = mas.Handle(P, mas.default_params(2, nrhs_max=64, max_coarse=300))
    R = torch.zeros((P.n0, 64), dtype=torch.float64, device=DEV)
    Z = torch.empty_like(R)
    rc = mas.lib.mas_apply_static(h.h, C.c_void_p(R.data_ptr()), C.c_void_p(Z.data_ptr()), 64, None)
    assert rc == mas.MAS_EINVAL and b"static scratch" in mas.lib.mas_last_error()
    h.close()
