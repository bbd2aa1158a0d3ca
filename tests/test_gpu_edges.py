"""Edge cases of the GPU path through the C-ABI: zero right-hand sides (alone
and beside non-zero columns), the largest batch (64 right-hand sides), a
batch size that is not a power of two, the smallest hierarchy (K1 is the
coarsest level, solved densely), a solve that hits max_it, and argument
errors that must not touch the device."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import dc  # noqa: E402
from paper_2306_06795_amd import mas  # noqa: E402
from parity import assert_parity  # noqa: E402
from paper_2306_06795_amd.inputs import make_problem  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def handle(P, nrhs_max=1, precision=mas.MAS_FP64, **over):
    kw = dict(precision=precision, nrhs_max=nrhs_max, max_coarse=30)
    kw.update(over)
    return mas.Handle(P, mas.default_params(P.dim, **kw))


def test_zero_rhs_alone_and_in_a_batch():
    print("[edges] zero right-hand sides", flush=True)
    P = make_problem(dim=2, n=8, forcing="gaussian", bc="zero", seed=2, nrhs=3)
    h = handle(P, nrhs_max=3)
    b = torch.zeros(P.n0, dtype=torch.float64, device=DEV)
    x = torch.full_like(b, 7.0)
    rc, info = h.solve(b, x)
    assert rc == mas.MAS_OK and info[0]["converged"] and info[0]["iters"] == 0
    assert torch.count_nonzero(x).item() == 0
    B = np.array(P.b)
    B[:, 1] = 0.0
    Bd = torch.tensor(B, device=DEV)
    Xd = torch.empty_like(Bd)
    rc, info = h.solve(Bd, Xd, rtol=1e-8, nrhs=3)
    X = Xd.cpu().numpy()
    assert rc == mas.MAS_OK
    assert info[1]["iters"] == 0 and np.all(X[:, 1] == 0.0)
    for k in (0, 2):
        assert np.linalg.norm(B[:, k] - P.K0 @ X[:, k]) <= 1e-8 * np.linalg.norm(B[:, k])
    h.close()


@pytest.mark.parametrize("nrhs", [64, 7])
def test_largest_and_ragged_batches(nrhs):
    print(f"[edges] nrhs={nrhs}", flush=True)
    P = make_problem(dim=2, n=8, forcing="gaussian", bc="lid", jitter=0.2, seed=4, nrhs=nrhs)
    h = handle(P, nrhs_max=nrhs, precision=mas.MAS_FP32)
    Bd = torch.tensor(P.b, device=DEV)
    Xd = torch.empty_like(Bd)
    rc, info = h.solve(Bd, Xd, rtol=1e-8, nrhs=nrhs)
    X = Xd.cpu().numpy()
    assert rc == mas.MAS_OK
    for k in range(nrhs):
        assert np.linalg.norm(P.b[:, k] - P.K0 @ X[:, k]) <= 1e-8 * np.linalg.norm(P.b[:, k]), k
    with pytest.raises(mas.MasError) as e:  # one more than the handle was built for
        h.solve(torch.zeros((P.n0, nrhs + 1), dtype=torch.float64, device=DEV),
                torch.zeros((P.n0, nrhs + 1), dtype=torch.float64, device=DEV), nrhs=nrhs + 1)
    assert e.value.code == mas.MAS_EINVAL
    h.close()


def test_two_level_hierarchy_matches_oracle():
    """max_coarse above the K1 size: K1 itself is the dense coarsest level."""
    P = make_problem(dim=2, n=6, forcing="gaussian", bc="lid", seed=3)
    par = dc.default_params(P, max_coarse=10 ** 6)
    pre = dc.DCPreconditioner(P, par)
    h = handle(P, max_coarse=10 ** 6)
    assert h.info()["n_levels"] == 2
    r = np.random.default_rng(0).standard_normal(P.n0)
    z = torch.empty(P.n0, dtype=torch.float64, device=DEV)
    h.apply(torch.tensor(r, device=DEV), z)
    torch.cuda.synchronize()
    ref = pre.apply(r)
    assert_parity(z.cpu().numpy(), ref, P.field0, 1e-11, "two-level")
    h.close()


def test_max_it_reports_not_converged():
    P = make_problem(dim=2, n=12, forcing="gaussian", bc="lid", seed=1)
    h = handle(P)
    b = torch.tensor(P.b, device=DEV)
    x = torch.empty_like(b)
    rc, info = h.solve(b, x, rtol=1e-14, max_it=3)
    assert rc == mas.MAS_NOT_CONVERGED and not info[0]["converged"] and info[0]["iters"] == 3
    res = np.linalg.norm(P.b - P.K0 @ x.cpu().numpy()) / np.linalg.norm(P.b)
    assert abs(res - info[0]["relres"]) <= 1e-6 * res  # the reported residual is the true one
    h.close()


def test_argument_errors():
    P = make_problem(dim=2, n=6)
    h = handle(P)
    b = torch.tensor(P.b, device=DEV)
    x = torch.empty_like(b)
    for kw in (dict(rtol=-1.0), dict(max_it=0), dict(nrhs=0), dict(rtol=[float("nan")], nrhs=1)):
        with pytest.raises(mas.MasError) as e:
            h.solve(b, x, **kw)
        assert e.value.code == mas.MAS_EINVAL, kw
    h.close()


@pytest.mark.parametrize("nrhs", [1, 5])
def test_classical_and_modified_gram_schmidt_agree(nrhs):
    """FGMRES with classical Gram-Schmidt (default) and modified (gram_schmidt):
    same iteration counts, solutions equal to rounding."""
    P = make_problem(dim=2, n=16, forcing="gaussian", bc="lid", jitter=0.2, seed=6, nrhs=nrhs)
    B = torch.tensor(P.b, device=DEV)
    out = {}
    for mgs in (False, True):
        h = handle(P, nrhs_max=nrhs, gram_schmidt=mas.MAS_GS_MODIFIED if mgs else mas.MAS_GS_CLASSICAL)
        X = torch.empty_like(B)
        rc, info = h.solve(B, X, rtol=1e-10, nrhs=nrhs)
        assert rc == mas.MAS_OK
        out[mgs] = (X.cpu().numpy(), [i["iters"] for i in info])
        h.close()
    (xc, ic), (xm, im) = out[False], out[True]
    print(f"[edges] nrhs={nrhs} its classical {ic} modified {im}", flush=True)
    assert ic == im
    assert np.linalg.norm(xc - xm) <= 1e-9 * np.linalg.norm(xm)
