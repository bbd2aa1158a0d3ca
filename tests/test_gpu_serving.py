"""Serving loop: viscosity scaling on a shared nu = 1 hierarchy, continuous
batching at slot level (a request admitted into a running batch equals its
solo solve), HBM-budget admission, release / re-upload of a handle.

Every result is checked against the operator assembled for its own viscosity
on the CPU: ||b - K_nu x|| <= rtol ||b||.  Batch invariance: a request solved
alone and the same request inside a mix of other requests and meshes give the
same solution, to 1e-9 relative with the FP64 cycle (the cycles agree to
rounding, so the iterates agree up to that rounding carried through the
Krylov method, or one iteration more or less at the threshold) and to 1e-6
with the FP32
cycle (the FP32 rounding of the batched and single-column patch kernels
differs; both solutions satisfy the residual bound, and 1e-6 is what the
cycle's FP32 rounding leaves after the FP64 outer iteration on these meshes).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2306_06795_amd import mas, serving  # noqa: E402
from paper_2306_06795_amd.inputs import make_problem, random_rhs  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
MESHES = {"a2": (2, 8), "b2": (2, 12), "c3": (3, 3)}


def mesh(dim, n, nu=1.0):
    return make_problem(dim=dim, n=n, disc="TH", forcing="gaussian", bc="zero", nu=nu, seed=1)


def make_server(budget=8 << 30, precision=mas.MAS_FP32, max_batch=8, workers=3, meshes=MESHES, sizes=None):
    srv = serving.StokesServer(budget, max_batch=max_batch, workers=workers, precision=precision,
                               params=dict(max_coarse=30))
    probs = {}
    for k, (d, n) in meshes.items():
        probs[k] = mesh(d, n)
        est = srv.add_mesh(k, probs[k])
        if sizes:
            assert est >= sizes[k], (k, est, sizes[k])  # the analysis estimate bounds the real size
            srv.add_mesh(k, probs[k], device_bytes=sizes[k])
    return srv, probs


def requests(probs, count, seed):
    rng = np.random.default_rng(seed)
    keys = sorted(probs)
    out = []
    for _ in range(count):
        k = keys[int(rng.integers(len(keys)))]
        nu = float(10.0 ** rng.uniform(-2, 0))
        out.append(serving.Request(mesh=k, nu=nu, b=random_rhs(probs[k], rng)))
    return out


def check_residual(req, dims):
    d, n = dims
    K = mesh(d, n, nu=req.nu).K0
    res = np.linalg.norm(req.b - K @ req.x) / np.linalg.norm(req.b)
    assert res <= req.rtol * (1 + 1e-6), (req.mesh, req.nu, res, req.iters)
    return res


@pytest.mark.parametrize("precision", [mas.MAS_FP32, mas.MAS_FP64])
def test_results_meet_their_viscosity_residual(precision):
    print(f"[serving] precision={precision}", flush=True)
    srv, probs = make_server(precision=precision)
    srv.start()
    reqs = requests(probs, 30, seed=7)
    for r in reqs:
        srv.submit(r)
    for r in reqs:
        assert r.done.wait(120)
    st = srv.stats()
    srv.shutdown()
    for r in reqs:
        assert r.error is None, r.error
        check_residual(r, MESHES[r.mesh])
        # zero-mean pressure carries over from the scaled solve
        P = probs[r.mesh]
        assert abs(P.p_weight0 @ r.x[P.meta["n_u"]:]) <= 1e-10 * np.abs(r.x).max()
    assert max(r.batch for r in reqs) > 1, st  # some requests advanced together
    print(f"  stats {st}")


@pytest.mark.parametrize("precision,tol", [(mas.MAS_FP64, 1e-9), (mas.MAS_FP32, 1e-6)])
def test_alone_equals_in_mix(precision, tol):
    print(f"[serving] alone vs mix precision={precision}", flush=True)
    srv, probs = make_server(precision=precision, max_batch=32)
    srv.start()
    rng = np.random.default_rng(3)
    probe = [serving.Request(mesh="b2", nu=nu, b=random_rhs(probs["b2"], rng)) for nu in (0.01, 0.3, 1.0)]
    alone = []
    for p in probe:
        r = serving.Request(mesh=p.mesh, nu=p.nu, b=p.b.copy())
        srv.submit(r)
        assert r.done.wait(120)
        assert r.error is None and r.batch == 1
        alone.append(r)
    # the same requests again, inside a burst of others on every mesh
    mix = requests(probs, 24, seed=9)
    for i, p in enumerate(probe):
        mix.insert(4 + 6 * i, p)
    srv.pause()  # the whole burst queues before the first batch forms
    for r in mix:
        srv.submit(r)
    srv.resume()
    for r in mix:
        assert r.done.wait(120)
    srv.shutdown()
    for a, p in zip(alone, probe):
        assert p.error is None
        assert p.batch > 1, "the probe was expected to share a batch"
        err = np.linalg.norm(a.x - p.x) / np.linalg.norm(a.x)
        print(f"  nu={p.nu}: alone {a.iters} its, in a batch of {p.batch}: {p.iters} its, rel diff {err:.2e}")
        assert err <= tol
        check_residual(p, MESHES["b2"])


def test_budget_admission_and_eviction():
    print("[serving] small budget", flush=True)
    probe, pprobs = make_server(budget=1 << 40)
    probe.start()
    for k in MESHES:  # one upload each: the registered sizes become the exact device bytes
        r = probe.submit(serving.Request(mesh=k, nu=1.0, b=random_rhs(pprobs[k], np.random.default_rng(0))))
        assert r.done.wait(120) and r.error is None
    est = {k: m.est_bytes for k, m in probe.meshes.items()}
    first = {k: m.handle.info()["device_bytes"] for k, m in probe.meshes.items()}
    assert est == first
    probe.shutdown()
    big = max(est.values())
    budget = big + min(est.values()) // 2  # the largest fits alone, no two of the larger ones together
    srv, probs = make_server(budget=budget, sizes=est)
    srv.start()
    reqs = requests(probs, 24, seed=11)
    for r in reqs:
        srv.submit(r)
        r.done.wait(120)  # one at a time, so the meshes alternate
    st = srv.stats()
    srv.shutdown()
    for r in reqs:
        assert r.error is None, r.error
        check_residual(r, MESHES[r.mesh])
    assert st["evictions"] > 0 and st["peak_resident_bytes"] <= budget, st
    print(f"  budget {budget} stats {st}")
    # a mesh whose hierarchy does not fit is refused at submission
    tiny, probs2 = make_server(budget=min(est.values()) - 1)
    tiny.start()
    r = tiny.submit(serving.Request(mesh="a2", nu=1.0, b=random_rhs(probs2["a2"], np.random.default_rng(0))))
    assert r.done.is_set() and "budget" in r.error
    tiny.shutdown()


def test_release_and_upload_roundtrip():
    P = mesh(2, 12)
    par = mas.default_params(2, max_coarse=30)
    h = mas.Handle(P, par)
    r = torch.tensor(np.random.default_rng(1).standard_normal(P.n0), device=DEV)
    z0 = torch.empty_like(r)
    h.apply(r, z0)
    torch.cuda.synchronize()
    assert h.info()["device_bytes"] > 0
    h.release()
    assert h.info()["device_bytes"] == 0
    with pytest.raises(mas.MasError):
        h.apply(r, torch.empty_like(r))
    h.upload()
    z1 = torch.empty_like(r)
    h.apply(r, z1)
    torch.cuda.synchronize()
    err = (torch.linalg.norm(z1 - z0) / torch.linalg.norm(z0)).item()
    assert err <= 1e-13, err
    h.close()
    # an analysed handle uploaded later equals a directly set-up one
    ha = mas.Handle(P, par, analyze_only=True)
    ha.upload()
    z2 = torch.empty_like(r)
    ha.apply(r, z2)
    torch.cuda.synchronize()
    assert (torch.linalg.norm(z2 - z0) / torch.linalg.norm(z0)).item() <= 1e-13
    ha.close()


@pytest.mark.parametrize("precision,tol", [(mas.MAS_FP64, 1e-9), (mas.MAS_FP32, 1e-6)])
def test_request_admitted_mid_batch_equals_its_solo_solve(precision, tol):
    """B enters a free slot after A's first restart cycle, while A keeps
    iterating from its own iterate; B's result equals B solved alone."""
    print(f"[serving] mid-batch admission precision={precision}", flush=True)
    meshes = {"b2": MESHES["b2"]}
    rng = np.random.default_rng(21)
    srv0, probs = make_server(precision=precision, max_batch=4, workers=1, meshes=meshes)
    P = probs["b2"]
    bA, bB = random_rhs(P, rng), random_rhs(P, rng)
    srv0.start()
    solo = serving.Request(mesh="b2", nu=0.2, b=bB.copy())
    srv0.submit(solo)
    assert solo.done.wait(120) and solo.error is None and solo.batch == 1
    srv0.shutdown()
    late = serving.Request(mesh="b2", nu=0.2, b=bB.copy())
    sent = []

    def on_step(key, running):
        if not sent and running:  # A is still iterating after its first cycle
            sent.append(srv.submit(late))

    srv, _ = make_server(precision=precision, max_batch=4, workers=1, meshes=meshes)
    srv.on_step = on_step
    srv.start()
    A = serving.Request(mesh="b2", nu=0.05, b=bA, rtol=1e-11)  # several restart cycles
    srv.submit(A)
    assert A.done.wait(120) and late.done.wait(120)
    srv.shutdown()
    assert sent and A.error is None and late.error is None
    assert late.joined_running and late.batch == 2 and A.iters > 20
    err = np.linalg.norm(late.x - solo.x) / np.linalg.norm(solo.x)
    print(f"  solo {solo.iters} its, admitted mid-batch {late.iters} its, rel diff {err:.2e}; A {A.iters} its")
    assert abs(late.iters - solo.iters) <= 1 and err <= tol
    check_residual(late, MESHES["b2"])
    check_residual(A, MESHES["b2"])
