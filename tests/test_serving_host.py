"""Host logic of the serving loop, on the CPU: batching by mesh in arrival
order, one tolerance per request, viscosity scaling (reading: K_nu = S K_1 S on
the free block, identity Dirichlet rows), HBM-budget admission with
least-recently-used eviction, refusals, failures that stay inside their
batch, and slot-level admission (requests join a running batch between steps,
converged ones leave at once).  The device is replaced by host arrays and the handle by an exact
least-squares solve of the nu = 1 system, so these tests check the server, not
the GPU path (tests/test_gpu_serving.py does that)."""
import contextlib
import threading

import numpy as np

from paper_2306_06795_amd import serving
from paper_2306_06795_amd.inputs import make_problem, random_rhs


class HostDevice:
    def new_stream(self):
        return None

    def stream_handle(self, stream):
        return None

    def on_stream(self, stream):
        return contextlib.nullcontext()

    def upload(self, a):
        return np.array(a, dtype=np.float64)

    def empty_like(self, t):
        return np.empty_like(t)

    def download(self, t):
        return t

    def stack_cols(self, cols):
        return np.ascontiguousarray(np.stack(cols, 1))

    def column(self, a, k):
        return np.ascontiguousarray(a[:, k])

    def zeros(self, n):
        return np.zeros(n)


class ExactHandle:
    """Stands in for an analysed libmas handle: solves K_1 y = c exactly."""

    log: list = []
    fail_solve: set = set()
    fail_upload: set = set()
    sizes: dict = {}
    lock = threading.Lock()

    def __init__(self, problem, par, key):
        self.P = problem
        self.key = key
        self.K = problem.K0.toarray()
        self.nu0 = problem.meta["n_u"]
        self.dir = np.nonzero(problem.dir0)[0]
        self.on = False

    def info(self):
        L = 2
        return dict(n_levels=L, n=[self.K.shape[0]] * L, nnz=[1000] * L, p_nnz=[0] * L,
                    factor_entries=[100] * L, patch_dofs=[100] * L, coarse_n=10,
                    device_bytes=self.sizes.get(self.key, 1 << 20) if self.on else 0)

    def upload(self, stream=None):
        if self.key in self.fail_upload:
            raise RuntimeError("out of memory")
        self.on = True

    def release(self):
        self.on = False

    def close(self):
        self.on = False

    def solve_step(self, b, x, rtol, fresh, cycles=1, nrhs=1, stream=None):
        """One step converges every column: its exact solution."""
        assert self.on, "solve on a released handle"
        if self.key in self.fail_solve:
            raise RuntimeError("device fault (test)")
        tols = list(np.atleast_1d(rtol))
        with self.lock:
            self.log.append((self.key, nrhs, tols))
        B = b.reshape(-1, nrhs)
        X = x.reshape(-1, nrhs)
        for k in range(nrhs):
            X[:, k] = np.linalg.lstsq(self.K, B[:, k], rcond=None)[0]
        return 0, [dict(iters=3, converged=True, relres=0.0) for _ in range(nrhs)]


MESHES = {"a": 6, "b": 8, "c": 5}


def mesh(n, nu=1.0):
    return make_problem(dim=2, n=n, disc="TH", forcing="gaussian", bc="zero", nu=nu, seed=1)


def server(budget=1 << 40, sizes=None, workers=2, max_batch=16):
    ExactHandle.log = []
    ExactHandle.fail_solve = set()
    ExactHandle.fail_upload = set()
    ExactHandle.sizes = dict(sizes or {})
    srv = serving.StokesServer(budget, max_batch=max_batch, workers=workers, device=HostDevice(),
                               handle_factory=None)
    probs = {}
    for k, n in MESHES.items():
        probs[k] = mesh(n)
        srv.handle_factory = (lambda key: (lambda P, par: ExactHandle(P, par, key)))(k)
        srv.add_mesh(k, probs[k], device_bytes=(sizes or {}).get(k))
    return srv, probs


def req(probs, key, nu, seed, rtol=1e-8):
    return serving.Request(mesh=key, nu=nu, b=random_rhs(probs[key], np.random.default_rng(seed)), rtol=rtol)


def test_viscosity_scaling_gives_the_nu_solution():
    srv, probs = server()
    srv.start()
    reqs = [req(probs, k, nu, i) for i, (k, nu) in enumerate([("a", 0.01), ("a", 0.3), ("b", 1.0), ("c", 0.05)])]
    for r in reqs:
        srv.submit(r)
    for r in reqs:
        assert r.done.wait(60)
    srv.shutdown()
    for r in reqs:
        assert r.error is None
        K = mesh(MESHES[r.mesh], nu=r.nu).K0
        res = np.linalg.norm(r.b - K @ r.x) / np.linalg.norm(r.b)
        assert res <= 1e-10, (r.mesh, r.nu, res)


def test_batches_by_mesh_in_arrival_order_with_own_tolerances():
    srv, probs = server(workers=1)
    srv.start()
    srv.pause()
    plan = [("a", 0.01), ("b", 0.5), ("a", 1.0), ("a", 0.2), ("b", 0.02), ("c", 1.0)]
    reqs = [req(probs, k, nu, i) for i, (k, nu) in enumerate(plan)]
    for r in reqs:
        srv.submit(r)
    srv.resume()
    for r in reqs:
        assert r.done.wait(60)
    srv.shutdown()
    log = ExactHandle.log
    # one worker: the mesh of the oldest waiting request goes first, with all its waiting requests
    assert [(k, n) for k, n, _ in log] == [("a", 3), ("b", 2), ("c", 1)]
    want = {k: [1e-8 / max(nu, 1 / nu) for kk, nu in plan if kk == k] for k in MESHES}
    for k, n, tols in log:
        assert np.allclose(tols, want[k]), (k, tols, want[k])
    assert [r.batch for r in reqs] == [3, 2, 3, 3, 2, 1]


def test_budget_admission_evicts_least_recently_used():
    srv, probs = server(budget=100, sizes={"a": 40, "b": 40, "c": 40}, workers=1)
    srv.start()
    for i, k in enumerate(["a", "b", "c", "a", "b"]):
        r = srv.submit(req(probs, k, 1.0, i))
        assert r.done.wait(60) and r.error is None
    st = srv.stats()
    resident = sorted(k for k, m in srv.meshes.items() if m.resident)
    srv.shutdown()
    # c evicts a (least recent), a evicts b, b evicts c
    assert st["evictions"] == 3 and st["uploads"] == 5, st
    assert resident == ["a", "b"]
    assert st["peak_resident_bytes"] <= 100


def test_refusals():
    srv, probs = server(budget=100, sizes={"a": 40, "b": 400, "c": 40})
    srv.start()
    r1 = srv.submit(req(probs, "b", 1.0, 0))
    r2 = srv.submit(serving.Request(mesh="zz", nu=1.0, b=np.zeros(3)))
    r3 = srv.submit(serving.Request(mesh="a", nu=1.0, b=np.zeros(7)))
    r4 = srv.submit(serving.Request(mesh="a", nu=-1.0, b=random_rhs(probs["a"], np.random.default_rng(0))))
    srv.shutdown()
    assert "budget" in r1.error
    assert "unknown" in r2.error
    assert "length" in r3.error
    assert "viscosity" in r4.error


def test_failures_stay_in_their_batch():
    srv, probs = server(workers=2)
    ExactHandle.fail_solve = {"b"}
    ExactHandle.fail_upload = {"c"}
    srv.start()
    reqs = [req(probs, k, 0.5, i) for i, k in enumerate(["a", "b", "c", "a", "b", "a"])]
    for r in reqs:
        srv.submit(r)
    for r in reqs:
        assert r.done.wait(60)
    st = srv.stats()
    srv.shutdown()
    for r in reqs:
        if r.mesh == "a":
            assert r.error is None and r.x is not None
        elif r.mesh == "b":
            assert "fault" in r.error
        else:
            assert "memory" in r.error
    # the failed upload gave its reservation back; a and b stay resident
    assert st["resident_bytes"] == 2 * (1 << 20), st


def test_parameters_may_depend_on_the_mesh():
    """params as a function of the problem: each mesh's analysis gets its own."""
    seen = {}

    def factory(key):
        def make(P, par):
            seen[key] = (par.relax, par.nrhs_max)
            return ExactHandle(P, par, key)
        return make

    srv = serving.StokesServer(1 << 40, max_batch=8, workers=1, device=HostDevice(),
                               params=lambda P: {"relax": 2} if P.meta["n"] == 8 else {})
    for k, n in MESHES.items():
        srv.handle_factory = factory(k)
        srv.add_mesh(k, mesh(n))
    srv.shutdown()
    assert seen == {"a": (0, 8), "b": (2, 8), "c": (0, 8)}


class CountingHandle(ExactHandle):
    """A column needs b[row] steps: every step adds 1 to its iterate (from 0
    when fresh) and reports 20 iterations; it converges once x[row] >= b[row]."""

    row = 0

    def solve_step(self, b, x, rtol, fresh, cycles=1, nrhs=1, stream=None):
        with self.lock:
            self.log.append((self.key, nrhs, list(fresh)))
        B = b.reshape(-1, nrhs)
        X = x.reshape(-1, nrhs)
        info = []
        for k in range(nrhs):
            if fresh[k]:
                X[:, k] = 0.0
            X[:, k] += 1.0
            info.append(dict(iters=20, converged=bool(X[self.row, k] >= B[self.row, k]), relres=0.0))
        return 0, info


def test_requests_join_a_running_batch_and_leave_when_converged():
    """Two slots: A (3 steps) and B (1 step) start together; B leaves after the
    first step and C takes its slot while A keeps iterating (C starts from
    zero, A does not restart); A finishes last after its three steps."""
    P = mesh(4)
    n0 = P.n0
    srv = serving.StokesServer(1 << 40, max_batch=2, workers=1, device=HostDevice(),
                               handle_factory=lambda P_, par: CountingHandle(P_, par, "m"))
    srv.add_mesh("m", P)
    CountingHandle.log = []
    srv.pause()
    srv.start()

    row = int(np.nonzero(~P.dir0)[0][0])  # a free velocity row
    CountingHandle.row = row

    def rhs(steps):
        b = np.zeros(n0)
        b[row] = steps
        return b

    A, B, C = (serving.Request(mesh="m", nu=1.0, b=rhs(s)) for s in (3, 1, 1))
    for r in (A, B, C):
        srv.submit(r)
    srv.resume()
    for r in (A, B, C):
        assert r.done.wait(60)
    srv.shutdown()
    assert all(r.error is None for r in (A, B, C))
    log = CountingHandle.log
    assert [(n, f) for _, n, f in log] == [(2, [True, True]), (2, [False, True]), (1, [False])]
    assert (A.iters, B.iters, C.iters) == (60, 20, 20)
    assert C.joined_running and not A.joined_running and not B.joined_running
    assert B.t_done <= C.t_done <= A.t_done
    assert A.x[row] == 3.0 and C.x[row] == 1.0
    assert (A.batch, B.batch, C.batch) == (2, 2, 2)
