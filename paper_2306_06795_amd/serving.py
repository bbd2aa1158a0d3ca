"""Continuous-batching request loop for Stokes solves on one GPU.

A request names a mesh, a viscosity nu and a right-hand side.  Each mesh is
analysed once on the host (Algorithm 1, patches) at registration.  Its device
half (operators, patch factors, coarse inverse, solver workspace for
``max_batch`` right-hand sides) is uploaded when a request for it is admitted
and stays resident until the HBM budget needs the room.

Viscosity: the hierarchy is built for nu = 1.  With
S = diag(sqrt(nu) I_u, I_p / sqrt(nu)) the free block of the nu operator is
S K_1 S, so a request is solved as c = S^-1 b (S b on Dirichlet rows),
K_1 y = c, x = S^-1 y (the scalings applied on the host when a request enters
and leaves its slot).  Residuals relate by
||b - K_nu x|| <= max(sqrt(nu), 1/sqrt(nu)) ||c - K_1 y|| and
||c|| <= max(sqrt(nu), 1/sqrt(nu)) ||b||, so solving the scaled system to
rtol / max(nu, 1/nu) bounds the relative residual of the nu system by rtol.

Scheduling (continuous batching at slot level): each worker thread owns a
stream.  It takes the mesh whose oldest waiting request is the oldest overall
(among meshes that are idle and fit the budget) and runs that mesh's slots:
up to ``max_batch`` right-hand sides advance together, one FGMRES restart
cycle per step (mas_solve_step), each column with its own tolerance and its
own iterate, so a result does not depend on its batch-mates.  Between steps,
every column that has converged is returned at once and its slot is given to
the next waiting request of the mesh, which starts from zero while the others
continue; the worker leaves the mesh when its slots and queue are empty.
Batches of different meshes run at the same time on their own streams.  Idle
hierarchies are released least-recently-used to admit a new one (their host
analysis stays, so re-admission costs one upload and factorisation); a mesh
whose hierarchy does not fit the budget even alone is refused at submission.
"""
from __future__ import annotations

import math
import threading
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import mas


@dataclass
class Request:
    mesh: str
    nu: float
    b: np.ndarray
    rtol: float = 1e-8
    t_arrival: float = 0.0
    t_start: float = 0.0
    t_done: float = 0.0
    x: np.ndarray | None = None
    iters: int = 0
    relres: float = float("nan")
    batch: int = 0           # most right-hand sides that advanced together with this one
    joined_running: bool = False  # admitted into a batch whose other slots were already iterating
    error: str | None = None
    done: threading.Event = field(default_factory=threading.Event)

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrival


class _Mesh:
    def __init__(self, key, problem, handle, est_bytes):
        self.key = key
        self.n0 = problem.K0.shape[0]
        self.nvel = int(np.count_nonzero(np.asarray(problem.field0) < problem.dim))
        self.dir = np.nonzero(np.asarray(problem.dir0))[0]
        self.handle: mas.Handle = handle  # analysed; on the device while resident
        self.est_bytes = est_bytes        # device bytes (estimate until the first upload)
        self.resident = False
        self.busy = False
        self.last_used = 0.0
        self.queue: deque[Request] = deque()


def estimate_device_bytes(info: dict, precision: int, max_batch: int) -> int:
    """Upper estimate of the device memory of a handle from its host analysis."""
    s = 4 if precision == mas.MAS_FP32 else 8
    L = info["n_levels"]
    R = max_batch
    # level operators (CSR + a sliced-ELL copy) and per-level vectors
    ops = sum(info["nnz"][l] * 2 * (s + 4) + info["n"][l] * (8 + 4 * s * R) for l in range(L))
    ops += sum(info["p_nnz"]) * 2 * 2 * (s + 4)  # P and P^T
    # patch factors, DoF lists, inverse maps, patch outputs
    pat = sum(info["factor_entries"][l] * s + info["patch_dofs"][l] * (16 + s * (1 + R)) for l in range(L))
    coarse = info["coarse_n"] ** 2 * 8 * 2
    # FP64 K0 copy and FGMRES(20) basis V, Z for R right-hand sides
    n0 = info["n"][0]
    k0 = info["nnz"][0] * 2 * 12 + n0 * 8 * (2 * 20 + 4) * R
    return int(1.3 * (ops + pat + coarse + k0)) + (16 << 20)


class TorchDevice:
    """Streams and device arrays of the server, through torch (one GPU)."""

    def __init__(self):
        import torch
        self.torch = torch

    def new_stream(self):
        return self.torch.cuda.Stream()  # default priority

    def stream_handle(self, stream):
        return stream.cuda_stream

    def on_stream(self, stream):
        return self.torch.cuda.stream(stream)

    def upload(self, a: np.ndarray):
        return self.torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")

    def empty_like(self, t):
        return self.torch.empty_like(t)

    def download(self, t) -> np.ndarray:
        return t.cpu().numpy()

    def stack_cols(self, cols):
        """n x k contiguous array (right-hand side fastest) from k vectors."""
        return self.torch.stack(cols, 1).contiguous()

    def column(self, a, k):
        return a[:, k].contiguous()

    def zeros(self, n):
        return self.torch.zeros(n, dtype=self.torch.float64, device="cuda:0")


def _analysed_handle(problem, par):
    return mas.Handle(problem, par, analyze_only=True)


class StokesServer:
    """``device`` (streams, arrays) and ``handle_factory(problem, params)``
    (an analysed handle with upload/release/info/solve_step/close) default to
    torch on cuda:0 and libmas; other implementations serve to test the
    scheduling on the host.  ``params``: overrides of the libmas parameters,
    a dict for every mesh or a function of the problem giving one (e.g. a
    different relaxation for 3D meshes)."""

    def __init__(self, hbm_budget: int, max_batch: int = 32, workers: int = 4,
                 precision: int = mas.MAS_FP32, params=None, device=None, handle_factory=None,
                 max_it: int = 1000, on_step=None):
        self.device = device
        self.handle_factory = handle_factory or _analysed_handle
        self.budget = int(hbm_budget)
        self.max_batch = int(max_batch)
        self.precision = precision
        self.params = params or {}
        self.meshes: dict[str, _Mesh] = {}
        self.cv = threading.Condition()
        self.stop = False
        self.paused = False
        self.resident = 0
        self.peak_resident = 0
        self.uploads = 0
        self.evictions = 0
        self.batches = 0
        self.batch_sizes: list[int] = []
        self.n_workers = workers
        self.threads: list[threading.Thread] = []
        self.max_it = int(max_it)
        self.on_step = on_step  # called as on_step(mesh_key, requests) after every step (tests)

    # ------------------------------------------------------------------ API
    def add_mesh(self, key: str, problem, device_bytes: int | None = None) -> int:
        """Analyse a mesh (host only) and register it; returns the device-byte
        figure used for admission: ``device_bytes`` when the caller knows it
        (from an earlier upload with the same parameters), else an upper
        estimate from the analysis.  The exact size replaces it at the first
        upload."""
        disc = mas.MAS_SV if problem.disc == "SV" else mas.MAS_TH
        extra = self.params(problem) if callable(self.params) else self.params
        par = mas.default_params(problem.dim, disc, precision=self.precision, nrhs_max=self.max_batch, **extra)
        h = self.handle_factory(problem, par)
        est = int(device_bytes) if device_bytes else estimate_device_bytes(h.info(), self.precision,
                                                                             self.max_batch)
        with self.cv:
            old = self.meshes.get(key)
            if old is not None:
                if old.busy or old.queue or old.resident:
                    h.close()
                    raise RuntimeError(f"mesh {key} is in use")
                old.handle.close()
            self.meshes[key] = _Mesh(key, problem, h, est)
        return est

    def start(self):
        if self.device is None:
            self.device = TorchDevice()
        self.threads = [threading.Thread(target=self._worker, daemon=True) for _ in range(self.n_workers)]
        for t in self.threads:
            t.start()

    def submit(self, req: Request) -> Request:
        req.t_arrival = time.perf_counter()
        with self.cv:
            m = self.meshes.get(req.mesh)
            err = None
            if m is None:
                err = "unknown mesh"
            elif m.est_bytes > self.budget:
                err = "hierarchy does not fit the HBM budget"
            elif np.shape(req.b) != (m.n0,):
                err = "right-hand side has the wrong length"
            elif not (req.nu > 0.0 and math.isfinite(req.nu)):
                err = "viscosity must be positive"
            if err is not None:
                req.error = err
                req.t_done = req.t_arrival
                req.done.set()
                return req
            m.queue.append(req)
            self.cv.notify()
        return req

    def pause(self):
        """Hold new batches (running ones finish); requests keep queueing."""
        with self.cv:
            self.paused = True

    def resume(self):
        with self.cv:
            self.paused = False
            self.cv.notify_all()

    def shutdown(self):
        with self.cv:
            self.stop = True
            self.cv.notify_all()
        for t in self.threads:
            t.join()
        self.threads = []
        for m in self.meshes.values():
            m.handle.close()
        self.meshes.clear()

    def stats(self) -> dict:
        with self.cv:
            return dict(resident_bytes=self.resident, peak_resident_bytes=self.peak_resident, uploads=self.uploads,
                        evictions=self.evictions, batches=self.batches,
                        mean_batch=float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0)

    # ------------------------------------------------------------ internals
    def _fits(self, m: _Mesh) -> bool:
        """Make room for m (evicting idle residents, least recently used first).
        Called with the lock held."""
        if m.resident or self.resident + m.est_bytes <= self.budget:
            return True
        idle = sorted((o for o in self.meshes.values() if o.resident and not o.busy), key=lambda o: o.last_used)
        need = self.resident + m.est_bytes - self.budget
        if sum(o.est_bytes for o in idle) < need:
            return False
        for o in idle:
            if self.resident + m.est_bytes <= self.budget:
                break
            o.handle.release()
            o.resident = False
            self.resident -= o.est_bytes
            self.evictions += 1
        return True

    def _pick(self):
        """Idle mesh with the oldest waiting request that fits (lock held)."""
        if self.paused:
            return None
        cands = sorted((m for m in self.meshes.values() if m.queue and not m.busy),
                       key=lambda m: m.queue[0].t_arrival)
        for m in cands:
            if self._fits(m):
                return m
        return None

    def _worker(self):
        dev = self.device
        stream = dev.new_stream()
        while True:
            with self.cv:
                while True:
                    if self.stop:
                        return
                    m = self._pick()
                    if m is not None:
                        break
                    self.cv.wait(0.05)
                m.busy = True
                if not m.resident:
                    self.resident += m.est_bytes  # reserved while uploading
                    self.peak_resident = max(self.peak_resident, self.resident)
            try:
                with dev.on_stream(stream):
                    self._run_slots(m, dev, stream)
            finally:
                with self.cv:
                    if not m.resident and m.handle.info()["device_bytes"] == 0:
                        self.resident -= m.est_bytes  # upload failed
                    m.busy = False
                    m.last_used = time.perf_counter()
                    self.cv.notify_all()

    def _fail(self, reqs, err):
        t = time.perf_counter()
        for r in reqs:
            r.error = err
            r.t_done = t
            r.done.set()

    def _scale_in(self, m: _Mesh, r: Request) -> np.ndarray:
        """c = S^-1 b on free rows, S b on Dirichlet rows (S = diag(sqrt(nu) I_u, I_p / sqrt(nu)))."""
        c = np.array(r.b, dtype=np.float64)
        c[:m.nvel] *= 1.0 / math.sqrt(r.nu)
        c[m.nvel:] *= math.sqrt(r.nu)
        c[m.dir] = np.asarray(r.b, dtype=np.float64)[m.dir] * math.sqrt(r.nu)
        return c

    def _scale_out(self, m: _Mesh, r: Request, y: np.ndarray) -> np.ndarray:
        """x = S^-1 y."""
        x = np.array(y, dtype=np.float64)
        x[:m.nvel] *= 1.0 / math.sqrt(r.nu)
        x[m.nvel:] *= math.sqrt(r.nu)
        return x

    def _run_slots(self, m: _Mesh, dev, stream):
        """Serve mesh m until its slots and queue are empty: admit waiting
        requests into free slots, advance every slot by one restart cycle,
        return the converged ones."""
        st = dev.stream_handle(stream)
        h = m.handle
        if not m.resident:
            try:
                h.upload(stream=st)
            except Exception as e:  # the mesh's waiting requests fail, the server keeps going
                with self.cv:
                    waiting = list(m.queue)
                    m.queue.clear()
                self._fail(waiting, str(e))
                return
            nbytes = h.info()["device_bytes"]
            with self.cv:
                self.resident += nbytes - m.est_bytes
                self.peak_resident = max(self.peak_resident, self.resident)
                m.est_bytes = nbytes  # exact from now on
                m.resident = True
                self.uploads += 1
        active: list = []  # [request, b column, x column, fresh]
        Bd = Xd = None     # stacked columns of the current slot set (rebuilt when it changes)
        while True:
            with self.cv:
                new = []
                # a new batch takes every waiting request of the mesh; a running one
                # takes more only while no idle mesh holds an older request
                while (len(active) + len(new) < self.max_batch and m.queue and not self.stop
                       and (not active or self._may_admit(m))):
                    new.append(m.queue.popleft())
            try:
                t0 = time.perf_counter()
                running = bool(active)  # slots already iterating when these requests enter
                for r in new:
                    r.t_start = t0
                    r.joined_running = running
                    active.append([r, dev.upload(self._scale_in(m, r)), dev.zeros(m.n0), True])
                if not active:
                    return
                nr = len(active)
                if new or Bd is None:
                    Bd = dev.stack_cols([a[1] for a in active])
                    Xd = dev.stack_cols([a[2] for a in active])
                new = []
                tols = [a[0].rtol / max(a[0].nu, 1.0 / a[0].nu) for a in active]
                _, info = h.solve_step(Bd, Xd, tols, [a[3] for a in active], cycles=1, nrhs=nr, stream=st)
                keep = []
                t1 = time.perf_counter()
                for k, a in enumerate(active):
                    r = a[0]
                    r.iters += info[k]["iters"]
                    r.batch = max(r.batch, nr)
                    a[3] = False
                    if info[k]["converged"] or r.iters >= self.max_it:
                        r.x = self._scale_out(m, r, dev.download(dev.column(Xd, k)))
                        r.relres = info[k]["relres"]
                        if not info[k]["converged"]:
                            r.error = "not converged"
                        r.t_done = t1
                        r.done.set()
                    else:
                        keep.append(k)
                if len(keep) < nr:  # some slots freed: the remaining columns, with their iterates
                    active = [[active[k][0], active[k][1], dev.column(Xd, k), False] for k in keep]
                    Bd = None
            except Exception as e:  # the slots fail, the server keeps going
                self._fail([a[0] for a in active if not a[0].done.is_set()] + new, str(e))
                return
            with self.cv:
                self.batches += 1
                self.batch_sizes.append(nr)
            if self.on_step is not None:
                self.on_step(m.key, [a[0] for a in active])

    def _may_admit(self, m: _Mesh) -> bool:
        """Whether no idle mesh holds a request older than m's next one (oldest
        first across meshes; lock held)."""
        head = m.queue[0].t_arrival
        for o in self.meshes.values():
            if o is not m and o.queue and not o.busy and o.queue[0].t_arrival < head:
                return False
        return True


def latency_percentiles(reqs, qs=(50, 99)) -> dict:
    lat = np.array([r.latency for r in reqs if r.error is None])
    if lat.size == 0:
        return {f"p{q}_ms": None for q in qs}
    return {f"p{q}_ms": float(np.percentile(lat, q) * 1e3) for q in qs}
