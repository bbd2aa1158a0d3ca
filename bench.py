"""Benchmark: Stokes solves/s to 1e-8 relative residual on one MI355X.

Workload (default): 3D Taylor-Hood P2/P1 on the unit cube, 32^3 cubes each
split into six tetrahedra (859,812 unknowns), seeded smooth forcing,
homogeneous Dirichlet velocity, the defect-correction preconditioner with
additive Vanka V(1,1) on every level but the coarsest, FP64 cycle (the plain
GPU form), FGMRES(20) to a 1e-8 relative residual.  The same solves with the
FP32 cycle (FP64 FGMRES, patch factorisation and coarse solve) are reported
beside it.  A step is one full solve from x0 = 0 with the right-hand side
already resident in HBM; setup is outside the timed region.  Prints one JSON
line (rank 0).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
WORKLOADS = {
    "th2d_256": "2D Taylor-Hood P2/P1, 256x256 squares split into triangles, interior vertices jittered "
                "U(-0.2h,0.2h), lid-driven cavity + Gaussian forcing",
    "th3d_32": "3D Taylor-Hood P2/P1, 32^3 cubes split into 6 tetrahedra, smooth random forcing, "
               "homogeneous Dirichlet",
    "th2d_16": "2D Taylor-Hood P2/P1, 16x16, manufactured solution",
    "sv2d_128x64": "2D Scott-Vogelius P2/P1disc on the Alfeld refinement of 128x128, 64 Gaussian right-hand "
                   "sides solved together",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="th3d_32")
    ap.add_argument("--relax", default="vanka", choices=["vanka", "dlsc", "vanka-dlsc"])
    ap.add_argument("--schedule", default="all", choices=["all", "skip1", "skip0", "ho"],
                    help="DC-all / DC-skip1 / DC-skip0, or HO-AMG (Algorithm 1 applied to K0)")
    ap.add_argument("--krylov-its", type=int, default=0,
                    help="FGMRES-wrapped Vanka relaxation with this many iterations (0: stationary sweeps)")
    ap.add_argument("--dlsc-amg", type=int, default=0,
                    help="DLSC continuity/pressure stages by one SA V-cycle with this many Jacobi sweeps (0: Chebyshev)")
    ap.add_argument("--theta", type=float, default=None,
                    help="strength-of-connection threshold of Algorithm 1 (default: the library's)")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--patch-kernel", type=int, default=None, choices=[0, 1, 2, 3, 4, 5],
                    help="kernel of the patches outside the buckets (0: timed at setup)")
    ap.add_argument("--share-blocks", type=int, default=None, choices=[0, 1],
                    help="0: one A^-1 per velocity component even where the components' blocks are identical")
    ap.add_argument("--bucket-min", type=int, default=None,
                    help="fewest patches of one shape that get a thread-per-patch bucket (default: the library's)")
    ap.add_argument("--mesh-n", type=int, default=None, help="another mesh size of the chosen workload family")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--no-companion", action="store_true",
                    help="skip the FP32-cycle solves reported beside an FP64 run")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-its", type=int, default=1)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="copy this many MiB with one plain device copy first (the scale of HBM byte counters)")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-load", type=float, default=0.8, help="arrival rate / closed-loop capacity")
    ap.add_argument("--serve-sweep", type=float, nargs="*", default=[])
    ap.add_argument("--serve-batch", type=int, default=32)
    ap.add_argument("--serve-workers", type=int, default=4)
    ap.add_argument("--serve-small-gb", type=float, default=0.0)
    ap.add_argument("--serve-baseline-open", action="store_true")
    ap.add_argument("--serve-relax-3d", default="vanka-dlsc", choices=["vanka", "vanka-dlsc"],
                    help="relaxation of the 3D meshes of the serving stream (2D meshes: Vanka)")
    return ap.parse_args()


def measured_traffic(config, precision, relax, kind):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary of this workload (FETCH_SIZE + WRITE_SIZE, scaled by a copy
    kernel of known size), or None when there is none or the kernel sources
    changed since the counters were taken."""
    import glob
    import hashlib
    hsh = hashlib.sha256()
    for fn in ("paper_2306_06795_amd/csrc/kernels.hpp", "paper_2306_06795_amd/csrc/mas.hip"):
        with open(os.path.join(ROOT, fn), "rb") as f:
            hsh.update(f.read())
    want = {"workload": config, "precision": precision, "relax": relax, "kind": kind, "sources": hsh.hexdigest()}
    for path in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        for line in open(path):
            if not line.startswith("traffic:"):
                continue
            kv = dict(t.split("=", 1) for t in line.split()[1:])
            if all(kv.get(k) == v for k, v in want.items()):
                return float(kv["bytes_per_launch"])
    return None


def stream_copy_gbs(torch, dev, mib=1024, reps=10):
    """Device-to-device copy bandwidth (read + write bytes per second, GB/s)."""
    src = torch.ones(mib << 18, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        dst.copy_(src)
    e1.record(st)
    torch.cuda.synchronize()
    gbs = 2.0 * (mib << 20) * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    return gbs


# Workloads whose oracle run would not fit the baseline's bounded sample (the
# 32^3 oracle re-factors ~4,300 dense 725 x 725 coarse patch matrices per sweep
# and needs tens of GB for them): the oracle is timed on a smaller mesh of the
# same family and its time per iteration scaled by the number of unknowns.
CPU_SAMPLE_MESH = {"th3d_32": ("th3d_16", dict(dim=3, n=16, disc="TH", forcing="smooth", bc="zero", seed=3))}


def cpu_baseline(prob, config, its_gpu, sample_its, relax="vanka", krylov_its=0, schedule="all", dlsc_amg=0,
                 theta=None):
    """The oracle on the host: setup untimed, then ``sample_its`` FGMRES
    iterations timed (first right-hand side) and scaled to one full solve of
    the workload."""
    from oracle import dc, fgmres

    from paper_2306_06795_amd.inputs import make_problem
    over = {} if theta is None else {"theta": theta}
    sub = CPU_SAMPLE_MESH.get(config)
    sprob, scale, where = prob, 1.0, "the same system"
    if sub is not None:
        sprob = make_problem(**sub[1])
        scale = prob.n0 / sprob.n0
        where = (f"{sub[0]} ({sprob.n0} unknowns, the same mesh family), time per iteration scaled by the "
                 f"unknown count x{scale:.1f}")
    pre = dc.DCPreconditioner(sprob, dc.default_params(sprob, relax, krylov_its=krylov_its, schedule=schedule,
                                                           dlsc_amg=dlsc_amg, **over))
    b0 = sprob.b if sprob.b.ndim == 1 else np.ascontiguousarray(sprob.b[:, 0])
    pre.apply(b0)  # untimed: builds the oracle's dense patch matrices once
    t0 = time.perf_counter()
    fgmres.fgmres(lambda v: sprob.K0 @ v, pre.apply, b0, rtol=0.0, restart=20, max_it=sample_its)
    dt = time.perf_counter() - t0
    per_it = dt / sample_its * scale
    cores = len(os.sched_getaffinity(0))
    return {"value": 1.0 / (per_it * its_gpu), "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": f"{sample_its} oracle FGMRES iteration(s) on {where} ({dt:.1f} s), scaled to the "
                      f"{its_gpu} iterations of one solve; oracle setup untimed"}


def timed_solves(torch, h, b, x, steps, warmup, rtol, nrhs):
    """``warmup`` untimed solves, then ``steps`` timed ones bracketed by device
    synchronisations; returns (seconds, iterations per solve, status, info)."""
    for _ in range(warmup):
        h.solve(b, x, rtol=rtol, nrhs=nrhs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    rc, sinfo = None, None
    for _ in range(steps):
        rc, sinfo = h.solve(b, x, rtol=rtol, nrhs=nrhs)
        iters.append(max(i["iters"] for i in sinfo))
    torch.cuda.synchronize()
    return time.perf_counter() - t0, iters, rc, sinfo


def vcycle_time(torch, h, n, nrhs, dev, nrep=20):
    """(mean, median, min) ms of one preconditioner application, HIP events on
    the stream the cycle runs on."""
    r = torch.randn(n, dtype=torch.float64, device=dev)
    z = torch.empty_like(r)
    h.apply(r, z, nrhs=nrhs)
    st = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(nrep + 1)]
    ev[0].record(st)
    for k in range(nrep):
        h.apply(r, z, nrhs=nrhs)
        ev[k + 1].record(st)
    torch.cuda.synchronize()
    per = sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(nrep))
    return ev[0].elapsed_time(ev[nrep]) / nrep, per[nrep // 2], per[0]


def true_relres(prob, xx):
    bb = prob.b.reshape(prob.n0, -1)
    return float(max(np.linalg.norm(bb[:, k] - prob.K0 @ xx[:, k]) / np.linalg.norm(bb[:, k])
                     for k in range(bb.shape[1])))


def rel_err(xx, ref):
    return float(max(np.linalg.norm(xx[:, k] - ref[:, k]) / np.linalg.norm(ref[:, k]) for k in range(ref.shape[1])))


def run_stream(srv, stream, rhs, rate, serving):
    """Submit the stream with Poisson arrivals at ``rate`` requests/s (0 = all
    at once, closed loop) and wait for every result."""
    reqs = [serving.Request(mesh=q["mesh"], nu=q["nu"], b=rhs[i]) for i, q in enumerate(stream)]
    t0 = time.perf_counter()
    t_next = t0
    for q, r in zip(stream, reqs):
        if rate > 0:
            t_next += q["gap"] / rate
            dt = t_next - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
        srv.submit(r)
    for r in reqs:
        assert r.done.wait(600), "request not finished after 600 s"
    t1 = max(r.t_done for r in reqs)
    bad = [r.error for r in reqs if r.error is not None]
    assert not bad, f"{len(bad)} requests failed: {bad[:3]}"
    out = {"solves_per_s": len(reqs) / (t1 - t0), "wall_s": t1 - t0,
           "mean_batch": float(np.mean([r.batch for r in reqs])),
           "iters_mean": float(np.mean([r.iters for r in reqs]))}
    out.update(serving.latency_percentiles(reqs))
    return out, reqs


def bench_serve(a):
    """Serving stream: 512 requests with Poisson arrivals over eight meshes
    (2D Taylor-Hood 32^2..256^2, 3D 8^3..24^3), viscosity log-uniform in
    [1e-2, 1], Gaussian forcing, hierarchies resident on the device."""
    import torch

    from paper_2306_06795_amd import mas, serving
    from paper_2306_06795_amd.inputs import SERVE_MESHES, make_serve_mesh, random_rhs, serve_stream

    t0 = time.perf_counter()
    probs = {f"th{d}d_{n}": make_serve_mesh(d, n) for d, n in SERVE_MESHES}
    stream = serve_stream(a.serve_requests, seed=5)
    rhs = [random_rhs(probs[q["mesh"]], np.random.default_rng(q["rhs_seed"])) for q in stream]
    t_gen = time.perf_counter() - t0
    full = int(torch.cuda.get_device_properties(0).total_memory * 0.8)

    def policy(P):
        if P.dim == 3 and a.serve_relax_3d == "vanka-dlsc":
            return {"relax": mas.MAS_RELAX_VANKA_DLSC}
        return {}

    def server(budget, precision, max_batch, workers):
        srv = serving.StokesServer(budget, max_batch=max_batch, workers=workers, precision=precision, params=policy)
        for k, P in probs.items():
            srv.add_mesh(k, P)
        srv.start()
        return srv

    def warm(srv):  # first upload of every hierarchy, outside the timed streams
        for k, P in probs.items():
            r = srv.submit(serving.Request(mesh=k, nu=1.0, b=random_rhs(P, np.random.default_rng(0))))
            assert r.done.wait(600), "warm-up request not finished after 600 s"
            assert r.error is None, r.error

    t0 = time.perf_counter()
    srv = server(full, mas.MAS_FP32, a.serve_batch, a.serve_workers)
    try:  # the worker threads must be joined before the interpreter exits, also on failure
        warm(srv)
        t_setup = time.perf_counter() - t0
        print(f"[serve] {len(stream)} requests, inputs {t_gen:.1f}s, analysis+upload {t_setup:.1f}s, "
              f"resident {srv.stats()['resident_bytes'] / 2**30:.2f} GiB", file=sys.stderr, flush=True)
        closed, _ = run_stream(srv, stream, rhs, 0.0, serving)
        cap = closed["solves_per_s"]
        print(f"[serve] closed loop: {closed}", file=sys.stderr, flush=True)
        rate = a.serve_load * cap
        main_run, reqs = run_stream(srv, stream, rhs, rate, serving)
        print(f"[serve] open loop at {rate:.1f}/s: {main_run}", file=sys.stderr, flush=True)
        sweep = {}
        for f in a.serve_sweep:
            sweep[f"{f:g}x"], _ = run_stream(srv, stream, rhs, f * cap, serving)
            print(f"[serve] {f:g}x: {sweep[f'{f:g}x']}", file=sys.stderr, flush=True)
        st_full = srv.stats()
    finally:
        srv.shutdown()
    # forced small budget: evictions and re-uploads inside the stream
    small = None
    if a.serve_small_gb > 0:
        srv = server(int(a.serve_small_gb * 2**30), mas.MAS_FP32, a.serve_batch, a.serve_workers)
        try:
            small, _ = run_stream(srv, stream, rhs, rate, serving)
            small.update(budget_gib=a.serve_small_gb, **{k: v for k, v in srv.stats().items()
                                                           if k in ("uploads", "evictions", "peak_resident_bytes")})
        finally:
            srv.shutdown()
        print(f"[serve] budget {a.serve_small_gb} GiB: {small}", file=sys.stderr, flush=True)
    # baseline: the same stream one request at a time, plain FP64 cycle
    srv = server(full, mas.MAS_FP64, 1, 1)
    try:
        warm(srv)
        base_closed, _ = run_stream(srv, stream, rhs, 0.0, serving)
        base_open, _ = run_stream(srv, stream, rhs, rate, serving) if a.serve_baseline_open else (None, None)
    finally:
        srv.shutdown()
    print(f"[serve] one-at-a-time FP64: {base_closed}", file=sys.stderr, flush=True)
    out = {
        "metric": "serving solves/s to 1e-8 rel. residual (p50/p99 latency)",
        "value": main_run["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": len(stream),
        "warmup": len(probs),
        "ms_per_step": 1e3 / main_run["solves_per_s"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 cycle / f64 FGMRES",
        "data": "synthetic",
        "config": {"workload": "serve: 512 Poisson-arrival requests (seed 5), Taylor-Hood meshes 2D 32^2/64^2/"
                               "128^2/256^2 and 3D 8^3/12^3/16^3/24^3, viscosity log-uniform [1e-2,1], Gaussian "
                               "forcing, homogeneous Dirichlet, FGMRES(20) rtol 1e-8",
                   "arrival_rate_per_s": rate, "load_factor": a.serve_load, "max_batch": a.serve_batch,
                   "workers": a.serve_workers, "hbm_budget_gib": full / 2**30,
                   "relaxation": f"2D Vanka, 3D {a.serve_relax_3d}"},
        "p50_ms": main_run["p50_ms"],
        "p99_ms": main_run["p99_ms"],
        "closed_loop": closed,
        "open_loop": main_run,
        "load_sweep": sweep,
        "small_budget": small,
        "baseline_one_at_a_time_fp64": {"closed_loop": base_closed, "open_loop_same_rate": base_open},
        "throughput_vs_one_at_a_time": cap / base_closed["solves_per_s"],
        "resident_gib": st_full["peak_resident_bytes"] / 2**30,
    }
    print(json.dumps(out))


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the multi-GPU layout is a design note, "
              "not built", file=sys.stderr)
        sys.exit(2)
    if a.config == "serve":
        return bench_serve(a)
    import torch

    from paper_2306_06795_amd import mas
    from paper_2306_06795_amd.inputs import make_config

    dev = "cuda:0"
    if a.copy_probe_mib > 0:  # one copy kernel of known size: reference for HBM byte counters
        src = torch.ones(a.copy_probe_mib << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        float(src.sum())  # a read-only pass over the same bytes
        torch.cuda.synchronize()
        del src, dst
    t0 = time.perf_counter()
    prob = make_config(a.config) if a.mesh_n is None else make_config(a.config, n=a.mesh_n)
    t_gen = time.perf_counter() - t0
    if a.mesh_n is not None:
        a.config = f"{a.config}@n={a.mesh_n}"
    relax = {"vanka": mas.MAS_RELAX_VANKA, "dlsc": mas.MAS_RELAX_DLSC, "vanka-dlsc": mas.MAS_RELAX_VANKA_DLSC}[a.relax]
    prec = mas.MAS_FP64 if a.precision == "fp64" else mas.MAS_FP32
    nrhs = prob.nrhs
    if a.krylov_its and (a.relax != "vanka" or nrhs != 1):
        sys.exit("--krylov-its wraps the Vanka relaxation of a single right-hand side")
    rname = a.relax + (f"+fgmres{a.krylov_its}" if a.krylov_its else "") + (f"+amg{a.dlsc_amg}" if a.dlsc_amg else "")
    label = rname
    sched = {"all": mas.MAS_DC_ALL, "skip1": mas.MAS_DC_SKIP1, "skip0": mas.MAS_DC_SKIP0, "ho": mas.MAS_HO_AMG}
    method = "HO-AMG" if a.schedule == "ho" else f"DC-{a.schedule}"
    if a.schedule != "all":
        label += f"+{a.schedule}"
    over = {} if a.theta is None else {"theta": a.theta, "soc": mas.MAS_SOC_SYMMETRIC}
    if a.theta is not None:  # another hierarchy: no counter figure of the default one applies
        label += f"+theta{a.theta:g}"
    if a.bucket_min is not None:
        over["bucket_min"] = a.bucket_min
        label += f"+bucket{a.bucket_min}"
    if a.share_blocks is not None:
        over["share_blocks"] = a.share_blocks
        label += f"+share{a.share_blocks}"
    if a.patch_kernel is not None:
        over["patch_kernel"] = a.patch_kernel
    mp = mas.default_params(prob.dim, mas.MAS_SV if prob.disc == "SV" else mas.MAS_TH, relax, precision=prec,
                            nrhs_max=nrhs, krylov_its=a.krylov_its, schedule=sched[a.schedule],
                            dlsc_amg=a.dlsc_amg, **over)
    t0 = time.perf_counter()
    h = mas.Handle(prob, mp)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    info = h.info()
    print(f"[bench] {a.config}: n0={prob.n0} levels={info['n']} patches={info['n_patches']} "
          f"bucket patches={info['bucket_patches']} patch kernel={info['patch_kernel']} "
          f"gen {t_gen:.1f}s setup {t_setup:.1f}s", file=sys.stderr, flush=True)
    b = torch.tensor(prob.b, device=dev)
    x = torch.empty_like(b)
    dt, iters, rc, sinfo = timed_solves(torch, h, b, x, a.steps, a.warmup, a.rtol, nrhs)
    assert rc == mas.MAS_OK, f"solve did not converge: {sinfo}"
    xx = x.cpu().numpy().reshape(prob.n0, -1)
    relres = true_relres(prob, xx)
    print(f"[bench] timed {a.steps} solves in {dt:.3f}s, iters {iters}, true relres {relres:.2e}",
          file=sys.stderr, flush=True)
    eager = None
    if prob.n0 < 20000:  # small systems are launch-bound: the same solves without the iteration graphs
        mp.graphs = 0
        he = mas.Handle(prob, mp)
        mp.graphs = 1
        xe = torch.empty_like(b)
        he.solve(b, xe, rtol=a.rtol, nrhs=nrhs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            he.solve(b, xe, rtol=a.rtol, nrhs=nrhs)
        torch.cuda.synchronize()
        eager = {"ms_per_step": 1e3 * (time.perf_counter() - t0) / a.steps,
                 "note": "same solves with every kernel launched from the host (no graph replay)"}
        he.close()
    # reference solution for the error of each result: the FP64 cycle's solve to 1e-12 (its cycle
    # application equals the oracle's to 1e-11 in the full-size parity tests)
    if prec == mas.MAS_FP64:
        h64 = h
    else:
        h64 = mas.Handle(prob, mas.default_params(prob.dim, mas.MAS_SV if prob.disc == "SV" else mas.MAS_TH,
                                                  relax, precision=mas.MAS_FP64, nrhs_max=nrhs,
                                                  krylov_its=a.krylov_its, schedule=sched[a.schedule],
                                                  dlsc_amg=a.dlsc_amg, **over))
    xref = torch.empty_like(b)
    h64.solve(b, xref, rtol=1e-12, nrhs=nrhs, max_it=2000)
    Xref = xref.cpu().numpy().reshape(prob.n0, -1)
    if h64 is not h:
        h64.close()
    del xref
    err_ref = rel_err(xx, Xref)
    companion = None
    if prec == mas.MAS_FP64 and not a.no_companion and a.krylov_its == 0:
        # the mixed-precision form beside the plain FP64 one: FP32 cycle, FP64 FGMRES
        mp32 = mas.default_params(prob.dim, mas.MAS_SV if prob.disc == "SV" else mas.MAS_TH, relax,
                                  precision=mas.MAS_FP32, nrhs_max=nrhs, schedule=sched[a.schedule],
                                  dlsc_amg=a.dlsc_amg, **over)
        t0 = time.perf_counter()
        h32 = mas.Handle(prob, mp32)
        torch.cuda.synchronize()
        setup32 = time.perf_counter() - t0
        x32 = torch.empty_like(b)
        dt32, it32, rc32, si32 = timed_solves(torch, h32, b, x32, a.steps, a.warmup, a.rtol, nrhs)
        assert rc32 == mas.MAS_OK, f"FP32-cycle solve did not converge: {si32}"
        xx32 = x32.cpu().numpy().reshape(prob.n0, -1)
        v32 = vcycle_time(torch, h32, prob.n0 * nrhs, nrhs, dev)
        companion = {"cycle_precision": "fp32 (FP64 FGMRES, patch factorisation and coarse solve)",
                     "value": a.steps * nrhs / dt32, "unit": "solves/s", "ms_per_step": 1e3 * dt32 / a.steps,
                     "speedup_vs_fp64": dt / dt32, "iters": it32[-1], "true_relres": true_relres(prob, xx32),
                     "err_vs_reference": rel_err(xx32, Xref), "vcycle_median_ms": v32[1], "setup_s": setup32}
        print(f"[bench] FP32 cycle: {companion}", file=sys.stderr, flush=True)
        h32.close()
        del x32
    # V-cycle (one preconditioner application) time, and the patch kernel measured with HIP events
    nrep = 20
    r = torch.randn(prob.n0 * nrhs, dtype=torch.float64, device=dev)
    z = torch.empty_like(r)
    vcycle_ms, vmed, vmin = vcycle_time(torch, h, prob.n0 * nrhs, nrhs, dev, nrep)
    # algorithmic bytes of one cycle: its timed patch kernels and sparse products
    h.set_timing(True)
    h.apply(r, z, nrhs=nrhs)
    cyc_bytes = sum(v[2] for v in h.timing().values())
    h.set_timing(False)
    copy_gbs = stream_copy_gbs(torch, dev)
    h.set_timing(True)
    h.solve(b, x, rtol=a.rtol, nrhs=nrhs)
    tm = h.timing()
    h.set_timing(False)
    # the dominant kernel of the solve, its launches timed with HIP events on its stream
    kind = max(tm, key=lambda k: tm[k][0])
    k_ms, k_launches, k_bytes = tm[kind]
    k_launches = max(1, k_launches)
    avg_launch_ms = k_ms / k_launches
    avg_bytes = k_bytes / k_launches
    achieved = avg_bytes / (avg_launch_ms * 1e-3) / 1e9
    kernel = {"tpp": "k_vanka_tpp (thread-per-patch bucket kernel)",
              "generic": "k_vanka_apply / k_vanka_col (workgroup- or wavefront-per-patch kernel, chosen per level)",
              "batched": "k_vanka_apply_nr (batched patch kernel)",
              "sell": "k_sell (sliced-ELL sparse product)",
              "csr": "k_csr (CSR sparse product)",
              "spmm": "k_spmm (batched CSR sparse product)"}[kind]
    total_ms = sum(v[0] for v in tm.values())
    its_last = sinfo[0]["iters"]
    out = {
        "metric": "Stokes solves/s to 1e-8 rel. residual",
        "value": a.steps * nrhs / dt,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * dt / a.steps,
        "rhs_per_step": nrhs,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == mas.MAS_FP64 else "f32 cycle / f64 FGMRES",
        "data": "synthetic",
        "config": {"workload": f"{a.config}: {WORKLOADS.get(a.config, a.config)}, {rname} {method}, "
                               f"FGMRES(20) rtol {a.rtol:g}",
                   "n0": prob.n0, "levels": info["n"], "relax": label, "cycle_precision": a.precision},
        "iters": iters[-1],
        "true_relres": relres,
        "err_vs_reference": err_ref,
        "reference": "FP64-cycle solve of the same system to 1e-12 relative residual",
        "fp32_cycle": companion,
        "eager": eager,
        "vcycle_ms": vcycle_ms,
        "vcycle": {"mean_ms": vcycle_ms, "median_ms": vmed, "min_ms": vmin, "applies": nrep,
                   "algorithmic_bytes": cyc_bytes,
                   "hbm_frac": cyc_bytes / (vmed * 1e-3) / 1e9 / HBM_PEAK_GBS,
                   "copy_frac": cyc_bytes / (vmed * 1e-3) / 1e9 / copy_gbs},
        "setup_s": t_setup,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "vcycle_hbm_frac": cyc_bytes / (vmed * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": measured_traffic(a.config, a.precision, label, kind),
                     "measured_copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs,
                     "kernel": kernel, "avg_launch_ms": avg_launch_ms,
                     "algorithmic_bytes_per_launch": avg_bytes, "launches_timed": k_launches,
                     "share_of_timed_kernels": k_ms / max(1e-12, total_ms)},
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, a.config, its_last, a.cpu_sample_its, a.relax, a.krylov_its,
                                           a.schedule, a.dlsc_amg, a.theta)
    print(json.dumps(out))
    h.close()


if __name__ == "__main__":
    main()
