"""Benchmark: Stokes solves/s to 1e-8 relative residual on one MI355X.

Workload (default): 2D Taylor-Hood P2/P1 on a 256x256 triangulated unit square,
interior vertices jittered by U(-0.2h, 0.2h), lid-driven cavity plus Gaussian
forcing (seeded), FP64 plain GPU form, additive Vanka V(1,1) on all levels,
FGMRES(20) to a 1e-8 relative residual.  A step is one full solve from x0 = 0
with the right-hand side already resident in HBM; setup is outside the timed
region.  Prints one JSON line (rank 0).
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
    ap.add_argument("--config", default="th2d_256")
    ap.add_argument("--relax", default="vanka", choices=["vanka", "dlsc"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-its", type=int, default=2)
    return ap.parse_args()


def cpu_baseline(prob, its_gpu, sample_its):
    """The oracle on the host: setup untimed, then ``sample_its`` FGMRES
    iterations of the same workload (first right-hand side) timed and scaled to
    one full solve."""
    from oracle import dc, fgmres
    pre = dc.DCPreconditioner(prob, dc.default_params(prob))
    b0 = prob.b if prob.b.ndim == 1 else np.ascontiguousarray(prob.b[:, 0])
    pre.apply(b0)  # untimed: builds the oracle's dense patch matrices once
    t0 = time.perf_counter()
    fgmres.fgmres(lambda v: prob.K0 @ v, pre.apply, b0, rtol=0.0, restart=20, max_it=sample_its)
    dt = time.perf_counter() - t0
    per_it = dt / sample_its
    cores = len(os.sched_getaffinity(0))
    return {"value": 1.0 / (per_it * its_gpu), "unit": "solves/s", "cores": cores, "kind": "oracle",
            "sample": f"{sample_its} oracle FGMRES iterations on the same system ({dt:.1f} s), scaled to the "
                      f"{its_gpu} iterations of one solve; oracle setup and patch-matrix extraction untimed"}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {a.gpus}); the multi-GPU layout is a design note, "
              "not built", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2306_06795_amd import mas
    from paper_2306_06795_amd.inputs import make_config

    dev = "cuda:0"
    t0 = time.perf_counter()
    prob = make_config(a.config)
    t_gen = time.perf_counter() - t0
    relax = mas.MAS_RELAX_VANKA if a.relax == "vanka" else mas.MAS_RELAX_DLSC
    prec = mas.MAS_FP64 if a.precision == "fp64" else mas.MAS_FP32
    nrhs = prob.nrhs
    mp = mas.default_params(prob.dim, mas.MAS_SV if prob.disc == "SV" else mas.MAS_TH, relax, precision=prec,
                            nrhs_max=nrhs)
    t0 = time.perf_counter()
    h = mas.Handle(prob, mp)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    info = h.info()
    print(f"[bench] {a.config}: n0={prob.n0} levels={info['n']} patches={info['n_patches']} "
          f"gen {t_gen:.1f}s setup {t_setup:.1f}s", file=sys.stderr, flush=True)
    b = torch.tensor(prob.b, device=dev)
    x = torch.empty_like(b)
    for _ in range(a.warmup):
        rc, sinfo = h.solve(b, x, rtol=a.rtol, nrhs=nrhs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    for _ in range(a.steps):
        rc, sinfo = h.solve(b, x, rtol=a.rtol, nrhs=nrhs)
        iters.append(max(i["iters"] for i in sinfo))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert rc == mas.MAS_OK, f"solve did not converge: {sinfo}"
    xs = x.cpu().numpy()
    bb = prob.b.reshape(prob.n0, -1)
    xx = xs.reshape(prob.n0, -1)
    relres = float(max(np.linalg.norm(bb[:, k] - prob.K0 @ xx[:, k]) / np.linalg.norm(bb[:, k])
                       for k in range(nrhs)))
    print(f"[bench] timed {a.steps} solves in {dt:.3f}s, iters {iters}, true relres {relres:.2e}",
          file=sys.stderr, flush=True)
    # V-cycle (one preconditioner application) time, and the patch kernel measured with HIP events
    nrep = 20
    r = torch.randn(prob.n0 * nrhs, dtype=torch.float64, device=dev)
    z = torch.empty_like(r)
    h.apply(r, z, nrhs=nrhs)
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(nrep):
        h.apply(r, z, nrhs=nrhs)
    e1.record(st)
    torch.cuda.synchronize()
    vcycle_ms = e0.elapsed_time(e1) / nrep
    h.set_timing(True)
    h.solve(b, x, rtol=a.rtol, nrhs=nrhs)
    tm = h.timing()
    h.set_timing(False)
    # the dominant kernel family of the cycle, timed with HIP events on its stream
    fam = "vanka" if tm["vanka_ms"] >= tm["spmv_ms"] else "spmv"
    launches = max(1, tm[fam + "_launches"])
    avg_launch_ms = tm[fam + "_ms"] / launches
    avg_bytes = tm[fam + "_bytes"] / launches
    achieved = avg_bytes / (avg_launch_ms * 1e-3) / 1e9
    kernel = "k_vanka_tpp/k_vanka_apply (patch solves)" if fam == "vanka" else "k_sell/k_csr (sparse products)"
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
        "config": {"workload": f"{a.config}: {WORKLOADS.get(a.config, a.config)}, {a.relax} DC-all, "
                               f"FGMRES(20) rtol {a.rtol:g}",
                   "n0": prob.n0, "levels": info["n"], "relax": a.relax, "cycle_precision": a.precision},
        "iters": iters[-1],
        "true_relres": relres,
        "vcycle_ms": vcycle_ms,
        "setup_s": t_setup,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": kernel, "avg_launch_ms": avg_launch_ms,
                     "algorithmic_bytes_per_launch": avg_bytes, "launches_timed": launches,
                     "share_of_timed_kernels": tm[fam + "_ms"] / max(1e-12, tm["vanka_ms"] + tm["spmv_ms"])},
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(prob, its_last, a.cpu_sample_its)
    print(json.dumps(out))
    h.close()


if __name__ == "__main__":
    main()
