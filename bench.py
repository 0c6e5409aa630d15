"""Benchmark: BDDC-SO PCG DoF/s to a relative residual of 1e-8 on one MI355X.

A step is one pass of the whole hot path over one synthetic input: the
numeric setup from rho (local factors, coarse basis, coarse factorization)
followed by the PCG solve to rtol.  Inputs (rho, f) are resident in HBM before
the timed region; the host classification and the device allocations happen
once, before it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload cfg2]
                    [--precision fp64|mixed] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

WORKLOADS = {
    # name: (builder, description)
    "cfg2": (W.config2, "3D Q1 96^3 (857,375 dofs), 8x8x8 subdomains of 12^3, subobjects 4h, "
                        "log10 rho ~ U[-3,3] per subdomain"),
    "cfg4": (W.config4, "cfg2 mesh and rho with subobjects of 2h"),
    "cfg1": (W.config1, "2D Q1 64^2, 4x4 subdomains of 16^2, subobjects 4h, rho = 1"),
    "cfg5": (W.config5, "3D Q1 64^3, 8x8x8 subdomains of 8^3, subobjects 4h"),
    "cfg2_small": (lambda: W.config2_like(48, 12, 4, cfg=2, name="cfg2_small"),
                   "cfg2 shapes on a 48^3 mesh (4x4x4 subdomains of 12^3)"),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cfg2", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--coarse", default="nd", choices=["nd", "dense"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--phases", action="store_true", help="also time setup and solve separately")
    return ap.parse_args()


def cpu_baseline():
    """The oracle, untuned, on a bounded sample: cfg2's subdomain and
    subobject shapes (12^3 elements, L = 4h, same rho law) on a 48^3 mesh,
    64 subdomains, 103,823 dofs; end-to-end setup + PCG to 1e-8."""
    from oracle import bddc, pcg

    p = W.config2_like(48, 12, 4, cfg=2, name="cfg2_sample")
    t0 = time.perf_counter()
    o = bddc.from_problem(p)
    t1 = time.perf_counter()
    r = pcg.solve(o, p.f[0], rtol=1e-8)
    t2 = time.perf_counter()
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": p.n_free / (t2 - t0), "unit": "DoF/s", "cores": threads, "kind": "oracle",
            "sample": f"cfg2 shapes on 48^3 ({p.n_free} dofs, 64 subdomains), setup {t1 - t0:.1f} s "
                      f"+ solve {t2 - t1:.1f} s, {r.iters} iterations"}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (the multi-GPU "
                                   "sharding is a design only)"}))
        sys.exit(2)
    import torch

    import paper_2001_07289_amd as pk

    build, desc = WORKLOADS[a.workload]
    p = build()
    prob = pk.Problem.from_workload(p)
    dev = torch.device("cuda:0")
    rho = torch.as_tensor(p.rho, device=dev)
    b = torch.as_tensor(np.ascontiguousarray(p.f[0]), device=dev)
    opts = dict(precision=1 if a.precision == "mixed" else 0, coarse_solver=1 if a.coarse == "dense" else 0,
                rtol=1e-8, maxit=500)
    t0 = time.perf_counter()
    pc = pk.Preconditioner(prob, rho, **opts)
    torch.cuda.synchronize()
    t_first = time.perf_counter() - t0

    def step():
        pc.refactor(rho)
        return pc.solve(b)

    for _ in range(a.warmup):
        x, st = step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        x, st = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / a.steps
    n = p.n_free
    # true residual of the last solve, on the device
    res = float(torch.linalg.norm(b - pc.operator(x)) / torch.linalg.norm(b))
    out = {
        "metric": "BDDC-SO PCG DoF/s to rel.res 1e-8",
        "value": n * a.steps / (t1 - t0),
        "unit": "DoF/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.precision == "fp64" else "f32-local/f64-outer",
        "data": "synthetic",
        "config": {"workload": a.workload, "description": desc, "n_free": n, "n_sub": prob.info()["n_sub"],
                   "n_coarse": pc.info()["n_coarse"], "precision": a.precision, "coarse": a.coarse,
                   "rtol": 1e-8},
        "iters": st["iters"][0], "kappa": st["kappa"][0], "true_relres": res,
        "first_setup_s": t_first, "device_bytes": pc.info()["device_bytes"],
    }
    if a.phases:
        reps = max(1, a.steps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            pc.refactor(rho)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(reps):
            pc.solve(b)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        out["setup_ms"] = (t1 - t0) * 1e3 / reps
        out["solve_ms"] = (t2 - t1) * 1e3 / reps
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
