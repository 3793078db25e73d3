"""Benchmark of the exact-gradient FE step on one MI355X.

A step is one iteration of the density-based optimisation loop on the
paper-scale cantilever (224 x 112 x 56 bricks, 1,404,928 design variables):
  rho = P x;  u = K(rho)^-1 f (warm-started CG to 1e-6);  dc = dc/drho;
  dcx = P^T dc;  x = OC(x, dcx, dv)   (volume fraction 0.12, move 0.2).
Warm-up steps run first; the timed steps continue the same trajectory.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, AMD published figure


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--grid", type=str, default="224x112x56")
    ap.add_argument("--precision", default="fp32_ir", choices=["fp64", "fp32_ir", "bf16_ir"])
    ap.add_argument("--precond", default="jacobi", choices=["jacobi", "gmg"])
    ap.add_argument("--mg-levels", type=int, default=3)
    ap.add_argument("--rtol", type=float, default=1e-6)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-grid", type=str, default="80x40x20")
    return ap.parse_args()


def traffic_from_profiles(kernel_key: str):
    """HBM bytes per launch measured by rocprofv3 counters, when the stored
    figure was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "kxu_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        from paper_2104_12282_amd.build import source_digest
        if rec.get("source_digest") != source_digest() or kernel_key not in rec.get("kernels", {}):
            return None
        return rec["kernels"][kernel_key]["bytes_per_launch"]
    except Exception:
        return None


def cpu_baseline(grid, rtol):
    """The FP64 oracle's own step (assembly, banded Cholesky, sensitivity,
    filter, OC) on a reduced grid of the same cantilever, timed on the host."""
    from oracle import fe_oracle as O
    from paper_2104_12282_amd import synth
    nx, ny, nz = grid
    ne = nx * ny * nz
    f = synth.cantilever_edge_load(nx, ny, nz)
    fixed = O.clamp_x0_fixed(nx, ny, nz)
    Ke = O.hex8_ke(0.3)
    x = np.full(ne, 0.12)
    t0 = time.perf_counter()
    P = O.filter_matrix(nx, ny, nz, 1.5)
    rho = P @ x
    u = O.solve_direct(nx, ny, nz, O.simp_modulus(rho), Ke, f, fixed)
    dc = O.sensitivity(nx, ny, nz, Ke, rho, u)
    dcx = P.T @ dc
    dv = P.T @ np.ones(ne)
    O.oc_update(x, dcx, dv, 0.12, 0.2)
    dt = time.perf_counter() - t0
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    return {"value": 1.0 / dt, "unit": f"FE solves/s ({nx}x{ny}x{nz} grid, {ne} elements)",
            "cores": cores, "kind": "oracle",
            "sample": (f"one full oracle optimisation step (CSR assembly, banded Cholesky, "
                       f"sensitivity, filter, OC) on the {nx}x{ny}x{nz} cantilever, "
                       f"{dt:.2f} s; the 224x112x56 step needs ~675 GB for the banded factor"),
            "seconds": dt}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch

    from paper_2104_12282_amd import fe, synth

    nx, ny, nz = (int(v) for v in args.grid.split("x"))
    ne = nx * ny * nz
    dev = "cuda:0"
    torch.cuda.set_device(0)
    T = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
    f = synth.cantilever_edge_load(nx, ny, nz)
    prob = fe.Problem(nx, ny, nz, T(f), device=dev, precision=args.precision,
                      precond=args.precond, mg_levels=args.mg_levels)
    x = torch.full((ne,), 0.12, dtype=torch.float64, device=dev)
    u = torch.zeros(prob.ndof, dtype=torch.float64, device=dev)
    rho = torch.empty_like(x)
    dc = torch.empty_like(x)
    dcx = torch.empty_like(x)
    dv = prob.filter(torch.ones_like(x), transpose=True)
    comp = torch.zeros(1, dtype=torch.float64, device=dev)
    change = torch.zeros(1, dtype=torch.float64, device=dev)
    iters = []

    def step():
        prob.filter(x, out=rho)
        _, info = prob.solve(rho, u=u, rtol=args.rtol)
        prob.sensitivity(rho, u, out=dc, compliance_out=comp)
        prob.filter(dc, transpose=True, out=dcx)
        prob.oc_update(x, dcx, dv, 0.12, 0.2, out=x, change_out=change)
        iters.append(info["iters"])
        return info

    print(f"bench: grid {nx}x{ny}x{nz} precision {args.precision} precond {args.precond}",
          file=sys.stderr, flush=True)
    for i in range(args.warmup):
        info = step()
        print(f"bench: warmup {i} iters {info['iters']} c {info['compliance']:.6g}",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    prob.kernel_stats(reset=True)
    prob.set_profiling(True)
    iters.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        info = step()
        print(f"bench: step {i} iters {info['iters']} outer {info['outer_iters']} "
              f"rel_res {info['rel_res']:.2e} c {info['compliance']:.6g}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prob.set_profiling(False)
    ks = prob.kernel_stats(reset=True)

    avg_ms = ks["total_ms"] / max(1, ks["launches"])
    achieved = ks["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9 if ks["launches"] else 0.0
    kkey = f"kxu_{'f64' if args.precision == 'fp64' else 'f32'}_{nx}x{ny}x{nz}"
    out = {
        "metric": "FE solves/s at 1.4M elements (one optimisation step = one solve)",
        "value": args.steps / dt,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32 (f64 refinement and dots)",
        "data": "synthetic (seeded cantilever, uniform start density 0.12)",
        "config": {"workload": f"cantilever {nx}x{ny}x{nz} optimisation step",
                   "grid": [nx, ny, nz], "elements": ne, "dofs": prob.ndof,
                   "precision": args.precision, "precond": args.precond,
                   "mg_levels": args.mg_levels if args.precond == "gmg" else None,
                   "rtol": args.rtol, "volfrac": 0.12, "filter_r": 1.5, "move": 0.2,
                   "cg_iters_per_solve": float(np.mean(iters)) if iters else None},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic_from_profiles(kkey),
                     "kernel": "matrix-free K*u", "launches": ks["launches"],
                     "avg_launch_us": avg_ms * 1e3,
                     "algorithmic_bytes_per_launch": ks["bytes_per_launch"]},
    }
    if not args.no_cpu_baseline:
        cg = tuple(int(v) for v in args.cpu_grid.split("x"))
        out["cpu_baseline"] = cpu_baseline(cg, args.rtol)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
