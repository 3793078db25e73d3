"""Benchmark of the exact-gradient FE step on one MI355X.

A step is one iteration of the density-based optimisation loop on the
paper-scale cantilever (224 x 112 x 56 bricks, 1,404,928 design variables):
  rho = P x;  u = K(rho)^-1 f (CG with a 4-level geometric multigrid
  preconditioner to 1e-6, each solve started from the extrapolation of the
  last two solutions);  dc = dc/drho;  dcx = P^T dc;
  x = OC(x, dcx, dv)   (volume fraction 0.12, move limit 0.2).
Warm-up steps run first; the design is then reset to the uniform start and
the timed steps are the first `--steps` iterations of the loop (50 by
default: the whole loop).  The same loop is then timed in the alternative
precision (float32 CG inside float64 refinement) and reported under "alt",
and profiled passes give the roofline records.  Prints one JSON line.
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
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--grid", type=str, default="224x112x56")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32_ir", "bf16_ir", "bf16x3_ir"])
    ap.add_argument("--alt-precision", default="fp32_ir", choices=["none", "fp64", "fp32_ir", "bf16_ir", "bf16x3_ir"])
    ap.add_argument("--precond", default="gmg", choices=["jacobi", "gmg"])
    ap.add_argument("--mg-levels", type=int, default=4)
    ap.add_argument("--mg-nu", type=int, default=1)
    ap.add_argument("--mg-omega", type=float, default=0.0, help="damped Jacobi weight (0: the library's default)")
    ap.add_argument("--mg-coarse", type=int, default=0,
                    help="coarsest-level Chebyshev degree (0: the library's default for the coarsest grid)")
    ap.add_argument("--f32-from", type=int, default=-1,
                    help="first multigrid level run in float32 inside float64 solves (-1: the library default; "
                         "0: all, the finest level's smoothing included; the number of levels: none)")
    ap.add_argument("--mg-coarse-ratio", type=float, default=0.0,
                    help="coarsest-level Chebyshev interval ratio (0: the library's default)")
    ap.add_argument("--study-mg-levels", type=int, default=3,
                    help="multigrid levels of the synthetic-gradient and two-scale coarse solves and of the "
                         "paper meshes below 1M elements (smaller grids: three levels)")
    ap.add_argument("--mg-cheb-from", type=int, default=-1,
                    help="first level smoothed by Chebyshev steps (-1: the library default; 0: damped Jacobi "
                         "on every level)")
    ap.add_argument("--mg-cheb-deg", type=int, default=6, help="Chebyshev smoothing steps (with --mg-cheb-from)")
    ap.add_argument("--mg-cheb-ratio", type=float, default=30.0,
                    help="Chebyshev smoothing interval ratio (with --mg-cheb-from)")
    ap.add_argument("--coarse-form", type=int, default=0,
                    help="coarsest-level Chebyshev launch form (0: the library's automatic choice; 3: pairs of "
                         "steps on 3D tiles, 2: pairs on z-marching tiles, 1: one step per launch)")
    ap.add_argument("--rtol", type=float, default=1e-6)
    ap.add_argument("--extrapolate", type=float, default=1.0,
                    help="initial guess of each loop solve: u + theta (u - u_prev) from the third "
                         "iteration on (fe_extrapolate; 0: the last solution alone)")
    ap.add_argument("--volfrac", type=float, default=0.12)
    ap.add_argument("--move", type=float, default=0.2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision-seeds", type=int, default=4,
                    help="seeded smoothed densities of the precision study (0 = skip it)")
    ap.add_argument("--mg-context", type=int, default=1,
                    help="also run the loop with the other hierarchy (3 levels with damped Jacobi smoothing "
                         "when the headline runs 4, else 4) as a context line")
    ap.add_argument("--two-scale", type=int, default=1,
                    help="time the coarse-scale solves of the two-scale scheme beside the fine solve")
    ap.add_argument("--adjoint", type=int, default=1,
                    help="time the adjoint gradient of a non-self-adjoint objective")
    ap.add_argument("--paper-meshes", type=int, default=200,
                    help="iterations of the runs on the paper's three cantilever meshes (0: skip)")
    ap.add_argument("--onsg-iters", type=int, default=40,
                    help="iterations of the online synthetic-gradient loop on the paper's mesh 2 (0: skip)")
    ap.add_argument("--cold", type=int, default=1024,
                    help="MB of the buffer streamed through before each cold-timed launch (0: no cold timing)")
    ap.add_argument("--c2", type=int, default=1,
                    help="run the 96x48x48 float64 Jacobi-PCG solve (to 1e-8) against the oracle")
    ap.add_argument("--serving", type=int, default=256,
                    help="requests of the serving stream to run (0: skip)")
    ap.add_argument("--serving-streams", type=int, default=5,
                    help="streams the serving engine's batches run on (one per grid size by default)")
    ap.add_argument("--serving-slots", type=int, default=16,
                    help="slots of each grid size's batch in the serving engine")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one device-to-device copy of 512 MiB (reference for counters)")
    return ap.parse_args()


# Fused-operand form of the CG-product launch: 3 when a float64 solve's
# preconditioner leaves z in float32 (the default), else 2; set by main().
PRODUCT_XIN = {"fp64": 3}


def product_xin(precision: str) -> int:
    return PRODUCT_XIN.get(precision, 2)


def traffic_from_profiles(precision: str, grid: str, field: str = "bytes", want: str | None = None):
    """HBM bytes (fetched + written) of one launch of a kernel on this grid
    (`want`: a substring of its name; by default the CG-product launch of the
    tiled K*u kernel), from rocprofv3 FETCH_SIZE / WRITE_SIZE counters scaled
    by a copy of known size (field "bytes"), or rocprofv3's average kernel
    duration of that launch in us (field "trace_work_avg_us"), when the stored
    figures were taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"loop_kernels_{grid}_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        from paper_2104_12282_amd.build import source_digest
        if rec.get("source_digest") != source_digest():
            return None
        want = want or f"kxu_tile_kernel<{'double' if precision == 'fp64' else 'float'}, 1, {product_xin(precision)}>"
        for name, k in rec["kernels"].items():
            if want in name:
                return k["fetch_bytes"] + k["write_bytes"] if field == "bytes" else k.get(field)
    except Exception:
        return None
    return None


def profile_record(grid: str):
    """The stored rocprofv3 figures of this grid when they were taken on the
    current kernel source, else None."""
    path = os.path.join(ROOT, "profiles", f"loop_kernels_{grid}_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
        from paper_2104_12282_amd.build import source_digest
        return rec if rec.get("source_digest") == source_digest() else None
    except Exception:
        return None


def initial_guess_text(args):
    """How each solve of an optimisation loop starts."""
    if args.extrapolate:
        return (f"u + {args.extrapolate:g} (u - u_prev) from the last two solutions, from the third solve on "
                "(fe_extrapolate); the last solution before")
    return "the last solution"


def apply_mg(prob, args):
    """Multigrid settings of the command line on a problem; 0 keeps the
    library's default for that problem's coarsest grid."""
    if args.precond != "gmg" or prob.cfg.precond != 1:
        return None
    if args.f32_from >= 0:
        prob.set_float32_levels(min(args.f32_from, prob.cfg.mg_levels))
    if args.coarse_form:
        prob.set_coarse_fusion(args.coarse_form)
    cur = prob.mg_params()
    prob.set_mg_params(nu=args.mg_nu, coarse_sweeps=args.mg_coarse or cur["coarse_sweeps"],
                       omega=args.mg_omega or cur["omega"],
                       coarse_ratio=args.mg_coarse_ratio or cur["coarse_ratio"])
    if args.mg_cheb_from == 0 or 1 <= args.mg_cheb_from <= prob.cfg.mg_levels - 2:
        prob.set_mg_smoother(args.mg_cheb_from, args.mg_cheb_deg, args.mg_cheb_ratio)
    return dict(prob.mg_params(), smoother=prob.mg_smoother())


def coarse_solve_record(nx, ny, nz, args, degree):
    """Roofline context of the coarsest-level Chebyshev launches (the largest
    share of GPU time in the multigrid solve): the launch form the library
    picks, algorithmic bytes per launch and rocprofv3's average duration
    from the stored kernel-trace run of the same source."""
    if args.precond != "gmg":
        return None
    cx, cy, cz = nx, ny, nz
    for _ in range(args.mg_levels - 1):  # each level has ceil(n / 2) elements per axis
        cx, cy, cz = (cx + 1) // 2, (cy + 1) // 2, (cz + 1) // 2
    nnode = (cx + 1) * (cy + 1) * (cz + 1)
    wide = args.precision == "fp64" and args.f32_from >= args.mg_levels  # the coarsest level in float64
    vb = 8.0 if wide else 4.0
    # d_k, r_k, acc read and r, acc, d_{k+s} written (3 dofs per node), moduli,
    # inverse diagonal, fixed-dof mask: each array once
    nbytes = vb * (6 * 3 * nnode + cx * cy * cz + nnode) + nnode
    form = args.coarse_form
    if form == 0:  # the library's automatic choice (fe_set_coarse_fusion)
        import torch
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        cols = ((cx + 4) // 4) * ((cy + 4) // 4)
        form = 5 if cols * ((cz + 4) // 4) <= cus else 4 if not wide and cols * ((cz + 8) // 8) <= cus else 2
    if form == 5 and wide:
        form = 3
    if form == 5:
        import torch
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        nblk = lambda ox, oy, oz: ((cx + ox) // ox) * ((cy + oy) // oy) * ((cz + oz) // oz)
        ox, oy = (2, 2) if nblk(2, 2, 4) <= cus else (2, 4) if nblk(2, 4, 4) <= cus else (4, 4)
        name, steps, shape = f"cheb3t_kernel<{ox}, {oy}, 4>", 3, f"3D tiles of {ox} x {oy} x 4 nodes"
        launches = 2 if degree == 4 else (degree + 2) // 3
    else:
        oz = 8 if form == 4 and not wide else 4
        name = f"cheb3d_kernel<{'double' if wide else 'float'}, {oz}>" if form >= 3 else \
            f"cheb2_kernel<{'double' if wide else 'float'}>"
        steps, shape = 2, (f"3D tiles of 4 x 4 x {oz} nodes" if form >= 3 else "z-marching tiles")
        launches = (degree + 1) // 2
    word = {2: "two", 3: "three"}[steps]
    out = {"kernel": f"{name}: {word} coarsest-level Chebyshev steps per launch on {shape}",
           "coarse_grid": [cx, cy, cz], "launches_per_vcycle": launches,
           "algorithmic_bytes_per_launch": nbytes, "bound": "latency",
           "note": "well under a MB per launch on a few-thousand-element grid: the launch is bound by its "
                   "chain of dependent memory round trips, LDS phases and barriers, not by HBM bandwidth"}
    rec = profile_record(f"{nx}x{ny}x{nz}")
    if rec:
        for t in rec.get("time_shares", []):
            if name.split("<")[0] in t["kernel"] and t.get("work_avg_us"):
                out["rocprofv3_avg_kernel_us"] = t["work_avg_us"]
                out["rocprofv3_share_of_gpu_time"] = t["share"]
                out["achieved_GBs"] = nbytes / (t["work_avg_us"] * 1e-6) / 1e9
                out["frac_of_hbm_peak"] = out["achieved_GBs"] / HBM_PEAK_GBS
                break
    return out


def oracle_reference(case: str, seed: int):
    """The oracle's stored solution of a workload (compliance, sensitivity),
    written by tests/golden/make_oracle_refs.py, or None if absent."""
    path = os.path.join(ROOT, "tests", "golden", f"oracle_{case}_seed{seed}.npz")
    if not os.path.exists(path):
        return None
    z = np.load(path)
    return {"compliance": float(z["compliance"]), "dc": z["dc"].astype(np.float64),
            "dc_absmax": float(z["dc_absmax"]), "iters": int(z["iters"]), "rel_res": float(z["rel_res"]),
            "file": os.path.relpath(path, ROOT)}


def cpu_baseline(grid, rtol, k1=2, k2=22):
    """The FP64 oracle on the headline workload (the first optimisation step
    of the 224x112x56 loop), timed on the host on a bounded sample: the
    filter, sensitivity, transpose filter and OC once at full size, and the
    oracle's Jacobi-PCG on the full operator for k1 and k2 iterations (setup
    and per-iteration time); the solve is scaled to the iteration count the
    oracle needs for this step (from the stored reference run)."""
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
    E = O.simp_modulus(rho)
    t_filter = time.perf_counter() - t0
    times = {}
    for k in (k1, k2):
        t0 = time.perf_counter()
        u, it, _ = O.solve_pcg(nx, ny, nz, E, Ke, f, fixed, rtol=rtol, max_iters=k, elementwise=True)
        times[k] = time.perf_counter() - t0
    t_iter = (times[k2] - times[k1]) / (k2 - k1)
    t_setup = times[k1] - k1 * t_iter
    t0 = time.perf_counter()
    dc = O.sensitivity(nx, ny, nz, Ke, rho, u)
    dcx = P.T @ dc
    dv = P.T @ np.ones(ne)
    O.oc_update(x, dcx, dv, 0.12, 0.2)
    t_rest = time.perf_counter() - t0
    ref_path = os.path.join(ROOT, "tests", "golden", "oracle_c3_step0.json")
    ref = json.load(open(ref_path)) if os.path.exists(ref_path) else None
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    sampled = t_filter + times[k2] + t_rest
    out = {"unit": "solves/s", "cores": cores, "kind": "oracle", "seconds_sampled": sampled,
           "seconds_per_pcg_iteration": t_iter, "seconds_pcg_setup": t_setup,
           "seconds_filter_sensitivity_oc": t_filter + t_rest}
    if ref:
        step = t_filter + t_setup + ref["iters"] * t_iter + t_rest
        out.update({"value": 1.0 / step, "seconds_per_step": step, "oracle_pcg_iterations": ref["iters"],
                    "sample": (f"the oracle's first step of the {nx}x{ny}x{nz} loop (uniform 0.12): filter, "
                               f"sensitivity, transpose filter and OC at full size, and its Jacobi-PCG on the "
                               f"full element-by-element operator for {k1} and {k2} iterations "
                               f"({sampled:.1f} s in all); one step = those parts + setup + "
                               f"{ref['iters']} PCG iterations to {ref['rtol']:g} (the count of the stored "
                               f"oracle run, {os.path.relpath(ref_path, ROOT)}); numpy's BLAS threads for the "
                               f"element products, the gathers and sums single-threaded")})
    else:
        out.update({"value": None, "sample": "the oracle's iteration count for this step is not stored"})
    return out


PREC_VARIANTS = (("fp32_ir", 1), ("bf16_ir", 2), ("bf16x3_ir", 4))


def kxu_rate(prob, rho, u, variant, reps=20, flush=None):
    """Average finest-grid K*u kernel time (HIP events around each launch on
    the problem's stream) and algorithmic GB/s of one fe_apply_K variant;
    with `flush` (a device buffer of >= 512 MB) every timed launch is
    preceded by a pass over it, so its operands come from HBM (cold)."""
    y = prob.apply_K(rho, u, variant=variant)
    prob.kernel_stats(reset=True)
    if flush is not None:
        prob.set_cache_flush(flush)
    prob.set_profiling(True)
    for _ in range(reps):
        prob.apply_K(rho, u, variant=variant, out=y)
    prob.set_profiling(False)
    if flush is not None:
        prob.set_cache_flush(None)
    ks = prob.kernel_stats(reset=True)
    us = ks["total_ms"] / max(1, ks["launches"]) * 1e3
    return us, ks["bytes_per_launch"] / (us * 1e-6) / 1e9


def precision_study(fe, synth, torch, nx, ny, nz, seeds, args, flush=None):
    """Smoothed random densities (U(0.01,1) through 5 filter passes): float64,
    float32, bf16 and split-bf16 element contractions (the reduced ones inside
    float64 refinement), each solved to 1e-8 and compared with the oracle's
    stored solution of the same design (Jacobi-PCG to 1e-12 on the CPU):
    relative compliance error and max sensitivity error relative to
    max |dc*|, with the solve status; and the K*u kernel rate of each variant,
    warm (operands resident in the caches after the conversions before it)
    and cold (every launch after a pass over a 1 GB buffer)."""
    dev = "cuda:0"
    T = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
    f = T(synth.cantilever_edge_load(nx, ny, nz))
    kw = dict(device=dev, precond=args.precond, mg_levels=args.mg_levels)
    probs = {p: fe.Problem(nx, ny, nz, f, precision=p, **kw) for p in ("fp64",) + tuple(v for v, _ in PREC_VARIANTS)}
    if args.precond == "gmg":
        for pr in probs.values():
            apply_mg(pr, args)
    keys = ("c_rel_err", "dc_rel_err", "c_rel_err_vs_gpu_fp64", "dc_rel_err_vs_gpu_fp64", "iters", "outer_iters",
            "rel_res", "ms", "status")
    res = {p: {k: [] for k in keys} for p in probs}
    refs = []
    for seed in range(seeds):
        ref = oracle_reference("c4", seed) if (nx, ny, nz) == (224, 112, 56) else None
        refs.append(ref["file"] if ref else None)
        a = T(synth.density_uniform(nx, ny, nz, seed))
        b = torch.empty_like(a)
        for _ in range(5):
            probs["fp64"].filter(a, out=b)
            a, b = b, a
        gpu64 = None
        for p, pr in probs.items():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            u, info = pr.solve(a, rtol=1e-8, allow_notconv=True)
            dc, c = pr.sensitivity(a, u)
            torch.cuda.synchronize()
            ms = 1e3 * (time.perf_counter() - t0)
            dcn, cv = dc.cpu().numpy(), float(c.item())
            if p == "fp64":
                gpu64 = (dcn, cv)
            r = res[p]
            r["status"].append(fe.STATUS_NAME[info["status"]])
            if ref:
                r["c_rel_err"].append(abs(cv - ref["compliance"]) / abs(ref["compliance"]))
                r["dc_rel_err"].append(float(np.abs(dcn - ref["dc"]).max() / ref["dc_absmax"]))
            r["c_rel_err_vs_gpu_fp64"].append(abs(cv - gpu64[1]) / abs(gpu64[1]))
            r["dc_rel_err_vs_gpu_fp64"].append(float(np.abs(dcn - gpu64[0]).max() / np.abs(gpu64[0]).max()))
            r["iters"].append(info["iters"])
            r["outer_iters"].append(info["outer_iters"])
            r["rel_res"].append(info["rel_res"])
            r["ms"].append(ms)
            err = (f"c_err {r['c_rel_err'][-1]:.2e} dc_err {r['dc_rel_err'][-1]:.2e} (oracle)" if ref
                   else "no oracle reference stored")
            print(f"bench[precision]: seed {seed} {p} {r['status'][-1]} iters {info['iters']} "
                  f"outer {info['outer_iters']} rel_res {info['rel_res']:.2e} {err}",
                  file=sys.stderr, flush=True)
    uu = T(np.random.default_rng(7).standard_normal(probs["fp64"].ndof))
    out = {"grid": [nx, ny, nz], "seeds": seeds, "density": "U(0.01,1) seeded, 5 filter passes (r=1.5)",
           "rtol": 1e-8, "reference": "the FP64 CPU oracle (Jacobi-PCG to 1e-12, stored per seed)",
           "reference_files": refs, "tolerance": {"c_rel_err": 1e-6, "dc_rel_err": 1e-5}, "variants": {}}
    for p, pr in probs.items():
        variant = 0 if p == "fp64" else dict(PREC_VARIANTS)[p]
        us, gbs = kxu_rate(pr, a, uu, variant)
        rec = {"kxu_variant": variant, "kxu_warm_us": us, "kxu_warm_gbs": gbs,
               "kxu_warm_frac_of_hbm_peak": gbs / HBM_PEAK_GBS}
        if flush is not None:
            cus, cgbs = kxu_rate(pr, a, uu, variant, flush=flush)
            rec.update({"kxu_cold_us": cus, "kxu_cold_gbs": cgbs, "kxu_cold_frac_of_hbm_peak": cgbs / HBM_PEAK_GBS})
        r = res[p]
        ok = [i for i, st in enumerate(r["status"]) if st == "FE_OK"]
        with_ref = [i for i in ok if refs[i]]
        rec.update({
            "statuses": r["status"], "converged": len(ok),
            "c_rel_err_max": max((r["c_rel_err"][i] for i in with_ref), default=None) if r["c_rel_err"] else None,
            "dc_rel_err_max": max((r["dc_rel_err"][i] for i in with_ref), default=None) if r["dc_rel_err"] else None,
            "c_rel_err_vs_gpu_fp64_max": max((r["c_rel_err_vs_gpu_fp64"][i] for i in ok), default=None),
            "dc_rel_err_vs_gpu_fp64_max": max((r["dc_rel_err_vs_gpu_fp64"][i] for i in ok), default=None),
            "errors_over": "converged solves (status FE_OK) with a stored oracle reference",
            "iters_mean": float(np.mean(r["iters"])), "outer_iters_mean": float(np.mean(r["outer_iters"])),
            "rel_res_max": max(r["rel_res"]), "solve_ms_mean": float(np.mean(r["ms"]))})
        out["variants"][p] = rec
        pr.close()
    return out


def c2_study(fe, synth, torch, flush=None, reps=3):
    """The medium-size plain solve: the cantilever on 96x48x48 (seed 0,
    U(0.01,1) through 3 filter passes), float64 Jacobi-PCG to 1e-8, then the
    sensitivity and its transpose filter; solve time (median of reps after
    one untimed solve), iterations, errors against the oracle's stored
    solution, and the float64 K*u kernel rate warm and cold."""
    dev = "cuda:0"
    nx, ny, nz = 96, 48, 48
    T = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
    prob = fe.Problem(nx, ny, nz, T(synth.cantilever_edge_load(nx, ny, nz)), device=dev, precision="fp64",
                      precond="jacobi")
    a = T(synth.density_uniform(nx, ny, nz, 0))
    b = torch.empty_like(a)
    for _ in range(3):
        prob.filter(a, out=b)
        a, b = b, a
    ms, info = [], None
    for rep in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, info = prob.solve(a, rtol=1e-8)
        dc, c = prob.sensitivity(a, u)
        dcx = prob.filter(dc, transpose=True)
        torch.cuda.synchronize()
        if rep:
            ms.append(1e3 * (time.perf_counter() - t0))
    ref = oracle_reference("c2", 0)
    out = {"grid": [nx, ny, nz], "density": "U(0.01,1) seed 0, 3 filter passes (r=1.5)", "precision": "fp64",
           "precond": "jacobi", "rtol": 1e-8, "iters": info["iters"], "rel_res": info["rel_res"],
           "status": fe.STATUS_NAME[info["status"]],
           "solve_sensitivity_filter_ms": float(np.median(ms)), "solves_per_s": 1e3 / float(np.median(ms))}
    if ref:
        dcn = dc.cpu().numpy()
        out.update({"reference": ref["file"], "c_rel_err": abs(float(c.item()) - ref["compliance"]) / ref["compliance"],
                    "dc_rel_err": float(np.abs(dcn - ref["dc"]).max() / ref["dc_absmax"])})
    del dcx
    uu = T(np.random.default_rng(7).standard_normal(prob.ndof))
    us, gbs = kxu_rate(prob, a, uu, 0)
    out.update({"kxu_fp64_warm_us": us, "kxu_fp64_warm_gbs": gbs})
    if flush is not None:
        cus, cgbs = kxu_rate(prob, a, uu, 0, flush=flush)
        out.update({"kxu_fp64_cold_us": cus, "kxu_fp64_cold_gbs": cgbs,
                    "kxu_fp64_cold_frac_of_hbm_peak": cgbs / HBM_PEAK_GBS})
    print(f"bench[c2]: jacobi fp64 {info['iters']} iterations, {out['solve_sensitivity_filter_ms']:.1f} ms, "
          f"c_err {out.get('c_rel_err', float('nan')):.2e} dc_err {out.get('dc_rel_err', float('nan')):.2e}, "
          f"K*u {us:.1f} us warm", file=sys.stderr, flush=True)
    prob.close()
    return out


def two_scale_study(fe, synth, torch, nx, ny, nz, args, block_sizes=(2, 4, 5, 7, 8), steps=20):
    """Cost of the coarse scale of the two-scale scheme, which solves the
    coarse problem at every optimisation iteration: the loop of the main
    benchmark (filter, warm-started solve, sensitivity, transpose filter, OC)
    runs `steps` iterations, and after each, per block size nb dividing the
    grid, the coarse step on the same design (block means, the coarse filter,
    the coarse solve warm-started from the previous u_C).  Each part is timed
    on its own (synchronised); the first iteration is left out of the means."""
    dev = "cuda:0"
    T = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
    ne = nx * ny * nz
    fine = fe.Problem(nx, ny, nz, T(synth.cantilever_edge_load(nx, ny, nz)), device=dev,
                      precision=args.precision, precond=args.precond, mg_levels=args.mg_levels)
    if args.precond == "gmg":
        apply_mg(fine, args)
    x = torch.full((ne,), args.volfrac, dtype=torch.float64, device=dev)
    u = torch.zeros(fine.ndof, dtype=torch.float64, device=dev)
    rho, dc, dcx = (torch.empty_like(x) for _ in range(3))
    dv = fine.filter(torch.ones_like(x), transpose=True)
    comp = torch.zeros(1, dtype=torch.float64, device=dev)
    change = torch.zeros(1, dtype=torch.float64, device=dev)
    coarse = {}
    for nb in block_sizes:
        if nx % nb or ny % nb or nz % nb:
            continue
        cx, cy, cz = nx // nb, ny // nb, nz // nb
        pc = fine.coarse_problem(nb, T(synth.cantilever_edge_load(cx, cy, cz)), mg_levels=args.study_mg_levels)
        apply_mg(pc, args)
        zc = torch.empty(cx * cy * cz, dtype=torch.float64, device=dev)
        coarse[nb] = {"prob": pc, "zc": zc, "rc": torch.empty_like(zc),
                      "uc": torch.zeros(pc.ndof, dtype=torch.float64, device=dev), "ms": [], "iters": []}
    fine_ms, fine_iters = [], []
    for it in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fine.filter(x, out=rho)
        _, info = fine.solve(rho, u=u, rtol=args.rtol)
        fine.sensitivity(rho, u, out=dc, compliance_out=comp)
        fine.filter(dc, transpose=True, out=dcx)
        torch.cuda.synchronize()
        fine_ms.append(1e3 * (time.perf_counter() - t0))
        fine_iters.append(info["iters"])
        for nb, c in coarse.items():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fine.block_mean(x, nb, out=c["zc"])
            c["prob"].filter(c["zc"], out=c["rc"])
            _, ci = c["prob"].solve(c["rc"], u=c["uc"], rtol=args.rtol)
            torch.cuda.synchronize()
            c["ms"].append(1e3 * (time.perf_counter() - t0))
            c["iters"].append(ci["iters"])
        fine.oc_update(x, dcx, dv, args.volfrac, args.move, out=x, change_out=change)
    mean = lambda v: float(np.mean(v[1:])) if len(v) > 1 else float(v[0])
    f_ms = mean(fine_ms)
    out = {"grid": [nx, ny, nz], "steps": steps, "rtol": args.rtol,
           "fine_step": {"ms": f_ms, "iters_mean": mean(fine_iters), "dofs": fine.ndof,
                         "parts": "filter, warm-started solve, sensitivity, transpose filter (OC not timed)"},
           "coarse": {}}
    print(f"bench[two-scale]: fine step {f_ms:.2f} ms, {mean(fine_iters):.1f} iterations", file=sys.stderr,
          flush=True)
    for nb, c in coarse.items():
        pc = c["prob"]
        precond = fe.PRECOND_NAME[pc.cfg.precond]
        rec = {"grid": [pc.nx, pc.ny, pc.nz], "dofs": pc.ndof, "precond": precond,
               "mg_levels": pc.cfg.mg_levels if precond == "gmg" else 0, "ms": mean(c["ms"]),
               "iters_mean": mean(c["iters"]), "ratio_to_fine_step": mean(c["ms"]) / f_ms}
        out["coarse"][str(nb)] = rec
        print(f"bench[two-scale]: nb {nb} coarse {pc.nx}x{pc.ny}x{pc.nz} ({precond}) {rec['ms']:.2f} ms, "
              f"{rec['iters_mean']:.1f} iterations, {rec['ratio_to_fine_step']:.3f} of the fine step",
              file=sys.stderr, flush=True)
        pc.close()
    fine.close()
    return out


def adjoint_study(fe, synth, torch, nx, ny, nz, args, reps=5):
    """The general adjoint gradient (Eq. 3) of a non-self-adjoint objective,
    J = -u_z at the middle of the loaded edge, on one smoothed random design
    (U(0.01,1) through 3 filter passes): the forward solve, the adjoint solve
    (load swapped to dJ/du and restored), and the state-equation term
    -lam^T dr/drho, against the compliance sensitivity kernel.  Medians of
    reps after one untimed run; kernel times from events on the stream."""
    dev = "cuda:0"
    T = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
    f = T(synth.cantilever_edge_load(nx, ny, nz))
    prob = fe.Problem(nx, ny, nz, f, device=dev, precision=args.precision, precond=args.precond,
                      mg_levels=args.mg_levels)
    apply_mg(prob, args)
    l = torch.zeros(prob.ndof, dtype=torch.float64, device=dev)
    l[3 * (nx + (nx + 1) * (ny // 2)) + 2] = -1.0
    rho = T(synth.density_uniform(nx, ny, nz, 0))
    tmp = torch.empty_like(rho)
    for _ in range(3):
        prob.filter(rho, out=tmp)
        rho, tmp = tmp, rho
    g = torch.empty_like(rho)

    def median_ms(fn):
        fn()
        ms = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            out = fn()
            torch.cuda.synchronize()
            ms.append(1e3 * (time.perf_counter() - t0))
        return float(np.median(ms)), out

    fwd_ms, (u, finfo) = median_ms(lambda: prob.solve(rho, rtol=args.rtol))

    def adjoint_solve():
        prob.set_load(l)
        try:
            return prob.solve(rho, rtol=args.rtol)
        finally:
            prob.set_load(f)

    adj_ms, (lam, ainfo) = median_ms(adjoint_solve)

    def kernel_us(fn, n=20):
        fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(n):
            fn()
        b.record()
        b.synchronize()
        return a.elapsed_time(b) * 1e3 / n

    dc = torch.empty_like(rho)
    adj_us = kernel_us(lambda: prob.sensitivity_adjoint(rho, u, lam, out=g))
    sens_us = kernel_us(lambda: prob.sensitivity(rho, u, out=dc))
    nbytes = 8.0 * (2 * prob.ndof + 2 * prob.nelem)  # u, lam, rho read, g written
    out = {"grid": [nx, ny, nz], "objective": "J = -u_z at node (nx, ny/2, 0)", "rtol": args.rtol,
           "forward_solve_ms": fwd_ms, "forward_iters": finfo["iters"],
           "adjoint_solve_ms": adj_ms, "adjoint_iters": ainfo["iters"],
           "adjoint_term_us": adj_us, "adjoint_term_algorithmic_bytes": nbytes,
           "adjoint_term_gbs": nbytes / (adj_us * 1e-6) / 1e9, "compliance_sensitivity_us": sens_us}
    print(f"bench[adjoint]: forward {fwd_ms:.2f} ms ({finfo['iters']} it), adjoint {adj_ms:.2f} ms "
          f"({ainfo['iters']} it), term {adj_us:.1f} us ({out['adjoint_term_gbs']:.0f} GB/s), "
          f"compliance sensitivity {sens_us:.1f} us", file=sys.stderr, flush=True)
    prob.close()
    return out


# Final objectives of the paper's standard optimizer on its cantilever meshes
# (Table II); its material constants are not stated, so they are context only.
PAPER_TABLE2_STANDARD = {70: 370.11, 100: 379.54, 180: 383.51}


def paper_mesh_study(fe, synth, torch, args, iters):
    """The standard optimizer on the paper's cantilever meshes (Sec. IV):
    the 2 x 1 x 1 domain in 70x35x35, 100x50x50 and 180x90x90 elements
    (h = 2 / nx), filter radius R = 0.08 (2.8, 4 and 7.2 elements), volume
    fraction 0.12, the edge load, `iters` iterations from the uniform design.
    Multigrid with the requested levels on every mesh (an odd axis coarsens
    to ceil(n / 2) elements)."""
    dev = "cuda:0"
    T = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
    out = {"domain": [2.0, 1.0, 1.0], "filter_R": 0.08, "volfrac": 0.12, "move": args.move,
           "rtol": args.rtol, "initial_guess": initial_guess_text(args), "iterations": iters, "meshes": {}}
    for nx in (70, 100, 180):
        ny = nz = nx // 2
        h = 2.0 / nx
        # four levels from ~1M elements on, as for the loop (180x90x90:
        # 2.87 s against 3.37 s with three; the smaller meshes: three)
        levels = 4 if nx * ny * nz >= 1_000_000 else args.study_mg_levels
        precond = args.precond
        prob = fe.Problem(nx, ny, nz, T(synth.cantilever_edge_load(nx, ny, nz)), device=dev, h=h,
                          filter_r=0.08 / h, precision=args.precision, precond=precond,
                          mg_levels=levels)
        mg = apply_mg(prob, args)
        ne = nx * ny * nz
        x = torch.full((ne,), 0.12, dtype=torch.float64, device=dev)
        u = torch.zeros(prob.ndof, dtype=torch.float64, device=dev)
        u_hist = torch.zeros_like(u)
        rho, dc, dcx = (torch.empty_like(x) for _ in range(3))
        dv = prob.filter(torch.ones_like(x), transpose=True)
        comp = torch.zeros(1, dtype=torch.float64, device=dev)
        change = torch.zeros(1, dtype=torch.float64, device=dev)
        cs, its = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for it in range(iters):
            prob.filter(x, out=rho)
            prob.extrapolate(u, u_hist, args.extrapolate if it >= 2 else 0.0)
            _, info = prob.solve(rho, u=u, rtol=args.rtol)
            prob.sensitivity(rho, u, out=dc, compliance_out=comp)
            prob.filter(dc, transpose=True, out=dcx)
            prob.oc_update(x, dcx, dv, 0.12, args.move, out=x, change_out=change)
            cs.append(info["compliance"])
            its.append(info["iters"])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rec = {"grid": [nx, ny, nz], "elements": ne, "dofs": prob.ndof, "h": h, "filter_r_elements": 0.08 / h,
               "precond": precond, "mg_levels": levels if precond == "gmg" else 0,
               "mg_coarse_chebyshev_degree": mg["coarse_sweeps"] if mg else None,
               "seconds": dt, "ms_per_iteration": 1e3 * dt / iters, "cg_iters_mean": float(np.mean(its)),
               "objective_first": cs[0], "objective_final": cs[-1],
               "objective_at": {str(k): cs[k - 1] for k in (10, 50, 100, 200) if k <= iters},
               "paper_table2_standard_objective": PAPER_TABLE2_STANDARD[nx]}
        out["meshes"][f"{nx}x{ny}x{nz}"] = rec
        print(f"bench[paper-mesh]: {nx}x{ny}x{nz} ({precond}{'' if precond != 'gmg' else f', {levels} levels'}) "
              f"{iters} iterations in {dt:.1f} s ({rec['ms_per_iteration']:.1f} ms each, "
              f"{rec['cg_iters_mean']:.0f} CG iterations), objective {cs[0]:.4g} -> {cs[-1]:.4g} "
              f"(paper, other constants: {PAPER_TABLE2_STANDARD[nx]})", file=sys.stderr, flush=True)
        prob.close()
    return out


def onsg_study(fe, synth, torch, args, K, nb=5, width=1000, steps=2000, batch=256, lr0=5e-4, halve=500,
               n_init=10, n_freq=10):
    """Alg. 1 on the paper's cantilever mesh 2 (100x50x50, h = 0.02, R = 0.08)
    with block size nb: every iteration coarse-grains the design and solves
    the coarse problem; iterations k < n_init and k = 0 mod n_freq take the
    exact gradient, add the blocks' samples and update the network (`steps`
    Adam steps on mini-batches of `batch` drawn uniformly from all samples so
    far), the others take the network's synthetic gradient; OC with either.
    The standard optimizer runs the same K iterations for comparison; both
    final designs are evaluated by one exact solve.  Samples are scaled by
    their iteration's max |u_C| and max |g| (inside the library)."""
    dev = "cuda:0"
    T = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
    nx, ny, nz = 100, 50, 50
    h = 2.0 / nx
    ne = nx * ny * nz
    cx, cy, cz = nx // nb, ny // nb, nz // nb

    def make():
        prob = fe.Problem(nx, ny, nz, T(synth.cantilever_edge_load(nx, ny, nz)), device=dev, h=h,
                          filter_r=0.08 / h, precision=args.precision, precond="gmg",
                          mg_levels=args.study_mg_levels)
        return prob

    def run(onsg):
        prob = make()
        coarse = prob.coarse_problem(nb, T(synth.cantilever_edge_load(cx, cy, cz)))
        x = torch.full((ne,), 0.12, dtype=torch.float64, device=dev)
        u = torch.zeros(prob.ndof, dtype=torch.float64, device=dev)
        uc = torch.zeros(coarse.ndof, dtype=torch.float64, device=dev)
        rho, dc, g = (torch.empty_like(x) for _ in range(3))
        zc = torch.empty(cx * cy * cz, dtype=torch.float64, device=dev)
        rc = torch.empty_like(zc)
        dv = prob.filter(torch.ones_like(x), transpose=True)
        change = torch.zeros(1, dtype=torch.float64, device=dev)
        model = None
        t = {"fine": 0.0, "coarse": 0.0, "train": 0.0, "predict": 0.0, "oc": 0.0}
        exact_iters, objective, err, losses = 0, [], [], []
        torch.cuda.synchronize()
        t_all = time.perf_counter()

        def clock(key, t0):
            torch.cuda.synchronize()
            t[key] += time.perf_counter() - t0

        for k in range(K):
            exact = (not onsg) or k < n_init or k % n_freq == 0
            if onsg:
                t0 = time.perf_counter()
                prob.block_mean(x, nb, out=zc)
                coarse.filter(zc, out=rc)
                coarse.solve(rc, u=uc, rtol=args.rtol)
                clock("coarse", t0)
            if exact:
                t0 = time.perf_counter()
                prob.filter(x, out=rho)
                _, info = prob.solve(rho, u=u, rtol=args.rtol)
                prob.sensitivity(rho, u, out=dc)
                prob.filter(dc, transpose=True, out=g)
                clock("fine", t0)
                objective.append(info["compliance"])
                exact_iters += 1
                if onsg:
                    if model is not None:
                        # the model's synthetic gradient for this design, before it sees it
                        gs = model.predict(x, uc)
                        # the prediction is in units of the iteration's largest gradient
                        gsc = gs * g.abs().max()
                        err.append({"iteration": k, "rel_l2": float((gsc - g).norm() / g.norm()),
                                    "cosine": float(torch.dot(gs, g) / (gs.norm() * g.norm()))})
                    t0 = time.perf_counter()
                    if model is None:
                        sizes = [nb ** 3 + 24, width, width, width, width, nb ** 3]
                        model = fe.SyntheticGradientModel(nx, ny, nz, nb, width,
                                                          (n_init + K // n_freq + 1) * cx * cy * cz, batch,
                                                          synth.mlp_init(sizes, 0), device=dev)
                    model.add_samples(x, uc, g)
                    ls = model.train(synth.minibatches(model.num_samples, steps, batch, seed=1000 + k), lr0, halve)
                    clock("train", t0)
                    losses.append({"iteration": k, "first": float(ls[0]), "last_50_mean": float(ls[-50:].mean())})
            else:
                t0 = time.perf_counter()
                model.predict(x, uc, out=g)
                clock("predict", t0)
            t0 = time.perf_counter()
            prob.oc_update(x, g, dv, 0.12, args.move, out=x, change_out=change)
            clock("oc", t0)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t_all
        prob.filter(x, out=rho)
        _, info = prob.solve(rho, u=u, rtol=args.rtol)
        rec = {"seconds": wall, "exact_iterations": exact_iters, "final_objective": info["compliance"],
               "objective_at_exact_iterations": objective, "seconds_by_part": t}
        if onsg:
            rec["synthetic_vs_exact"] = err
            rec["training_loss"] = losses
        if model is not None:
            model.close()
        coarse.close()
        prob.close()
        return rec

    std = run(False)
    ons = run(True)
    flops = 6.0 * batch * sum(i * o for i, o in zip([nb ** 3 + 24] + [width] * 4, [width] * 4 + [nb ** 3]))
    out = {"mesh": [nx, ny, nz], "h": h, "filter_r_elements": 0.08 / h, "nb": nb, "iterations": K,
           "n_init": n_init, "n_freq": n_freq, "network": {"hidden": [width] * 4, "steps_per_update": steps,
                                                          "batch": batch, "lr0": lr0, "halve_every": halve},
           "standard": std, "onsg": ons,
           "training_tflops": flops * steps * (ons["exact_iterations"]) / max(ons["seconds_by_part"]["train"], 1e-9)
           / 1e12,
           "final_objective_rel_diff": ons["final_objective"] / std["final_objective"] - 1.0,
           "speedup": std["seconds"] / ons["seconds"]}
    for e in ons["synthetic_vs_exact"]:
        print(f"bench[onsg]: iteration {e['iteration']}: synthetic vs exact gradient rel. l2 error "
              f"{e['rel_l2']:.3f}, cosine {e['cosine']:.3f}", file=sys.stderr, flush=True)
    for e in ons["training_loss"]:
        print(f"bench[onsg]: update at {e['iteration']}: loss {e['first']:.3g} -> {e['last_50_mean']:.3g}",
              file=sys.stderr, flush=True)
    print(f"bench[onsg]: {K} iterations on 100x50x50 (nb {nb}): standard {std['seconds']:.2f} s, objective "
          f"{std['final_objective']:.4g}; ONSG {ons['seconds']:.2f} s ({ons['exact_iterations']} exact, "
          f"train {ons['seconds_by_part']['train']:.2f} s at {out['training_tflops']:.1f} TFLOP/s, coarse "
          f"{ons['seconds_by_part']['coarse']:.2f} s), objective {ons['final_objective']:.4g}",
          file=sys.stderr, flush=True)
    return out


def serving_bench(n, torch, nslots=16, nstreams=5):
    """Serving stream of n seeded requests over the five grid sizes: the same
    requests one at a time (blocking solves); through the batched engine
    (one fe_batch of nslots per size, designs sharing launches) all at once
    (throughput) and as Poisson arrivals at 0.5x and 2x the sequential rate
    and at 0.8x the batched throughput (latency under load); and, for
    comparison, through the engine that overlaps per-design launches on
    streams."""
    from paper_2104_12282_amd import serve, synth
    reqs = synth.serving_requests(n, seed=0)
    # each request arrives with its design: inputs in pinned host memory,
    # generated before any clock starts (every engine copies them the same way)
    serve.attach_payloads(reqs)
    serve.run_engine_batched(reqs[:8], None, nslots=nslots, n_streams=nstreams)  # warm-up: kernels, graphs
    serve.run_engine(reqs[:8], None)
    _, seq = serve.run_sequential(reqs)
    print(f"bench[serving]: sequential {seq['designs_per_s']:.1f} designs/s", file=sys.stderr, flush=True)
    _, sat = serve.run_engine_batched(reqs, None, nslots=nslots, n_streams=nstreams)
    print(f"bench[serving]: batched engine {sat['designs_per_s']:.1f} designs/s", file=sys.stderr, flush=True)
    _, streams = serve.run_engine(reqs, None)
    print(f"bench[serving]: stream engine {streams['designs_per_s']:.1f} designs/s", file=sys.stderr, flush=True)
    out = {"requests": n, "grids": [list(g) for g in synth.SERVING_GRIDS],
           "per_request": "load at a random node of x = nx (random direction), density U(0.01,1) "
                          "(both arriving with the request in pinned host memory, copied to the device "
                          "asynchronously) through 3 filter passes, float32 CG with 4-level multigrid "
                          "inside float64 refinement to 1e-8, then sensitivity",
           "engine": f"fe_batch per grid size, {nslots} slots each; CG chunks of all slots in shared "
                     "launches; designs admitted into free slots between replays",
           "sequential": seq, "batched_all_at_once": sat, "stream_engine_all_at_once": streams,
           "poisson": {}}
    for name, rate in (("0.5x_sequential_rate", 0.5 * seq["designs_per_s"]),
                       ("2.0x_sequential_rate", 2.0 * seq["designs_per_s"]),
                       ("0.8x_batched_throughput", 0.8 * sat["designs_per_s"])):
        arr = synth.poisson_arrivals(n, rate, seed=1)
        _, st = serve.run_engine_batched(reqs, arr, nslots=nslots, n_streams=nstreams)
        st["arrival_rate_per_s"] = rate
        out["poisson"][name] = st
        print(f"bench[serving]: poisson {name}: {st['designs_per_s']:.1f} designs/s p50 "
              f"{st['p50_latency_s']*1e3:.1f} ms p99 {st['p99_latency_s']*1e3:.1f} ms", file=sys.stderr,
              flush=True)
    out["speedup_vs_sequential"] = sat["designs_per_s"] / seq["designs_per_s"]
    return out


def run_loop(fe, synth, torch, nx, ny, nz, precision, args, steps, warmup, profile, flush=None, prof_mode=1):
    """Warm-up steps, then `steps` timed optimisation steps from the start
    design (the timed steps are iterations 0 .. steps-1 of the loop).  With
    profile, HIP event nodes bracket every CG-product launch (prof_mode 1)
    or every coarsest-level Chebyshev pair launch (prof_mode 7); with flush as
    well, a pass over that buffer precedes each one (cold operands)."""
    ne = nx * ny * nz
    dev = "cuda:0"
    T = lambda a: torch.as_tensor(a, dtype=torch.float64, device=dev)
    f = synth.cantilever_edge_load(nx, ny, nz)
    prob = fe.Problem(nx, ny, nz, T(f), device=dev, precision=precision, precond=args.precond,
                      mg_levels=args.mg_levels)
    if args.precond == "gmg":
        rec_mg = apply_mg(prob, args)
    else:
        rec_mg = None
    x = torch.empty(ne, dtype=torch.float64, device=dev)
    u = torch.empty(prob.ndof, dtype=torch.float64, device=dev)
    u_hist = torch.empty_like(u)  # the solution before the last (initial-guess extrapolation)
    rho = torch.empty_like(x)
    dc = torch.empty_like(x)
    dcx = torch.empty_like(x)
    dv = prob.filter(torch.ones_like(x), transpose=True)
    comp = torch.zeros(1, dtype=torch.float64, device=dev)
    change = torch.zeros(1, dtype=torch.float64, device=dev)
    rec = {"iters": [], "outer": [], "compliance": [], "mg": rec_mg}

    def reset():
        x.fill_(args.volfrac)
        u.zero_()
        rec["n"] = 0

    def step():
        prob.filter(x, out=rho)
        # from the third solve on the guess extrapolates the last two solutions
        prob.extrapolate(u, u_hist, args.extrapolate if rec["n"] >= 2 else 0.0)
        rec["n"] += 1
        _, info = prob.solve(rho, u=u, rtol=args.rtol)
        prob.sensitivity(rho, u, out=dc, compliance_out=comp)
        prob.filter(dc, transpose=True, out=dcx)
        prob.oc_update(x, dcx, dv, args.volfrac, args.move, out=x, change_out=change)
        rec["iters"].append(info["iters"])
        rec["outer"].append(info["outer_iters"])
        rec["compliance"].append(info["compliance"])
        return info

    reset()
    for i in range(warmup):
        info = step()
        print(f"bench[{precision}]: warmup {i} iters {info['iters']} c {info['compliance']:.6g}",
              file=sys.stderr, flush=True)
    reset()
    rec["iters"].clear()
    rec["outer"].clear()
    rec["compliance"].clear()
    torch.cuda.synchronize()
    prob.kernel_stats(reset=True)
    if flush is not None:
        prob.set_cache_flush(flush)
    prob.set_profiling(profile, mode=prof_mode)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        info = step()
        if i % 10 == 0 or i == steps - 1:
            print(f"bench[{precision}]: step {i} iters {info['iters']} outer {info['outer_iters']} "
                  f"rel_res {info['rel_res']:.2e} c {info['compliance']:.6g}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prob.set_profiling(False)
    ks = prob.kernel_stats(reset=True)
    prob.close()
    return dt, rec, ks, prob.ndof


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU: --gpus must be 1"}))
        sys.exit(2)
    import torch

    from paper_2104_12282_amd import fe, synth

    nx, ny, nz = (int(v) for v in args.grid.split("x"))
    ne = nx * ny * nz
    PRODUCT_XIN["fp64"] = 3 if args.precond == "gmg" and args.f32_from <= 0 else 2
    torch.cuda.set_device(0)
    probe = None
    if args.copy_probe:
        nbytes = 512 << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        probe = {"bytes": nbytes}
    print(f"bench: grid {nx}x{ny}x{nz} precision {args.precision} precond {args.precond}",
          file=sys.stderr, flush=True)
    # the headline: unprofiled
    dt, rec, _, ndof = run_loop(fe, synth, torch, nx, ny, nz, args.precision, args, args.steps,
                                args.warmup, profile=False)
    print(f"bench: {args.steps} steps in {dt:.3f} s ({args.steps / dt:.2f} solves/s)", file=sys.stderr, flush=True)
    # the same steps again with event nodes around every CG-product launch
    dtp, recp, ks, _ = run_loop(fe, synth, torch, nx, ny, nz, args.precision, args, args.steps, 0,
                                profile=True)
    avg_ms = ks["total_ms"] / max(1, ks["launches"])
    achieved = ks["bytes_per_launch"] / (avg_ms * 1e-3) / 1e9 if ks["launches"] else 0.0
    flush = None
    if args.cold:
        flush = torch.empty(args.cold << 20, dtype=torch.uint8, device="cuda:0")
        flush.zero_()
    cold = None
    if flush is not None:
        # a few steps with every CG-product launch preceded by a pass over 1 GB: operands from HBM
        _, _, ksc, _ = run_loop(fe, synth, torch, nx, ny, nz, args.precision, args, min(args.steps, 3), 0,
                                profile=True, flush=flush)
        cms = ksc["total_ms"] / max(1, ksc["launches"])
        cold = {"launches": ksc["launches"], "avg_launch_us": cms * 1e3,
                "achieved": ksc["bytes_per_launch"] / (cms * 1e-3) / 1e9 if ksc["launches"] else 0.0,
                "note": f"first {min(args.steps, 3)} steps of the loop; every timed launch follows a kernel that "
                        f"streams through a {args.cold} MB buffer, so its operands come from HBM"}
        cold["frac"] = cold["achieved"] / HBM_PEAK_GBS
    product = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": achieved / HBM_PEAK_GBS,
               "measured_on": "a second pass over the same timed steps with event nodes (the headline "
                              "pass runs without them); warm: the loop's own cache state",
               "profiled_pass_solves_per_s": args.steps / dtp,
               "cold": cold,
               "traffic": traffic_from_profiles(args.precision, f"{nx}x{ny}x{nz}"),
               "traffic_of": "one CG-product launch (rocprofv3 counters, copy-scaled)",
               "kernel": "kxu_tile_kernel<" + ("double" if args.precision == "fp64" else "float")
                         + f", 1, {product_xin(args.precision)}>: CG product on the finest grid "
                         "(direction p = z + beta p fused into the matrix-free K*u, p^T K p partials"
                         + ("; z read in float32" if product_xin(args.precision) == 3 else "") + ")",
               "launches": ks["launches"], "avg_launch_us": avg_ms * 1e3,
               "rocprofv3_avg_kernel_us": traffic_from_profiles(args.precision, f"{nx}x{ny}x{nz}",
                                                                "trace_work_avg_us"),
               "timing_note": "avg_launch_us brackets each launch with HIP event nodes inside the "
                              "captured CG graph (includes the nodes' own dispatch time); "
                              "rocprofv3_avg_kernel_us is the kernel-trace average of the same "
                              "kernel in the profiled run of this command; both leave out the "
                              "launches that met the CG stop flag (a converged solve's remaining "
                              "iterations in its last chunk return at once)",
               "algorithmic_bytes_per_launch": ks["bytes_per_launch"]}
    roofline = product
    coarse = coarse_solve_record(nx, ny, nz, args, rec["mg"]["coarse_sweeps"]) if rec["mg"] else None
    if coarse:
        # the coarsest-level Chebyshev launches take the largest share of a
        # multigrid solve's GPU time: they are the dominant kernel of the
        # roofline line
        dtq, _, ksq, _ = run_loop(fe, synth, torch, nx, ny, nz, args.precision, args, args.steps, 0,
                                  profile=True, prof_mode=7)
        # one event pair brackets each coarse solve (its launches_per_vcycle
        # launches back to back, the gaps between them included)
        per = coarse["launches_per_vcycle"]
        sms = ksq["total_ms"] / max(1, ksq["launches"])  # one coarse solve
        qms = sms / per
        qach = ksq["bytes_per_launch"] / (sms * 1e-3) / 1e9 if ksq["launches"] else 0.0
        name = coarse["kernel"].split(":")[0]
        roofline = {"bound": "hbm", "achieved": qach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": qach / HBM_PEAK_GBS,
                    "limiter": "latency: a fraction of a MB per launch on the coarsest grid, one workgroup "
                               "per tile on a quarter of the compute units; the launch time is its chain of one "
                               "memory round trip, the brick and node phases in LDS (two per step) and the "
                               "stores, not HBM bandwidth",
                    "measured_on": "a third pass over the same timed steps with event nodes around every "
                                   "coarse solve (the headline pass runs without them); warm",
                    "profiled_pass_solves_per_s": args.steps / dtq,
                    "traffic": traffic_from_profiles(args.precision, f"{nx}x{ny}x{nz}", want=name.split("<")[0]),
                    "traffic_of": "one coarse launch (rocprofv3 counters, copy-scaled)",
                    "kernel": coarse["kernel"],
                    "launches": ksq["launches"] * per, "avg_launch_us": qms * 1e3,
                    "rocprofv3_avg_kernel_us": traffic_from_profiles(args.precision, f"{nx}x{ny}x{nz}",
                                                                     "trace_work_avg_us",
                                                                     want=name.split("<")[0]),
                    "timing_note": "one HIP event pair inside the captured CG graph brackets each coarse solve "
                                   f"({per} launches back to back); avg_launch_us is its time over {per}, so the "
                                   "short gaps between the launches are included; rocprofv3_avg_kernel_us is the "
                                   "kernel-trace average of the same kernel in the profiled run of this command; "
                                   "both leave out the launches that met the CG stop flag",
                    "algorithmic_bytes_per_launch": ksq["bytes_per_launch"] / per,
                    "cg_product": product}
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
        "dtype": ("f64" if args.precond != "gmg" or args.f32_from >= args.mg_levels
                  else "f64 (CG operator, vectors and reductions; multigrid preconditioner in f32)")
        if args.precision == "fp64" else "f32 (f64 refinement and dots)",
        "data": "synthetic (seeded cantilever, uniform start density 0.12)",
        "config": {"workload": f"cantilever {nx}x{ny}x{nz} optimisation loop, first {args.steps} "
                               f"iterations",
                   "grid": [nx, ny, nz], "elements": ne, "dofs": ndof,
                   "precision": args.precision, "precond": args.precond,
                   "mg_levels": args.mg_levels if args.precond == "gmg" else None,
                   "mg_smoothing_sweeps": args.mg_nu if args.precond == "gmg" else None,
                   "mg_coarse_chebyshev_degree": rec["mg"]["coarse_sweeps"] if rec["mg"] else None,
                   "mg_coarse_chebyshev_ratio": rec["mg"]["coarse_ratio"] if rec["mg"] else None,
                   "mg_chebyshev_smoothing": rec["mg"]["smoother"] if rec["mg"] else None,
                   "preconditioner_float32_from_level": ((args.f32_from if args.f32_from >= 0 else 0)
                                                         if args.precision == "fp64" else 0) if rec["mg"] else None,
                   "rtol": args.rtol, "volfrac": args.volfrac, "filter_r": 1.5, "move": args.move,
                   "initial_guess": initial_guess_text(args),
                   "cg_iters_per_solve": float(np.mean(rec["iters"])),
                   "cg_iters_max": int(np.max(rec["iters"])),
                   "refinement_steps_per_solve": float(np.mean(rec["outer"])),
                   "compliance_first": rec["compliance"][0], "compliance_last": rec["compliance"][-1]},
        "roofline": roofline,
    }
    rec_prof = profile_record(f"{nx}x{ny}x{nz}")
    if rec_prof and rec_prof.get("time_shares"):
        out["roofline"]["rocprofv3_time_shares"] = [
            {"kernel": t["kernel"], "share": round(t["share"], 4), "avg_us": round(t["avg_us"], 2)}
            for t in rec_prof["time_shares"][:8]]
    if coarse:
        out["roofline"]["coarse_solve"] = coarse
    if probe:
        out["copy_probe"] = probe
    if args.alt_precision != "none":
        dt2, rec2, _, _ = run_loop(fe, synth, torch, nx, ny, nz, args.alt_precision, args, args.steps,
                                   0, profile=False)
        c1, c2 = np.array(rec["compliance"]), np.array(rec2["compliance"])
        out["alt"] = {"precision": args.alt_precision, "value": args.steps / dt2,
                      "ms_per_step": 1e3 * dt2 / args.steps,
                      "cg_iters_per_solve": float(np.mean(rec2["iters"])),
                      "refinement_steps_per_solve": float(np.mean(rec2["outer"])),
                      "compliance_max_rel_diff": float(np.max(np.abs(c2 - c1) / np.abs(c1)))}
    if args.precision == "fp64" and args.precond == "gmg" and args.alt_precision != "none":
        # context: the same loop with the preconditioner in float64 throughout
        a64 = argparse.Namespace(**{**vars(args), "f32_from": args.mg_levels})
        dt6, rec6, _, _ = run_loop(fe, synth, torch, nx, ny, nz, args.precision, a64, args.steps, 1,
                                   profile=False)
        out["fp64_preconditioner_context"] = {"value": args.steps / dt6, "ms_per_step": 1e3 * dt6 / args.steps,
                                              "cg_iters_per_solve": float(np.mean(rec6["iters"]))}
    if args.mg_context and args.precond == "gmg":
        lv = 3 if args.mg_levels == 4 else 4
        a4 = argparse.Namespace(**{**vars(args), "mg_levels": lv, "mg_coarse": 0, "mg_cheb_from": -1})
        dt4, rec4, _, _ = run_loop(fe, synth, torch, nx, ny, nz, args.precision, a4, args.steps, 1,
                                   profile=False)
        out[f"gmg{lv}_context"] = {"precision": args.precision, "mg_levels": lv, "value": args.steps / dt4,
                                   "ms_per_step": 1e3 * dt4 / args.steps,
                                   "cg_iters_per_solve": float(np.mean(rec4["iters"])),
                                   "mg": rec4["mg"]}
    if args.c2:
        out["c2_jacobi"] = c2_study(fe, synth, torch, flush=flush)
    if args.precision_seeds > 0:
        out["precision_study"] = precision_study(fe, synth, torch, nx, ny, nz, args.precision_seeds, args,
                                                 flush=flush)
    if args.onsg_iters > 0:
        out["onsg"] = onsg_study(fe, synth, torch, args, args.onsg_iters)
    if args.paper_meshes > 0:
        out["paper_meshes"] = paper_mesh_study(fe, synth, torch, args, args.paper_meshes)
    if args.adjoint:
        out["adjoint"] = adjoint_study(fe, synth, torch, nx, ny, nz, args)
    if args.two_scale:
        out["two_scale"] = two_scale_study(fe, synth, torch, nx, ny, nz, args)
    if args.serving > 0:
        out["serving"] = serving_bench(args.serving, torch, nslots=args.serving_slots, nstreams=args.serving_streams)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline((nx, ny, nz), args.rtol)
        print(f"bench[cpu]: oracle {out['cpu_baseline']['seconds_sampled']:.1f} s sampled, "
              f"{out['cpu_baseline']['seconds_per_pcg_iteration']:.3f} s per PCG iteration", file=sys.stderr,
              flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
