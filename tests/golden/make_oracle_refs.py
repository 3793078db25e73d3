"""Writes the oracle's reference solutions of the medium and paper-scale
cantilever workloads into this folder.  Calls only the CPU oracle (and the
seeded input generators); nothing here touches the HIP path.

    python tests/golden/make_oracle_refs.py c2          # 96x48x48, seed 0, P^3
    python tests/golden/make_oracle_refs.py c4 0 1 2 3  # 224x112x56, seeds 0-3, P^5
    python tests/golden/make_oracle_refs.py c3step      # 224x112x56 uniform 0.12: oracle PCG to 1e-6

The solve K(rho) u = f (Sec. III-D, Eq. (4)) is too large here for the
banded Cholesky factor (40 GB at 96x48x48, 675 GB at 224x112x56), so the
oracle's Jacobi-preconditioned CG runs to a relative residual of 1e-12 with
the element-by-element operator.  Stored per case: the compliance f^T u
(float64), the sensitivity of Eq. (5) (float32: its rounding, 6e-8 of an
entry, is far below the 1e-5 of max |dc| that results are held to), the
iteration count, the final relative residual and the command.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import fe_oracle as O  # noqa: E402
from paper_2104_12282_amd import synth  # noqa: E402

CASES = {"c2": ((96, 48, 48), 3), "c4": ((224, 112, 56), 5)}


def smoothed_density(nx, ny, nz, seed, passes, P):
    rho = synth.density_uniform(nx, ny, nz, seed)
    for _ in range(passes):
        rho = P @ rho
    return rho


def reference(case, seed, rtol=1e-12):
    (nx, ny, nz), passes = CASES[case]
    t0 = time.perf_counter()
    P = O.filter_matrix(nx, ny, nz, 1.5)
    rho = smoothed_density(nx, ny, nz, seed, passes, P)
    Ke = O.hex8_ke(0.3)
    f = synth.cantilever_edge_load(nx, ny, nz)
    fixed = O.clamp_x0_fixed(nx, ny, nz)
    tag = f"{case} seed {seed}"
    u, it, rel = O.solve_pcg(nx, ny, nz, O.simp_modulus(rho), Ke, f, fixed, rtol=rtol, elementwise=True,
                             progress=lambda i, r: print(f"{tag}: iteration {i} rel {r:.3e}", flush=True)
                             if i % 500 == 0 else None)
    c = O.compliance(f, u)
    dc = O.sensitivity(nx, ny, nz, Ke, rho, u)
    dt = time.perf_counter() - t0
    path = os.path.join(HERE, f"oracle_{case}_seed{seed}.npz")
    np.savez_compressed(
        path, grid=np.array([nx, ny, nz]), seed=seed, filter_passes=passes, filter_r=1.5,
        compliance=c, dc=dc.astype(np.float32), dc_absmax=np.abs(dc).max(), iters=it, rel_res=rel,
        rtol=rtol, solver="oracle Jacobi-PCG, element-by-element K, float64",
        command=f"python tests/golden/make_oracle_refs.py {case} {seed}")
    print(f"{tag}: {it} iterations, rel {rel:.3e}, c {c:.15g}, {dt:.0f} s -> {path}", flush=True)


def c3_step(rtol=1e-6):
    """The first step of the optimisation loop at 224x112x56 (uniform design
    0.12, volume fraction 0.12): iterations of the oracle's PCG from zero to
    the loop's tolerance, for the timed CPU baseline."""
    nx, ny, nz = CASES["c4"][0]
    x = np.full(nx * ny * nz, 0.12)
    rho = O.filter_matrix(nx, ny, nz, 1.5) @ x
    Ke = O.hex8_ke(0.3)
    f = synth.cantilever_edge_load(nx, ny, nz)
    fixed = O.clamp_x0_fixed(nx, ny, nz)
    t0 = time.perf_counter()
    u, it, rel = O.solve_pcg(nx, ny, nz, O.simp_modulus(rho), Ke, f, fixed, rtol=rtol, elementwise=True,
                             progress=lambda i, r: print(f"c3step: iteration {i} rel {r:.3e}", flush=True)
                             if i % 500 == 0 else None)
    dt = time.perf_counter() - t0
    rec = {"grid": [nx, ny, nz], "design": "uniform 0.12", "rtol": rtol, "iters": it, "rel_res": rel,
           "compliance": O.compliance(f, u), "solve_seconds_here": dt,
           "solver": "oracle Jacobi-PCG, element-by-element K, float64, from u = 0",
           "command": "python tests/golden/make_oracle_refs.py c3step"}
    with open(os.path.join(HERE, "oracle_c3_step0.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    what = sys.argv[1]
    if what == "c3step":
        c3_step()
    else:
        for s in (sys.argv[2:] or ["0"]):
            reference(what, int(s))
