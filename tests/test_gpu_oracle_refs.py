"""Solves of the medium (96x48x48) and paper-scale (224x112x56) workloads
against the oracle's stored solutions of the same designs
(tests/golden/oracle_*.npz: the CPU oracle's Jacobi-PCG to a relative
residual of 1e-12, written by tests/golden/make_oracle_refs.py, which calls
nothing but the oracle and the input generators).

The bar is the one stated for every result of the path: relative compliance
error <= 1e-6 and max |dc - dc*| <= 1e-5 max |dc*|, for the plain float64
solve (Jacobi and multigrid) and for the float32, bf16 and split-bf16
contractions inside float64 refinement, each solved to 1e-8 and required to
converge (status FE_OK).  The stored dc* is rounded to float32 (6e-8 of an
entry), which the 1e-5 bar leaves untouched."""
import os

import numpy as np
import pytest
import torch

from oracle import fe_oracle as O
from paper_2104_12282_amd import fe, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
CASES = {"c2": ((96, 48, 48), 3), "c4": ((224, 112, 56), 5)}


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def _reference(case, seed):
    path = os.path.join(GOLDEN, f"oracle_{case}_seed{seed}.npz")
    assert os.path.exists(path), f"{path} missing: run tests/golden/make_oracle_refs.py"
    z = np.load(path)
    assert float(z["rel_res"]) <= 1e-12
    return float(z["compliance"]), z["dc"].astype(np.float64), float(z["dc_absmax"])


def _density(case, seed):
    """The stored design, rebuilt on the CPU by the oracle's filter (the
    reference script's recipe: U(0.01, 1) through `passes` filter passes)."""
    (nx, ny, nz), passes = CASES[case]
    P = O.filter_matrix(nx, ny, nz, 1.5)
    rho = synth.density_uniform(nx, ny, nz, seed)
    for _ in range(passes):
        rho = P @ rho
    return rho


def _check(case, seed, precision, precond, rtol=1e-8, levels=3):
    (nx, ny, nz), _ = CASES[case]
    c_ref, dc_ref, dc_max = _reference(case, seed)
    rho = _density(case, seed)
    kw = {"mg_levels": levels} if precond == "gmg" else {}
    prob = fe.Problem(nx, ny, nz, T(synth.cantilever_edge_load(nx, ny, nz)), device=DEV, precision=precision,
                      precond=precond, **kw)
    print(f"oracle-ref: {case} seed {seed} {precision} {precond} levels {levels}", flush=True)
    u, info = prob.solve(T(rho), rtol=rtol)
    dc, c = prob.sensitivity(T(rho), u)
    torch.cuda.synchronize()
    prob.close()
    assert info["status"] == fe.FE_OK and info["rel_res"] <= rtol
    c_err = abs(float(c.item()) - c_ref) / c_ref
    dc_err = float(np.abs(dc.cpu().numpy() - dc_ref).max()) / dc_max
    assert c_err <= 1e-6, (case, seed, precision, precond, c_err)
    assert dc_err <= 1e-5, (case, seed, precision, precond, dc_err)
    return info


def test_c2_jacobi_fp64_as_configured():
    """96x48x48, float64 Jacobi-PCG to 1e-8, then sensitivity (the plain
    medium-size configuration)."""
    _check("c2", 0, "fp64", "jacobi")


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_c2_multigrid(precision):
    _check("c2", 0, precision, "gmg")


@pytest.mark.parametrize("levels", [3, 4])
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir", "bf16_ir", "bf16x3_ir"])
def test_c4_seed0_every_precision(precision, levels):
    """224x112x56 against the oracle's stored solution in every precision,
    with three levels and with the loop's four (Chebyshev-smoothed level 2,
    three-step coarse launches)."""
    _check("c4", 0, precision, "gmg", levels=levels)


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_c4_other_seeds(seed, precision):
    _check("c4", seed, precision, "gmg")
