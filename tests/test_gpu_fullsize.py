"""Parity at the workload sizes (96x48x48 and the paper-scale 224x112x56),
in the configuration bench.py runs.  The oracle computes sampled K u rows
and sampled sensitivities one by one, the whole filter and OC, and the
compliance identity; the solve itself is checked through properties that
hold at any size (float64 residual, energy identity, precision agreement)."""
import numpy as np
import pytest
import torch

from oracle import fe_oracle as O
from paper_2104_12282_amd import fe, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
T = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def N(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _sample_nodes(nx, ny, nz, n, seed):
    rng = np.random.default_rng(seed)
    nn = (nx + 1) * (ny + 1) * (nz + 1)
    picks = list(rng.integers(0, nn, n))
    # tile seams of the K*u kernel (15-node blocks), domain faces and corners
    for i in (0, 1, 14, 15, 16, 29, 30, nx - 1, nx):
        for j in (0, 14, 15, ny):
            for k in (0, 7, 8, nz):
                if i <= nx and j <= ny and k <= nz:
                    picks.append(i + (nx + 1) * (j + (ny + 1) * k))
    return np.unique(np.array(picks))


@pytest.fixture(scope="module")
def Ke():
    return O.hex8_ke(0.3)


@pytest.mark.parametrize("grid", [(96, 48, 48), (224, 112, 56)])
def test_fullsize_kxu_sampled_rows(Ke, grid):
    nx, ny, nz = grid
    rho = synth.density_uniform(nx, ny, nz, seed=0)
    u = np.random.default_rng(1).standard_normal(3 * (nx + 1) * (ny + 1) * (nz + 1))
    fixed = O.clamp_x0_fixed(nx, ny, nz)
    nodes = _sample_nodes(nx, ny, nz, 400, seed=2)
    ref = O.apply_K_rows(nx, ny, nz, O.simp_modulus(rho), Ke, fixed, u, nodes)
    scale = np.abs(ref).max()
    for prec, variant, tol in (("fp64", 0, 1e-12), ("fp32_ir", 1, 5e-6)):
        prob = fe.Problem(nx, ny, nz, T(synth.cantilever_edge_load(nx, ny, nz)), device=DEV,
                          precision=prec, precond="gmg", mg_levels=3)
        y = N(prob.apply_K(T(rho), T(u), variant=variant)).reshape(-1, 3)[nodes]
        assert np.abs(y - ref).max() <= tol * scale, prec
        prob.close()


@pytest.mark.parametrize("grid,passes", [((96, 48, 48), 3), ((224, 112, 56), 5)])
def test_fullsize_solve_properties_and_sampled_sensitivity(Ke, grid, passes):
    nx, ny, nz = grid
    ne = nx * ny * nz
    f = synth.cantilever_edge_load(nx, ny, nz)
    P = O.filter_matrix(nx, ny, nz, 1.5)
    rho = synth.density_uniform(nx, ny, nz, seed=0)
    for _ in range(passes):
        rho = P @ rho
    res = {}
    for prec in ("fp64", "fp32_ir"):
        prob = fe.Problem(nx, ny, nz, T(f), device=DEV, precision=prec, precond="gmg", mg_levels=3)
        # the GPU filter reproduces the oracle's smoothing at full size
        xf = N(prob.filter(T(synth.density_uniform(nx, ny, nz, seed=0))))
        assert np.abs(xf - P @ synth.density_uniform(nx, ny, nz, seed=0)).max() <= 1e-14
        u, info = prob.solve(T(rho), rtol=1e-8)
        dc, c = prob.sensitivity(T(rho), u)
        res[prec] = (N(u), N(dc), float(N(c)[0]), info)
        assert info["rel_res"] <= 1e-8
        prob.close()
    u64, dc64, c64, _ = res["fp64"]
    # compliance identity f^T u = sum_e E_e u_e^T Ke u_e (energy of the GPU u, by the oracle)
    E = O.simp_modulus(rho)
    energy = float(np.sum(E * O.element_energies(nx, ny, nz, Ke, u64)))
    assert abs(energy - c64) / c64 <= 1e-6
    # sampled sensitivities recomputed by the oracle from the same u
    rng = np.random.default_rng(4)
    el = np.unique(np.concatenate([rng.integers(0, ne, 500), [0, nx - 1, ne - 1, ne // 2]]))
    ref = O.sensitivity_elements(nx, ny, nz, Ke, rho, u64, el)
    # the dense quadratic form u_e^T Ke u_e cancels the large rigid part of u_e
    # in floating point (24 x 24 terms of size |u_e|^2 |Ke|); the kernel's
    # factorised form drops translations exactly.  1e-10 of max |dc| bounds that.
    assert np.abs(dc64[el] - ref).max() <= 1e-10 * np.abs(dc64).max()
    # mixed precision reaches the float64 answer within the stated tolerances
    u32, dc32, c32, _ = res["fp32_ir"]
    assert abs(c32 - c64) / c64 <= 1e-6
    assert np.abs(dc32 - dc64).max() / np.abs(dc64).max() <= 1e-5


@pytest.mark.parametrize("grid", [(96, 48, 48), (224, 112, 56)])
def test_fullsize_filter_and_oc(grid):
    nx, ny, nz = grid
    ne = nx * ny * nz
    P = O.filter_matrix(nx, ny, nz, 1.5)
    rng = np.random.default_rng(5)
    x = rng.uniform(0.01, 0.6, ne)
    dcx = -rng.uniform(1e-6, 1.0, ne)
    prob = fe.Problem(nx, ny, nz, T(synth.cantilever_edge_load(nx, ny, nz)), device=DEV,
                      precond="gmg", mg_levels=3)
    for tr in (False, True):
        y = N(prob.filter(T(x), transpose=tr))
        y_ref = (P.T @ x) if tr else (P @ x)
        assert np.abs(y - y_ref).max() <= 1e-14
    dv = P.T @ np.ones(ne)
    xn_ref, _, ch_ref = O.oc_update(x, dcx, dv, 0.2, 0.2)
    xn, ch = prob.oc_update(T(x), T(dcx), T(dv), 0.2, 0.2)
    xn = N(xn)
    assert np.abs(xn - xn_ref).max() <= 1e-9
    assert abs(float(N(ch)[0]) - ch_ref) <= 1e-9


def test_fullsize_oc_near_binary():
    """A late design: most elements at a bound or a move limit over the whole
    multiplier bracket, a few hundred crossing a bound inside it; repeated
    calls give the same bits."""
    nx, ny, nz = 96, 48, 48
    ne = nx * ny * nz
    rng = np.random.default_rng(6)
    solid = rng.random(ne) < 0.2
    x = np.where(solid, 1.0 - rng.uniform(0.0, 1e-3, ne), rng.uniform(1e-3, 2e-3, ne))
    mid = rng.random(ne) < 0.01
    x[mid] = rng.uniform(0.05, 0.95, mid.sum())
    dcx = -np.where(solid | mid, rng.uniform(0.5, 2.0, ne), rng.uniform(1e-9, 1e-6, ne))
    dv = O.filter_matrix(nx, ny, nz, 1.5).T @ np.ones(ne)
    prob = fe.Problem(nx, ny, nz, T(synth.cantilever_edge_load(nx, ny, nz)), device=DEV)
    for volfrac, move in ((0.21, 0.2), (0.2, 0.05)):
        xn_ref, _, ch_ref = O.oc_update(x, dcx, dv, volfrac, move)
        xn, ch = prob.oc_update(T(x), T(dcx), T(dv), volfrac, move)
        xn2, _ = prob.oc_update(T(x), T(dcx), T(dv), volfrac, move)
        assert torch.equal(xn, xn2)
        assert np.abs(N(xn) - xn_ref).max() <= 1e-9
        assert abs(float(N(ch)[0]) - ch_ref) <= 1e-9
