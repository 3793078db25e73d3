"""The coarse scale of the two-scale scheme on the GPU against the oracle:
block means of the design variables, and the coarse solve K_C(z_C) u_C = f_C
(block means, the filter of the same physical radius, SIMP, element edge
nb h) through fe_block_mean and an fe_problem of the coarse grid.

Tolerances: a block mean sums nb^3 values, so it may differ from the
oracle's (pairwise) sum by nb^3 roundings of max |z|; the coarse solves use
the contract's 1e-6 relative compliance."""
import numpy as np
import pytest
import torch

from oracle import fe_oracle as O
from paper_2104_12282_amd import fe, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
EPS = np.finfo(np.float64).eps


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def N(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _fine(nx, ny, nz, **kw):
    kw.setdefault("precond", "gmg")
    kw.setdefault("mg_levels", 2)
    return fe.Problem(nx, ny, nz, T(synth.cantilever_edge_load(nx, ny, nz)), device=DEV, **kw)


@pytest.mark.parametrize("grid,nbs", [((24, 12, 12), (1, 2, 3, 4, 6, 12)), ((30, 10, 20), (5, 10)),
                                      ((14, 14, 14), (7,)), ((2, 2, 2), (1, 2))])
def test_block_mean_parity(grid, nbs):
    nx, ny, nz = grid
    z = synth.density_uniform(nx, ny, nz, seed=11)
    prob = _fine(nx, ny, nz, precond="jacobi")
    for nb in nbs:
        zc = N(prob.block_mean(T(z), nb))
        ref = O.block_mean(nx, ny, nz, z, nb)
        if nb == 1:
            assert np.array_equal(zc, ref)
        else:
            assert zc.shape == ref.shape
            assert np.abs(zc - ref).max() <= nb ** 3 * EPS * np.abs(z).max()


def test_block_mean_rejects_bad_arguments():
    prob = _fine(12, 6, 6, precond="jacobi")
    z = T(np.ones(12 * 6 * 6))
    for nb in (0, -1, 4, 5, 7):
        with pytest.raises(fe.FEError):
            prob.block_mean(z, nb)
    with pytest.raises(fe.FEError):
        prob.block_mean(z, 1, out=z)
    with pytest.raises(fe.FEError):
        prob.coarse_problem(5, T(np.zeros(3)))


@pytest.mark.parametrize("nb", [2, 3, 4])
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_coarse_solve_parity(nb, precision):
    nx, ny, nz = 24, 12, 12
    z = synth.density_uniform(nx, ny, nz, seed=5)
    fine = _fine(nx, ny, nz, precision=precision, mg_levels=3)
    cx, cy, cz = nx // nb, ny // nb, nz // nb
    f_c = synth.cantilever_edge_load(cx, cy, cz)
    coarse = fine.coarse_problem(nb, T(f_c))
    zc = fine.block_mean(T(z), nb)
    coarse_rho = coarse.filter(zc)
    u, info = coarse.solve(coarse_rho, rtol=1e-10)
    zc_ref, u_ref, c_ref = O.coarse_scale_solve(nx, ny, nz, z, nb, f_c)
    assert np.abs(N(zc) - zc_ref).max() <= nb ** 3 * EPS
    assert abs(info["compliance"] - c_ref) / c_ref <= 1e-6
    assert np.abs(N(u) - u_ref).max() <= 1e-6 * np.abs(u_ref).max()
    _, c = coarse.sensitivity(coarse_rho, u)
    assert abs(float(N(c)[0]) - c_ref) / c_ref <= 1e-6


def test_block_size_one_is_the_fine_problem():
    nx, ny, nz = 16, 8, 8
    z = T(synth.density_uniform(nx, ny, nz, seed=2))
    fine = _fine(nx, ny, nz, mg_levels=3)
    coarse = fine.coarse_problem(1, fine.f)
    assert torch.equal(fine.block_mean(z, 1), z)
    rho = fine.filter(z)
    assert torch.equal(coarse.filter(z), rho)
    u1, i1 = fine.solve(rho, rtol=1e-9)
    u2, i2 = coarse.solve(rho, rtol=1e-9)
    assert i1["iters"] == i2["iters"] and torch.equal(u1, u2)


@pytest.mark.parametrize("nb", [2, 4, 7, 8])
def test_fullsize_block_means(nb):
    nx, ny, nz = 224, 112, 56
    z = synth.density_uniform(nx, ny, nz, seed=0)
    prob = fe.Problem(nx, ny, nz, T(synth.cantilever_edge_load(nx, ny, nz)), device=DEV, precond="gmg",
                      mg_levels=3)
    zc = N(prob.block_mean(T(z), nb))
    assert np.abs(zc - O.block_mean(nx, ny, nz, z, nb)).max() <= nb ** 3 * EPS


def test_fullsize_coarse_solves():
    """224x112x56 design, block sizes 8 (28x14x7, 3-level multigrid whose
    coarse levels overhang the odd axis: checked against the oracle's direct
    solve) and 4 (56x28x14, 3-level multigrid: float64
    residual and the energy identity by the oracle)."""
    nx, ny, nz = 224, 112, 56
    P = O.filter_matrix(nx, ny, nz, 1.5)
    z = synth.density_uniform(nx, ny, nz, seed=0)
    for _ in range(3):
        z = P @ z
    fine = fe.Problem(nx, ny, nz, T(synth.cantilever_edge_load(nx, ny, nz)), device=DEV, precond="gmg",
                      mg_levels=3)
    for nb in (8, 4):
        cx, cy, cz = nx // nb, ny // nb, nz // nb
        f_c = synth.cantilever_edge_load(cx, cy, cz)
        coarse = fine.coarse_problem(nb, T(f_c))
        rho_c = coarse.filter(fine.block_mean(T(z), nb))
        u, info = coarse.solve(rho_c, rtol=1e-9)
        assert info["rel_res"] <= 1e-9
        if nb == 8:
            _, u_ref, c_ref = O.coarse_scale_solve(nx, ny, nz, z, nb, f_c)
            assert abs(info["compliance"] - c_ref) / c_ref <= 1e-6
            assert np.abs(N(u) - u_ref).max() <= 1e-6 * np.abs(u_ref).max()
        else:
            Ke = O.hex8_ke(0.3, h=nb)
            E = O.simp_modulus(N(rho_c))
            energy = float(np.sum(E * O.element_energies(cx, cy, cz, Ke, N(u))))
            assert abs(energy - info["compliance"]) / info["compliance"] <= 1e-6
        coarse.close()
