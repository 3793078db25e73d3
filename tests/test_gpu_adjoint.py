"""The general adjoint gradient (Sec. III-A, Eq. 3) on the GPU against the
oracle: the state-equation term -lam^T dr/drho of fe_sensitivity_adjoint,
and the gradient of a linear objective J = l^T u through a second solve
with the load swapped by fe_set_load.

Tolerances: the kernel evaluates the bilinear form lam_e^T Ke u_e in the
factorised basis, the oracle with the dense 24 x 24 Ke: rounding of a
24 x 24-term sum, 1e-11 of max |g| for random fields; whole gradients use
the contract's 1e-5 relative max error."""
import numpy as np
import pytest
import torch

from oracle import fe_oracle as O
from paper_2104_12282_amd import fe, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


def N(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def Ke():
    return O.hex8_ke(0.3)


@pytest.mark.parametrize("grid", [(24, 12, 12), (13, 7, 5), (1, 1, 1), (2, 9, 3)])
def test_adjoint_term_parity(Ke, grid):
    nx, ny, nz = grid
    rng = np.random.default_rng(3)
    rho = synth.density_uniform(nx, ny, nz, seed=1)
    nd = 3 * (nx + 1) * (ny + 1) * (nz + 1)
    u, lam = rng.standard_normal(nd), rng.standard_normal(nd)
    prob = fe.Problem(nx, ny, nz, T(synth.cantilever_edge_load(nx, ny, nz)), device=DEV)
    g = N(prob.sensitivity_adjoint(T(rho), T(u), T(lam)))
    ref = O.adjoint_sensitivity(nx, ny, nz, Ke, rho, u, lam)
    assert np.abs(g - ref).max() <= 1e-11 * np.abs(ref).max()
    # symmetric in (u, lam); lam = u is the compliance sensitivity
    g2 = N(prob.sensitivity_adjoint(T(rho), T(lam), T(u)))
    assert np.abs(g2 - g).max() <= 1e-13 * np.abs(g).max()
    dc, _ = prob.sensitivity(T(rho), T(u))
    gu = N(prob.sensitivity_adjoint(T(rho), T(u), T(u)))
    assert np.abs(gu - N(dc)).max() <= 1e-13 * np.abs(gu).max()


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
@pytest.mark.parametrize("precond", ["jacobi", "gmg"])
def test_linear_objective_gradient_parity(Ke, precision, precond):
    nx, ny, nz = 24, 12, 12
    rho = synth.density_around(nx, ny, nz, 0)
    f = synth.cantilever_edge_load(nx, ny, nz)
    fixed = O.clamp_x0_fixed(nx, ny, nz)
    rng = np.random.default_rng(9)
    l = rng.standard_normal(f.size)
    prob = fe.Problem(nx, ny, nz, T(f), device=DEV, precision=precision, precond=precond, mg_levels=3)
    g, u, lam = prob.linear_objective_gradient(T(rho), T(l), rtol=1e-10)
    u_ref, lam_ref, g_ref = O.linear_objective_gradient(nx, ny, nz, Ke, rho, f, np.where(fixed, 0.0, l), fixed)
    assert np.abs(N(u) - u_ref).max() <= 1e-6 * np.abs(u_ref).max()
    assert np.abs(N(lam) - lam_ref).max() <= 1e-6 * np.abs(lam_ref).max()
    assert np.abs(N(g) - g_ref).max() <= 1e-5 * np.abs(g_ref).max()
    # the load is restored: the next solve is the forward solve again
    u2, info = prob.solve(T(rho), rtol=1e-10)
    assert abs(info["compliance"] - f @ u_ref) <= 1e-6 * abs(f @ u_ref)


def test_set_load_rejects_bad_arguments():
    prob = fe.Problem(6, 3, 3, T(synth.cantilever_edge_load(6, 3, 3)), device=DEV)
    with pytest.raises(fe.FEError):
        fe._check(fe.load_library().fe_set_load(prob._h, None))
    # a zero load gives the zero solution at once
    prob.set_load(T(np.zeros(prob.ndof)))
    u, info = prob.solve(T(np.full(54, 0.5)), rtol=1e-8)
    assert info["iters"] == 0 and not N(u).any()


@pytest.mark.parametrize("grid", [(96, 48, 48), (224, 112, 56)])
def test_fullsize_tip_displacement_gradient(Ke, grid):
    """J = -u_z at the middle of the loaded edge (a compliant-mechanism-like
    objective, not self-adjoint): the adjoint solve's float64 residual, and
    sampled gradient entries recomputed by the oracle from the GPU's u and
    lam (the factorised form drops rigid parts exactly, the dense one in
    floating point: 1e-10 of max |g| bounds that)."""
    nx, ny, nz = grid
    P = O.filter_matrix(nx, ny, nz, 1.5)
    rho = synth.density_uniform(nx, ny, nz, seed=0)
    for _ in range(3):
        rho = P @ rho
    f = synth.cantilever_edge_load(nx, ny, nz)
    l = np.zeros_like(f)
    l[3 * O.node_index(nx, ny, nz, nx, ny // 2, 0) + 2] = -1.0
    prob = fe.Problem(nx, ny, nz, T(f), device=DEV, precond="gmg", mg_levels=3)
    u, _ = prob.solve(T(rho), rtol=1e-9)
    prob.set_load(T(l))
    lam, info = prob.solve(T(rho), rtol=1e-9)
    assert info["rel_res"] <= 1e-9
    prob.set_load(T(f))
    g = N(prob.sensitivity_adjoint(T(rho), u, lam))
    ne = nx * ny * nz
    rng = np.random.default_rng(4)
    el = np.unique(np.concatenate([rng.integers(0, ne, 400), [0, nx - 1, ne - 1, ne // 2]]))
    ref = O.adjoint_sensitivity_elements(nx, ny, nz, Ke, rho, N(u), N(lam), el)
    assert np.abs(g[el] - ref).max() <= 1e-10 * np.abs(g).max()
    # Betti: the adjoint solve's f^T lam equals J = l^T u
    assert abs(float(N(u) @ l) - float(N(lam) @ f)) <= 1e-7 * abs(float(N(u) @ l))
