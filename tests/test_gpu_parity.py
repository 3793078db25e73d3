"""Parity of the HIP path with the FP64 CPU oracle on seeded synthetic inputs.

Tolerances (stated by the build contract for floating point):
  compliance   |c - c*| / |c*|              <= 1e-6
  sensitivity  ||dc - dc*||_inf / ||dc*||_inf <= 1e-5
Kernel-level checks use tolerances derived from the arithmetic: float64
rounding of a 24-term sum (1e-12 relative to max |y*|), float32 (5e-6).
"""
import numpy as np
import pytest
import torch

from oracle import fe_oracle as O
from paper_2104_12282_amd import fe, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
NU = 0.3

# grids spanning several workgroups with ragged tails, plus degenerate ones
GRIDS = [(24, 12, 12), (13, 7, 5), (37, 19, 11), (1, 1, 1), (5, 1, 1), (2, 9, 3), (31, 16, 17),
         (16, 29, 9)]


def T(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def N(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def Ke():
    return O.hex8_ke(NU)


def _problem(nx, ny, nz, precision="fp64", f=None, fixed=None, **kw):
    if f is None:
        f = synth.cantilever_edge_load(nx, ny, nz)
    fx = None if fixed is None else T(fixed, torch.uint8)
    return fe.Problem(nx, ny, nz, T(f), fx, device=DEV, precision=precision, nu=NU, **kw)


@pytest.mark.parametrize("grid", GRIDS)
@pytest.mark.parametrize("variant", [0, 1, 3])
def test_kxu_matches_assembled_K(Ke, grid, variant):
    nx, ny, nz = grid
    rho = synth.density_uniform(nx, ny, nz, seed=3)
    E = O.simp_modulus(rho)
    rng = np.random.default_rng(4)
    u = rng.standard_normal(3 * (nx + 1) * (ny + 1) * (nz + 1))
    fixed = O.clamp_x0_fixed(nx, ny, nz)
    y_ref = O.apply_K_free(O.assemble_K(nx, ny, nz, E, Ke), fixed, u)
    prob = _problem(nx, ny, nz, precision="fp32_ir" if variant == 1 else "fp64")
    y = N(prob.apply_K(T(rho), T(u), variant=variant))
    scale = np.abs(y_ref).max()
    tol = 5e-6 if variant == 1 else 1e-12
    assert np.abs(y - y_ref).max() <= tol * scale


def test_kxu_general_fixed_mask(Ke):
    nx, ny, nz = 11, 6, 4
    rng = np.random.default_rng(9)
    fixed = rng.random(3 * (nx + 1) * (ny + 1) * (nz + 1)) < 0.1
    rho = synth.density_uniform(nx, ny, nz, seed=5)
    u = rng.standard_normal(fixed.size)
    y_ref = O.apply_K_free(O.assemble_K(nx, ny, nz, O.simp_modulus(rho), Ke), fixed, u)
    prob = _problem(nx, ny, nz, fixed=fixed.astype(np.uint8))
    y = N(prob.apply_K(T(rho), T(u)))
    assert np.abs(y - y_ref).max() <= 1e-12 * np.abs(y_ref).max()


def _solve_case(Ke, nx, ny, nz, seed, precision, rtol, density="around"):
    if density == "around":
        rho = synth.density_around(nx, ny, nz, seed)
    else:
        P = O.filter_matrix(nx, ny, nz, 1.5)
        rho = P @ (P @ (P @ synth.density_uniform(nx, ny, nz, seed)))
    f = synth.cantilever_edge_load(nx, ny, nz)
    fixed = O.clamp_x0_fixed(nx, ny, nz)
    u_ref = O.solve_direct(nx, ny, nz, O.simp_modulus(rho), Ke, f, fixed)
    c_ref = O.compliance(f, u_ref)
    dc_ref = O.sensitivity(nx, ny, nz, Ke, rho, u_ref)
    prob = _problem(nx, ny, nz, precision=precision)
    u, info = prob.solve(T(rho), rtol=rtol)
    dc, c = prob.sensitivity(T(rho), u)
    return dict(u=N(u), info=info, dc=N(dc), c=float(N(c)[0]), u_ref=u_ref, c_ref=c_ref,
                dc_ref=dc_ref)


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
@pytest.mark.parametrize("grid", [(24, 12, 12), (13, 7, 5), (20, 9, 6)])
def test_solve_compliance_sensitivity(Ke, grid, precision):
    r = _solve_case(Ke, *grid, seed=0, precision=precision, rtol=1e-10)
    assert r["info"]["rel_res"] <= 1e-10
    assert abs(r["c"] - r["c_ref"]) / abs(r["c_ref"]) <= 1e-6
    assert abs(r["info"]["compliance"] - r["c_ref"]) / abs(r["c_ref"]) <= 1e-6
    err = np.abs(r["dc"] - r["dc_ref"]).max() / np.abs(r["dc_ref"]).max()
    assert err <= 1e-5, err
    assert np.abs(r["u"] - r["u_ref"]).max() <= 1e-6 * np.abs(r["u_ref"]).max()


def test_solve_smoothed_density(Ke):
    r = _solve_case(Ke, 16, 8, 8, seed=1, precision="fp64", rtol=1e-10, density="smoothed")
    assert abs(r["c"] - r["c_ref"]) / abs(r["c_ref"]) <= 1e-6
    assert np.abs(r["dc"] - r["dc_ref"]).max() / np.abs(r["dc_ref"]).max() <= 1e-5


def test_sensitivity_kernel_given_u(Ke):
    nx, ny, nz = 37, 19, 11
    rho = synth.density_uniform(nx, ny, nz, seed=8)
    u = np.random.default_rng(1).standard_normal(3 * (nx + 1) * (ny + 1) * (nz + 1))
    prob = _problem(nx, ny, nz)
    dc, _ = prob.sensitivity(T(rho), T(u))
    dc_ref = O.sensitivity(nx, ny, nz, Ke, rho, u)
    assert np.abs(N(dc) - dc_ref).max() <= 1e-12 * np.abs(dc_ref).max()


@pytest.mark.parametrize("grid", GRIDS)
@pytest.mark.parametrize("r", [1.5, 2.3, 2.8, 4.0, 7.2, 8.0])
def test_filter_parity(grid, r):
    """Radii from the 19-point stencil to the paper's 0.08 on its finest mesh
    (7.2 elements, 1,560 points) and the largest supported (8).  The kernel
    sums in stencil order, the oracle in column order: n terms of at most
    max |y| each, so 2e-16 n relative (at least 1e-14) bounds the difference."""
    nx, ny, nz = grid
    x = synth.density_uniform(nx, ny, nz, seed=2)
    prob = _problem(nx, ny, nz, filter_r=r)
    P = O.filter_matrix(nx, ny, nz, r)
    R = int(np.ceil(r))
    d = np.arange(-R, R + 1)
    nst = int(np.sum(r - np.sqrt(d[:, None, None] ** 2 + d[None, :, None] ** 2 + d[None, None, :] ** 2) > 0))
    tol = max(1e-14, 2e-16 * nst)
    for tr in (False, True):
        y = N(prob.filter(T(x), transpose=tr))
        y_ref = (P.T @ x) if tr else (P @ x)
        assert np.abs(y - y_ref).max() <= tol * max(1.0, np.abs(y_ref).max())


@pytest.mark.parametrize("grid", [(24, 12, 12), (37, 19, 11), (3, 2, 1)])
def test_oc_parity(grid):
    nx, ny, nz = grid
    n = nx * ny * nz
    rng = np.random.default_rng(13)
    x = rng.uniform(0.01, 0.6, n)
    dcx = -rng.uniform(1e-4, 5.0, n)
    dcx[rng.random(n) < 0.05] = 0.0
    prob = _problem(nx, ny, nz)
    dv = N(prob.filter(T(np.ones(n)), transpose=True))
    dv_ref = O.filter_matrix(nx, ny, nz, 1.5).T @ np.ones(n)
    assert np.abs(dv - dv_ref).max() <= 1e-14
    volfrac, move = 0.3, 0.2
    xn_ref, lam_ref, ch_ref = O.oc_update(x, dcx, dv_ref, volfrac, move)
    xn, ch = prob.oc_update(T(x), T(dcx), T(dv_ref), volfrac, move)
    xn = N(xn)
    assert np.abs(xn - xn_ref).max() <= 1e-9
    assert abs(float(N(ch)[0]) - ch_ref) <= 1e-9
    assert abs(np.sum(dv_ref * xn) - volfrac * n) <= 1e-10 * volfrac * n


def test_oc_in_place():
    nx, ny, nz = 9, 5, 4
    n = nx * ny * nz
    rng = np.random.default_rng(2)
    x = rng.uniform(0.05, 0.5, n)
    dcx = -rng.uniform(0.1, 1.0, n)
    dv = np.ones(n)
    prob = _problem(nx, ny, nz)
    xt = T(x)
    prob.oc_update(xt, T(dcx), T(dv), 0.25, 0.2, out=xt)
    xn_ref, _, _ = O.oc_update(x, dcx, dv, 0.25, 0.2)
    assert np.abs(N(xt) - xn_ref).max() <= 1e-9


def test_oc_graph_replays():
    """Repeated calls on the same arrays replay one captured OC graph (the
    first call launches directly, the second captures): with eager writes of
    new inputs between the calls every replay matches the directly launched
    update of the same inputs bit for bit, and the oracle."""
    nx, ny, nz = 40, 20, 12
    n = nx * ny * nz
    rng = np.random.default_rng(31)
    dv = O.filter_matrix(nx, ny, nz, 1.5).T @ np.ones(n)
    cases = [(rng.uniform(0.01, 0.9, n), -rng.uniform(1e-5, 2.0, n)) for _ in range(5)]
    # directly launched references: every call has its own arrays (kept alive,
    # so no two calls share an address)
    ref_prob = _problem(nx, ny, nz)
    keep, refs = [], []
    for x, dcx in cases:
        a, b, c = T(x), T(dcx), T(dv)
        xn, ch = ref_prob.oc_update(a, b, c, 0.3, 0.2)
        keep += [a, b, c, xn, ch]
        refs.append((xn, ch))
    prob = _problem(nx, ny, nz)
    xt, dct, dvt = T(np.zeros(n)), T(np.zeros(n)), T(dv)
    out = torch.empty_like(xt)
    chg = torch.zeros(1, dtype=torch.float64, device=DEV)
    for (x, dcx), (xr, cr) in zip(cases, refs):
        xt.copy_(T(x))
        dct.copy_(T(dcx))
        prob.oc_update(xt, dct, dvt, 0.3, 0.2, out=out, change_out=chg)
        torch.cuda.synchronize()
        assert torch.equal(out, xr) and torch.equal(chg, cr)
        xn_ref, _, ch_ref = O.oc_update(x, dcx, dv, 0.3, 0.2)
        assert np.abs(N(out) - xn_ref).max() <= 1e-9
        assert abs(float(N(chg)[0]) - ch_ref) <= 1e-9
    # in place (x_new = x), as an optimisation loop calls it
    for x, dcx in cases[:3]:
        xt.copy_(T(x))
        dct.copy_(T(dcx))
        prob.oc_update(xt, dct, dvt, 0.3, 0.2, out=xt, change_out=chg)
        xn_ref, _, _ = O.oc_update(x, dcx, dv, 0.3, 0.2)
        assert np.abs(N(xt) - xn_ref).max() <= 1e-9


def test_solve_deterministic():
    nx, ny, nz = 20, 9, 6
    rho = synth.density_around(nx, ny, nz, 4)
    prob = _problem(nx, ny, nz)
    u1, i1 = prob.solve(T(rho), rtol=1e-9)
    u2, i2 = prob.solve(T(rho), rtol=1e-9)
    assert i1["iters"] == i2["iters"]
    assert torch.equal(u1, u2)


def test_notconv_and_warm_start():
    nx, ny, nz = 20, 9, 6
    rho = synth.density_around(nx, ny, nz, 4)
    prob = _problem(nx, ny, nz)
    with pytest.raises(fe.FEError) as ei:
        prob.solve(T(rho), rtol=1e-12, max_iters=3)
    assert ei.value.status == fe.FE_ENOTCONV
    u, info = prob.solve(T(rho), rtol=1e-12, max_iters=3, allow_notconv=True)
    assert info["status"] == fe.FE_ENOTCONV and info["iters"] == 3
    u_full, info_full = prob.solve(T(rho), rtol=1e-9)
    u_warm, info_warm = prob.solve(T(rho), u=u_full.clone(), rtol=1e-9)
    assert info_warm["iters"] == 0


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_every_iteration_count_moves_the_iterate(Ke, precision):
    """Multigrid CG applies its x update every second iteration, for two
    steps; a solve stopped after an iteration that deferred its step applies
    it at the end.  CG minimises the energy 1/2 u^T K u - f^T u over growing
    Krylov spaces, so after k = 1, 2, ... iterations (stopped by the cap) the
    energy of the returned u (oracle K) falls strictly with k: a lost step
    at an odd or even count would leave u where it was one iteration
    earlier."""
    nx, ny, nz = 16, 8, 8
    rho = synth.density_around(nx, ny, nz, 2)
    f = synth.cantilever_edge_load(nx, ny, nz)
    fixed = O.clamp_x0_fixed(nx, ny, nz)
    K = O.assemble_K(nx, ny, nz, O.simp_modulus(rho), Ke)
    prob = _problem(nx, ny, nz, precision, precond="gmg", mg_levels=3)
    energies = []
    for k in range(1, 8):
        u, info = prob.solve(T(rho), rtol=1e-14, max_iters=k, allow_notconv=True)
        assert info["status"] == fe.FE_ENOTCONV and info["iters"] == k
        un = N(u)
        Ku = O.apply_K_free(K, fixed, un)
        energies.append(0.5 * float(un @ Ku) - float(f @ un))
    drops = -np.diff(energies)
    assert (drops > 1e-9 * abs(energies[-1])).all(), energies


def test_breakdown_on_nan_density():
    nx, ny, nz = 6, 3, 3
    rho = synth.density_around(nx, ny, nz, 1)
    rho[5] = np.nan
    prob = _problem(nx, ny, nz)
    with pytest.raises(fe.FEError) as ei:
        prob.solve(T(rho), rtol=1e-8, max_iters=100)
    assert ei.value.status == fe.FE_EBREAKDOWN


@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
@pytest.mark.parametrize("grid,levels", [((24, 12, 12), 3), ((16, 8, 8), 2), ((32, 16, 8), 4),
                                         ((13, 7, 5), 3), ((25, 12, 9), 3), ((30, 15, 15), 3), ((21, 11, 7), 4)])
def test_gmg_solve_parity(Ke, grid, levels, precision):
    nx, ny, nz = grid
    rho = synth.density_around(nx, ny, nz, 3)
    f = synth.cantilever_edge_load(nx, ny, nz)
    u_ref = O.solve_direct(nx, ny, nz, O.simp_modulus(rho), Ke, f, O.clamp_x0_fixed(nx, ny, nz))
    c_ref = O.compliance(f, u_ref)
    dc_ref = O.sensitivity(nx, ny, nz, Ke, rho, u_ref)
    prob = _problem(nx, ny, nz, precision=precision, precond="gmg", mg_levels=levels)
    u, info = prob.solve(T(rho), rtol=1e-10)
    dc, c = prob.sensitivity(T(rho), u)
    assert info["rel_res"] <= 1e-10
    assert abs(float(N(c)[0]) - c_ref) / c_ref <= 1e-6
    assert np.abs(N(dc) - dc_ref).max() / np.abs(dc_ref).max() <= 1e-5
    # the multigrid preconditioner must beat Jacobi on the same system
    jac = _problem(nx, ny, nz, precision=precision)
    _, info_j = jac.solve(T(rho), rtol=1e-10)
    assert info["iters"] < info_j["iters"]


@pytest.mark.parametrize("grid,levels", [((28, 14, 14), 2), ((30, 15, 15), 3)])
@pytest.mark.parametrize("precond", ["jacobi", "gmg"])
def test_paper_domain_step_parity(Ke, precond, grid, levels):
    """The paper's cantilever geometry (2 x 1 x 1 domain, h = 2 / nx, filter
    radius 0.08 = 1.12-1.2 elements here) on 28x14x14 and on 30x15x15 (odd
    like the paper's 70x35x35 mesh: its coarse levels overhang the mesh):
    one optimisation step's filter, solve, compliance and sensitivity
    against the oracle with Ke of edge h."""
    nx, ny, nz = grid
    h = 2.0 / nx
    r = 0.08 / h
    x = synth.density_uniform(nx, ny, nz, seed=8)
    f = synth.cantilever_edge_load(nx, ny, nz)
    prob = fe.Problem(nx, ny, nz, T(f), device=DEV, h=h, filter_r=r, precond=precond, mg_levels=levels)
    rho = prob.filter(T(x))
    P = O.filter_matrix(nx, ny, nz, r)
    rho_ref = P @ x
    assert np.abs(N(rho) - rho_ref).max() <= 1e-14
    u, info = prob.solve(rho, rtol=1e-10)
    Keh = O.hex8_ke(NU, h=h)
    u_ref = O.solve_direct(nx, ny, nz, O.simp_modulus(rho_ref), Keh, f, O.clamp_x0_fixed(nx, ny, nz))
    c_ref = O.compliance(f, u_ref)
    assert abs(info["compliance"] - c_ref) / c_ref <= 1e-6
    dc, _ = prob.sensitivity(rho, u)
    dc_ref = O.sensitivity(nx, ny, nz, Keh, rho_ref, u_ref)
    assert np.abs(N(dc) - dc_ref).max() <= 1e-5 * np.abs(dc_ref).max()


@pytest.mark.parametrize("grid,levels", [((24, 12, 12), 3), ((32, 16, 16), 3), ((20, 10, 6), 2)])
def test_float32_levels_in_float64_solves(Ke, grid, levels):
    """Float64 solves with their multigrid levels from k on in float32 (k =
    0, the default, includes the finest level's smoothing; k = levels keeps
    float64) reach the oracle's
    answer to the contract's tolerances; float32 rounding in the
    preconditioner costs some iterations near a tight tolerance (1e-10 here:
    up to a quarter more); levels outside [1, levels] are rejected."""
    nx, ny, nz = grid
    rho = synth.density_uniform(nx, ny, nz, seed=3)
    f = synth.cantilever_edge_load(nx, ny, nz)
    fixed = O.clamp_x0_fixed(nx, ny, nz)
    u_ref = O.solve_direct(nx, ny, nz, O.simp_modulus(rho), Ke, f, fixed)
    c_ref = O.compliance(f, u_ref)
    dc_ref = O.sensitivity(nx, ny, nz, Ke, rho, u_ref)
    its = {}
    for first in range(0, levels + 1):
        prob = _problem(nx, ny, nz, precond="gmg", mg_levels=levels)
        prob.set_float32_levels(first)
        u, info = prob.solve(T(rho), rtol=1e-10)
        assert info["rel_res"] <= 1e-10
        assert abs(info["compliance"] - c_ref) / c_ref <= 1e-6
        dc, _ = prob.sensitivity(T(rho), u)
        assert np.abs(N(dc) - dc_ref).max() <= 1e-5 * np.abs(dc_ref).max()
        its[first] = info["iters"]
        for bad in (-1, levels + 1):
            with pytest.raises(fe.FEError):
                prob.set_float32_levels(bad)
        prob.close()
    for first in range(0, levels):
        assert its[first] <= 2 + 1.25 * its[levels]
    # the default is the whole preconditioner in float32
    prob = _problem(nx, ny, nz, precond="gmg", mg_levels=levels)
    u, info = prob.solve(T(rho), rtol=1e-10)
    assert info["iters"] == its[0]


def test_gmg_params_validation():
    prob = _problem(16, 8, 8, precond="gmg", mg_levels=3)
    with pytest.raises(fe.FEError):
        prob.set_mg_params(nu=0)
    with pytest.raises(fe.FEError):  # unstable smoother: omega * 5.32 >= 2
        prob.set_mg_params(omega=0.6)
    with pytest.raises(fe.FEError):  # empty Chebyshev interval
        prob.set_mg_params(coarse_ratio=1.0)
    prob.set_mg_params(nu=2, coarse_sweeps=10, omega=0.3)
    rho = synth.density_around(16, 8, 8, 1)
    _, info = prob.solve(T(rho), rtol=1e-9)
    assert info["rel_res"] <= 1e-9
    # a wide interval (the residual polynomial stays in (0, 1) below it):
    # still a symmetric positive definite preconditioner
    prob.set_mg_params(coarse_sweeps=30, coarse_ratio=1e8)
    _, info = prob.solve(T(rho), rtol=1e-9)
    assert info["rel_res"] <= 1e-9


def test_gmg_default_coarse_chebyshev_follows_the_coarsest_grid():
    """Defaults: degree 2 clamp(round(12 n / 28), 4, 24) and interval ratio
    max(50, 5000 min(1, (n / 56)^2)) for the coarsest grid's longest
    dimension n; fe_set_mg_params overrides them and fe_get_mg_params reads
    what is in effect."""
    cases = {(224, 112, 56): (48, 5000.0), (32, 16, 16): (8, 5000.0 * (8 / 56) ** 2),
             (96, 48, 48): (20, 5000.0 * (24 / 56) ** 2), (8, 4, 4): (8, 50.0)}
    for (nx, ny, nz), (deg, ratio) in cases.items():
        prob = fe.Problem(nx, ny, nz, T(synth.cantilever_edge_load(nx, ny, nz)), device=DEV, precond="gmg",
                          mg_levels=3)
        mg = prob.mg_params()
        assert mg["coarse_sweeps"] == deg and abs(mg["coarse_ratio"] - ratio) <= 1e-9 * ratio
        assert mg["nu"] == 1 and mg["omega"] == 0.35
        prob.set_mg_params(nu=2, coarse_sweeps=13, omega=0.3, coarse_ratio=700.0)
        assert prob.mg_params() == {"nu": 2, "coarse_sweeps": 13, "omega": 0.3, "coarse_ratio": 700.0}
        prob.close()


def test_oc_extreme_dynamic_range():
    """Late designs have void elements with x ~ 1e-50 and dc ~ 1e-80: the
    multiplier then lies hundreds of decades below the largest a-scale."""
    nx, ny, nz = 20, 10, 6
    n = nx * ny * nz
    rng = np.random.default_rng(21)
    x = np.where(rng.random(n) < 0.7, 10.0 ** rng.uniform(-60, -20, n), rng.uniform(0.2, 1.0, n))
    dcx = -np.where(x < 1e-10, 10.0 ** rng.uniform(-90, -40, n), rng.uniform(1e-3, 1.0, n))
    x[:40] = 0.0            # elements driven to zero
    x[40:80] = 1e-310       # subnormal densities
    dcx[80:90] = 0.0        # no descent information
    dv = O.filter_matrix(nx, ny, nz, 1.5).T @ np.ones(n)
    move = 0.2
    prob = _problem(nx, ny, nz)
    # reachable target (between the all-lower and all-upper volumes 0.128, 0.383)
    volfrac = 0.2
    xn_ref, lam_ref, ch_ref = O.oc_update(x, dcx, dv, volfrac, move)
    xn, ch = prob.oc_update(T(x), T(dcx), T(dv), volfrac, move)
    xn = N(xn)
    assert abs(np.sum(dv * xn) - volfrac * n) <= 1e-10 * volfrac * n
    assert np.abs(xn - xn_ref).max() <= 1e-9
    # unreachable target below the all-lower volume: every element at its lower bound
    xn2, _ = prob.oc_update(T(x), T(dcx), T(dv), 0.12, move)
    assert np.array_equal(N(xn2), np.maximum(0.0, x - move))
    xn2_ref, _, _ = O.oc_update(x, dcx, dv, 0.12, move)
    assert np.abs(xn2_ref - np.maximum(0.0, x - move)).max() <= 1e-300


@pytest.mark.parametrize("precond", ["jacobi", "gmg"])
def test_optimisation_trajectory(Ke, precond):
    """Twelve iterations of the whole loop (filter, solve, sensitivity,
    transpose filter, OC) from the uniform start: the GPU's compliance history
    follows the oracle's."""
    nx, ny, nz = 32, 16, 8
    ne = nx * ny * nz
    f = synth.cantilever_edge_load(nx, ny, nz)
    fixed = O.clamp_x0_fixed(nx, ny, nz)
    P = O.filter_matrix(nx, ny, nz, 1.5)
    dv_ref = P.T @ np.ones(ne)
    x_ref = np.full(ne, 0.12)
    c_ref = []
    for _ in range(12):
        rho = P @ x_ref
        u = O.solve_direct(nx, ny, nz, O.simp_modulus(rho), Ke, f, fixed)
        c_ref.append(O.compliance(f, u))
        dc = O.sensitivity(nx, ny, nz, Ke, rho, u)
        x_ref, _, _ = O.oc_update(x_ref, P.T @ dc, dv_ref, 0.12, 0.2)
    prob = _problem(nx, ny, nz, precond=precond, mg_levels=3)
    x = T(np.full(ne, 0.12))
    u = torch.zeros(prob.ndof, dtype=torch.float64, device=DEV)
    dv = prob.filter(torch.ones_like(x), transpose=True)
    c_gpu = []
    for _ in range(12):
        rho = prob.filter(x)
        _, info = prob.solve(rho, u=u, rtol=1e-10)
        c_gpu.append(info["compliance"])
        dc, _ = prob.sensitivity(rho, u)
        x, _ = prob.oc_update(x, prob.filter(dc, transpose=True), dv, 0.12, 0.2)
    rel = np.abs(np.array(c_gpu) - np.array(c_ref)) / np.array(c_ref)
    assert rel.max() <= 1e-6, rel
    assert np.abs(N(x) - x_ref).max() <= 1e-6


@pytest.mark.parametrize("grid", [(24, 12, 12), (37, 19, 11), (31, 16, 17)])
def test_kxu_bf16_mfma_accuracy(Ke, grid):
    """bf16 operands, float32 accumulation: rows agree with float64 to the
    bf16 rounding of Ke and of the corner-0-relative brick displacements."""
    nx, ny, nz = grid
    rho = synth.density_uniform(nx, ny, nz, seed=3)
    E = O.simp_modulus(rho)
    fixed = O.clamp_x0_fixed(nx, ny, nz)
    K = O.assemble_K(nx, ny, nz, E, Ke)
    prob = _problem(nx, ny, nz, precision="bf16_ir")
    rng = np.random.default_rng(4)
    # a rough field and a smooth (bending-like) field plus a large translation
    nn = (nx + 1) * (ny + 1) * (nz + 1)
    X = np.stack([np.arange(nn) % (nx + 1), (np.arange(nn) // (nx + 1)) % (ny + 1),
                  np.arange(nn) // ((nx + 1) * (ny + 1))], axis=1).astype(float)
    smooth = np.stack([0.01 * X[:, 0] * X[:, 2], 0.002 * X[:, 1] ** 2, -0.01 * X[:, 0] ** 2], axis=1)
    for u, tol in ((rng.standard_normal(3 * nn), 2e-2), ((smooth + 50.0).ravel(), 2e-2)):
        y_ref = O.apply_K_free(K, fixed, u)
        y = N(prob.apply_K(T(rho), T(u), variant=2))
        assert np.abs(y - y_ref).max() <= tol * np.abs(y_ref).max()


@pytest.mark.parametrize("precond", ["jacobi", "gmg"])
def test_bf16_refined_solve_parity(Ke, precond):
    nx, ny, nz = 24, 12, 12
    rho = synth.density_around(nx, ny, nz, 0)
    f = synth.cantilever_edge_load(nx, ny, nz)
    u_ref = O.solve_direct(nx, ny, nz, O.simp_modulus(rho), Ke, f, O.clamp_x0_fixed(nx, ny, nz))
    c_ref = O.compliance(f, u_ref)
    dc_ref = O.sensitivity(nx, ny, nz, Ke, rho, u_ref)
    prob = _problem(nx, ny, nz, precision="bf16_ir", precond=precond, mg_levels=3)
    u, info = prob.solve(T(rho), rtol=1e-10)
    dc, c = prob.sensitivity(T(rho), u)
    assert info["rel_res"] <= 1e-10 and info["outer_iters"] >= 2
    assert abs(float(N(c)[0]) - c_ref) / c_ref <= 1e-6
    assert np.abs(N(dc) - dc_ref).max() / np.abs(dc_ref).max() <= 1e-5


@pytest.mark.parametrize("nu", [2, 3])
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_gmg_smoothing_sweeps_parity(Ke, nu, precision):
    """More than one smoothing sweep takes the fused first sweep through a
    smoothing launch (and, for nu = 3, the ping-pong of the later sweeps)."""
    nx, ny, nz = 24, 12, 12
    rho = synth.density_around(nx, ny, nz, 0)
    f = synth.cantilever_edge_load(nx, ny, nz)
    u_ref = O.solve_direct(nx, ny, nz, O.simp_modulus(rho), Ke, f, O.clamp_x0_fixed(nx, ny, nz))
    c_ref = O.compliance(f, u_ref)
    dc_ref = O.sensitivity(nx, ny, nz, Ke, rho, u_ref)
    prob = _problem(nx, ny, nz, precision=precision, precond="gmg", mg_levels=3)
    prob.set_mg_params(nu=nu, coarse_sweeps=12)
    u, info = prob.solve(T(rho), rtol=1e-10)
    dc, c = prob.sensitivity(T(rho), u)
    assert info["rel_res"] <= 1e-10
    assert abs(float(N(c)[0]) - c_ref) / c_ref <= 1e-6
    assert np.abs(N(dc) - dc_ref).max() / np.abs(dc_ref).max() <= 1e-5


def test_profiling_selector():
    nx, ny, nz = 32, 16, 16
    prob = _problem(nx, ny, nz, precond="gmg", mg_levels=3)
    rho = T(synth.density_around(nx, ny, nz, 0))
    with pytest.raises(fe.FEError):
        fe._check(fe.load_library().fe_set_profiling(prob._h, 10))
    # form 7: each coarsest-level Chebyshev solve, its launches bracketed as
    # one (coarsest grid 8 x 4 x 4, float32: three steps per launch, the
    # remainder in pairs, a last four as two pairs): one per V-cycle
    prob.set_profiling(True, mode=7)
    _, info = prob.solve(rho, rtol=1e-8)
    prob.set_profiling(False)
    ks = prob.kernel_stats(reset=True)
    deg = prob.mg_params()["coarse_sweeps"]
    launches = 2 if deg == 4 else (deg + 2) // 3
    assert info["iters"] + 1 <= ks["launches"] <= info["iters"] + 9
    cn, ce = 9 * 5 * 5, 8 * 4 * 4
    assert ks["bytes_per_launch"] == pytest.approx(launches * (4.0 * (19 * cn + ce) + cn), rel=1e-12)
    # pairs when asked for (one event pair still brackets the whole solve)
    prob.set_coarse_fusion(3)
    prob.set_profiling(True, mode=7)
    prob.solve(rho, rtol=1e-8)
    prob.set_profiling(False)
    ks = prob.kernel_stats(reset=True)
    assert ks["bytes_per_launch"] == pytest.approx((deg + 1) // 2 * (4.0 * (19 * cn + ce) + cn), rel=1e-12)
    prob.set_coarse_fusion(0)
    prob.set_profiling(True, mode=1)
    _, info = prob.solve(rho, rtol=1e-8)
    prob.set_profiling(False)
    ks = prob.kernel_stats(reset=True)
    # one CG-product launch per iteration, plus the unused tail of the last chunk
    assert info["iters"] <= ks["launches"] <= info["iters"] + 8
    nd, ne = prob.ndof, nx * ny * nz
    # z read (float32: the preconditioner's result), the previous direction
    # read, q and the new direction written, E read
    assert ks["bytes_per_launch"] == pytest.approx(8.0 * (3 * nd + ne) + 4.0 * nd, rel=1e-12)
    prob.set_profiling(True)
    prob.solve(rho, rtol=1e-8)
    prob.set_profiling(False)
    assert prob.kernel_stats()["launches"] > ks["launches"]
    # with the preconditioner in float64, z is read in float64
    prob.kernel_stats(reset=True)
    prob.set_float32_levels(3)
    prob.set_profiling(True, mode=1)
    prob.solve(rho, rtol=1e-8)
    prob.set_profiling(False)
    assert prob.kernel_stats()["bytes_per_launch"] == pytest.approx(8.0 * (4 * nd + ne), rel=1e-12)


@pytest.mark.parametrize("deg", [1, 2, 3, 8])
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_coarse_chebyshev_degrees_parity(Ke, deg, precision):
    """Low coarse Chebyshev degrees (a poor coarse solve, the first step from
    zero alone for degree 1) still give a symmetric positive definite
    V-cycle: CG reaches the oracle's answer."""
    nx, ny, nz = 32, 16, 16
    rho = synth.density_around(nx, ny, nz, 2)
    f = synth.cantilever_edge_load(nx, ny, nz)
    u_ref = O.solve_direct(nx, ny, nz, O.simp_modulus(rho), Ke, f, O.clamp_x0_fixed(nx, ny, nz))
    c_ref = O.compliance(f, u_ref)
    dc_ref = O.sensitivity(nx, ny, nz, Ke, rho, u_ref)
    prob = _problem(nx, ny, nz, precision=precision, precond="gmg", mg_levels=3)
    prob.set_mg_params(coarse_sweeps=deg)
    u, info = prob.solve(T(rho), rtol=1e-10)
    dc, c = prob.sensitivity(T(rho), u)
    assert info["rel_res"] <= 1e-10
    assert abs(float(N(c)[0]) - c_ref) / c_ref <= 1e-6
    assert np.abs(N(dc) - dc_ref).max() / np.abs(dc_ref).max() <= 1e-5


@pytest.mark.parametrize("grid,precond,levels", [((1, 1, 1), "jacobi", 1), ((5, 1, 1), "jacobi", 1),
                                                 ((2, 9, 3), "jacobi", 1), ((2, 2, 2), "gmg", 2),
                                                 ((4, 2, 2), "gmg", 2), ((8, 4, 4), "gmg", 3),
                                                 ((3, 1, 1), "gmg", 2), ((5, 3, 1), "gmg", 3)])
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_solve_degenerate_grids(Ke, grid, precond, levels, precision):
    """One-element-thick grids and multigrid hierarchies whose coarsest
    level is a single element layer."""
    nx, ny, nz = grid
    rho = synth.density_around(nx, ny, nz, 3)
    f = synth.cantilever_edge_load(nx, ny, nz)
    fixed = O.clamp_x0_fixed(nx, ny, nz)
    u_ref = O.solve_direct(nx, ny, nz, O.simp_modulus(rho), Ke, f, fixed)
    c_ref = O.compliance(f, u_ref)
    dc_ref = O.sensitivity(nx, ny, nz, Ke, rho, u_ref)
    kw = {"precond": precond}
    if precond == "gmg":
        kw["mg_levels"] = levels
    prob = _problem(nx, ny, nz, precision=precision, **kw)
    u, info = prob.solve(T(rho), rtol=1e-10)
    dc, c = prob.sensitivity(T(rho), u)
    assert info["rel_res"] <= 1e-10
    assert abs(float(N(c)[0]) - c_ref) / c_ref <= 1e-6
    assert np.abs(N(dc) - dc_ref).max() / np.abs(dc_ref).max() <= 1e-5


@pytest.mark.parametrize("grid,levels,deg", [((32, 16, 16), 3, 40), ((60, 32, 28), 3, 7), ((8, 4, 4), 3, 4),
                                             ((26, 14, 2), 2, 5), ((80, 80, 40), 2, 6),
                                             ((208, 208, 64), 2, 6), ((27, 13, 9), 3, 6)])
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
def test_coarse_fusion_bitwise(grid, levels, deg, precision):
    """Pairs of coarse Chebyshev steps in one launch (each workgroup
    recomputing the ring of first-step values its second step needs) give
    bitwise the solve of one launch per step: coarse grids of one or several
    13-column tiles, one-element-thick coarse grids, z chunks of one level
    and of many, even and odd degrees."""
    nx, ny, nz = grid
    rho = T(synth.density_around(nx, ny, nz, 4))
    out = []
    for per_launch in (1, 2):
        prob = _problem(nx, ny, nz, precision=precision, precond="gmg", mg_levels=levels)
        prob.set_mg_params(coarse_sweeps=deg)
        prob.set_coarse_fusion(per_launch)
        u, info = prob.solve(rho, rtol=1e-6)
        out.append((N(u), info))
        if per_launch == 2:
            for bad in (-1, 6):
                with pytest.raises(fe.FEError):
                    prob.set_coarse_fusion(bad)
        prob.close()
    (u1, i1), (u2, i2) = out
    assert i1["rel_res"] <= 1e-6
    assert i1["iters"] == i2["iters"] and i1["outer_iters"] == i2["outer_iters"]
    assert np.array_equal(u1, u2)


@pytest.mark.parametrize("grid,levels,deg", [((32, 16, 16), 3, 40), ((60, 32, 28), 3, 7), ((8, 4, 4), 3, 4),
                                             ((26, 14, 2), 2, 5), ((80, 80, 40), 2, 6),
                                             ((208, 208, 64), 2, 6), ((27, 13, 9), 3, 6), ((224, 112, 56), 3, 48)])
@pytest.mark.parametrize("precision", ["fp64", "fp32_ir"])
@pytest.mark.parametrize("form", [3, 4, 5])
def test_coarse_3d_tiles(grid, levels, deg, precision, form):
    """Pairs of coarse Chebyshev steps on 3D tiles (the default launch form)
    apply the same polynomial as one launch per step, up to the rounding of
    their node sums (another order): to a tight tolerance both solves need
    the same CG iterations (within two in float64, within 15% with float32
    inner solves) and reach the same displacement;
    two solves with 3D tiles agree bit for bit (no atomics).  Blocks of
    4 x 4 x 4 and 4 x 4 x 8 nodes (float32 coarse levels; float64 ones take
    the former), coarse grids of one tile and of many, one-element-thick
    ones, odd degrees."""
    nx, ny, nz = grid
    rho = T(synth.density_around(nx, ny, nz, 4))
    out = []
    for per_launch in (1, form, form):
        prob = _problem(nx, ny, nz, precision=precision, precond="gmg", mg_levels=levels)
        prob.set_mg_params(coarse_sweeps=deg)
        prob.set_coarse_fusion(per_launch)
        u, info = prob.solve(rho, rtol=1e-9)
        out.append((N(u), info))
        prob.close()
    (u1, i1), (u3, i3), (u3b, i3b) = out
    assert i1["rel_res"] <= 1e-9 and i3["rel_res"] <= 1e-9
    # float32 inner solves restart at each refinement step and feel the
    # rounding of the preconditioner more: a looser iteration bound there
    slack = 2 if precision == "fp64" else 2 + 0.15 * max(i1["iters"], i3["iters"])
    assert abs(i1["iters"] - i3["iters"]) <= slack, (i1["iters"], i3["iters"])
    assert np.abs(u3 - u1).max() <= 1e-6 * np.abs(u1).max()
    assert np.array_equal(u3, u3b) and i3["iters"] == i3b["iters"]


def test_extrapolate():
    """fe_extrapolate: u <- u + theta (u - u_hist), u_hist <- the old u,
    exactly (one multiply-add per dof in float64); validation."""
    nx, ny, nz = 9, 5, 4
    prob = _problem(nx, ny, nz)
    rng = np.random.default_rng(4)
    u0 = rng.standard_normal(prob.ndof)
    h0 = rng.standard_normal(prob.ndof)
    for theta in (0.0, 1.0, 0.5):
        u, h = T(u0), T(h0)
        prob.extrapolate(u, h, theta)
        want = u0 + theta * (u0 - h0)
        assert np.array_equal(N(h), u0)
        assert np.abs(N(u) - want).max() <= 1e-15 * np.abs(want).max()
    u = T(u0)
    for bad in (-0.1, 5.0, float("nan")):
        with pytest.raises(fe.FEError):
            prob.extrapolate(u, T(h0), bad)
    with pytest.raises(fe.FEError):
        prob.extrapolate(u, u, 1.0)
