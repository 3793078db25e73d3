"""Pins of the FP64 CPU oracle against facts the paper and the mechanics fix
independently of the oracle's own code: Table I counts, closed-form strain
energies, rigid-body null space, the patch test, beam theory, finite
differences, filter identities and brute force on tiny inputs."""
import json
import math
import os

import numpy as np
import pytest

from oracle import fe_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
NU = 0.3


@pytest.fixture(scope="module")
def Ke():
    return O.hex8_ke(NU)


def _round_k(n):
    """Format a count the way Table I prints it (86K, 1.5M, ...)."""
    if n >= 1_000_000:
        return f"{n / 1e6:.1f}M"
    return f"{round(n / 1000)}K"


# --------------------------------------------------------------------- mesh
def test_table1_counts():
    g = json.load(open(os.path.join(GOLDEN, "table1_counts.json")))
    nb = g["block_size"]
    for m in g["meshes"]:
        nx, ny, nz = m["grid"]
        c = O.mesh_counts(nx, ny, nz)
        cc = O.mesh_counts(nx // nb, ny // nb, nz // nb)
        assert _round_k(c["nelem"]) == m["dvs_printed"], m
        assert _round_k(c["ndof"]) == m["kdim_printed"], m
        assert _round_k(cc["ndof"]) == m["kc_printed"], m
    # exact derived values (3 * nodes)
    assert O.mesh_counts(70, 35, 35)["ndof"] == 276048
    assert O.mesh_counts(100, 50, 50)["ndof"] == 788103
    assert O.mesh_counts(180, 90, 90)["ndof"] == 4496583


def test_element_dofs_layout():
    edof = O.element_dofs(3, 2, 2)
    # element (1,1,1) -> e = 1 + 3*(1 + 2*1) = 10; its local node 6 is (2,2,2)
    n = O.node_index(3, 2, 2, 2, 2, 2)
    assert edof[10, 18:21].tolist() == [3 * n, 3 * n + 1, 3 * n + 2]
    assert edof[0, 0:3].tolist() == [0, 1, 2]


# ---------------------------------------------------------------------- Ke
def test_ke_symmetric_and_six_rigid_modes(Ke):
    assert np.allclose(Ke, Ke.T, rtol=0, atol=1e-15)
    w = np.linalg.eigvalsh(Ke)
    scale = w.max()
    assert np.sum(np.abs(w) < 1e-12 * scale) == 6
    assert np.all(w[6:] > 1e-3 * scale)
    R = O.rigid_body_modes(O.LOCAL_NODES.astype(float))
    assert np.abs(Ke @ R).max() < 1e-13


def test_ke_diagonal_equal_and_quadrature_exact(Ke):
    d = np.diag(Ke)
    assert np.ptp(d) < 1e-15
    Ke3 = O.hex8_ke(NU, nq=3)
    assert np.abs(Ke3 - Ke).max() < 1e-14
    assert np.abs(O.hex8_ke(NU, h=2.5) - 2.5 * Ke).max() < 1e-13
    assert np.abs(O.hex8_ke(NU, E=7.0) - 7.0 * Ke).max() < 1e-13


def test_ke_linear_in_lame():
    # Ke(E, nu) = lam * K_lam + mu * K_mu: three moduli pairs must agree
    def split(E, nu):
        return O.lame(E, nu)
    K1, K2, K3 = O.hex8_ke(0.3), O.hex8_ke(0.2), O.hex8_ke(0.45)
    A = np.array([split(1, 0.3), split(1, 0.2)])
    coef = np.linalg.solve(A.T, np.array(split(1, 0.45)))
    assert np.abs(coef[0] * K1 + coef[1] * K2 - K3).max() < 1e-12


@pytest.mark.parametrize("case", ["uniaxial", "shear_xy", "shear_yz", "volumetric", "mixed"])
def test_ke_constant_strain_energy_closed_form(case):
    """For a linear displacement field u = G x the element energy is
    h^3 * (lam * tr(eps)^2 + 2 mu eps:eps) exactly, eps = sym(G)."""
    h = 1.7
    E, nu = 2.0, 0.27
    lam, mu = O.lame(E, nu)
    G = {"uniaxial": np.diag([1.0, 0, 0]),
         "shear_xy": np.array([[0, 1.0, 0], [0, 0, 0], [0, 0, 0]]),
         "shear_yz": np.array([[0, 0, 0], [0, 0, 0.5], [0, 0.5, 0]]),
         "volumetric": np.eye(3),
         "mixed": np.array([[0.3, -0.2, 0.7], [0.1, -0.5, 0.4], [0.25, 0.6, 0.9]])}[case]
    X = h * O.LOCAL_NODES.astype(float)
    u = (X @ G.T).ravel()
    eps = 0.5 * (G + G.T)
    energy = h ** 3 * (lam * np.trace(eps) ** 2 + 2 * mu * np.sum(eps * eps))
    Ke = O.hex8_ke(nu, E=E, h=h)
    assert abs(u @ Ke @ u - energy) < 1e-12 * max(1.0, energy)


# ------------------------------------------------------------ assembly, K
def _nodes_xyz(nx, ny, nz):
    n = np.arange((nx + 1) * (ny + 1) * (nz + 1))
    i = n % (nx + 1)
    j = (n // (nx + 1)) % (ny + 1)
    k = n // ((nx + 1) * (ny + 1))
    return np.stack([i, j, k], axis=1).astype(float)


def test_global_K_rigid_modes_and_symmetry(Ke):
    nx, ny, nz = 4, 3, 2
    rng = np.random.default_rng(1)
    E = rng.uniform(0.1, 1.0, nx * ny * nz)
    K = O.assemble_K(nx, ny, nz, E, Ke)
    R = O.rigid_body_modes(_nodes_xyz(nx, ny, nz))
    assert np.abs(K @ R).max() < 1e-12
    x, y = rng.standard_normal((2, K.shape[0]))
    assert abs(x @ (K @ y) - y @ (K @ x)) < 1e-11


def test_patch_test(Ke):
    """Constant strain is reproduced: interior rows of K (A x + b) vanish and a
    solve with the boundary held at A x + b returns A x + b inside."""
    nx, ny, nz = 4, 4, 3
    X = _nodes_xyz(nx, ny, nz)
    A = np.array([[0.01, 0.02, -0.03], [0.005, -0.01, 0.02], [0.03, 0.0, 0.015]])
    b = np.array([0.1, -0.2, 0.3])
    ulin = (X @ A.T + b).ravel()
    K = O.assemble_K(nx, ny, nz, np.ones(nx * ny * nz), Ke)
    i, j, k = X[:, 0], X[:, 1], X[:, 2]
    interior = (i > 0) & (i < nx) & (j > 0) & (j < ny) & (k > 0) & (k < nz)
    idof = np.repeat(interior, 3)
    assert np.abs((K @ ulin)[idof]).max() < 1e-13
    # Dirichlet solve on the interior
    fixed = ~idof
    rhs = -(K @ np.where(fixed, ulin, 0.0))
    Kii = K[idof][:, idof].toarray()
    ui = np.linalg.solve(Kii, rhs[idof])
    assert np.abs(ui - ulin[idof]).max() < 1e-12


# --------------------------------------------------------------- solves
def _end_face_load(nx, ny, nz, total=1.0):
    f = np.zeros(3 * (nx + 1) * (ny + 1) * (nz + 1))
    wj = np.ones(ny + 1); wj[[0, -1]] = 0.5
    wk = np.ones(nz + 1); wk[[0, -1]] = 0.5
    s = wj.sum() * wk.sum()
    for j in range(ny + 1):
        for k in range(nz + 1):
            f[3 * O.node_index(nx, ny, nz, nx, j, k) + 2] -= total * wj[j] * wk[k] / s
    return f, np.outer(wj, wk).ravel() / s


@pytest.mark.slow
def test_cantilever_beam_theory(Ke):
    """Solid cantilever, L/H = 8, unit end shear: tip deflection approaches
    Timoshenko's PL^3/(3EI) + PL/(kappa G A) from below, monotonically, within
    5% at 64x8x8 (the full-integration brick is slightly stiff in bending)."""
    ratios = []
    for n in (2, 4, 8):
        nx, ny, nz = 8 * n, n, n
        f, w = _end_face_load(nx, ny, nz)
        u = O.solve_direct(nx, ny, nz, np.ones(nx * ny * nz), Ke, f,
                           O.clamp_x0_fixed(nx, ny, nz))
        L, H = nx, n
        I, A = H ** 4 / 12.0, H * H
        G = 1.0 / (2 * (1 + NU))
        kappa = 10 * (1 + NU) / (12 + 11 * NU)
        dT = L ** 3 / (3 * I) + L / (kappa * G * A)
        uz = np.array([u[3 * O.node_index(nx, ny, nz, nx, j, k) + 2]
                       for j in range(ny + 1) for k in range(nz + 1)])
        ratios.append(-(uz @ w) / dT)
    assert ratios[0] < ratios[1] < ratios[2] <= 1.0
    assert ratios[2] > 0.95


def _c1_problem(nx=8, ny=4, nz=4, seed=0):
    rng = np.random.default_rng(seed)
    rho = np.clip(0.3 + rng.uniform(-0.1, 0.1, nx * ny * nz), 0.01, 1.0)
    f = np.zeros(3 * (nx + 1) * (ny + 1) * (nz + 1))
    for j in range(ny + 1):
        w = 0.5 if j in (0, ny) else 1.0
        f[3 * O.node_index(nx, ny, nz, nx, j, 0) + 2] = -w / ny
    return rho, f, O.clamp_x0_fixed(nx, ny, nz)


def test_uniform_density_scaling(Ke):
    nx, ny, nz = 6, 3, 3
    _, f, fixed = _c1_problem(nx, ny, nz)
    u1 = O.solve_direct(nx, ny, nz, np.ones(nx * ny * nz), Ke, f, fixed)
    a = 0.12
    Ea = O.simp_modulus(np.full(nx * ny * nz, a))
    ua = O.solve_direct(nx, ny, nz, Ea, Ke, f, fixed)
    assert abs(O.compliance(f, ua) / O.compliance(f, u1) - 1.0 / Ea[0]) < 1e-10 / Ea[0]


def test_betti_linearity_mirror(Ke):
    nx, ny, nz = 6, 4, 3
    rho, f, fixed = _c1_problem(nx, ny, nz, seed=3)
    E = O.simp_modulus(rho)
    rng = np.random.default_rng(5)
    f2 = np.where(fixed, 0.0, rng.standard_normal(f.size))
    u1 = O.solve_direct(nx, ny, nz, E, Ke, f, fixed)
    u2 = O.solve_direct(nx, ny, nz, E, Ke, f2, fixed)
    assert abs(f @ u2 - f2 @ u1) < 1e-10 * abs(f @ u2)
    u12 = O.solve_direct(nx, ny, nz, E, Ke, 2 * f - 3 * f2, fixed)
    assert np.abs(u12 - (2 * u1 - 3 * u2)).max() < 1e-9 * np.abs(u12).max()
    # y-mirror symmetric density + symmetric edge load -> mirrored solution
    r3 = rho.reshape(nz, ny, nx)
    rs = 0.5 * (r3 + r3[:, ::-1, :])
    us = O.solve_direct(nx, ny, nz, O.simp_modulus(rs.ravel()), Ke, f, fixed)
    U = us.reshape(nz + 1, ny + 1, nx + 1, 3)
    Um = U[:, ::-1, :, :] * np.array([1, -1, 1])
    assert np.abs(U - Um).max() < 1e-9 * np.abs(U).max()


def test_cholesky_vs_pcg(Ke):
    nx, ny, nz = 10, 5, 5
    rho, f, fixed = _c1_problem(nx, ny, nz, seed=2)
    E = O.simp_modulus(rho)
    ud = O.solve_direct(nx, ny, nz, E, Ke, f, fixed)
    up, it, rel = O.solve_pcg(nx, ny, nz, E, Ke, f, fixed, rtol=1e-13)
    assert rel <= 1e-13
    assert np.abs(ud - up).max() < 1e-9 * np.abs(ud).max()
    K = O.assemble_K(nx, ny, nz, E, Ke)
    r = np.where(fixed, 0.0, f - K @ ud)
    assert np.linalg.norm(r) < 1e-10 * np.linalg.norm(f)
    # the element-by-element operator (the paper-scale references) reaches the same u
    ue, it_e, rel_e = O.solve_pcg(nx, ny, nz, E, Ke, f, fixed, rtol=1e-13, elementwise=True)
    assert rel_e <= 1e-13
    assert np.abs(ud - ue).max() < 1e-9 * np.abs(ud).max()


def test_elementwise_operator(Ke):
    """K u formed brick by brick equals the assembled K_ff u_f, annihilates
    the rigid motions when nothing is fixed, and is symmetric."""
    nx, ny, nz = 5, 4, 3
    rng = np.random.default_rng(8)
    E = rng.uniform(0.1, 1.0, nx * ny * nz)
    u = rng.standard_normal(3 * (nx + 1) * (ny + 1) * (nz + 1))
    fixed = O.clamp_x0_fixed(nx, ny, nz)
    ref = O.apply_K_free(O.assemble_K(nx, ny, nz, E, Ke), fixed, u)
    y = O.apply_K_elementwise(nx, ny, nz, E, Ke, fixed, u)
    assert np.abs(y - ref).max() < 1e-13 * np.abs(ref).max()
    none = np.zeros_like(fixed)
    n = np.arange((nx + 1) * (ny + 1) * (nz + 1))
    xyz = np.stack([n % (nx + 1), (n // (nx + 1)) % (ny + 1), n // ((nx + 1) * (ny + 1))], axis=1)
    R = O.rigid_body_modes(xyz.astype(float))
    for m in range(6):
        assert np.abs(O.apply_K_elementwise(nx, ny, nz, E, Ke, none, R[:, m])).max() < 1e-12
    v = rng.standard_normal(u.size)
    a = v @ O.apply_K_elementwise(nx, ny, nz, E, Ke, fixed, u)
    b = u @ O.apply_K_elementwise(nx, ny, nz, E, Ke, fixed, v)
    assert abs(a - b) < 1e-12 * abs(a)


# ----------------------------------------------------- compliance, dc
def test_compliance_identities(Ke):
    nx, ny, nz = 6, 3, 3
    rho, f, fixed = _c1_problem(nx, ny, nz, seed=4)
    E = O.simp_modulus(rho)
    u = O.solve_direct(nx, ny, nz, E, Ke, f, fixed)
    K = O.assemble_K(nx, ny, nz, E, Ke)
    c = O.compliance(f, u)
    assert abs(c - u @ (K @ u)) < 1e-11 * c
    assert abs(c - np.sum(E * O.element_energies(nx, ny, nz, Ke, u))) < 1e-11 * c


@pytest.mark.parametrize("grid", [(4, 2, 2), (6, 3, 3)])
def test_sensitivity_central_fd(Ke, grid):
    nx, ny, nz = grid
    rng = np.random.default_rng(7)
    rho = rng.uniform(0.2, 1.0, nx * ny * nz)
    _, f, fixed = _c1_problem(nx, ny, nz)
    penal, E0, Emin = 3.0, 1.0, 1e-9

    def c_of(r):
        u = O.solve_direct(nx, ny, nz, O.simp_modulus(r, E0, Emin, penal), Ke, f, fixed)
        return O.compliance(f, u), u

    c0, u = c_of(rho)
    dc = O.sensitivity(nx, ny, nz, Ke, rho, u, E0, Emin, penal)
    idx = rng.choice(rho.size, size=min(8, rho.size), replace=False)
    for e in idx:
        step = 1e-6 * rho[e]
        rp, rm = rho.copy(), rho.copy()
        rp[e] += step
        rm[e] -= step
        fd = (c_of(rp)[0] - c_of(rm)[0]) / (2 * step)
        assert abs(fd - dc[e]) <= 1e-6 * np.abs(dc).max(), (e, fd, dc[e])
    # homogeneity: sum rho dc = -p (c - Emin sum u_e^T Ke u_e)
    ee = O.element_energies(nx, ny, nz, Ke, u)
    assert abs(np.sum(rho * dc) + penal * (c0 - Emin * ee.sum())) < 1e-10 * c0


@pytest.mark.parametrize("grid", [(4, 2, 2), (6, 3, 3)])
def test_adjoint_gradient_central_fd(Ke, grid):
    """J = l^T u(rho) for a random l (not self-adjoint): the gradient (3)
    against central finite differences; with l = f it is the compliance
    sensitivity; swapping f and l leaves it unchanged (Betti)."""
    nx, ny, nz = grid
    rng = np.random.default_rng(11)
    rho = rng.uniform(0.2, 1.0, nx * ny * nz)
    _, f, fixed = _c1_problem(nx, ny, nz)
    l = np.where(fixed, 0.0, rng.standard_normal(f.size))
    u, lam, g = O.linear_objective_gradient(nx, ny, nz, Ke, rho, f, l, fixed)

    def J(r):
        return l @ O.solve_direct(nx, ny, nz, O.simp_modulus(r), Ke, f, fixed)

    for e in rng.choice(rho.size, size=min(8, rho.size), replace=False):
        step = 1e-6 * rho[e]
        rp, rm = rho.copy(), rho.copy()
        rp[e] += step
        rm[e] -= step
        fd = (J(rp) - J(rm)) / (2 * step)
        assert abs(fd - g[e]) <= 1e-6 * np.abs(g).max(), (e, fd, g[e])
    _, _, g_ff = O.linear_objective_gradient(nx, ny, nz, Ke, rho, f, f, fixed)
    assert np.abs(g_ff - O.sensitivity(nx, ny, nz, Ke, rho, u)).max() <= 1e-12 * np.abs(g_ff).max()
    _, _, g_sw = O.linear_objective_gradient(nx, ny, nz, Ke, rho, l, f, fixed)
    assert np.abs(g_sw - g).max() <= 1e-10 * np.abs(g).max()


# ----------------------------------------------------------------- filter
def test_filter_closed_form_weights():
    P = O.filter_matrix(7, 7, 7, 1.5)
    e = 3 + 7 * (3 + 7 * 3)  # interior element
    row = P.getrow(e)
    W = 1.5 + 6 * 0.5 + 12 * (1.5 - math.sqrt(2.0))
    assert abs(W - 5.5294372515) < 1e-9
    assert row.nnz == 19
    vals = np.sort(row.data)
    assert abs(vals[-1] - 1.5 / W) < 1e-15
    assert np.allclose(vals[:12], (1.5 - math.sqrt(2.0)) / W, rtol=0, atol=1e-15)
    assert np.allclose(vals[12:18], 0.5 / W, rtol=0, atol=1e-15)


def test_filter_identities_and_brute_force():
    nx, ny, nz, r = 5, 4, 3, 1.5
    P = O.filter_matrix(nx, ny, nz, r)
    n = nx * ny * nz
    assert np.abs(P @ np.ones(n) - 1.0).max() < 1e-14
    rng = np.random.default_rng(0)
    x, y = rng.standard_normal((2, n))
    assert abs((P @ x) @ y - x @ (P.T @ y)) < 1e-12
    # brute force: all centroid pairs
    e = np.arange(n)
    C = np.stack([e % nx, (e // nx) % ny, e // (nx * ny)], axis=1) + 0.5
    d = np.linalg.norm(C[:, None, :] - C[None, :, :], axis=2)
    H = np.maximum(0.0, r - d)
    Pd = H / H.sum(axis=1, keepdims=True)
    assert np.abs(P.toarray() - Pd).max() < 1e-15
    for r2 in (1.0 + 1e-9, 2.3):
        P2 = O.filter_matrix(nx, ny, nz, r2).toarray()
        H2 = np.maximum(0.0, r2 - d)
        assert np.abs(P2 - H2 / H2.sum(axis=1, keepdims=True)).max() < 1e-15


# --------------------------------------------------------------------- OC
def test_oc_volume_bounds_and_brute_force():
    rng = np.random.default_rng(11)
    n = 60
    x = rng.uniform(0.05, 0.5, n)
    dcx = -rng.uniform(0.01, 3.0, n)
    dcx[:3] = 0.0  # no descent information -> lower bound
    dv = rng.uniform(0.8, 1.2, n)
    volfrac, move = 0.25, 0.2
    xn, lam, change = O.oc_update(x, dcx, dv, volfrac, move)
    target = volfrac * n
    assert abs(np.sum(dv * xn) - target) <= 1e-10 * target
    assert np.all(xn >= np.maximum(0, x - move) - 1e-15)
    assert np.all(xn <= np.minimum(1, x + move) + 1e-15)
    assert np.allclose(xn[:3], np.maximum(0, x[:3] - move))
    assert abs(change - np.abs(xn - x).max()) == 0
    # brute force: volume is non-increasing in lambda; a fine log grid brackets lam
    grid = np.logspace(-6, 6, 4001)
    vols = np.array([np.sum(dv * np.clip(x * np.sqrt(np.maximum(0, -dcx) / dv / g),
                                         np.maximum(0, x - move), np.minimum(1, x + move)))
                     for g in grid])
    assert np.all(np.diff(vols) <= 1e-12)
    k = np.searchsorted(-vols, -target)
    assert grid[k - 1] <= lam <= grid[k]


# ------------------------------------------------ planted-mistake checks
def test_pins_catch_planted_mistakes(monkeypatch):
    """A wrong shear modulus in D, or a sign error in a shape-function
    derivative, must break at least one of the closed-form pins above."""
    good_D = O.isotropic_D

    def bad_D(E, nu):
        D = good_D(E, nu)
        D[3, 3] *= 2.0  # tensor instead of engineering shear
        return D

    monkeypatch.setattr(O, "isotropic_D", bad_D)
    Ke_bad = O.hex8_ke(NU)
    G = np.array([[0, 0, 0], [0, 0, 1.0], [0, 0, 0]])  # pure yz shear
    X = O.LOCAL_NODES.astype(float)
    u = (X @ G.T).ravel()
    lam, mu = O.lame(1.0, NU)
    eps = 0.5 * (G + G.T)
    energy = lam * np.trace(eps) ** 2 + 2 * mu * np.sum(eps * eps)
    assert abs(u @ Ke_bad @ u - energy) > 1e-3
    monkeypatch.setattr(O, "isotropic_D", good_D)

    good_B = O.hex8_B

    def bad_B(t, h):
        B = good_B(t, h)
        B[5, 0::3] *= -1.0  # sign slip in the xy shear row
        return B

    monkeypatch.setattr(O, "hex8_B", bad_B)
    Ke_bad = O.hex8_ke(NU)
    R = O.rigid_body_modes(O.LOCAL_NODES.astype(float))
    assert np.abs(Ke_bad @ R).max() > 1e-3


def test_row_and_element_samplers_agree_with_full_forms(Ke):
    nx, ny, nz = 5, 4, 3
    rng = np.random.default_rng(3)
    E = rng.uniform(0.1, 1.0, nx * ny * nz)
    u = rng.standard_normal(3 * (nx + 1) * (ny + 1) * (nz + 1))
    fixed = O.clamp_x0_fixed(nx, ny, nz)
    y = O.apply_K_free(O.assemble_K(nx, ny, nz, E, Ke), fixed, u).reshape(-1, 3)
    nodes = np.arange(y.shape[0])
    assert np.abs(O.apply_K_rows(nx, ny, nz, E, Ke, fixed, u, nodes) - y).max() < 1e-13
    rho = rng.uniform(0.1, 1.0, nx * ny * nz)
    el = np.array([0, 7, 33, 59])
    assert np.abs(O.sensitivity_elements(nx, ny, nz, Ke, rho, u, el)
                  - O.sensitivity(nx, ny, nz, Ke, rho, u)[el]).max() < 1e-13
    lam = rng.standard_normal(u.size)
    full = O.adjoint_sensitivity(nx, ny, nz, Ke, rho, u, lam)
    part = O.adjoint_sensitivity_elements(nx, ny, nz, Ke, rho, u, lam, el)
    assert np.abs(part - full[el]).max() < 1e-13 * np.abs(full).max()
    # lam and u enter as lam_e^T Ke u_e: swapping them changes nothing (Ke symmetric),
    # and lam = u is the compliance sensitivity
    assert np.abs(O.adjoint_sensitivity_elements(nx, ny, nz, Ke, rho, lam, u, el) - part).max() \
        < 1e-13 * np.abs(full).max()
    assert np.abs(O.adjoint_sensitivity_elements(nx, ny, nz, Ke, rho, u, u, el)
                  - O.sensitivity_elements(nx, ny, nz, Ke, rho, u, el)).max() < 1e-13
