"""Pins of the oracle's coarse scale of the two-scale scheme (block means of
the design variables, the coarse stiffness and load) against closed forms,
brute force and the Galerkin identity of nested trilinear spaces."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import fe_oracle as O

NU = 0.3


def _edge_load(nx, ny, nz):
    """Consistent nodal loads of a unit downward line load on the edge
    (x = nx, z = 0): trapezoid weights 1/ny inside, 1/(2 ny) at the ends."""
    f = np.zeros(3 * (nx + 1) * (ny + 1) * (nz + 1))
    for j in range(ny + 1):
        f[3 * O.node_index(nx, ny, nz, nx, j, 0) + 2] = -(0.5 if j in (0, ny) else 1.0) / ny
    return f


def _prolongation(nx, ny, nz, nb):
    """Trilinear interpolation from the coarse mesh (edge nb) to the fine mesh,
    by evaluating every coarse nodal hat function at every fine node."""
    cx, cy, cz = nx // nb, ny // nb, nz // nb
    rows, cols, vals = [], [], []
    hat = lambda t: max(0.0, 1.0 - abs(t))
    for k in range(nz + 1):
        for j in range(ny + 1):
            for i in range(nx + 1):
                nf = O.node_index(nx, ny, nz, i, j, k)
                for K in range(cz + 1):
                    for J in range(cy + 1):
                        for I in range(cx + 1):
                            w = hat(i / nb - I) * hat(j / nb - J) * hat(k / nb - K)
                            if w == 0.0:
                                continue
                            nc = O.node_index(cx, cy, cz, I, J, K)
                            for c in range(3):
                                rows.append(3 * nf + c)
                                cols.append(3 * nc + c)
                                vals.append(w)
    return sp.csr_matrix((vals, (rows, cols)),
                         shape=(3 * (nx + 1) * (ny + 1) * (nz + 1), 3 * (cx + 1) * (cy + 1) * (cz + 1)))


def test_block_mean_closed_forms_and_brute_force():
    nx, ny, nz = 12, 6, 9
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    # element e = i + nx (j + ny k): build the field in that order
    lin = lambda a, b, c, d: (a * i + b * j + c * k + d).transpose(2, 1, 0).ravel()
    z = lin(0.5, -1.25, 2.0, 0.3)
    assert np.array_equal(O.block_mean(nx, ny, nz, z, 1), z)
    for nb in (3,):
        zc = O.block_mean(nx, ny, nz, z, nb)
        I, J, K = np.meshgrid(np.arange(nx // nb), np.arange(ny // nb), np.arange(nz // nb), indexing="ij")
        m = (nb - 1) / 2.0
        ref = (0.5 * (nb * I + m) - 1.25 * (nb * J + m) + 2.0 * (nb * K + m) + 0.3).transpose(2, 1, 0).ravel()
        assert np.abs(zc - ref).max() <= 1e-13
    # brute force: scatter every fine element into its block
    rng = np.random.default_rng(0)
    for nb, (gx, gy, gz) in ((2, (4, 6, 2)), (3, (6, 3, 9)), (5, (5, 10, 5))):
        z = rng.uniform(0.0, 1.0, gx * gy * gz)
        cx, cy = gx // nb, gy // nb
        acc = np.zeros((gx // nb) * (gy // nb) * (gz // nb))
        for e in range(z.size):
            a, b, c = e % gx, (e // gx) % gy, e // (gx * gy)
            acc[a // nb + cx * (b // nb + cy * (c // nb))] += z[e]
        zc = O.block_mean(gx, gy, gz, z, nb)
        assert np.abs(zc - acc / nb ** 3).max() <= 1e-15
        assert abs(zc.sum() * nb ** 3 - z.sum()) <= 1e-12 * z.sum()
    with pytest.raises(ValueError):
        O.block_mean(6, 4, 4, np.zeros(96), 4)


def test_block_mean_pin_catches_transposed_blocks(monkeypatch):
    """A block mean that numbers the coarse grid with x slowest must fail the
    linear-field closed form."""
    good = O.block_mean

    def bad(nx, ny, nz, z, nb):
        return good(nx, ny, nz, z, nb).reshape(nz // nb, ny // nb, nx // nb).transpose(2, 1, 0).ravel()

    nx, ny, nz, nb = 12, 6, 9, 3
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    z = (0.5 * i - 1.25 * j + 2.0 * k).transpose(2, 1, 0).ravel()
    I, J, K = np.meshgrid(np.arange(4), np.arange(2), np.arange(3), indexing="ij")
    ref = (0.5 * (3 * I + 1) - 1.25 * (3 * J + 1) + 2.0 * (3 * K + 1)).transpose(2, 1, 0).ravel()
    monkeypatch.setattr(O, "block_mean", bad)
    assert np.abs(O.block_mean(nx, ny, nz, z, nb) - ref).max() > 1.0


@pytest.mark.parametrize("nb", [2, 3])
def test_coarse_stiffness_and_load_are_galerkin_products(nb):
    """The coarse trilinear space is a subspace of the fine one.  For a design
    that is constant on every block, the coarse stiffness of edge nb equals
    P^T K P exactly, and the coarse edge load equals P^T f."""
    nx, ny, nz = 2 * nb * 3, nb * 2, nb * 2
    cx, cy, cz = nx // nb, ny // nb, nz // nb
    rng = np.random.default_rng(nb)
    zc_true = rng.uniform(0.1, 1.0, cx * cy * cz)
    e = np.arange(nx * ny * nz)
    a, b, c = e % nx, (e // nx) % ny, e // (nx * ny)
    z = zc_true[a // nb + cx * (b // nb + cy * (c // nb))]
    zc = O.block_mean(nx, ny, nz, z, nb)
    assert np.abs(zc - zc_true).max() <= 1e-15
    P = _prolongation(nx, ny, nz, nb)
    Kf = O.assemble_K(nx, ny, nz, O.simp_modulus(z), O.hex8_ke(NU))
    Kc = O.assemble_K(cx, cy, cz, O.simp_modulus(zc), O.hex8_ke(NU, h=nb))
    G = (P.T @ Kf @ P).toarray()
    assert np.abs(G - Kc.toarray()).max() <= 1e-12 * np.abs(G).max()
    fc = _edge_load(cx, cy, cz)
    assert np.abs(P.T @ _edge_load(nx, ny, nz) - fc).max() <= 1e-15
    # the coarse solve (filter radius below one coarse element: identity) is
    # the Galerkin solve of the fine problem on the coarse subspace
    _, uc, cc = O.coarse_scale_solve(nx, ny, nz, z, nb, fc, r=0.5)
    fixed = O.clamp_x0_fixed(cx, cy, cz)
    free = np.flatnonzero(~fixed)
    ug = np.zeros(fc.size)
    ug[free] = spla.spsolve(sp.csr_matrix(G[np.ix_(free, free)]), fc[free])
    assert np.abs(uc - ug).max() <= 1e-9 * np.abs(ug).max()
    # nested spaces: the coarse solution is stiffer
    uf = O.solve_direct(nx, ny, nz, O.simp_modulus(z), O.hex8_ke(NU), _edge_load(nx, ny, nz),
                        O.clamp_x0_fixed(nx, ny, nz))
    assert 0.0 < cc <= O.compliance(_edge_load(nx, ny, nz), uf)


def test_coarse_scale_block_size_one_is_the_fine_solve():
    nx, ny, nz = 8, 4, 4
    rng = np.random.default_rng(7)
    z = rng.uniform(0.05, 1.0, nx * ny * nz)
    f = _edge_load(nx, ny, nz)
    zc, uc, cc = O.coarse_scale_solve(nx, ny, nz, z, 1, f)
    assert np.array_equal(zc, z)
    rho = O.filter_matrix(nx, ny, nz, 1.5) @ z
    u = O.solve_direct(nx, ny, nz, O.simp_modulus(rho), O.hex8_ke(NU), f, O.clamp_x0_fixed(nx, ny, nz))
    assert np.array_equal(uc, u)
    assert cc == O.compliance(f, u)


def test_coarse_compliance_decreases_with_block_size():
    """Uniform density: the spaces of block sizes 4, 2, 1 are nested, so the
    compliance cannot increase as the blocks grow."""
    nx, ny, nz = 16, 4, 4
    z = np.full(nx * ny * nz, 0.4)
    cs = [O.coarse_scale_solve(nx, ny, nz, z, nb, _edge_load(nx // nb, ny // nb, nz // nb))[2]
          for nb in (1, 2, 4)]
    assert cs[0] >= cs[1] >= cs[2] > 0.0
