"""Plain FP64 CPU oracle for the exact-gradient step of minimum-compliance
topology optimisation (Zhang et al., "Speeding up Computational Morphogenesis
with Online Neural Synthetic Gradients", Sec. III-D, Eq. (4)-(5)).

TEST INFRASTRUCTURE ONLY.  This module is imported by ``tests/``, by
``__graft_entry__.smoke()`` and by the ``cpu_baseline`` leg of ``bench.py``;
nothing in the product path (the HIP library and its Python binding) imports,
links or calls it, and it imports nothing from the product package.

Everything here is written from the definitions, in float64, with NumPy/SciPy
primitives as single steps (sparse matrix-vector products, a banded Cholesky
factorisation from LAPACK).  There is no blocking, fusion or reordering beyond
what the definitions state, so each function can be checked by eye.

Conventions (structured hex8 voxel mesh, element size h):
  element e = i + nx*(j + ny*k)            (0 <= i < nx, ...)
  node    n = i + (nx+1)*(j + (ny+1)*k)    (0 <= i <= nx, ...)
  dof       = 3*n + c,  c in {x, y, z}
  local node order of an element (offsets along x, y, z):
  (0,0,0) (1,0,0) (1,1,0) (0,1,0) (0,0,1) (1,0,1) (1,1,1) (0,1,1);
  local dof = 3*a + c.

Readings where the paper is silent:
  * the element is the trilinear 8-node brick with full 2x2x2 Gauss
    quadrature; the PDE is isotropic linear elasticity (Sec. III-D: K(z)u = f);
  * the stiffness interpolation is SIMP, E(rho) = Emin + rho^p (E0 - Emin);
  * the stiffness is driven by the filtered (physical) density rho = P z;
  * the density filter P is the linear cone w_ij = max(0, r - |c_i - c_j|)
    over element centroids, truncated at the domain boundary and
    row-normalised;
  * the optimality-criteria update uses the square-root rule with a move
    limit and bisects the multiplier until the bracket is relatively 1e-12
    wide.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg
import scipy.sparse as sp

# Local node offsets of the hex8 element, in the fixed local order.
LOCAL_NODES = np.array(
    [[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
     [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], dtype=np.int64)


# ---------------------------------------------------------------------------
# Mesh (Sec. IV, Table I: dimension of K = 3 x number of nodes)
# ---------------------------------------------------------------------------
def mesh_counts(nx: int, ny: int, nz: int) -> dict:
    """Element, node and dof counts of an nx*ny*nz brick mesh.

    Table I counts the dimension of K over every node of the mesh, clamped or
    not, with three displacement components per node.
    """
    nelem = nx * ny * nz
    nnode = (nx + 1) * (ny + 1) * (nz + 1)
    return {"nelem": nelem, "nnode": nnode, "ndof": 3 * nnode}


def node_index(nx, ny, nz, i, j, k):
    return i + (nx + 1) * (j + (ny + 1) * k)


def element_dofs(nx: int, ny: int, nz: int) -> np.ndarray:
    """(nelem, 24) array: global dof of local dof 3a+c of every element."""
    e = np.arange(nx * ny * nz)
    i = e % nx
    j = (e // nx) % ny
    k = e // (nx * ny)
    edof = np.empty((e.size, 24), dtype=np.int64)
    for a, (di, dj, dk) in enumerate(LOCAL_NODES):
        n = node_index(nx, ny, nz, i + di, j + dj, k + dk)
        for c in range(3):
            edof[:, 3 * a + c] = 3 * n + c
    return edof


def clamp_x0_fixed(nx: int, ny: int, nz: int) -> np.ndarray:
    """Boolean dof mask of the cantilever support: every dof of the nodes on
    the face x = 0 is fixed (Sec. IV, benchmark problems)."""
    n = np.arange((nx + 1) * (ny + 1) * (nz + 1))
    on_face = (n % (nx + 1)) == 0
    return np.repeat(on_face, 3)


# ---------------------------------------------------------------------------
# Element stiffness Ke = integral over the brick of B^T D B
# ---------------------------------------------------------------------------
def lame(E: float, nu: float) -> tuple[float, float]:
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def isotropic_D(E: float, nu: float) -> np.ndarray:
    """6x6 elasticity matrix, Voigt order (xx, yy, zz, yz, xz, xy) with
    engineering shear strains."""
    lam, mu = lame(E, nu)
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[0, 0] = D[1, 1] = D[2, 2] = lam + 2.0 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    return D


def hex8_B(t: np.ndarray, h: float) -> np.ndarray:
    """Strain-displacement matrix (6x24) at reference point t in [0,1]^3 of
    a cube of edge h.  Shape functions are products of phi_0(s) = 1 - s and
    phi_1(s) = s along each axis."""
    def phi(a, s):
        return s if a == 1 else 1.0 - s

    def dphi(a):
        return 1.0 if a == 1 else -1.0

    B = np.zeros((6, 24))
    for a, off in enumerate(LOCAL_NODES):
        g = np.empty(3)
        for d in range(3):
            val = dphi(off[d]) / h
            for d2 in range(3):
                if d2 != d:
                    val *= phi(off[d2], t[d2])
            g[d] = val
        cx, cy, cz = 3 * a, 3 * a + 1, 3 * a + 2
        B[0, cx] = g[0]
        B[1, cy] = g[1]
        B[2, cz] = g[2]
        B[3, cy] = g[2]
        B[3, cz] = g[1]
        B[4, cx] = g[2]
        B[4, cz] = g[0]
        B[5, cx] = g[1]
        B[5, cy] = g[0]
    return B


def hex8_ke(nu: float, E: float = 1.0, h: float = 1.0, nq: int = 2) -> np.ndarray:
    """24x24 element stiffness of the trilinear brick by nq^3 Gauss points.
    nq = 2 integrates B^T D B exactly (degree <= 2 per axis)."""
    pts, wts = np.polynomial.legendre.leggauss(nq)
    pts = 0.5 * (pts + 1.0)  # map [-1,1] -> [0,1]
    wts = 0.5 * wts
    D = isotropic_D(E, nu)
    Ke = np.zeros((24, 24))
    for qx, wx in zip(pts, wts):
        for qy, wy in zip(pts, wts):
            for qz, wz in zip(pts, wts):
                B = hex8_B(np.array([qx, qy, qz]), h)
                Ke += (wx * wy * wz * h ** 3) * (B.T @ D @ B)
    return Ke


def rigid_body_modes(nodes_xyz: np.ndarray) -> np.ndarray:
    """(3*nnode, 6) matrix of the three translations and the three
    infinitesimal rotations omega x X evaluated at the given node coordinates."""
    n = nodes_xyz.shape[0]
    R = np.zeros((3 * n, 6))
    for c in range(3):
        R[c::3, c] = 1.0
    x, y, z = nodes_xyz[:, 0], nodes_xyz[:, 1], nodes_xyz[:, 2]
    # rotation about x: (0, -z, y); about y: (z, 0, -x); about z: (-y, x, 0)
    R[1::3, 3], R[2::3, 3] = -z, y
    R[0::3, 4], R[2::3, 4] = z, -x
    R[0::3, 5], R[1::3, 5] = -y, x
    return R


# ---------------------------------------------------------------------------
# SIMP interpolation and the global stiffness K(rho) = sum_e E_e A_e^T Ke A_e
# ---------------------------------------------------------------------------
def simp_modulus(rho, E0=1.0, Emin=1e-9, penal=3.0):
    return Emin + np.asarray(rho, dtype=np.float64) ** penal * (E0 - Emin)


def assemble_K(nx, ny, nz, E_elem, Ke) -> sp.csr_matrix:
    """Global stiffness by element-wise accumulation (duplicates summed)."""
    edof = element_dofs(nx, ny, nz)
    ndof = 3 * (nx + 1) * (ny + 1) * (nz + 1)
    rows = np.repeat(edof, 24, axis=1).ravel()
    cols = np.tile(edof, (1, 24)).ravel()
    vals = (np.asarray(E_elem, dtype=np.float64)[:, None] * Ke.ravel()[None, :]).ravel()
    K = sp.coo_matrix((vals, (rows, cols)), shape=(ndof, ndof)).tocsr()
    K.sum_duplicates()
    return K


def apply_K_rows(nx, ny, nz, E_elem, Ke, fixed, u, nodes):
    """Rows of y = K_ff u_f at the given nodes, one node at a time from the
    (up to) eight bricks around it: y_n = sum_e E_e (Ke u_e)[local(n, e)].
    Returns an (len(nodes), 3) array (zero on fixed dofs)."""
    uf = np.where(fixed, 0.0, u)
    out = np.zeros((len(nodes), 3))
    for r, n in enumerate(nodes):
        i = n % (nx + 1)
        j = (n // (nx + 1)) % (ny + 1)
        k = n // ((nx + 1) * (ny + 1))
        for a, (di, dj, dk) in enumerate(LOCAL_NODES):
            ei, ej, ek = i - di, j - dj, k - dk
            if not (0 <= ei < nx and 0 <= ej < ny and 0 <= ek < nz):
                continue
            dofs = []
            for b, (bi, bj, bk) in enumerate(LOCAL_NODES):
                m = node_index(nx, ny, nz, ei + bi, ej + bj, ek + bk)
                dofs.extend((3 * m, 3 * m + 1, 3 * m + 2))
            e = ei + nx * (ej + ny * ek)
            out[r] += E_elem[e] * (Ke[3 * a:3 * a + 3, :] @ uf[dofs])
        for c in range(3):
            if fixed[3 * n + c]:
                out[r, c] = 0.0
    return out


def apply_K_elementwise(nx, ny, nz, E_elem, Ke, fixed, u, edof=None):
    """y = K_ff u_f on free dofs, 0 on fixed dofs, evaluated from the
    definition K = sum_e E_e A_e^T Ke A_e without assembling K: gather each
    brick's 24 values, multiply by E_e Ke, add the products back into the
    global vector (np.bincount sums them in element order).  Memory grows
    with the mesh, not with the nonzeros of K, so it serves grids whose
    assembled K does not fit in host memory."""
    if edof is None:
        edof = element_dofs(nx, ny, nz)
    uf = np.where(fixed, 0.0, u)
    Y = (uf[edof] @ Ke) * np.asarray(E_elem, dtype=np.float64)[:, None]  # Ke symmetric
    y = np.bincount(edof.ravel(), weights=Y.ravel(), minlength=u.size)
    return np.where(fixed, 0.0, y)


def apply_K_free(K: sp.csr_matrix, fixed: np.ndarray, u: np.ndarray) -> np.ndarray:
    """y = K_ff u_f on free dofs, 0 on fixed dofs (fixed entries of u are
    ignored)."""
    free = ~fixed
    uf = np.where(free, u, 0.0)
    return np.where(free, K @ uf, 0.0)


# ---------------------------------------------------------------------------
# Solve K_ff u_f = f_f
# ---------------------------------------------------------------------------
def _longest_axis_slowest_perm(nx, ny, nz):
    """Dof permutation that numbers the longest grid axis slowest (smallest
    band of the banded Cholesky factor)."""
    dims = [nx + 1, ny + 1, nz + 1]
    order = sorted(range(3), key=lambda d: dims[d])  # fastest .. slowest
    ii, jj, kk = np.meshgrid(np.arange(dims[0]), np.arange(dims[1]),
                             np.arange(dims[2]), indexing="ij")
    idx = [ii.ravel(), jj.ravel(), kk.ravel()]
    new = idx[order[0]] + dims[order[0]] * (idx[order[1]] + dims[order[1]] * idx[order[2]])
    old = node_index(nx, ny, nz, idx[0], idx[1], idx[2])
    node_perm = np.empty_like(old)
    node_perm[new] = old          # new position -> old node
    dof_perm = (3 * node_perm[:, None] + np.arange(3)[None, :]).ravel()
    return dof_perm


def solve_direct(nx, ny, nz, E_elem, Ke, f, fixed) -> np.ndarray:
    """u = K^-1 f with fixed dofs eliminated, by banded Cholesky (LAPACK
    pbtrf/pbtrs) after numbering the longest axis slowest."""
    K = assemble_K(nx, ny, nz, E_elem, Ke)
    perm = _longest_axis_slowest_perm(nx, ny, nz)
    perm = perm[~fixed[perm]]                 # free dofs, banded order
    Kff = K[perm][:, perm].tocoo()
    upper = Kff.col >= Kff.row
    r, c, v = Kff.row[upper], Kff.col[upper], Kff.data[upper]
    bw = int(np.max(c - r))
    ab = np.zeros((bw + 1, perm.size))
    ab[bw + r - c, c] = v
    cb = scipy.linalg.cholesky_banded(ab, lower=False, check_finite=False)
    uf = scipy.linalg.cho_solve_banded((cb, False), f[perm], check_finite=False)
    u = np.zeros(K.shape[0])
    u[perm] = uf
    return u


def solve_pcg(nx, ny, nz, E_elem, Ke, f, fixed, rtol=1e-12, max_iters=100000,
              u0=None, elementwise=False, progress=None):
    """Fallback for grids too large for the banded factor: Jacobi-preconditioned
    CG on K_ff, stopped at ||f - K u|| <= rtol ||f|| over the free dofs.
    K_ff is the assembled CSR matrix, or with elementwise=True the
    element-by-element product apply_K_elementwise (the same K, for grids
    whose assembled matrix does not fit in host memory); the Jacobi diagonal
    is then sum_e E_e Ke_dd over the bricks that hold the dof.  progress, if
    given, is called as progress(iteration, relative residual) every 100
    iterations.  Returns (u, iterations, relative residual)."""
    free = ~fixed
    if elementwise:
        edof = element_dofs(nx, ny, nz)
        E = np.asarray(E_elem, dtype=np.float64)
        dfull = np.bincount(edof.ravel(), weights=(E[:, None] * np.diag(Ke)[None, :]).ravel(),
                            minlength=f.size)

        def matvec(v):
            full = np.zeros(f.size)
            full[free] = v
            return apply_K_elementwise(nx, ny, nz, E, Ke, fixed, full, edof)[free]
        d = dfull[free]
    else:
        K = assemble_K(nx, ny, nz, E_elem, Ke)
        Kff = K[free][:, free].tocsr()
        d = Kff.diagonal()

        def matvec(v):
            return Kff @ v
    b = f[free]
    x = np.zeros(b.size) if u0 is None else u0[free].copy()
    r = b - matvec(x)
    z = r / d
    p = z.copy()
    rz = r @ z
    bnorm = np.linalg.norm(b)
    it = 0
    rel = np.linalg.norm(r) / bnorm
    while rel > rtol and it < max_iters:
        q = matvec(p)
        alpha = rz / (p @ q)
        x += alpha * p
        r -= alpha * q
        z = r / d
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
        it += 1
        rel = np.linalg.norm(r) / bnorm
        if progress is not None and it % 100 == 0:
            progress(it, rel)
    u = np.zeros(f.size)
    u[free] = x
    return u, it, rel


# ---------------------------------------------------------------------------
# Compliance (Eq. 4) and its gradient (Eq. 5)
# ---------------------------------------------------------------------------
def compliance(f, u) -> float:
    return float(np.dot(f, u))


def element_energies(nx, ny, nz, Ke, u) -> np.ndarray:
    """u_e^T Ke u_e of every element (unit modulus)."""
    Ue = u[element_dofs(nx, ny, nz)]
    return np.einsum("ei,ij,ej->e", Ue, Ke, Ue)


def sensitivity_elements(nx, ny, nz, Ke, rho, u, elems, E0=1.0, Emin=1e-9, penal=3.0):
    """Eq. (5) for the given elements only (same formula as sensitivity)."""
    edof = element_dofs(nx, ny, nz)[elems]
    Ue = u[edof]
    ee = np.einsum("ei,ij,ej->e", Ue, Ke, Ue)
    return -penal * np.asarray(rho)[elems] ** (penal - 1.0) * (E0 - Emin) * ee


def sensitivity(nx, ny, nz, Ke, rho, u, E0=1.0, Emin=1e-9, penal=3.0):
    """dc/drho_e = -u^T (dK/drho_e) u = -p rho_e^(p-1) (E0 - Emin) u_e^T Ke u_e.
    The compliance is self-adjoint, so the adjoint of Eq. (3) is u itself."""
    ee = element_energies(nx, ny, nz, Ke, u)
    return -penal * np.asarray(rho) ** (penal - 1.0) * (E0 - Emin) * ee


def adjoint_sensitivity(nx, ny, nz, Ke, rho, u, lam, E0=1.0, Emin=1e-9, penal=3.0):
    """The state-equation term of the gradient (3) for r(rho, u) = K(rho) u - f:
    -lam^T (dr/drho_e) = -p rho_e^(p-1) (E0 - Emin) lam_e^T Ke u_e, where lam
    solves K^T lam = dJ/du (K is symmetric)."""
    edof = element_dofs(nx, ny, nz)
    return -penal * np.asarray(rho) ** (penal - 1.0) * (E0 - Emin) * np.einsum(
        "ei,ij,ej->e", lam[edof], Ke, u[edof])


def adjoint_sensitivity_elements(nx, ny, nz, Ke, rho, u, lam, elems, E0=1.0, Emin=1e-9, penal=3.0):
    """adjoint_sensitivity for the given elements only (same formula)."""
    edof = element_dofs(nx, ny, nz)[elems]
    return -penal * np.asarray(rho)[elems] ** (penal - 1.0) * (E0 - Emin) * np.einsum(
        "ei,ij,ej->e", lam[edof], Ke, u[edof])


def linear_objective_gradient(nx, ny, nz, Ke, rho, f, l, fixed, E0=1.0, Emin=1e-9, penal=3.0):
    """dJ/drho of J = l^T u(rho) by the gradient (3): J has no explicit
    dependence on rho and dJ/du = l, so u solves K u = f, lam solves
    K lam = l (both with the fixed dofs eliminated) and the gradient is
    adjoint_sensitivity(u, lam).  Returns (u, lam, gradient)."""
    E = simp_modulus(rho, E0, Emin, penal)
    u = solve_direct(nx, ny, nz, E, Ke, f, fixed)
    lam = solve_direct(nx, ny, nz, E, Ke, l, fixed)
    return u, lam, adjoint_sensitivity(nx, ny, nz, Ke, rho, u, lam, E0, Emin, penal)


# ---------------------------------------------------------------------------
# Density filter P (Eq. 4) and its transpose (gradient of the volume, Sec. III-D)
# ---------------------------------------------------------------------------
def filter_matrix(nx, ny, nz, r) -> sp.csr_matrix:
    """Row-normalised cone filter over element centroids (element units):
    w_ij = max(0, r - dist), truncated at the domain boundary."""
    R = int(math.ceil(r))
    e = np.arange(nx * ny * nz)
    i = e % nx
    j = (e // nx) % ny
    k = e // (nx * ny)
    rows, cols, vals = [], [], []
    for dk in range(-R, R + 1):
        for dj in range(-R, R + 1):
            for di in range(-R, R + 1):
                w = r - math.sqrt(di * di + dj * dj + dk * dk)
                if w <= 0.0:
                    continue
                ii, jj, kk = i + di, j + dj, k + dk
                ok = (ii >= 0) & (ii < nx) & (jj >= 0) & (jj < ny) & (kk >= 0) & (kk < nz)
                rows.append(e[ok])
                cols.append((ii + nx * (jj + ny * kk))[ok])
                vals.append(np.full(int(ok.sum()), w))
    H = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(e.size, e.size)).tocsr()
    W = np.asarray(H.sum(axis=1)).ravel()
    return sp.diags(1.0 / W) @ H


def apply_filter(nx, ny, nz, r, x, transpose=False) -> np.ndarray:
    P = filter_matrix(nx, ny, nz, r)
    return (P.T @ x) if transpose else (P @ x)


# ---------------------------------------------------------------------------
# Optimality-criteria update (Sec. III-D, with the volume of Eq. (4))
# ---------------------------------------------------------------------------
def oc_update(x, dcx, dv, volfrac, move, rel_tol=1e-12):
    """x_new(lam) = clamp(x * sqrt(max(0, -dcx) / (lam * dv)),
                          max(0, x - move), min(1, x + move)),
    with lam found by bisection so that sum(dv * x_new) = volfrac * N.
    Returns (x_new, lam, max |x_new - x|)."""
    x = np.asarray(x, dtype=np.float64)
    target = volfrac * x.size
    lo = np.maximum(0.0, x - move)
    hi = np.minimum(1.0, x + move)
    B = np.maximum(0.0, -np.asarray(dcx)) / np.asarray(dv)

    def x_of(lam):
        return np.clip(x * np.sqrt(B / lam), lo, hi)

    l1, l2 = 0.0, 1e9
    while np.sum(dv * x_of(l2)) > target and l2 < 1e300:   # widen until the bracket holds
        l2 *= 10.0
    while (l2 - l1) > rel_tol * (l1 + l2):
        lmid = 0.5 * (l1 + l2)
        if np.sum(dv * x_of(lmid)) > target:
            l1 = lmid
        else:
            l2 = lmid
    lam = 0.5 * (l1 + l2)
    xn = x_of(lam)
    return xn, lam, float(np.max(np.abs(xn - x)))


# ---------------------------------------------------------------------------
# Coarse scale of the two-scale scheme (Sec. III-C, Sec. III-E; the
# coarse-graining and coarse-solve steps of Alg. 1)
# ---------------------------------------------------------------------------
def block_mean(nx, ny, nz, z, nb) -> np.ndarray:
    """z_C: each coarse element takes the mean of the design variables over
    its nb x nb x nb block of fine elements (nb divides nx, ny, nz).  Coarse
    element (I, J, K) holds fine elements i = nb I .. nb I + nb - 1 (and so on);
    the coarse grid is numbered like the fine one."""
    if nb < 1 or nx % nb or ny % nb or nz % nb:
        raise ValueError("nb must be >= 1 and divide nx, ny, nz")
    z = np.asarray(z, dtype=np.float64).reshape(nz // nb, nb, ny // nb, nb, nx // nb, nb)
    return z.mean(axis=(1, 3, 5)).ravel()


def coarse_scale_solve(nx, ny, nz, z, nb, f_c, nu=0.3, h=1.0, r=1.5, E0=1.0, Emin=1e-9, penal=3.0):
    """u_C of K_C(z_C) u_C = f_C on the coarse mesh of (nx/nb, ny/nb, nz/nb)
    elements of edge nb h, with the design-to-stiffness map of the fine
    scale: z_C = block_mean(z), the density filter of the same physical
    radius (r / nb coarse elements), SIMP, supports clamped at x = 0.  With
    nb = 1 this is the fine-scale solve.  Returns (z_C, u_C, c_C)."""
    ncx, ncy, ncz = nx // nb, ny // nb, nz // nb
    zc = block_mean(nx, ny, nz, z, nb)
    rho_c = filter_matrix(ncx, ncy, ncz, r / nb) @ zc
    Ke = hex8_ke(nu, h=nb * h)
    u = solve_direct(ncx, ncy, ncz, simp_modulus(rho_c, E0, Emin, penal), Ke, f_c,
                     clamp_x0_fixed(ncx, ncy, ncz))
    return zc, u, compliance(f_c, u)
