"""MI355X (gfx950) HIP implementation of the exact-gradient finite-element step
of minimum-compliance topology optimisation: matrix-free K(rho)u, Jacobi and
multigrid preconditioned CG with float64 refinement, compliance sensitivity,
density filter and optimality-criteria update, behind the C ABI of
include/fe_abi.h.  ``fe`` is the ctypes binding, ``synth`` the seeded inputs."""
