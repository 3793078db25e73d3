"""Continuous batching: every design's result is the same alone and in the
mix, admission respects the HBM budget, and one result matches the oracle."""
import numpy as np
import pytest
import torch

from oracle import fe_oracle as O
from paper_2104_12282_amd import serve, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _requests(n, seed=0):
    grids = ((32, 16, 16), (48, 24, 24), (16, 8, 8))
    return synth.serving_requests(n, seed=seed, grids=grids)


def test_results_same_alone_and_in_the_mix():
    reqs = _requests(10)
    arrivals = np.linspace(0.0, 0.02, len(reqs))  # arrive while others are on the GPU
    mix, st = serve.run_engine(reqs, arrivals, device=DEV, max_active=6, keep_outputs=True)
    alone, _ = serve.run_sequential(reqs, device=DEV, keep_outputs=True)
    assert st["requests"] == len(reqs) and st["max_active"] > 1
    for r in reqs:
        a, b = mix[r["id"]], alone[r["id"]]
        assert a["iters"] == b["iters"]
        assert np.array_equal(a["u"], b["u"])      # same arithmetic, bitwise
        assert np.array_equal(a["dc"], b["dc"])
        assert a["rel_res"] <= 1e-8


def test_admission_by_footprint():
    reqs = _requests(5, seed=3)
    fps = [serve.request_footprint(*r["grid"], precision="fp32_ir", precond="gmg", mg_levels=3)
           for r in reqs]
    budget = max(fps) + 1  # room for one design at a time
    res, st = serve.run_engine(reqs, None, device=DEV, max_active=8, hbm_budget=budget)
    assert st["requests"] == len(reqs)
    assert st["max_active"] == 1
    # admissions never overlap: each admits after the previous finished
    seq = sorted(res.values(), key=lambda r: r["admit"])
    for prev, nxt in zip(seq, seq[1:]):
        assert nxt["admit"] >= prev["finish"] - 1e-3


def test_served_design_matches_oracle():
    req = {"id": 0, "grid": (16, 8, 8), "seed": 1234}
    res, _ = serve.run_engine([req], None, device=DEV, keep_outputs=True)
    nx, ny, nz = req["grid"]
    f, rho0 = serve.prepare_inputs(req, DEV)
    P = O.filter_matrix(nx, ny, nz, 1.5)
    rho = P @ (P @ (P @ rho0))
    Ke = O.hex8_ke(0.3)
    u = O.solve_direct(nx, ny, nz, O.simp_modulus(rho), Ke, f, O.clamp_x0_fixed(nx, ny, nz))
    c_ref = O.compliance(f, u)
    dc_ref = O.sensitivity(nx, ny, nz, Ke, rho, u)
    r = res[0]
    assert abs(r["compliance"] - c_ref) / c_ref <= 1e-6
    assert np.abs(r["dc"] - dc_ref).max() / np.abs(dc_ref).max() <= 1e-5


@pytest.mark.parametrize("precision,grid,levels", [("fp32_ir", (16, 8, 8), 3), ("fp64", (16, 8, 8), 3),
                                                   ("fp32_ir", (13, 7, 5), 3), ("fp64", (13, 7, 5), 3),
                                                   ("fp32_ir", (96, 48, 48), 3), ("fp32_ir", (128, 64, 64), 3),
                                                   ("fp64", (192, 32, 32), 4), ("fp32_ir", (192, 32, 32), 4)])
def test_batch_slots_match_lone_solves(precision, grid, levels):
    """Designs sharing a batch's launches (one slot idle, slots reused)
    give bitwise the result of the same design solved alone, also on an odd
    grid whose coarse levels overhang the mesh, and with four levels whose
    level 2 is smoothed by Chebyshev steps (on by default over a coarsest
    grid of 24 elements) -- as long as the batch's coarse Chebyshev launches
    take the lone solve's form.  The forms follow the workgroups of a launch
    (3D tiles while every slot's blocks get a compute unit each, else the
    z-march), so on the largest serving grid the batch of three marches
    where the lone solve takes 3D tiles: the same polynomial with its node
    sums rounded in another order, hence the same iterations within a few
    and the same displacement to 1e-6 of its largest entry."""
    from paper_2104_12282_amd import fe
    nx, ny, nz = grid
    T = lambda a: torch.as_tensor(a, dtype=torch.float64, device=DEV)
    designs = [(synth.point_load(nx, ny, nz, s), synth.density_uniform(nx, ny, nz, s)) for s in (11, 12, 13, 14)]
    alone = []
    for f, rho in designs:
        p = fe.Problem(nx, ny, nz, T(f), device=DEV, precision=precision, precond="gmg", mg_levels=levels)
        u, info = p.solve(T(rho), rtol=1e-8)
        alone.append((u.cpu().numpy(), info))
        p.close()
    b = fe.Batch(nx, ny, nz, 3, device=DEV, precision=precision, mg_levels=levels)
    got = {}
    todo = list(range(len(designs)))
    live = {}
    free = [0, 1]  # slot 2 stays idle
    rounds = 0
    while todo or live:
        while todo and free:
            d, s = todo.pop(0), free.pop(0)
            f, rho = designs[d]
            prob = b.setup_slot(s, T(f))
            u = torch.zeros(prob.ndof, dtype=torch.float64, device=DEV)
            prob.solve_begin(T(rho), u, rtol=1e-8)
            live[s] = (d, prob, u)
        b.round_begin()
        b.round_end()
        rounds += 1
        assert rounds < 5000
        for s, (d, prob, u) in list(live.items()):
            if prob.solve_step():
                got[d] = (u.cpu().numpy(), prob.solve_end())
                del live[s]
                free.append(s)
    b.close()
    # the library's choice of coarse launch form (fe_set_coarse_fusion)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    cx, cy, cz = nx, ny, nz
    for _ in range(levels - 1):
        cx, cy, cz = (cx + 1) // 2, (cy + 1) // 2, (cz + 1) // 2
    cols = ((cx + 4) // 4) * ((cy + 4) // 4)
    n4, n8 = cols * ((cz + 4) // 4), cols * ((cz + 8) // 8)
    same_form = (n4 <= cus) == (n4 * 3 <= cus or n8 * 3 <= cus)
    for d in range(len(designs)):
        ua, ia = alone[d]
        ub, ib = got[d]
        assert ib["rel_res"] <= 1e-8
        if same_form:
            assert ia["iters"] == ib["iters"] and ia["outer_iters"] == ib["outer_iters"]
            assert np.array_equal(ua, ub)
        else:
            assert abs(ia["iters"] - ib["iters"]) <= 2 + 0.15 * ia["iters"]
            assert np.abs(ua - ub).max() <= 1e-6 * np.abs(ua).max()


def test_batched_engine_matches_sequential():
    reqs = _requests(12, seed=5)
    arrivals = np.linspace(0.0, 0.03, len(reqs))
    mix, st = serve.run_engine_batched(reqs, arrivals, device=DEV, nslots=3, keep_outputs=True)
    alone, _ = serve.run_sequential(reqs, device=DEV, keep_outputs=True)
    assert st["requests"] == len(reqs) and st["max_active"] > 1
    for r in reqs:
        a, b = mix[r["id"]], alone[r["id"]]
        assert a["iters"] == b["iters"]
        assert np.array_equal(a["u"], b["u"])
        assert np.array_equal(a["dc"], b["dc"])
        assert a["rel_res"] <= 1e-8


def test_batched_engine_budget_of_one_batch_two_sizes():
    """A budget that holds one size's batch at a time: requests of two sizes
    alternate, each size's batch is released once idle so the other's can
    be created, every request finishes and the admitted footprint never
    exceeds the budget."""
    from paper_2104_12282_amd import fe
    cfg = {"precision": "fp32_ir", "precond": "gmg", "mg_levels": 3}
    grids = ((16, 8, 8), (24, 12, 12))
    reqs = [{"id": i, "grid": grids[i % 2], "seed": 500 + i} for i in range(6)]

    def need(g):
        ne, nd = g[0] * g[1] * g[2], 3 * (g[0] + 1) * (g[1] + 1) * (g[2] + 1)
        return fe.Batch.workspace_bytes(*g, 2, **cfg) + 8 * (2 * nd + 3 * ne)

    budget = max(need(g) for g in grids) + 1
    res, st = serve.run_engine_batched(reqs, None, device=DEV, nslots=2, hbm_budget=budget, cfg_kw=cfg)
    assert st["requests"] == len(reqs)
    assert st["peak_bytes"] <= budget
    assert all(r["rel_res"] <= 1e-8 for r in res.values())


def test_sequential_reuse_matches_fresh_problems():
    """The sequential baseline with one problem kept per size (load swapped
    in) gives bitwise the results of a fresh problem per request."""
    reqs = _requests(6, seed=9)
    a, _ = serve.run_sequential(reqs, device=DEV, keep_outputs=True, reuse=True)
    b, _ = serve.run_sequential(reqs, device=DEV, keep_outputs=True, reuse=False)
    for r in reqs:
        assert a[r["id"]]["iters"] == b[r["id"]]["iters"]
        assert np.array_equal(a[r["id"]]["u"], b[r["id"]]["u"])
        assert np.array_equal(a[r["id"]]["dc"], b[r["id"]]["dc"])


def test_pinned_payloads_match_generated_inputs():
    """Requests that arrive with their inputs in pinned host memory (copied
    to the device asynchronously on each design's stream, the compliance
    read back through a pinned slot) give bitwise the results of inputs
    generated and copied synchronously, in every engine."""
    import copy
    reqs = _requests(8, seed=11)
    paid = serve.attach_payloads(copy.deepcopy(reqs))
    base, _ = serve.run_sequential(reqs, device=DEV, keep_outputs=True)
    for run in (lambda r: serve.run_sequential(r, device=DEV, keep_outputs=True),
                lambda r: serve.run_engine(r, None, device=DEV, keep_outputs=True),
                lambda r: serve.run_engine_batched(r, None, device=DEV, nslots=3, keep_outputs=True)):
        got, _ = run(paid)
        for r in reqs:
            a, b = base[r["id"]], got[r["id"]]
            assert a["iters"] == b["iters"]
            assert a["compliance"] == b["compliance"]
            assert np.array_equal(a["u"], b["u"])
            assert np.array_equal(a["dc"], b["dc"])
