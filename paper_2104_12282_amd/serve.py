"""Continuous batching of design solves on one GPU.

Requests (grid, load, density seed) arrive over time and are admitted in
arrival order whenever a slot is free and the device footprint of what is
admitted stays within the HBM budget.  Every admitted design keeps its u,
rho and multigrid hierarchy resident in its own workspace.  Two engines:

* run_engine_batched: designs of one grid size share an fe_batch (one
  workspace, nslots slots); their CG iterations run as one captured graph
  whose every launch covers all slots, and designs join a batch (free slot)
  and leave it (finished) between replays -- the batches of the different
  sizes advance in overlapping rounds on their own streams;
* run_engine: every design on its own, advancing through the non-blocking
  ABI (fe_solve_begin / fe_solve_step / fe_solve_end) on a few streams so
  that the designs' launches overlap.

A design's arithmetic does not depend on the mix: in a batch the launch
forms follow only the grid and the batch's slot count, and it is that of a
lone fe_solve except where a large batch's coarse Chebyshev launches march
while the lone solve takes 3D tiles (the same polynomial, node sums rounded
in another order).  Per request the engines record arrival,
admission and completion times (completion = sensitivity finished on the
device, observed by the host); they report designs/s and p50/p99 latency.
"""
from __future__ import annotations

import collections
import time

import numpy as np
import torch

from . import fe, synth

# Solver of a served design: float32 CG inside float64 refinement, four
# multigrid levels (on the serving grids up to 128 x 64 x 64 a fourth level
# was faster than three: 213 against 198 designs/s one at a time, 546-589
# against 476-518 batched)
SERVE_CFG = {"precision": "fp32_ir", "precond": "gmg", "mg_levels": 4}


def request_footprint(nx, ny, nz, **cfg_kw) -> int:
    """Device bytes one design holds while admitted: its workspace plus load,
    density (two buffers), displacement and sensitivity arrays."""
    cfg = fe.make_config(nx, ny, nz, **cfg_kw)
    ne, nd = nx * ny * nz, 3 * (nx + 1) * (ny + 1) * (nz + 1)
    return fe.workspace_size(cfg) + 8 * (2 * nd + 3 * ne)


class _Slot:
    def __init__(self, req, prob, stream, rho, u, dc, comp, admit_t, footprint):
        self.req, self.prob, self.stream = req, prob, stream
        self.rho, self.u, self.dc, self.comp = rho, u, dc, comp
        self.admit_t, self.footprint = admit_t, footprint
        self.info = None
        self.event = None  # sensitivity completion


def prepare_inputs(req, device):
    """Host-side seeded inputs of one request (load, raw density): its
    payload when one is attached, else generated now."""
    if "payload" in req:
        return req["payload"]["f"], req["payload"]["rho0"]
    nx, ny, nz = req["grid"]
    f = synth.point_load(nx, ny, nz, req["seed"])
    rho0 = synth.density_uniform(nx, ny, nz, req["seed"])
    return f, rho0


def attach_payloads(requests):
    """Gives every request its inputs in pinned host memory (load, raw
    density, and a pinned slot for the returned compliance), as a request
    that arrives with its design carries them: the engines then copy them
    to the device asynchronously on the design's stream and read the
    compliance without a synchronising copy."""
    for req in requests:
        if "payload" in req:
            continue
        nx, ny, nz = req["grid"]
        f = torch.from_numpy(synth.point_load(nx, ny, nz, req["seed"])).pin_memory()
        rho0 = torch.from_numpy(synth.density_uniform(nx, ny, nz, req["seed"])).pin_memory()
        req["payload"] = {"f": f, "rho0": rho0,
                          "comp": torch.zeros(1, dtype=torch.float64).pin_memory()}
    return requests


def _dev(x, device):
    """A request input on the device, copied on the current stream (pinned
    payloads asynchronously)."""
    if isinstance(x, torch.Tensor):
        return x.to(device, non_blocking=True)
    return torch.as_tensor(x, device=device)


def _comp_out(req, comp):
    """Queues the compliance's copy into the request's pinned slot on the
    current stream (read after the stream's completion event); None without
    a payload."""
    if "payload" not in req:
        return None
    host = req["payload"]["comp"]
    host.copy_(comp, non_blocking=True)
    return host


def _comp_value(host, comp):
    return float(host[0]) if host is not None else float(comp.item())


def _start(req, stream, device, cfg_kw, rtol, filter_passes):
    nx, ny, nz = req["grid"]
    f, rho0 = prepare_inputs(req, device)
    with torch.cuda.stream(stream):
        prob = fe.Problem(nx, ny, nz, _dev(f, device), device=device, stream=stream, **cfg_kw)
        a = _dev(rho0, device)
        b = torch.empty_like(a)
        for _ in range(filter_passes):  # smoothed density, on the device
            prob.filter(a, out=b)
            a, b = b, a
        u = torch.zeros(prob.ndof, dtype=torch.float64, device=device)
        dc = torch.empty_like(a)
        comp = torch.zeros(1, dtype=torch.float64, device=device)
        prob.solve_begin(a, u, rtol=rtol)
    return prob, a, u, dc, comp


def run_engine(requests, arrivals=None, *, device="cuda:0", max_active=16, n_streams=4,
               hbm_budget=64 << 30, rtol=1e-8, filter_passes=3, keep_outputs=False,
               cfg_kw=None, log=None):
    """Serves `requests` (dicts with id, grid, seed) arriving at `arrivals`
    (seconds after the start; None = all at once).  Returns (results, stats)."""
    cfg_kw = dict(cfg_kw or SERVE_CFG)
    if arrivals is None:
        arrivals = np.zeros(len(requests))
    order = np.argsort(arrivals, kind="stable")
    pending = collections.deque((float(arrivals[i]), requests[i]) for i in order)
    queue = collections.deque()
    streams = [torch.cuda.Stream(device=device) for _ in range(n_streams)]
    active: list[_Slot] = []
    used = 0
    results = {}
    max_q = max_act = 0
    t0 = time.perf_counter()
    rr = 0
    while pending or queue or active:
        now = time.perf_counter() - t0
        while pending and pending[0][0] <= now:
            t_arr, req = pending.popleft()
            queue.append((t_arr, req))
        # admission: FIFO, slot and memory permitting
        while queue and len(active) < max_active:
            t_arr, req = queue[0]
            fp = request_footprint(*req["grid"], **cfg_kw)
            if used + fp > hbm_budget and active:
                break
            queue.popleft()
            stream = streams[rr % n_streams]
            rr += 1
            prob, rho, u, dc, comp = _start(req, stream, device, cfg_kw, rtol, filter_passes)
            s = _Slot(req, prob, stream, rho, u, dc, comp, time.perf_counter() - t0, fp)
            s.arrival = t_arr
            active.append(s)
            used += fp
        max_q = max(max_q, len(queue))
        max_act = max(max_act, len(active))
        # advance every admitted design by at most one stage
        still = []
        for s in active:
            if s.info is None:
                if s.prob.solve_step():
                    s.info = s.prob.solve_end()
                    with torch.cuda.stream(s.stream):
                        s.prob.sensitivity(s.rho, s.u, out=s.dc, compliance_out=s.comp)
                        s.comp_host = _comp_out(s.req, s.comp)
                        s.event = torch.cuda.Event()
                        s.event.record(s.stream)
                still.append(s)
            elif s.event.query():
                t_done = time.perf_counter() - t0
                rec = {"id": s.req["id"], "grid": s.req["grid"], "arrival": s.arrival,
                       "admit": s.admit_t, "finish": t_done, "latency": t_done - s.arrival,
                       "iters": s.info["iters"], "outer_iters": s.info["outer_iters"],
                       "rel_res": s.info["rel_res"], "compliance": _comp_value(s.comp_host, s.comp)}
                if keep_outputs:
                    rec["u"] = s.u.cpu().numpy()
                    rec["dc"] = s.dc.cpu().numpy()
                results[s.req["id"]] = rec
                used -= s.footprint
                s.prob.close()
                if log:
                    log(rec)
            else:
                still.append(s)
        active = still
        if not active and queue == collections.deque() and pending:
            # idle until the next arrival
            wait = pending[0][0] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.01))
    torch.cuda.synchronize(device)
    wall = time.perf_counter() - t0
    lat = np.array([r["latency"] for r in results.values()])
    stats = {"requests": len(results), "wall_s": wall, "designs_per_s": len(results) / wall,
             "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
             "max_queue": max_q, "max_active": max_act}
    return results, stats


def run_sequential(requests, *, device="cuda:0", rtol=1e-8, filter_passes=3, keep_outputs=False,
                   cfg_kw=None, reuse=True):
    """The same requests one at a time with the blocking fe_solve (no
    overlap, no admission), for comparison.  With reuse (the default) one
    problem per grid size is set up once and kept: a request swaps in its
    load (fe_set_load) and reuses the size's workspace and captured graphs,
    as the batched engine reuses its slots; reuse=False sets up a fresh
    problem per request."""
    cfg_kw = dict(cfg_kw or SERVE_CFG)
    stream = torch.cuda.current_stream(device)
    results = {}
    probs = {}
    t0 = time.perf_counter()
    for req in requests:
        ts = time.perf_counter() - t0
        nx, ny, nz = req["grid"]
        f, rho0 = prepare_inputs(req, device)
        ft = _dev(f, device)
        prob = probs.get(tuple(req["grid"])) if reuse else None
        if prob is None:
            prob = fe.Problem(nx, ny, nz, ft, device=device, stream=stream, **cfg_kw)
            if reuse:
                probs[tuple(req["grid"])] = prob
        else:
            prob.set_load(ft)
        a = _dev(rho0, device)
        b = torch.empty_like(a)
        for _ in range(filter_passes):
            prob.filter(a, out=b)
            a, b = b, a
        u = torch.zeros(prob.ndof, dtype=torch.float64, device=device)
        _, info = prob.solve(a, u=u, rtol=rtol)
        dc, comp = prob.sensitivity(a, u)
        torch.cuda.synchronize(device)
        t_done = time.perf_counter() - t0
        rec = {"id": req["id"], "grid": req["grid"], "start": ts, "finish": t_done,
               "latency": t_done - ts, "iters": info["iters"], "rel_res": info["rel_res"],
               "compliance": float(comp.item())}
        if keep_outputs:
            rec["u"] = u.cpu().numpy()
            rec["dc"] = dc.cpu().numpy()
        results[req["id"]] = rec
        if not reuse:
            prob.close()
    wall = time.perf_counter() - t0
    for prob in probs.values():
        prob.close()
    lat = np.array([r["latency"] for r in results.values()])
    return results, {"requests": len(results), "wall_s": wall, "designs_per_s": len(results) / wall,
                     "p50_latency_s": float(np.percentile(lat, 50)),
                     "p99_latency_s": float(np.percentile(lat, 99)),
                     "problem_reuse": bool(reuse)}


def run_engine_batched(requests, arrivals=None, *, device="cuda:0", nslots=16, n_streams=4,
                       hbm_budget=64 << 30, rtol=1e-8, filter_passes=3, keep_outputs=False, cfg_kw=None,
                       log=None):
    """Serves `requests` with one fe_batch per grid size (nslots slots each,
    created when the first request of that size is admitted)."""
    cfg_kw = dict(cfg_kw or SERVE_CFG)
    if arrivals is None:
        arrivals = np.zeros(len(requests))
    order = np.argsort(arrivals, kind="stable")
    pending = collections.deque((float(arrivals[i]), requests[i]) for i in order)
    queue = []
    streams = [torch.cuda.Stream(device=device) for _ in range(n_streams)]
    classes = {}  # grid -> {"batch", "free", "live"}
    used = 0
    results = {}
    finishing = []  # (slot record, event)
    max_q = max_act = 0
    peak = 0  # largest admitted footprint (batch workspaces + per-request arrays)
    t0 = time.perf_counter()

    def release_idle(keep):
        """Closes the batches (other than size `keep`) that hold no design,
        live or finishing, returning their workspaces to the budget."""
        nonlocal used
        busy = {rec["cls"] for rec, _ in finishing}
        for gi in [gi for gi, ci in classes.items() if gi != keep and not ci["live"] and gi not in busy]:
            classes.pop(gi)["batch"].close()
            used -= fe.Batch.workspace_bytes(*gi, nslots, **cfg_kw)

    def per_request_bytes(grid):
        nx, ny, nz = grid
        ne, nd = nx * ny * nz, 3 * (nx + 1) * (ny + 1) * (nz + 1)
        return 8 * (2 * nd + 3 * ne)

    while pending or queue or finishing or any(c["live"] for c in classes.values()):
        now = time.perf_counter() - t0
        while pending and pending[0][0] <= now:
            queue.append(pending.popleft())
        # admission in arrival order: a request whose size has a free slot (or
        # whose size's batch fits the budget) is admitted
        rest = []
        for t_arr, req in queue:
            g = tuple(req["grid"])
            c = classes.get(g)
            if c is None:
                nbytes = fe.Batch.workspace_bytes(*g, nslots, **cfg_kw)
                if used + nbytes + per_request_bytes(g) > hbm_budget:
                    release_idle(g)
                if used + nbytes + per_request_bytes(g) > hbm_budget and (classes or finishing):
                    rest.append((t_arr, req))
                    continue
                stream = streams[len(classes) % n_streams]
                with torch.cuda.stream(stream):
                    b = fe.Batch(*g, nslots, device=device, stream=stream, **cfg_kw)
                c = classes[g] = {"batch": b, "free": list(range(nslots - 1, -1, -1)), "live": {}, "open": False}
                used += nbytes
                peak = max(peak, used)
            if c["free"] and used + per_request_bytes(g) > hbm_budget:
                release_idle(g)
            # a slot is set up only between its batch's rounds
            if c["open"] or not c["free"] or used + per_request_bytes(g) > hbm_budget:
                rest.append((t_arr, req))
                continue
            slot = c["free"].pop()
            b = c["batch"]
            f, rho0 = prepare_inputs(req, device)
            with torch.cuda.stream(b.stream):
                prob = b.setup_slot(slot, _dev(f, device))
                a = _dev(rho0, device)
                tmp = torch.empty_like(a)
                for _ in range(filter_passes):
                    prob.filter(a, out=tmp)
                    a, tmp = tmp, a
                u = torch.zeros(prob.ndof, dtype=torch.float64, device=device)
                prob.solve_begin(a, u, rtol=rtol)
            c["live"][slot] = {"req": req, "arrival": t_arr, "admit": time.perf_counter() - t0, "prob": prob,
                               "rho": a, "u": u, "slot": slot, "cls": g}
            used += per_request_bytes(g)
            peak = max(peak, used)
        if rest and len(rest) == len(queue) and not pending and not finishing \
                and not any(c["live"] for c in classes.values()):
            # nothing runs, nothing arrives, nothing was admitted: it never will be
            raise RuntimeError("a request cannot be admitted within the HBM budget")
        queue = rest
        max_q = max(max_q, len(queue))
        max_act = max(max_act, sum(len(c["live"]) for c in classes.values()))
        # every batch runs its rounds on its own stream: a batch whose round
        # has completed is advanced and started again at once, without
        # waiting for the rounds of the other sizes
        active = [c for c in classes.values() if c["live"] or c["open"]]
        for c in active:
            if c["open"]:
                if not c["batch"].round_ready():
                    continue
                c["batch"].round_end()
                c["open"] = False
            for slot, rec in list(c["live"].items()):
                if not rec["prob"].solve_step():
                    continue
                prob = rec["prob"]
                rec["info"] = prob.solve_end()
                with torch.cuda.stream(c["batch"].stream):
                    rec["dc"], rec["comp"] = prob.sensitivity(rec["rho"], rec["u"])
                    rec["comp_host"] = _comp_out(rec["req"], rec["comp"])
                    ev = torch.cuda.Event()
                    ev.record(c["batch"].stream)
                finishing.append((rec, ev))
                del c["live"][slot]
                c["free"].append(slot)  # stream order: the next design's setup follows the sensitivity
            if c["live"]:
                c["batch"].round_begin()
                c["open"] = True
        still = []
        for rec, ev in finishing:
            if not ev.query():
                still.append((rec, ev))
                continue
            t_done = time.perf_counter() - t0
            info = rec["info"]
            out = {"id": rec["req"]["id"], "grid": rec["req"]["grid"], "arrival": rec["arrival"],
                   "admit": rec["admit"], "finish": t_done, "latency": t_done - rec["arrival"],
                   "iters": info["iters"], "outer_iters": info["outer_iters"], "rel_res": info["rel_res"],
                   "compliance": _comp_value(rec["comp_host"], rec["comp"]), "slot": rec["slot"]}
            if keep_outputs:
                out["u"] = rec["u"].cpu().numpy()
                out["dc"] = rec["dc"].cpu().numpy()
            results[rec["req"]["id"]] = out
            used -= per_request_bytes(rec["cls"])
            if log:
                log(out)
        finishing = still
        if not active and not finishing and pending and (not queue or not classes):
            wait = pending[0][0] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.01))
    torch.cuda.synchronize(device)
    wall = time.perf_counter() - t0
    for c in classes.values():
        c["batch"].close()
    lat = np.array([r["latency"] for r in results.values()])
    return results, {"requests": len(results), "wall_s": wall, "designs_per_s": len(results) / wall,
                     "p50_latency_s": float(np.percentile(lat, 50)),
                     "p99_latency_s": float(np.percentile(lat, 99)), "max_queue": max_q,
                     "max_active": max_act, "slots_per_size": nslots, "peak_bytes": peak}
