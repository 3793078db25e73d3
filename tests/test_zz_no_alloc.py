"""The allocation-free OC entry point (oc_update_noalloc, static per-device
scratch) against the problem-bound oc_update it varies: the same kernels in
the same order, so x_new and the change must agree bit for bit.  Two calls
in a row, the second on a smaller design, show that nothing left in the
shared scratch by the first call leaks into the second; the oracle's update
of the same inputs checks both against the definition."""
import numpy as np
import pytest
import torch

from oracle import fe_oracle as O
from paper_2104_12282_amd import fe

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _inputs(nx, ny, nz, seed, xmax):
    """A design in [0.01, xmax] (its mean near the volume fraction, so the
    target is reachable within the move limit), a compliance-like
    sensitivity spanning six decades (near-void elements carry tiny
    gradients) and dv = P^T 1."""
    rng = np.random.default_rng(seed)
    n = nx * ny * nz
    x = rng.uniform(0.01, xmax, n)
    dcx = -(10.0 ** rng.uniform(-6.0, 0.0, n)) * x ** 2
    dv = O.apply_filter(nx, ny, nz, 1.5, np.ones(n), transpose=True)
    return x, dcx, dv


def _t(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=DEV)


@pytest.mark.parametrize("volfrac,move,xmax", [(0.3, 0.2, 0.6), (0.12, 0.05, 0.22)])
def test_noalloc_matches_oc_update_twice(volfrac, move, xmax):
    # the second call is on a smaller design than the first
    for (nx, ny, nz), seed in (((40, 20, 12), 1), ((13, 7, 5), 2)):
        x, dcx, dv = _inputs(nx, ny, nz, seed, xmax)
        n = x.size
        print(f"noalloc: grid {nx}x{ny}x{nz} volfrac {volfrac} move {move}", flush=True)
        xs, dcs, dvs = _t(x), _t(dcx), _t(dv)
        out = torch.full((n,), -1.0, dtype=torch.float64, device=DEV)
        ch = torch.full((1,), -1.0, dtype=torch.float64, device=DEV)
        fe.oc_update_noalloc(xs, dcs, dvs, volfrac, move, out, ch)
        prob = fe.Problem(nx, ny, nz, torch.zeros(3 * (nx + 1) * (ny + 1) * (nz + 1), dtype=torch.float64,
                                                  device=DEV), device=DEV)
        ref, ref_ch = prob.oc_update(xs, dcs, dvs, volfrac, move)
        torch.cuda.synchronize()
        prob.close()
        assert torch.equal(out, ref), (nx, ny, nz)
        assert torch.equal(ch, ref_ch)
        xo, _, cho = O.oc_update(x, dcx, dv, volfrac, move)
        got = out.cpu().numpy()
        assert np.abs(got - xo).max() <= 1e-9
        assert abs(float(ch.item()) - cho) <= 1e-9
        assert abs(float(np.dot(dv, got)) - volfrac * n) <= 1e-10 * volfrac * n


def test_noalloc_in_place_on_a_side_stream():
    nx, ny, nz = 24, 12, 8
    x, dcx, dv = _inputs(nx, ny, nz, 3, 0.6)
    xs, dcs, dvs = _t(x), _t(dcx), _t(dv)
    side = torch.cuda.Stream(device=DEV)
    side.wait_stream(torch.cuda.current_stream(DEV))
    xa = xs.clone()
    with torch.cuda.stream(side):
        fe.oc_update_noalloc(xa, dcs, dvs, 0.3, 0.2, xa, None, stream=side)
    side.synchronize()
    xb = torch.empty_like(xs)
    fe.oc_update_noalloc(xs, dcs, dvs, 0.3, 0.2, xb)
    torch.cuda.synchronize()
    assert torch.equal(xa, xb)


def test_noalloc_rejects_bad_arguments():
    x = torch.zeros(8, dtype=torch.float64, device=DEV)
    with pytest.raises(fe.FEError):
        fe.oc_update_noalloc(x, x, x, 1.5, 0.2, x.clone())
    lib = fe.load_library()
    assert lib.oc_update_noalloc(0, None, None, None, 0.3, 0.2, None, None, None) == fe.FE_EINVAL
    p = fe._ptr(x)
    assert lib.oc_update_noalloc(0, p, p, p, 0.3, 0.2, p, None, None) == fe.FE_EINVAL
    assert lib.oc_update_noalloc(2 ** 31, p, p, p, 0.3, 0.2, p, None, None) == fe.FE_EINVAL
