"""Seeded synthetic inputs of the cantilever workloads (numpy, float64).

This module holds problem data only (densities, loads, supports, arrival
times); none of the method's arithmetic lives here.  Both the HIP path and
the CPU oracle take their inputs from it.

Canonical orders: element e = i + nx*(j + ny*k); node n = i + (nx+1)*(j +
(ny+1)*k); dof 3n + c.
"""
from __future__ import annotations

import numpy as np


def counts(nx, ny, nz):
    return nx * ny * nz, (nx + 1) * (ny + 1) * (nz + 1)


def density_around(nx, ny, nz, seed, base=0.3, spread=0.1, lo=0.01, hi=1.0):
    """clip(base + U(-spread, spread), lo, hi) per element."""
    rng = np.random.default_rng(seed)
    ne = nx * ny * nz
    return np.clip(base + rng.uniform(-spread, spread, ne), lo, hi)


def density_uniform(nx, ny, nz, seed, lo=0.01, hi=1.0):
    """U(lo, hi) per element (to be smoothed by the density filter)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, nx * ny * nz)


def cantilever_edge_load(nx, ny, nz, total=1.0):
    """Unit downward (-z) load spread along the bottom edge (k = 0) of the
    face x = nx with consistent (trapezoid) weights: interior nodes total/ny,
    the two end nodes total/(2 ny)."""
    _, nn = counts(nx, ny, nz)
    f = np.zeros(3 * nn)
    for j in range(ny + 1):
        w = 0.5 if j in (0, ny) else 1.0
        n = nx + (nx + 1) * j
        f[3 * n + 2] = -total * w / ny
    return f


def point_load(nx, ny, nz, seed):
    """Unit force at a uniformly drawn node of the face x = nx, direction
    uniform on the sphere (normalised Gaussian)."""
    rng = np.random.default_rng(seed)
    j = int(rng.integers(0, ny + 1))
    k = int(rng.integers(0, nz + 1))
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    _, nn = counts(nx, ny, nz)
    f = np.zeros(3 * nn)
    n = nx + (nx + 1) * (j + (ny + 1) * k)
    f[3 * n:3 * n + 3] = d
    return f


def clamp_x0(nx, ny, nz):
    """uint8 dof mask: all dofs of the nodes on the face x = 0 are fixed."""
    _, nn = counts(nx, ny, nz)
    n = np.arange(nn)
    return np.repeat((n % (nx + 1)) == 0, 3).astype(np.uint8)


def poisson_arrivals(n, rate, seed):
    """Arrival times (s) of n requests of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n))


SERVING_GRIDS = ((32, 16, 16), (48, 24, 24), (64, 32, 32), (96, 48, 48), (128, 64, 64))


def serving_requests(n, seed=0, grids=SERVING_GRIDS):
    """Request i: grid drawn uniformly from `grids`, its own seed 1000 + i for
    the load and the density draw."""
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, len(grids), n)
    return [{"id": i, "grid": tuple(grids[int(idx[i])]), "seed": 1000 + i} for i in range(n)]


def mlp_init(sizes, seed):
    """Initial parameters of a fully-connected network with layer sizes
    `sizes`: per layer W (out x in, row-major) from the He-uniform
    U(-sqrt(6/in), sqrt(6/in)), then a zero bias; float64, flat."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, o in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / i)
        parts.append(rng.uniform(-lim, lim, o * i))
        parts.append(np.zeros(o))
    return np.concatenate(parts)


def minibatches(n_samples, steps, batch, seed):
    """steps x batch sample indices drawn uniformly with replacement (int32)."""
    return np.random.default_rng(seed).integers(0, n_samples, size=(steps, batch)).astype(np.int32)
