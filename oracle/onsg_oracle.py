"""Plain CPU oracle of the online neural synthetic gradients (Sec. III-B/C/E,
Alg. 1): per-block training samples of the two-scale scheme, the
fully-connected network, its mean-squared-error loss, back-propagation and
Adam, written from their definitions in float64 NumPy.

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``;
nothing in the product path imports, links or calls it, and it
imports nothing from the product package.

Readings where the paper is silent:
  * a sample is one block of nb^3 fine elements: its input is the block's
    design variables (local order x fastest, then y, then z) followed by the
    24 coarse displacements of its coarse element (local node order of
    fe_oracle.LOCAL_NODES, 3 dofs each) divided by a scale s_u; its target
    is the exact gradient dJ/dz of the block's elements divided by a scale
    s_g (the optimisation loop takes each iteration's max |u_C| and
    max |dJ/dz|: the OC update is blind to a positive factor on the
    gradient, its multiplier absorbs it);
  * the network has 4 hidden layers with ReLU and a linear output layer;
    parameters are stored per layer as W (out x in, row-major) then b (out);
  * the loss is the mean of the squared errors over the mini-batch and the
    outputs; Adam (beta1 0.9, beta2 0.999, eps 1e-8) with bias correction,
    the learning rate halved every `halve_every` steps of an update; each
    model update is a fresh Adam run (moments and schedule restart) from the
    current weights, on mini-batches whose sample indices are given.
"""
from __future__ import annotations

import numpy as np

from oracle.fe_oracle import LOCAL_NODES as CORNERS


def layer_sizes(nb: int, width: int) -> list[int]:
    """Input nb^3 + 24, four hidden layers of `width`, output nb^3."""
    return [nb ** 3 + 24, width, width, width, width, nb ** 3]


def n_params(sizes) -> int:
    return sum(o * i + o for i, o in zip(sizes[:-1], sizes[1:]))


def unpack(params, sizes):
    """List of (W, b) per layer from the flat parameter vector."""
    out, k = [], 0
    for i, o in zip(sizes[:-1], sizes[1:]):
        W = params[k:k + o * i].reshape(o, i)
        k += o * i
        b = params[k:k + o]
        k += o
        out.append((W, b))
    return out


def block_samples(nx, ny, nz, nb, z, uc, g=None, s_u=1.0, s_g=1.0):
    """Inputs (nblocks, nb^3 + 24) and, with g, targets (nblocks, nb^3) of the
    blocks in coarse element order (I fastest); uc is the coarse-mesh
    displacement ((nx/nb + 1)(ny/nb + 1)(nz/nb + 1) nodes, 3 dofs)."""
    cx, cy, cz = nx // nb, ny // nb, nz // nb
    z = np.asarray(z, dtype=np.float64).reshape(nz, ny, nx)
    zb = z.reshape(cz, nb, cy, nb, cx, nb).transpose(0, 2, 4, 1, 3, 5).reshape(cz * cy * cx, nb ** 3)
    I, J, K = np.meshgrid(np.arange(cx), np.arange(cy), np.arange(cz), indexing="ij")
    I, J, K = (a.transpose(2, 1, 0).ravel() for a in (I, J, K))
    feats = []
    for a, b, c in CORNERS:
        node = (I + a) + (cx + 1) * ((J + b) + (cy + 1) * (K + c))
        feats.append(np.stack([uc[3 * node + d] for d in range(3)], axis=1))
    X = np.concatenate([zb, np.concatenate(feats, axis=1) / s_u], axis=1)
    if g is None:
        return X, None
    gb = np.asarray(g, dtype=np.float64).reshape(cz, nb, cy, nb, cx, nb).transpose(0, 2, 4, 1, 3, 5)
    return X, gb.reshape(cz * cy * cx, nb ** 3) / s_g


def scatter_blocks(nx, ny, nz, nb, Y, s_g=1.0):
    """Per-element gradient from per-block outputs (inverse of the target
    layout of block_samples), times s_g."""
    cx, cy, cz = nx // nb, ny // nb, nz // nb
    g = np.asarray(Y, dtype=np.float64).reshape(cz, cy, cx, nb, nb, nb).transpose(0, 3, 1, 4, 2, 5)
    return g.reshape(-1) * s_g


def forward(params, sizes, X):
    """Activations a_0 = X, a_l = relu(a_{l-1} W^T + b) for the hidden layers,
    and the linear output."""
    acts = [np.asarray(X, dtype=np.float64)]
    layers = unpack(params, sizes)
    for li, (W, b) in enumerate(layers):
        z = acts[-1] @ W.T + b
        acts.append(np.maximum(z, 0.0) if li < len(layers) - 1 else z)
    return acts


def loss_and_grad(params, sizes, X, Y):
    """Mean squared error over the batch and outputs, and its gradient with
    respect to the flat parameters (back-propagation)."""
    acts = forward(params, sizes, X)
    layers = unpack(params, sizes)
    diff = acts[-1] - Y
    loss = float(np.mean(diff * diff))
    dz = 2.0 * diff / diff.size
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        grads[li] = (dz.T @ acts[li], dz.sum(axis=0))
        if li > 0:
            dz = (dz @ W) * (acts[li] > 0.0)
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def adam_train(params, sizes, DX, DY, batch_idx, lr0, halve_every, beta1=0.9, beta2=0.999, eps=1e-8):
    """One model update: len(batch_idx) Adam steps from fresh moments on the
    mini-batches DX[idx], DY[idx]; the learning rate is lr0 halved every
    halve_every steps.  Returns (new parameters, loss of each step's batch
    before its update)."""
    p = np.array(params, dtype=np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    losses = []
    for t, idx in enumerate(batch_idx, start=1):
        loss, g = loss_and_grad(p, sizes, DX[idx], DY[idx])
        losses.append(loss)
        m = beta1 * m + (1.0 - beta1) * g
        v = beta2 * v + (1.0 - beta2) * g * g
        mh = m / (1.0 - beta1 ** t)
        vh = v / (1.0 - beta2 ** t)
        lr = lr0 * 0.5 ** ((t - 1) // halve_every)
        p = p - lr * mh / (np.sqrt(vh) + eps)
    return p, np.array(losses)
