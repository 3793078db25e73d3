"""Pins of the synthetic-gradient oracle: block samples against brute force
and closed forms, back-propagation against central finite differences, Adam
against its closed form under a constant gradient."""
import numpy as np
import pytest

from oracle import onsg_oracle as S
from paper_2104_12282_amd import synth


def test_block_samples_brute_force_and_round_trip():
    nx, ny, nz, nb = 6, 4, 8, 2
    cx, cy, cz = nx // nb, ny // nb, nz // nb
    rng = np.random.default_rng(0)
    z = rng.uniform(0, 1, nx * ny * nz)
    g = rng.standard_normal(nx * ny * nz)
    uc = rng.standard_normal(3 * (cx + 1) * (cy + 1) * (cz + 1))
    X, Y = S.block_samples(nx, ny, nz, nb, z, uc, g, s_u=2.0, s_g=4.0)
    assert X.shape == (cx * cy * cz, nb ** 3 + 24) and Y.shape == (cx * cy * cz, nb ** 3)
    for blk in range(cx * cy * cz):
        I, J, K = blk % cx, (blk // cx) % cy, blk // (cx * cy)
        for c in range(nb):
            for b in range(nb):
                for a in range(nb):
                    e = (nb * I + a) + nx * ((nb * J + b) + ny * (nb * K + c))
                    loc = a + nb * (b + nb * c)
                    assert X[blk, loc] == z[e] and Y[blk, loc] == g[e] / 4.0
        corners = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)]
        for q, (a, b, c) in enumerate(corners):
            n = (I + a) + (cx + 1) * ((J + b) + (cy + 1) * (K + c))
            for d in range(3):
                assert X[blk, nb ** 3 + 3 * q + d] == uc[3 * n + d] / 2.0
    assert np.array_equal(S.scatter_blocks(nx, ny, nz, nb, Y, s_g=4.0), g)


@pytest.mark.parametrize("nb,width", [(1, 6), (2, 5)])
def test_backprop_against_central_differences(nb, width):
    sizes = S.layer_sizes(nb, width)
    p = synth.mlp_init(sizes, seed=3)
    rng = np.random.default_rng(4)
    # biases away from zero keep every ReLU clear of its kink under the steps
    k = 0
    for i, o in zip(sizes[:-1], sizes[1:]):
        k += o * i
        p[k:k + o] = rng.uniform(0.05, 0.2, o)
        k += o
    X = rng.uniform(0, 1, (7, sizes[0]))
    Y = rng.standard_normal((7, sizes[-1]))
    loss, grad = S.loss_and_grad(p, sizes, X, Y)
    acts = S.forward(p, sizes, X)
    assert abs(loss - np.mean((acts[-1] - Y) ** 2)) <= 1e-15 * loss
    for j in rng.choice(p.size, size=25, replace=False):
        h = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[j] += h
        pm[j] -= h
        fd = (S.loss_and_grad(pp, sizes, X, Y)[0] - S.loss_and_grad(pm, sizes, X, Y)[0]) / (2 * h)
        assert abs(fd - grad[j]) <= 1e-7 * max(1.0, np.abs(grad).max()), (j, fd, grad[j])


def test_adam_closed_form_under_constant_gradient(monkeypatch):
    """With a constant gradient g the bias-corrected moments are g and g^2 at
    every step, so step t moves each parameter by -lr_t g / (|g| + eps)."""
    sizes = S.layer_sizes(1, 3)
    n = S.n_params(sizes)
    g = np.linspace(-2.0, 3.0, n)
    monkeypatch.setattr(S, "loss_and_grad", lambda p, s, X, Y: (0.0, g))
    p0 = np.zeros(n)
    steps, lr0, halve = 7, 1e-2, 3
    p, _ = S.adam_train(p0, sizes, np.zeros((1, sizes[0])), np.zeros((1, sizes[-1])),
                        np.zeros((steps, 1), dtype=np.int32), lr0, halve)
    lrs = [lr0 * 0.5 ** (t // halve) for t in range(steps)]
    ref = -sum(lrs) * g / (np.abs(g) + 1e-8)
    assert np.abs(p - ref).max() <= 1e-14


def test_training_fits_a_smooth_target():
    """A network of this shape must fit a smooth map of its inputs: the loss
    of 400 Adam steps falls below a tenth of the first batch's."""
    sizes = S.layer_sizes(1, 32)
    rng = np.random.default_rng(1)
    X = rng.uniform(0, 1, (256, sizes[0]))
    Y = np.sin(X[:, :3].sum(axis=1, keepdims=True))
    p, losses = S.adam_train(synth.mlp_init(sizes, 0), sizes, X, Y, synth.minibatches(256, 400, 32, 2), 5e-3, 200)
    assert losses[-20:].mean() < 0.1 * losses[0]


def _copy_net(nb, pick):
    """Parameters (per layer W out x in row-major, then b) of a network whose
    output k equals input pick[k]: relu(x) - relu(-x) = x through identity
    hidden layers of width 2 nin."""
    sizes = S.layer_sizes(nb, 2 * (nb ** 3 + 24))
    nin, w = sizes[0], sizes[1]
    eye = np.eye(nin)
    parts = [np.vstack([eye, -eye]).ravel(), np.zeros(w)]
    for _ in range(3):
        parts += [np.eye(w).ravel(), np.zeros(w)]
    Wo = np.zeros((nb ** 3, w))
    for k, src in enumerate(pick):
        Wo[k, src] = 1.0
        Wo[k, nin + src] = -1.0
    parts += [Wo.ravel(), np.zeros(nb ** 3)]
    return sizes, np.concatenate(parts)


@pytest.mark.parametrize("nb", [1, 2])
def test_forward_copies_picked_inputs(nb):
    """Signed inputs pass the copy network unchanged only if the hidden
    layers (and not the output layer) apply ReLU and every W is read as
    out x in, row-major, ahead of its bias."""
    rng = np.random.default_rng(11)
    nin = nb ** 3 + 24
    X = rng.standard_normal((9, nin))
    for pick in (list(range(nb ** 3)), [nin - 1 - (k % nin) for k in range(nb ** 3)]):
        sizes, p = _copy_net(nb, pick)
        assert p.size == S.n_params(sizes)
        out = S.forward(p, sizes, X)[-1]
        assert np.array_equal(out, X[:, pick])


# a network of widths 2 -> 3 -> 2 worked by hand, biases nonzero:
# z1 = W1 x + b1 = (1 - 4 + 0.5, 2 - 1, 3 - 2 + 2) = (-2.5, 1, 3); relu -> (0, 1, 3);
# out = W2 a1 + b2 = (0 + 1 + 3 - 1, 0 + 0 - 3 + 0.25) = (3, -2.75), linear (no ReLU).
HAND_X = np.array([[1.0, -2.0]])
HAND_W1 = np.array([[1.0, 2.0], [0.0, -1.0], [3.0, 1.0]])
HAND_B1 = np.array([0.5, -1.0, 2.0])
HAND_W2 = np.array([[1.0, 1.0, 1.0], [2.0, 0.0, -1.0]])
HAND_B2 = np.array([-1.0, 0.25])
HAND_OUT = np.array([[3.0, -2.75]])


def _hand_case_holds():
    sizes = [2, 3, 2]
    p = np.concatenate([HAND_W1.ravel(), HAND_B1, HAND_W2.ravel(), HAND_B2])
    layers = S.unpack(p, sizes)
    ok = (len(layers) == 2 and np.array_equal(layers[0][0], HAND_W1) and np.array_equal(layers[0][1], HAND_B1)
          and np.array_equal(layers[1][0], HAND_W2) and np.array_equal(layers[1][1], HAND_B2))
    return ok and np.array_equal(S.forward(p, sizes, HAND_X)[-1], HAND_OUT)


def test_unpack_layout_and_hand_computed_forward():
    assert _hand_case_holds()
    # the hidden activation as worked by hand
    sizes = [2, 3, 2]
    p = np.concatenate([HAND_W1.ravel(), HAND_B1, HAND_W2.ravel(), HAND_B2])
    assert np.array_equal(S.forward(p, sizes, HAND_X)[1], np.array([[0.0, 1.0, 3.0]]))


def test_pins_catch_planted_network_mistakes(monkeypatch):
    good_unpack, good_forward = S.unpack, S.forward

    def bias_first(params, sizes):  # b ahead of W in the flat vector
        out, k = [], 0
        for i, o in zip(sizes[:-1], sizes[1:]):
            b = params[k:k + o]
            k += o
            out.append((params[k:k + o * i].reshape(o, i), b))
            k += o * i
        return out

    def transposed(params, sizes):  # W read in x out
        return [(W.reshape(W.shape[1], W.shape[0]).T if W.shape[0] != W.shape[1] else W.T, b)
                for W, b in good_unpack(params, sizes)]

    def no_bias(params, sizes, X):
        acts = [np.asarray(X, dtype=np.float64)]
        layers = good_unpack(params, sizes)
        for li, (W, _) in enumerate(layers):
            z = acts[-1] @ W.T
            acts.append(np.maximum(z, 0.0) if li < len(layers) - 1 else z)
        return acts

    def relu_on_output(params, sizes, X):
        acts = good_forward(params, sizes, X)
        acts[-1] = np.maximum(acts[-1], 0.0)
        return acts

    for name, fn in (("unpack", bias_first), ("unpack", transposed), ("forward", no_bias),
                     ("forward", relu_on_output)):
        monkeypatch.setattr(S, name, fn)
        assert not _hand_case_holds(), fn.__name__
        monkeypatch.setattr(S, "unpack", good_unpack)
        monkeypatch.setattr(S, "forward", good_forward)
    assert _hand_case_holds()
