"""The synthetic-gradient network on the GPU (fe_onsg_*) against the oracle:
sample layout and forward pass exactly (a network built to copy chosen
inputs to its outputs), and an Adam update's loss trajectory and
predictions against the float64 oracle on the same float32-rounded samples,
initial parameters and mini-batches.

Tolerances: the GPU computes in float32, the oracle in float64; the first
batch loss (forward only) agrees to float32 rounding (1e-5 relative); later
steps differ by Adam's amplification of rounding in the updates (its
per-parameter normalisation turns a rounding of a small gradient into a
step of up to the learning rate).  Measured over these 60 steps: at most
2.4e-6 of the first loss and 1.7e-6 of the target scale for the
predictions; the bound is 1e-4 for both (a larger network, width 1000,
drifts by tens of percent over 60 steps at this learning rate, which is
why the cases stay small).
Inputs and targets of an iteration are scaled by that iteration's largest
|u_C| and |dJ/dz|; predictions come in units of the latter."""
import numpy as np
import pytest
import torch

from oracle import onsg_oracle as S
from paper_2104_12282_amd import fe, synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def T(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def N(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _copy_net(nb, pick):
    """Parameters of a network whose output k equals input pick[k] exactly:
    relu(x) - relu(-x) = x through identity hidden layers of width 2 in."""
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


@pytest.mark.parametrize("grid,nb", [((8, 4, 6), 2), ((9, 6, 3), 3), ((4, 4, 4), 1)])
def test_samples_layout_and_forward_exact(grid, nb):
    nx, ny, nz = grid
    cx, cy, cz = nx // nb, ny // nb, nz // nb
    rng = np.random.default_rng(1)
    z = rng.uniform(0, 1, nx * ny * nz)
    uc = rng.standard_normal(3 * (cx + 1) * (cy + 1) * (cz + 1))
    s_u = np.abs(uc).max()  # the library scales by the input's own maximum
    X, _ = S.block_samples(nx, ny, nz, nb, z, uc, s_u=s_u)
    Xf = X.astype(np.float32).astype(np.float64)
    nin = nb ** 3 + 24
    for pick in (list(range(nb ** 3)), [nb ** 3 + (k % 24) for k in range(nb ** 3)]):
        sizes, params = _copy_net(nb, pick)
        m = fe.SyntheticGradientModel(nx, ny, nz, nb, sizes[1], 4, 16, params, device=DEV)
        g = N(m.predict(T(z), T(uc)))
        ref = S.scatter_blocks(nx, ny, nz, nb, Xf[:, pick])
        assert np.array_equal(g, ref), (grid, nb, pick[:3])
        assert np.array_equal(N(m.params()), params.astype(np.float32).astype(np.float64))
        m.close()
    assert nin == sizes[0]


# the second case has a batch and an output width that are not multiples of
# the bias-gradient kernel's 16-wide slices or of its 4-row unrolling, and a
# loss sum over more than 4096 values (the unrolled part of the loss kernel)
@pytest.mark.parametrize("grid,nb,width,batch", [((8, 4, 4), 2, 16, 8), ((12, 9, 6), 3, 40, 200)])
def test_update_matches_oracle(grid, nb, width, batch):
    (nx, ny, nz), steps = grid, 60
    cx, cy, cz = nx // nb, ny // nb, nz // nb
    sizes = S.layer_sizes(nb, width)
    p0 = synth.mlp_init(sizes, seed=5)
    rng = np.random.default_rng(6)
    m = fe.SyntheticGradientModel(nx, ny, nz, nb, width, 64, batch, p0, device=DEV)
    DX, DY = [], []
    for it in range(2):  # two exact iterations of samples, each scaled by its own maxima
        z = rng.uniform(0, 1, nx * ny * nz)
        uc = rng.standard_normal(3 * (cx + 1) * (cy + 1) * (cz + 1)) * (1 + 4 * it)
        g = -np.abs(rng.standard_normal(nx * ny * nz)) * (1.0 + z) * (10.0 ** it)
        m.add_samples(T(z), T(uc), T(g))
        X, Y = S.block_samples(nx, ny, nz, nb, z, uc, g, s_u=np.abs(uc).max(), s_g=np.abs(g).max())
        DX.append(X)
        DY.append(Y)
    assert m.num_samples == 2 * cx * cy * cz
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    DX, DY = f32(np.concatenate(DX)), f32(np.concatenate(DY))
    idx = synth.minibatches(m.num_samples, steps, batch, seed=7)
    losses = N(m.train(idx, lr0=1e-2, halve_every=20))
    p_ref, losses_ref = S.adam_train(f32(p0), sizes, DX, DY, idx, 1e-2, 20)
    assert abs(losses[0] - losses_ref[0]) <= 1e-5 * losses_ref[0]
    assert np.all(np.abs(losses - losses_ref) <= 1e-4 * losses_ref[0])
    assert losses_ref[-10:].mean() < losses_ref[0]
    # predictions of the trained networks on the last iteration's design
    pred = N(m.predict(T(z), T(uc)))
    acts = S.forward(p_ref, sizes, S.block_samples(nx, ny, nz, nb, z, uc, s_u=np.abs(uc).max())[0])
    pred_ref = S.scatter_blocks(nx, ny, nz, nb, acts[-1])
    assert np.abs(pred - pred_ref).max() <= 1e-4 * np.abs(DY).max()
    m.close()


def test_bad_arguments():
    lib = fe.load_library()
    assert lib.fe_onsg_workspace_size(8, 4, 4, 3, 16, 10, 8) == 0      # nb does not divide
    assert lib.fe_onsg_workspace_size(8, 4, 4, 2, 0, 10, 8) == 0       # width
    assert lib.fe_onsg_num_params(2, 16) == S.n_params(S.layer_sizes(2, 16))
    sizes = S.layer_sizes(2, 8)
    m = fe.SyntheticGradientModel(8, 4, 4, 2, 8, 8, 4, synth.mlp_init(sizes, 0), device=DEV)
    z = T(np.full(128, 0.5))
    uc = T(np.zeros(3 * 5 * 3 * 3))
    with pytest.raises(fe.FEError):  # 16 samples per iteration exceed max_samples = 8
        m.add_samples(z, uc, z)
    with pytest.raises(fe.FEError):  # no samples yet
        m.train(np.zeros((1, 4), dtype=np.int32))
    with pytest.raises(ValueError):
        m.train(np.zeros((1, 3), dtype=np.int32))
    m.close()
