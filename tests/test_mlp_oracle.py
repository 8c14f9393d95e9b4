"""Pins of the FP64 MLP reference (CPU): its BF16 rounding against torch's
independent conversion, GELU against torch's tanh-approximate GELU, the
analytic gradient against finite differences (rounding off), and the Adam
step against torch.optim.Adam."""
import math

import numpy as np
import pytest
import torch

from oracle import mlp


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    vals = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.uniform(-30, 30, 5000),
                           np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38, 1e-40, -2.5])])
    ref = torch.tensor(vals.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16_round(vals), ref)
    # ties go to even: 1 + 2^-8 sits halfway between 1 and 1 + 2^-7
    assert mlp.bf16_round(1.0 + 2.0 ** -8) == 1.0
    assert mlp.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6


def test_gelu_matches_torch_tanh_form():
    z = np.linspace(-8, 8, 2001)
    ref = torch.nn.functional.gelu(torch.tensor(z), approximate="tanh").numpy()
    np.testing.assert_allclose(mlp.gelu(z), ref, rtol=1e-14, atol=1e-15)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(z), fd, rtol=1e-7, atol=1e-9)


def _setup(n_in=5, n_out=4, hidden=8, layers=2, B=7, seed=3):
    rng = np.random.default_rng(seed)
    shapes = mlp.layer_shapes(n_in, n_out, hidden, layers)
    w = np.concatenate([np.concatenate([rng.standard_normal(fo * fi) / np.sqrt(fi), 0.1 * rng.standard_normal(fo)])
                        for fo, fi in shapes])
    norm = np.zeros(64)
    norm[:n_in] = rng.standard_normal(n_in)
    norm[16:16 + n_in] = rng.uniform(0.5, 2, n_in)
    norm[32:32 + n_out] = rng.standard_normal(n_out)
    norm[48:48 + n_out] = rng.uniform(0.5, 2, n_out)
    X = rng.standard_normal((B, n_in))
    Y = rng.standard_normal((B, n_out))
    return w, norm, X, Y


def test_gradient_matches_finite_differences():
    w, norm, X, Y = _setup()
    net = mlp.MLP(5, 4, 8, 2, rounding=False)
    loss, g = net.gradients(w, norm, X, Y)
    fd = np.zeros_like(w)
    h = 1e-6
    for i in range(w.size):
        e = np.zeros_like(w)
        e[i] = h
        fd[i] = (net.loss(w + e, norm, X, Y) - net.loss(w - e, norm, X, Y)) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9)
    assert loss == pytest.approx(net.loss(w, norm, X, Y))


def test_gradient_matches_torch_autograd():
    """The same function in torch (float64, no rounding) differentiated by
    autograd."""
    n_in, n_out, hidden, layers = 5, 4, 8, 2
    w, norm, X, Y = _setup()
    net = mlp.MLP(n_in, n_out, hidden, layers, rounding=False)
    _, g = net.gradients(w, norm, X, Y)
    wt = torch.tensor(w, requires_grad=True)
    parts, off = [], 0
    for fo, fi in mlp.layer_shapes(n_in, n_out, hidden, layers):
        parts.append((wt[off:off + fo * fi].reshape(fo, fi), wt[off + fo * fi:off + fo * fi + fo]))
        off += fo * fi + fo
    a = (torch.tensor(X) - torch.tensor(norm[:n_in])) / torch.tensor(norm[16:16 + n_in])
    for W, b in parts[:-1]:
        a = torch.nn.functional.gelu(a @ W.T + b, approximate="tanh")
    out = a @ parts[-1][0].T + parts[-1][1]
    t = (torch.tensor(Y) - torch.tensor(norm[32:32 + n_out])) / torch.tensor(norm[48:48 + n_out])
    torch.mean((out - t) ** 2).backward()
    np.testing.assert_allclose(g, wt.grad.numpy(), rtol=1e-12, atol=1e-14)


def test_adam_matches_torch():
    rng = np.random.default_rng(1)
    w = rng.standard_normal(20)
    wt = torch.tensor(w.copy(), requires_grad=True)
    opt = torch.optim.Adam([wt], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    for step in range(1, 4):
        g = rng.standard_normal(20)
        w, m, v = mlp.adam_step(w, g, m, v, step, 1e-3)
        wt.grad = torch.tensor(g)
        opt.step()
        np.testing.assert_allclose(w, wt.detach().numpy(), rtol=1e-13, atol=1e-15)


# --------------------------------------------------------------------------
# the cell <-> network map
# --------------------------------------------------------------------------

def test_features_hand_worked():
    """atoms (1, 2): n = (1e3, 499500) has n_nuc = 1e3 + 2 * 499500 = 1e6,
    so the fractions are 1e-3 (log -3) and 0.4995; a missing species sits on
    the 1e-20 floor (log -20); T = 1e3 K gives 3, h = 1e-4 s gives -4."""
    atoms = np.array([1.0, 2.0])
    n = np.array([[1e3, 0.0], [499500.0, 5e5]])
    X = mlp.features(atoms, n, np.array([1e3, 10.0]), np.array([1e-4, 1.0]))
    assert X.shape == (2, 4)
    assert X[0, 0] == -3.0 and X[0, 1] == pytest.approx(math.log10(0.4995), abs=1e-15)
    assert X[0, 2] == 3.0 and X[0, 3] == -4.0
    # second cell: all nuclei in the diatomic species (fraction 1/2), the
    # atom is absent
    assert X[1, 0] == -20.0 and X[1, 1] == pytest.approx(math.log10(0.5), abs=1e-15)
    assert X[1, 2] == 1.0 and X[1, 3] == 0.0
    # a scalar step applies to every cell
    np.testing.assert_array_equal(mlp.features(atoms, n, np.array([1e3, 10.0]), 1e-4)[:, 3], -4.0)


def test_targets_hand_worked():
    """Same nuclei (1e6) before and after: the atom falls from 1e3 to 1e2
    (change -1), T doubles (change log10 2)."""
    atoms = np.array([1.0, 2.0])
    nb = np.array([[1e3], [499500.0]])
    na = np.array([[1e2], [499950.0]])
    Y = mlp.targets(atoms, nb, np.array([1e3]), na, np.array([2e3]))
    assert Y[0, 0] == pytest.approx(-1.0, abs=1e-15)
    assert Y[0, 1] == pytest.approx(math.log10(0.49995) - math.log10(0.4995), abs=1e-15)
    assert Y[0, 2] == pytest.approx(math.log10(2.0), abs=1e-15)


def test_starting_point_identity_and_round_trip():
    """A zero predicted change returns the state (species on the floor come
    back at 1e-20 n_nuc); the change between two states, fed back through
    the output normalisation, lands on the second state."""
    atoms = np.array([1.0, 2.0])
    nb = np.array([[1e3, 0.0], [499500.0, 5e5]])
    Tb = np.array([1e3, 10.0])
    norm = np.zeros(64)
    norm[48:] = 1.0
    y = mlp.starting_point(atoms, nb, Tb, np.zeros((2, 3)), norm)
    np.testing.assert_allclose(y[:, 0], [1e3, 499500.0, 1e3], rtol=1e-14)
    np.testing.assert_allclose(y[:, 1], [1e-20 * 1e6, 5e5, 10.0], rtol=1e-14)
    na = np.array([[1e2, 3e2], [499950.0, 499850.0]])
    Ta = np.array([2e3, 12.5])
    Y = mlp.targets(atoms, nb, Tb, na, Ta)
    # through a non-trivial output normalisation: out = (Y - mu) / sd
    norm[32:35] = [0.3, -0.2, 0.1]
    norm[48:51] = [2.0, 0.5, 4.0]
    out = (Y - norm[32:35]) / norm[48:51]
    y = mlp.starting_point(atoms, nb, Tb, out, norm)
    # the atom of cell 1 starts on the floor, so its change is measured from
    # 1e-20 n_nuc: the round trip is exact for it as well
    np.testing.assert_allclose(y[:2], na, rtol=1e-12)
    np.testing.assert_allclose(y[2], Ta, rtol=1e-13)
