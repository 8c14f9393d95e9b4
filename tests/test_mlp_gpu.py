"""GPU checks of the learned-guess kernels against the FP64 reference with
the same BF16 rounding points (oracle/mlp.py), and of the guess inside the
integrator (the Newton residual decides: results equal the plain oracle's)."""
import numpy as np
import pytest

import synthetic as sy

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _kr():
    import paper_2504_04941_amd as kr
    return kr


@pytest.fixture(scope="module")
def setup():
    kr = _kr()
    desc = sy.network_h_o_n(1)
    knet = kr.Network(desc)
    model = kr.GuessModel(knet, hidden=256, layers=3, seed=11)
    rng = np.random.default_rng(5)
    norm = np.zeros(64, np.float32)
    norm[16:] = 1.0
    norm[:11] = rng.standard_normal(11)
    norm[16:27] = rng.uniform(0.5, 3.0, 11)
    norm[32:42] = rng.standard_normal(10) * 0.1
    norm[48:58] = rng.uniform(0.5, 2.0, 10)
    norm[27:32] = 1.0
    norm[58:64] = 1.0
    model.set_normalization(norm)
    yield kr, desc, knet, model, norm
    model.close()
    knet.close()


def _oracle_mlp():
    from oracle import mlp
    return mlp


def test_param_roundtrip_and_layout(setup):
    kr, desc, knet, model, norm = setup
    w = model.get_params()
    assert w.size == model.n_params == (11 * 256 + 256) + 2 * (256 * 256 + 256) + (256 * 10 + 10)
    bound = 1 / np.sqrt(np.array([11] * (11 * 256 + 256) + [256] * (w.size - 11 * 256 - 256)))
    assert np.all(np.abs(w) <= bound + 1e-7)
    model.set_params(w * 0.5)
    np.testing.assert_array_equal(model.get_params(), (w * 0.5).astype(np.float32))
    model.set_params(w)
    np.testing.assert_array_equal(model.get_normalization(), norm)


@pytest.mark.parametrize("B", [1, 200, 1000])
def test_forward_matches_reference(setup, B):
    kr, desc, knet, model, norm = setup
    mlp = _oracle_mlp()
    rng = np.random.default_rng(B)
    X = rng.standard_normal((B, 11)).astype(np.float32) * 3
    out = model.forward(torch.tensor(X, device="cuda")).cpu().numpy()
    ref, _ = mlp.MLP(11, 10, 256, 3).forward(model.get_params().astype(np.float64), norm.astype(np.float64), X)
    err = np.abs(out - ref)
    scale = np.abs(ref).max()
    # FP32 accumulation order differs; a BF16 rounding of an activation can
    # land on the other side (one BF16 ulp, 2^-8 relative) now and then
    assert err.max() <= 1e-2 * scale
    assert np.percentile(err, 99) <= 1e-4 * scale


@pytest.mark.parametrize("B", [64, 257])
def test_gradients_match_reference(setup, B):
    kr, desc, knet, model, norm = setup
    mlp = _oracle_mlp()
    rng = np.random.default_rng(100 + B)
    X = (rng.standard_normal((B, 11)) * 3).astype(np.float32)
    Y = (rng.standard_normal((B, 10)) * 0.3).astype(np.float32)
    g, loss = model.gradients(torch.tensor(X, device="cuda"), torch.tensor(Y, device="cuda"))
    g = g.cpu().numpy().astype(np.float64)
    ref_loss, ref = mlp.MLP(11, 10, 256, 3).gradients(model.get_params().astype(np.float64),
                                                      norm.astype(np.float64), X, Y)
    assert loss == pytest.approx(ref_loss, rel=1e-4)
    for ws, bs, fo, fi in model.layer_slices():
        for sl in (ws, bs):
            a, b = g[sl], ref[sl]
            rel = np.linalg.norm(a - b) / np.linalg.norm(b)
            assert rel < 1e-3, (sl, rel)


def test_adam_step_matches_reference(setup):
    kr, desc, knet, model, norm = setup
    mlp = _oracle_mlp()
    w0 = model.get_params()
    rng = np.random.default_rng(9)
    B = 128
    X = (rng.standard_normal((B, 11)) * 3).astype(np.float32)
    Y = (rng.standard_normal((B, 10)) * 0.3).astype(np.float32)
    # seed 0 = the batch is the B rows in order; one step of lr 1e-3
    m2 = kr.GuessModel(knet, hidden=256, layers=3, seed=11)
    m2.set_normalization(norm)
    m2.set_params(w0)
    m2.train(torch.tensor(X, device="cuda"), torch.tensor(Y, device="cuda"), steps=1, batch=B,
             lr=1e-3, lr_min=1e-3, seed=0)
    w1 = m2.get_params().astype(np.float64)
    m2.close()
    _, g = mlp.MLP(11, 10, 256, 3).gradients(w0.astype(np.float64), norm.astype(np.float64), X, Y)
    ref, _, _ = mlp.adam_step(w0.astype(np.float64), g, 0 * g, 0 * g, 1, 1e-3)
    # the first Adam step moves each weight by ~lr sign(g): compare where the
    # gradient is not tiny (elsewhere its sign is rounding noise)
    big = np.abs(g) > 1e-3 * np.abs(g).max()
    assert np.max(np.abs(w1 - ref)[big]) < 5e-5
    assert np.max(np.abs(w1 - w0)) <= 1.0001e-3 + 1e-7


def test_training_reduces_loss_on_substep_pairs(setup):
    kr, desc, knet, model, norm = setup
    from paper_2504_04941_amd import learned
    m = kr.GuessModel(knet, hidden=256, layers=3, seed=3)
    X, Y, keep = learned.single_step_pairs(knet, m, desc, 1 << 14, salt=7)
    assert X.shape[0] > 0.9 * (1 << 14)
    m.fit_normalization(X, Y)
    _, loss0 = m.gradients(X[:4096].contiguous(), Y[:4096].contiguous())
    hist = learned.train(m, X, Y, steps=400, batch=1024, lr=2e-3, lr_min=1e-4)
    _, loss1 = m.gradients(X[:4096].contiguous(), Y[:4096].contiguous())
    assert loss1 < 0.3 * loss0, (loss0, loss1, hist)
    m.close()


def test_guess_keeps_the_plain_result(setup, oracle_lib):
    """A guess (here from an untrained network) changes only the Newton
    starting point: statuses and results match the plain oracle, and a
    failing guess falls back to the plain start."""
    kr, desc, knet, model, norm = setup
    cs = sy.cells_h_o_n(desc, 300, 1, salt=31)
    n = torch.tensor(cs.n, device="cuda")
    T = torch.tensor(cs.T, device="cuda")
    dt = torch.full((300,), 3e-7, dtype=torch.float64, device="cuda")
    guess = model.predict(n, T, dt=dt)
    counters = torch.zeros(8, dtype=torch.int64, device="cuda")
    status = torch.empty(300, dtype=torch.int32, device="cuda")
    kr.chem_integrate(knet, n, T, dt=dt, rtol=1e-6, opts=kr.guess_options(guess, counters),
                      status=status)
    torch.cuda.synchronize()
    c = counters.cpu().numpy()
    assert c[0] == 300 and 0 <= c[1] <= 300
    on = oracle_lib.OracleNet(desc)
    n_o, T_o, st_o, _ = on.integrate(cs.n, cs.T, dt=np.full(300, 3e-7))
    np.testing.assert_array_equal(status.cpu().numpy(), st_o)
    ng = n.cpu().numpy()
    nnuc = cs.n.sum(axis=0)
    res = set(int(r) for r in desc.reservoir)
    for s in range(desc.n_species):
        slack = 1e-11 * nnuc if s in res else 0.0
        err = np.maximum(np.abs(ng[s] - n_o[s]) - slack, 0) / np.maximum(np.abs(n_o[s]), 1e-20 * nnuc)
        assert err.max() <= 1e-6, (s, err.max())
    np.testing.assert_allclose(T.cpu().numpy(), T_o, rtol=1e-6)
