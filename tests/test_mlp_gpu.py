"""GPU checks of the learned-guess kernels against the FP64 reference with
the same BF16 rounding points (oracle/mlp.py), and of the guess inside the
integrator (the Newton residual decides: results equal the plain oracle's)."""
import numpy as np
import pytest

import synthetic as sy
from tests.test_parity_gpu import reservoir_slack

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
    scale = mlp.MLP(11, 10, 256, 3).gradient_scales(model.get_params().astype(np.float64),
                                                    norm.astype(np.float64), X, Y)
    # element by element, against each entry's own scale (its sum taken over
    # absolute terms): FP32 accumulation over B rows contributes ~B 2^-24 of
    # the scale, and a BF16 rounding of an activation or of dz that lands on
    # the other side of a rounding boundary (the FP32 intermediate differs
    # from the FP64 one in its last bits) one BF16 ulp, 2^-8, of one term
    tol = 2.0 ** -7
    for ws, bs, fo, fi in model.layer_slices():
        for sl in (ws, bs):
            a, b, sc = g[sl], ref[sl], scale[sl]
            err = np.abs(a - b) / np.maximum(sc, 1e-30)
            assert err.max() <= tol, (sl, err.max())
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
    n_o, T_o, st_o, stats_o = on.integrate(cs.n, cs.T, dt=np.full(300, 3e-7))
    np.testing.assert_array_equal(status.cpu().numpy(), st_o)
    ng = n.cpu().numpy()
    nnuc = cs.n.sum(axis=0)
    slack = reservoir_slack(desc, cs, stats_o)
    for s in range(desc.n_species):
        err = np.maximum(np.abs(ng[s] - n_o[s]) - slack[s], 0) / np.maximum(np.abs(n_o[s]), 1e-20 * nnuc)
        assert err.max() <= 1e-6, (s, err.max())
    np.testing.assert_allclose(T.cpu().numpy(), T_o, rtol=1e-6)


def test_feature_target_and_start_map(setup):
    """kr_guess_features / kr_guess_targets / kr_guess_predict against the
    oracle's map (oracle/mlp.py: features, targets, starting_point), element
    by element: features and targets are FP64 values rounded once to FP32 on
    the device, so they equal the oracle's rounded to FP32 (1 ulp where the
    two FP64 values straddle an FP32 rounding boundary); the starting point
    is FP64 from the network's FP32 outputs."""
    kr, desc, knet, model, norm = setup
    mlp = _oracle_mlp()
    cs = sy.cells_h_o_n(desc, 300, 1, salt=77)
    rng = np.random.default_rng(8)
    n = cs.n.copy()
    n[rng.integers(9, size=40), rng.integers(300, size=40)] = 0.0     # below the floor
    h = 10.0 ** rng.uniform(-10, -4, 300)
    atoms = np.abs(np.asarray(desc.composition)[:desc.n_elem]).sum(axis=0).astype(float)
    nd, Td, hd = (torch.tensor(a, device="cuda") for a in (n, cs.T, h))
    X = model.features(nd, Td, dt=hd).cpu().numpy()
    Xo = mlp.features(atoms, n, cs.T, h)
    ulp = np.spacing(np.abs(Xo).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(X - Xo.astype(np.float32)) <= ulp)
    assert np.mean(X == Xo.astype(np.float32)) > 0.999
    # targets between two states of the same cells
    n2 = n * np.exp(0.01 * rng.standard_normal(n.shape))
    T2 = cs.T * (1 + 0.01 * rng.standard_normal(300))
    Y = model.targets(nd, Td, torch.tensor(n2, device="cuda"), torch.tensor(T2, device="cuda")).cpu().numpy()
    Yo = mlp.targets(atoms, n, cs.T, n2, T2)
    ulp = np.spacing(np.abs(Yo).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(Y - Yo.astype(np.float32)) <= ulp)
    # the starting point from the network's own outputs on those features
    out = model.forward(torch.tensor(X, device="cuda")).cpu().numpy()
    guess = model.predict(nd, Td, dt=hd).cpu().numpy()
    yo = mlp.starting_point(atoms, n, cs.T, out, norm.astype(np.float64))
    np.testing.assert_allclose(guess, yo, rtol=1e-12, atol=0)


def test_fp32lu_with_non_conserving_guess(oracle_lib):
    """Form (1) started from a guess that does not conserve the element
    totals, in single-substep mode (the guessed substep is accepted): the
    projection must bring the iterate back to the substep start's totals.
    Statuses, abundances and element residuals match the plain start and
    the oracle, in both precisions."""
    kr = _kr()
    desc = sy.network_h_o_n(1)
    knet = kr.Network(desc)
    cs = sy.cells_h_o_n(desc, 256, 1, salt=55)
    rng = np.random.default_rng(21)
    h = 10.0 ** rng.uniform(-10, -6, 256)
    on = oracle_lib.OracleNet(desc)
    o = oracle_lib.default_opts()
    o.mode = oracle_lib.FIXED
    o.n_fixed = 1
    n_o, T_o, st_o, stats_o = on.integrate(cs.n, cs.T, dt=h, opts=o)
    assert np.all(st_o == 0)
    # most of the way to the root, each species by its own fraction: the
    # element totals are off by ~5 % of the substep's change
    f = 0.95 + 0.05 * rng.standard_normal((10, 256))
    y0 = np.vstack([cs.n, cs.T[None, :]])
    yr = np.vstack([n_o, T_o[None, :]])
    guess = y0 + (yr - y0) * f
    comp = np.asarray(desc.composition, float)
    drift = np.abs(comp @ (guess[:9] - cs.n)) / (np.abs(comp) @ cs.n)
    assert np.median(drift.max(axis=0)) > 1e-10      # the guess does not conserve
    nnuc = cs.n.sum(axis=0)
    for prec in (kr.KR_FP64, kr.KR_FP32LU_REFINE):
        n = torch.tensor(cs.n, device="cuda")
        T = torch.tensor(cs.T, device="cuda")
        g = torch.tensor(guess, device="cuda")
        counters = torch.zeros(8, dtype=torch.int64, device="cuda")
        status = torch.empty(256, dtype=torch.int32, device="cuda")
        kr.chem_integrate(knet, n, T, dt=torch.tensor(h, device="cuda"), rtol=1e-6,
                          opts=kr.guess_options(g, counters, mode=kr.KR_FIXED_STEP, n_fixed=1,
                                                precision=prec), status=status)
        resid = torch.zeros(256, dtype=torch.float64, device="cuda")
        kr.element_residual(knet, torch.tensor(cs.n, device="cuda"), n, resid=resid)
        torch.cuda.synchronize()
        c = counters.cpu().numpy()
        assert c[0] == 256
        assert c[1] < 0.5 * 256, c            # most guessed substeps are kept
        np.testing.assert_array_equal(status.cpu().numpy(), st_o)
        assert resid.cpu().numpy().max() < 1e-12
        ng = n.cpu().numpy()
        slack = reservoir_slack(desc, cs, stats_o)
        for s in range(9):
            err = np.maximum(np.abs(ng[s] - n_o[s]) - slack[s], 0) / np.maximum(np.abs(n_o[s]), 1e-20 * nnuc)
            assert err.max() <= 1e-6, (prec, s, err.max())
        np.testing.assert_allclose(T.cpu().numpy(), T_o, rtol=1e-6)
    knet.close()
