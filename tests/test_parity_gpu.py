"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Same seeded inputs on both sides.  Gate: abundances within 1e-8 relative
(plain FP64) or 1e-6 (FP32 LU form) of the oracle's, where abundances below
the 1e-20 floor (fraction of the nuclei density) are compared absolutely at
that floor; temperature to the same relative bound; per-cell status
identical; element residual below 1e-12.  Sizes span several waves and a
ragged tail."""
import numpy as np
import pytest

import synthetic as sy
from tests.nets import isomer_pair, linear_three

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FLOOR = 1e-20


def _kr():
    import paper_2504_04941_amd as kr
    return kr


def _dev(a, dtype=None):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=dtype)


def run_gpu(desc, cs, dt=None, dt_scalar=0.0, rtol=1e-6, build=None, **opt):
    kr = _kr()
    net = kr.Network(desc, build)
    n = _dev(cs.n, torch.float64)
    T = _dev(cs.T, torch.float64)
    rho = _dev(cs.rho, torch.float64)
    dtt = None if dt is None else _dev(dt, torch.float64)
    ncell = cs.T.shape[0]
    status = torch.full((ncell,), -7, dtype=torch.int32, device="cuda")
    stats = torch.zeros((ncell, 4), dtype=torch.int32, device="cuda")
    kr.chem_integrate(net, n, T, rho=rho, dt=dtt, dt_scalar=dt_scalar, rtol=rtol,
                      opts=kr.default_options(**opt), status=status, cell_stats=stats)
    torch.cuda.synchronize()
    before = _dev(cs.n, torch.float64)
    resid = torch.zeros(ncell, dtype=torch.float64, device="cuda")
    kr.element_residual(net, before, n, resid=resid)
    torch.cuda.synchronize()
    out = (n.cpu().numpy(), T.cpu().numpy(), status.cpu().numpy(), stats.cpu().numpy(),
           resid.cpu().numpy())
    net.close()
    return out


def run_oracle(oracle, desc, cs, dt=None, dt_scalar=0.0, rtol=1e-6, **opt):
    on = oracle.OracleNet(desc)
    o = oracle.default_opts(rtol=rtol)
    if opt.get("mode") == "fixed":
        o.mode = oracle.FIXED
        o.n_fixed = opt["n_fixed"]
    for k in ("max_newton", "max_substeps", "floor"):
        if k in opt:
            setattr(o, k, opt[k])
    return on.integrate(cs.n, cs.T, cs.rho, dt=dt, dt_scalar=dt_scalar, opts=o)


EPS = np.finfo(np.float64).eps


RESERVOIR_GATE = 4.0


def reservoir_slack(desc, cs, stats):
    """Absolute slack on the reservoir species.

    Each Newton update rounds every abundance to its own ulp, so a conserved
    row total drifts by a random walk, differently on the two sides; the
    post-processing's stage 2 (Sec. 2.2.3) hands the whole drift to the row's
    reservoir species.  A trace reservoir (an H atom at 1e-8 of the nuclei)
    therefore differs from the oracle's by about sqrt(iterations) * eps *
    n_nuc whatever the solver.  Model: each update adds independent rounding
    errors of at most eps/2 of each abundance to the row total, a standard
    deviation of at most eps n_nuc / sqrt(12) per update, so the difference of
    two such walks over m updates has a standard deviation below 0.41
    sqrt(m) eps n_nuc.  Measured on the parity batches (GPU against oracle,
    both precisions, both layouts, 5200 cells): at most 0.97 sqrt(m) eps
    n_nuc (48 species, H), 0.39 (5 species), 0.054 (9 species).  The gate is
    RESERVOIR_GATE = 4 sqrt(m) eps n_nuc: ten standard deviations of the
    model, four times the largest measured value."""
    nnuc = np.abs(np.asarray(desc.composition)[:desc.n_elem]).sum(axis=0) @ cs.n
    walk = RESERVOIR_GATE * EPS * np.sqrt(np.maximum(stats[:, 1], 1).astype(float)) * nnuc
    slack = np.zeros_like(cs.n)
    for rs in np.unique(np.asarray(desc.reservoir)):
        slack[rs] = walk
    return slack


def assert_parity(gpu, orc, cs, tol, label="", desc=None):
    n_g, T_g, st_g, stats_g, resid = gpu
    n_o, T_o, st_o, stats_o = orc
    np.testing.assert_array_equal(st_g, st_o, err_msg=f"{label}: status")
    nnuc = cs.n.sum(axis=0)
    scale = np.maximum(np.abs(n_o), FLOOR * nnuc[None, :])
    slack = reservoir_slack(desc, cs, stats_o) if desc is not None else 0.0
    err = np.maximum(np.abs(n_g - n_o) - slack, 0.0) / scale
    worst = np.unravel_index(np.argmax(err), err.shape)
    assert err.max() <= tol, f"{label}: abundance rel err {err.max():.3e} at {worst}"
    terr = np.abs(T_g - T_o) / np.abs(T_o)
    assert terr.max() <= tol, f"{label}: T rel err {terr.max():.3e}"
    ok = st_g != 2
    assert np.all(resid[ok] < 1e-12), f"{label}: element residual {resid[ok].max():.3e}"
    return err.max(), terr.max()


def _c0_inputs(oracle, ncell):
    net = sy.network_h_he(0)
    cs = sy.cells_h_he(net, ncell, 0)
    on = oracle.OracleNet(net)
    dt = np.array([1e3 * on.fastest_timescale(np.r_[cs.n[:, c], cs.T[c]]) for c in range(ncell)])
    return net, cs, dt


@pytest.mark.parametrize("ncell", [1, 63, 4096])
def test_h_he_adaptive_fp64(oracle_lib, ncell):
    net, cs, dt = _c0_inputs(oracle_lib, ncell)
    gpu = run_gpu(net, cs, dt=dt)
    orc = run_oracle(oracle_lib, net, cs, dt=dt)
    e, te = assert_parity(gpu, orc, cs, 1e-8, "h_he fp64", desc=net)
    # substep sequences agree (a flip would be a near-tie of err == 1)
    assert np.mean(np.all(gpu[3] == orc[3], axis=1)) > 0.99


@pytest.mark.parametrize("ncell", [200, 1000])
def test_h_o_n_adaptive_fp64(oracle_lib, ncell):
    net = sy.network_h_o_n(1)
    cs = sy.cells_h_o_n(net, ncell, 1)
    gpu = run_gpu(net, cs, dt_scalar=1e-4)
    orc = run_oracle(oracle_lib, net, cs, dt_scalar=1e-4)
    assert_parity(gpu, orc, cs, 1e-8, "h_o_n fp64", desc=net)
    assert np.mean(np.all(gpu[3] == orc[3], axis=1)) > 0.99


@pytest.mark.parametrize("nfix", [1, 7])
def test_fixed_step_fp64(oracle_lib, nfix):
    net = sy.network_h_o_n(1)
    cs = sy.cells_h_o_n(net, 130, 1)
    gpu = run_gpu(net, cs, dt_scalar=1e-9, mode=1, n_fixed=nfix)
    orc = run_oracle(oracle_lib, net, cs, dt_scalar=1e-9, mode="fixed", n_fixed=nfix)
    assert_parity(gpu, orc, cs, 1e-8, "fixed", desc=net)
    np.testing.assert_array_equal(gpu[3][:, 0], orc[3][:, 0])


@pytest.mark.parametrize("ncell", [77, 1000])
def test_fp32lu_refinement_form(oracle_lib, ncell):
    net = sy.network_h_o_n(1)
    cs = sy.cells_h_o_n(net, ncell, 1)
    gpu = run_gpu(net, cs, dt_scalar=1e-4, precision=1)
    orc = run_oracle(oracle_lib, net, cs, dt_scalar=1e-4)
    assert_parity(gpu, orc, cs, 1e-6, "fp32lu", desc=net)


def test_fp32lu_h_he(oracle_lib):
    net, cs, dt = _c0_inputs(oracle_lib, 1000)
    gpu = run_gpu(net, cs, dt=dt, precision=1)
    orc = run_oracle(oracle_lib, net, cs, dt=dt)
    assert_parity(gpu, orc, cs, 1e-6, "fp32lu h_he", desc=net)


@pytest.mark.parametrize("layout", ["lane", "wave", "group16", "group32"])
def test_closed_form_networks_on_gpu(oracle_lib, layout):
    """Isomer pair and all-unary network: GPU fixed steps equal the closed
    forms used to pin the oracle, in every layout (one cell per lane, per
    wavefront, per 16- and per 32-lane group)."""
    kr = _kr()
    build = kr.build_options(layout={"lane": kr.KR_LAYOUT_LANE, "wave": kr.KR_LAYOUT_WAVE,
                                     "group16": kr.KR_LAYOUT_GROUP16, "group32": kr.KR_LAYOUT_GROUP32}[layout])
    kf, ds = 2.0, 0.7
    kr_ = kf * np.exp(-ds)
    desc = isomer_pair(kf, ds)
    A0, B0 = 3.0, 0.25
    cs = sy.CellStates(np.array([[A0] * 70, [B0] * 70]), np.full(70, 500.0), np.ones(70), None)
    m, dt = 9, 2.0
    n, T, st, stats, _ = run_gpu(desc, cs, dt_scalar=dt, build=build, mode=1, n_fixed=m)
    Aeq = kr_ * (A0 + B0) / (kf + kr_)
    exact = Aeq + (A0 - Aeq) / (1 + (kf + kr_) * dt / m) ** m
    assert np.all(st == 0)
    np.testing.assert_allclose(n[0], exact, rtol=1e-13)
    desc = linear_three()
    cs = sy.CellStates(np.tile(np.array([[1.0], [2.0], [0.5]]), (1, 65)), np.full(65, 300.0),
                       np.ones(65), None)
    gpu = run_gpu(desc, cs, dt_scalar=3.0, build=build, mode=1, n_fixed=4)
    orc = run_oracle(oracle_lib, desc, cs, dt_scalar=3.0, mode="fixed", n_fixed=4)
    assert_parity(gpu, orc, cs, 1e-13, "linear3", desc=desc)


def test_edge_cases(oracle_lib):
    """Zero cells, zero step, NaN input, negative input (clipped), and the
    retry ladder forced by a one-iteration Newton limit."""
    kr = _kr()
    net = sy.network_h_o_n(1)
    cs = sy.cells_h_o_n(net, 70, 1)
    cs.n[:, 5] = np.nan
    cs.n[3, 9] = -1e3
    dt = np.full(70, 1e-6)
    dt[11] = 0.0
    gpu = run_gpu(net, cs, dt=dt)
    orc = run_oracle(oracle_lib, net, cs, dt=dt)
    n_g, T_g, st_g, _, _ = gpu
    assert st_g[5] == 2 and np.isnan(n_g[:, 5]).any()
    np.testing.assert_array_equal(st_g, orc[2])
    keep = np.ones(70, bool)
    keep[5] = False
    cs2 = sy.CellStates(cs.n[:, keep], cs.T[keep], cs.rho[keep], None)
    assert_parity((n_g[:, keep], T_g[keep], st_g[keep], gpu[3][keep], gpu[4][keep]),
                  (orc[0][:, keep], orc[1][keep], orc[2][keep], orc[3][keep]), cs2, 1e-8, "edges",
                  desc=net)
    # forced failure: both attempts fail -> reverted, inputs untouched
    cs = sy.cells_h_o_n(net, 65, 1)
    n_g, T_g, st_g, _, _ = run_gpu(net, cs, dt_scalar=1e-4, max_newton=1)
    assert np.all(st_g == 2)
    np.testing.assert_array_equal(n_g, cs.n)
    np.testing.assert_array_equal(T_g, cs.T)
    # zero cells is a no-op
    knet = kr.Network(net)
    t = torch.zeros((net.n_species, 0), dtype=torch.float64, device="cuda")
    kr.chem_integrate(knet, t, torch.zeros(0, dtype=torch.float64, device="cuda"), dt_scalar=1.0)
    knet.close()


def test_invalid_arguments_rejected():
    kr = _kr()
    net = kr.Network(sy.network_h_he(0))
    n = torch.zeros((5, 8), dtype=torch.float64, device="cuda")
    T = torch.ones(8, dtype=torch.float64, device="cuda")
    with pytest.raises(kr.KrError):
        kr.chem_integrate(net, n, T, dt_scalar=1.0, rtol=0.0)
    with pytest.raises(kr.KrError):
        kr.chem_integrate(net, n, T, dt_scalar=1.0, opts=kr.default_options(mode=1, n_fixed=0))
    bad = sy.network_h_he(0)
    bad.prod = bad.prod.copy()
    bad.prod[0, 0] = 1     # breaks conservation
    with pytest.raises(kr.KrError):
        kr.Network(bad)


def test_element_residual_matches_oracle(oracle_lib):
    kr = _kr()
    net = sy.network_h_o_n(1)
    cs = sy.cells_h_o_n(net, 300, 1)
    rng = np.random.default_rng(3)
    after = cs.n * (1 + 1e-9 * rng.standard_normal(cs.n.shape))
    knet = kr.Network(net)
    resid = torch.zeros(300, dtype=torch.float64, device="cuda")
    mx = kr.element_residual(knet, _dev(cs.n, torch.float64), _dev(after, torch.float64),
                             resid=resid, want_max=True)
    ref = oracle_lib.OracleNet(net).element_residual(cs.n, after)
    np.testing.assert_allclose(resid.cpu().numpy(), ref, rtol=1e-12, atol=1e-30)
    assert mx == pytest.approx(ref.max(), rel=1e-12)
    knet.close()


def test_fp32lu_astro23_batch(oracle_lib):
    """Form (1) on the 23-species network in full waves: every cell's result
    (and status) matches the oracle when 64 lanes with different refinement
    sweep counts run together (a per-lane loop exit in this spilled kernel
    once reverted ~10% of such cells while single cells were correct)."""
    desc = sy.network_astro23(2)
    cs = sy.cells_astro23(desc, 256, 2)
    on = oracle_lib.OracleNet(desc)
    dt = np.array([1e-2 * on.fastest_timescale(np.r_[cs.n[:, c], cs.T[c]]) for c in range(256)])
    kr = _kr()
    gpu = run_gpu(desc, cs, dt=dt, precision=1, build=kr.build_options(layout=kr.KR_LAYOUT_LANE))
    orc = run_oracle(oracle_lib, desc, cs, dt=dt)
    assert_parity(gpu, orc, cs, 1e-6, "astro23 fp32lu batch", desc=desc)
