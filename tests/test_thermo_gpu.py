"""GPU parity of the temperature-dependent heat capacities and the tabulated
rate factors (kr_network_desc.cv_poly, tab_of / tab_log2k) against the FP64
oracle, through the C ABI, in both device layouts:

* the combustion network with NASA-style c_V(T) and four tabulated
  reactions (synthetic.network_h_o_n_tcv): adaptive FP64 within 1e-8, the
  FP32 LU form within 1e-6, fixed steps within 1e-8, per-cell substep and
  Newton counts equal for > 99 % of the cells;
* the adiabatic equilibrium of an exothermic isomer pair with c_V rising in
  T: the GPU's long-time state equals the independent root of energy
  conservation plus detailed balance (tests/test_thermo_oracle.py) to 1e-10,
  and the frozen-c_V control comes out hotter;
* tables sampled from power laws give the Arrhenius (A, b, 0) results;
* the single- and mixed-precision modes run the same network (every cell
  ok; the FP32 error model of tests/test_precision_gpu.py applies);
* several networks in one launch, one of them with c_V(T) and tables.
"""
import numpy as np
import pytest

import synthetic as sy
from tests.test_parity_gpu import assert_parity, run_gpu, run_oracle
from tests.test_thermo_oracle import _equilibrium, _exo_pair, _power_law_pair

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _kr():
    import paper_2504_04941_amd as kr
    return kr


def _layout(kr, wave):
    return kr.build_options(layout=kr.KR_LAYOUT_WAVE if wave else kr.KR_LAYOUT_LANE)


@pytest.mark.parametrize("wave", [False, True])
@pytest.mark.parametrize("ncell", [200, 77])
def test_tcv_tables_fp64(oracle_lib, wave, ncell):
    kr = _kr()
    net = sy.network_h_o_n_tcv()
    cs = sy.cells_h_o_n(net, ncell, 1)
    gpu = run_gpu(net, cs, dt_scalar=1e-4, build=_layout(kr, wave))
    orc = run_oracle(oracle_lib, net, cs, dt_scalar=1e-4)
    assert_parity(gpu, orc, cs, 1e-8, f"tcv fp64 wave={wave}", desc=net)
    assert np.mean(np.all(gpu[3] == orc[3], axis=1)) > 0.99


@pytest.mark.parametrize("wave", [False, True])
def test_tcv_tables_fp32lu(oracle_lib, wave):
    kr = _kr()
    net = sy.network_h_o_n_tcv()
    cs = sy.cells_h_o_n(net, 130, 1)
    gpu = run_gpu(net, cs, dt_scalar=1e-4, build=_layout(kr, wave), precision=kr.KR_FP32LU_REFINE)
    orc = run_oracle(oracle_lib, net, cs, dt_scalar=1e-4)
    assert_parity(gpu, orc, cs, 1e-6, f"tcv fp32lu wave={wave}", desc=net)


@pytest.mark.parametrize("wave", [False, True])
def test_tcv_tables_fixed_steps(oracle_lib, wave):
    kr = _kr()
    net = sy.network_h_o_n_tcv()
    cs = sy.cells_h_o_n(net, 100, 1)
    gpu = run_gpu(net, cs, dt_scalar=1e-8, build=_layout(kr, wave), mode=1, n_fixed=5)
    orc = run_oracle(oracle_lib, net, cs, dt_scalar=1e-8, mode="fixed", n_fixed=5)
    assert_parity(gpu, orc, cs, 1e-8, f"tcv fixed wave={wave}", desc=net)


@pytest.mark.parametrize("wave", [False, True])
def test_adiabatic_equilibrium_on_gpu(wave):
    kr = _kr()
    cvB = np.array([1.5, 1.0e-3, 0.0, 0.0, 0.0])
    T0, n0 = 400.0, 1.0e10
    out = {}
    for frozen in (None, T0):
        desc = _exo_pair(cvB, frozen_T=frozen)
        cs = sy.CellStates(np.array([[n0] * 64, [0.0] * 64]), np.full(64, T0), np.ones(64), None)
        n, T, st, _, _ = run_gpu(desc, cs, dt_scalar=1.0, build=_layout(kr, wave))
        np.testing.assert_array_equal(st, 0)
        T_ref, x_ref = _equilibrium(desc, T0, n0)
        assert np.max(np.abs(T - T_ref)) <= 1e-10 * T_ref, (frozen, T[:3], T_ref)
        assert np.max(np.abs(n[1] / n0 - x_ref)) <= 1e-10, (frozen, n[1, :3] / n0, x_ref)
        out[frozen] = T[0]
    assert out[T0] > 1.05 * out[None], out


@pytest.mark.parametrize("wave", [False, True])
def test_power_law_tables_equal_arrhenius(wave):
    kr = _kr()
    ref, tab, _, _ = _power_law_pair()
    cs = sy.cells_h_o_n(ref, 128, 1)
    a = run_gpu(ref, cs, dt_scalar=1e-5, build=_layout(kr, wave))
    b = run_gpu(tab, cs, dt_scalar=1e-5, build=_layout(kr, wave))
    np.testing.assert_array_equal(a[2], b[2])
    nnuc = cs.n.sum(axis=0)
    assert np.max(np.abs(a[0] - b[0]) / np.maximum(np.abs(a[0]), 1e-20 * nnuc)) <= 1e-8
    np.testing.assert_allclose(a[1], b[1], rtol=1e-10)


def test_fp32_modes_with_tcv_tables(oracle_lib):
    kr = _kr()
    net = sy.network_h_o_n_tcv()
    cs = sy.cells_h_o_n(net, 256, 1)
    orc = run_oracle(oracle_lib, net, cs, dt_scalar=1e-6)
    nnuc = cs.n.sum(axis=0)
    for prec in (kr.KR_SINGLE, kr.KR_MIXED):
        n, T, st, stats, resid = run_gpu(net, cs, dt_scalar=1e-6, precision=prec)
        np.testing.assert_array_equal(st, 0)
        assert resid.max() <= 1e-12
        # major species and T: FP32 accuracy (the rate exponents here are
        # below 400, the substeps below 2000: u (m + L) < 2e-4)
        major = np.abs(orc[0]) > 1e-4 * nnuc[None, :]
        assert np.max(np.abs(n - orc[0])[major] / np.abs(orc[0])[major]) <= 1e-3
        assert np.max(np.abs(T - orc[1]) / orc[1]) <= 1e-4


def test_multi_launch_with_tcv_network(oracle_lib):
    """A several-network launch holding the c_V(T)/table network (lane
    layout) beside the 5-species (lane) and 23-species (wave) networks."""
    kr = _kr()
    descs = [sy.network_h_he(0), sy.network_h_o_n_tcv(), sy.network_astro23(2)]
    cells = [sy.cells_h_he(descs[0], 64, 0), sy.cells_h_o_n(descs[1], 96, 1), sy.cells_astro23(descs[2], 64, 2)]
    dts = [1e-9, 1e-6, 1e-9]
    nets = [kr.Network(d) for d in descs]
    multi = kr.Multi(nets, kr.build_options())
    bufs = []
    for cs, dt in zip(cells, dts):
        m = cs.T.shape[0]
        bufs.append({"states": torch.tensor(cs.n, device="cuda"), "T": torch.tensor(cs.T, device="cuda"),
                     "dt": torch.full((m,), dt, dtype=torch.float64, device="cuda"),
                     "status": torch.empty(m, dtype=torch.int32, device="cuda"),
                     "cell_stats": torch.empty((m, 4), dtype=torch.int32, device="cuda")})
    multi.integrate(bufs, rtol=1e-6, opts=kr.default_options())
    torch.cuda.synchronize()
    for desc, cs, dt, b in zip(descs, cells, dts, bufs):
        orc = run_oracle(oracle_lib, desc, cs, dt_scalar=dt)
        resid = np.zeros(cs.T.shape[0])
        gpu = (b["states"].cpu().numpy(), b["T"].cpu().numpy(), b["status"].cpu().numpy(),
               b["cell_stats"].cpu().numpy(), resid)
        assert_parity(gpu, orc, cs, 1e-8, f"multi {desc.name}", desc=desc)
    multi.close()
    for n in nets:
        n.close()
