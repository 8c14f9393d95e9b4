"""GPU parity of the one-wavefront-per-cell layout (large networks) against
the FP64 oracle, through the C ABI: the 48-species network at its own
shapes, and the smaller networks with the layout forced, so that the two
layouts are also checked against each other's oracle on the same inputs."""
import numpy as np
import pytest

import synthetic as sy
from tests.test_parity_gpu import assert_parity, run_gpu, run_oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _kr():
    import paper_2504_04941_amd as kr
    return kr


def _wave(kr):
    return kr.build_options(layout=kr.KR_LAYOUT_WAVE)


def _large_inputs(ncell, cap):
    desc = sy.network_large48(3)
    cs = sy.cells_large48(desc, ncell, 3)
    return desc, cs, np.minimum(cs.dt, cap)


@pytest.mark.parametrize("prec,tol", [(0, 1e-8), (1, 1e-6)])
@pytest.mark.parametrize("ncell", [1, 96])
def test_large48_matches_oracle(oracle_lib, prec, tol, ncell):
    """48 species / 200 reversible reactions / 5 element rows; per-cell
    steps log-uniform in [1e-8, 1e-5] s (substeps from 1 to ~1e4)."""
    kr = _kr()
    desc, cs, dt = _large_inputs(ncell, 1e-5)
    print(f"large48 prec={prec} ncell={ncell}", flush=True)
    gpu = run_gpu(desc, cs, dt=dt, precision=prec)
    orc = run_oracle(oracle_lib, desc, cs, dt=dt)
    assert_parity(gpu, orc, cs, tol, f"large48 prec {prec}", desc=desc)
    if prec == 0:
        assert np.mean(np.all(gpu[3] == orc[3], axis=1)) > 0.95


@pytest.mark.parametrize("which", ["h_he", "h_o_n", "astro23"])
@pytest.mark.parametrize("prec,tol", [(0, 1e-8), (1, 1e-6)])
def test_small_networks_in_wave_layout(oracle_lib, which, prec, tol):
    kr = _kr()
    if which == "h_he":
        desc = sy.network_h_he(0)
        cs = sy.cells_h_he(desc, 130, 0)
    elif which == "h_o_n":
        desc = sy.network_h_o_n(1)
        cs = sy.cells_h_o_n(desc, 70, 1)
    else:
        desc = sy.network_astro23(2)
        cs = sy.cells_astro23(desc, 100, 2)
    on = oracle_lib.OracleNet(desc)
    tau = np.array([on.fastest_timescale(np.r_[cs.n[:, c], cs.T[c]]) for c in range(cs.n_cells)])
    dt = np.minimum(20.0 * tau, 1e-5)
    print(f"{which} prec={prec} wave layout", flush=True)
    gpu = run_gpu(desc, cs, dt=dt, build=_wave(kr), precision=prec)
    orc = run_oracle(oracle_lib, desc, cs, dt=dt)
    assert_parity(gpu, orc, cs, tol, f"{which} wave prec {prec}", desc=desc)


def test_wave_layout_fixed_steps(oracle_lib):
    kr = _kr()
    desc, cs, dt = _large_inputs(40, 1e-7)
    gpu = run_gpu(desc, cs, dt=dt, mode=kr.KR_FIXED_STEP, n_fixed=3)
    orc = run_oracle(oracle_lib, desc, cs, dt=dt, mode="fixed", n_fixed=3)
    assert_parity(gpu, orc, cs, 1e-8, "large48 fixed", desc=desc)
    assert np.all(gpu[3][:, 0][gpu[2] != 2] == 3)


def test_wave_layout_edge_cells(oracle_lib):
    """zero step (pre-processing only), a non-finite input (reverted,
    untouched), negative input abundances (clipped)."""
    kr = _kr()
    desc, cs, dt = _large_inputs(5, 1e-6)
    cs.n[:, 1] *= -1.0
    cs.n[3, 2] = np.nan
    dt[0] = 0.0
    gpu = run_gpu(desc, cs, dt=dt)
    orc = run_oracle(oracle_lib, desc, cs, dt=dt)
    np.testing.assert_array_equal(gpu[2], orc[2])
    assert gpu[2][2] == 2 and np.isnan(gpu[0][3, 2])
    ok = gpu[2] != 2
    np.testing.assert_allclose(gpu[0][:, ok], orc[0][:, ok], rtol=1e-8, atol=1e-20 * cs.n.sum())
    np.testing.assert_allclose(gpu[1][ok], orc[1][ok], rtol=1e-8)


def test_wave_layout_timescale(oracle_lib):
    kr = _kr()
    desc, cs, _ = _large_inputs(200, 1e-6)
    net = kr.Network(desc)
    tau = kr.fastest_timescale(net, torch.as_tensor(cs.n, device="cuda"),
                               torch.as_tensor(cs.T, device="cuda")).cpu().numpy()
    on = oracle_lib.OracleNet(desc)
    ref = np.array([on.fastest_timescale(np.r_[cs.n[:, c], cs.T[c]]) for c in range(200)])
    np.testing.assert_allclose(tau, ref, rtol=1e-11)
    net.close()


def _counted(kr, desc, cs, dt, build):
    """FP32 LU form on the GPU with its statistics counters."""
    net = kr.Network(desc, build)
    n = torch.as_tensor(cs.n, device="cuda").clone()
    T = torch.as_tensor(cs.T, device="cuda").clone()
    status = torch.empty(cs.n_cells, dtype=torch.int32, device="cuda")
    stats = torch.zeros((cs.n_cells, 4), dtype=torch.int32, device="cuda")
    counters = torch.zeros(8, dtype=torch.int64, device="cuda")
    o = kr.default_options(precision=kr.KR_FP32LU_REFINE)
    o.counters = counters.data_ptr()
    kr.chem_integrate(net, n, T, dt=torch.as_tensor(dt, device="cuda"), rtol=1e-6, opts=o, status=status,
                      cell_stats=stats)
    resid = torch.zeros(cs.n_cells, dtype=torch.float64, device="cuda")
    kr.element_residual(net, torch.as_tensor(cs.n, device="cuda"), n, resid=resid)
    torch.cuda.synchronize()
    net.close()
    return ((n.cpu().numpy(), T.cpu().numpy(), status.cpu().numpy(), stats.cpu().numpy(), resid.cpu().numpy()),
            counters.cpu().numpy())


@pytest.mark.parametrize("ncell,cap", [(96, 1e-5), (64, 1e-2)])
def test_large48_mfma_blocked_lu(oracle_lib, ncell, cap):
    """The FP32 LU with its trailing updates on MFMA tiles (panels of 1, 16,
    16, 16 columns for 49 unknowns) against the oracle at 1e-6, in full
    waves, steps up to 1e-5 s and over the configuration's whole range
    [1e-8, 1e-2] s.  The FP32 form falls back to the FP64 LU where
    refinement does not settle, which would hide a broken factorisation:
    the blocked LU must need no more refinement sweeps and FP64 fallbacks
    per Newton iteration than the unblocked one, within a few percent."""
    kr = _kr()
    desc, cs, dt = _large_inputs(ncell, cap)
    src = kr.network_check(desc, build=kr.build_options(lu_mfma=1))
    assert "#define KR_LU_MFMA 1" in src
    g, c = _counted(kr, desc, cs, dt, kr.build_options(lu_mfma=1))
    g0, c0 = _counted(kr, desc, cs, dt, kr.build_options(lu_mfma=0))
    orc = run_oracle(oracle_lib, desc, cs, dt=dt)
    assert_parity(g, orc, cs, 1e-6, "large48 fp32lu mfma", desc=desc)
    assert_parity(g0, orc, cs, 1e-6, "large48 fp32lu valu", desc=desc)
    it, it0 = g[3][:, 1].sum(), g0[3][:, 1].sum()
    print(f"mfma: sweeps {c[3]} fallbacks {c[4]} iterations {it}; valu: sweeps {c0[3]} "
          f"fallbacks {c0[4]} iterations {it0}", flush=True)
    assert c[3] / it <= 1.05 * c0[3] / it0
    assert c[4] <= 1.05 * c0[4] + 0.001 * it
