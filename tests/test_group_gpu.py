"""GPU parity of the lane-group layout (one cell per group of 16 or 32
lanes, several cells per wavefront) against the FP64 oracle, through the C
ABI:

* the 23-species network in 32-lane groups (two cells per wavefront), the
  9- and 5-species networks in 16-lane groups (four per wavefront) and the
  9-species one in 32-lane groups: FP64 within 1e-8, the FP32 LU form within
  1e-6, per-cell substep and Newton counts equal to the oracle's for > 95 %
  of the cells; batches of 1 cell, odd sizes (the last wavefront partly
  idle) and several hundred cells (groups claiming cells at different
  times);
* c_V(T) and tabulated rates in 16-lane groups;
* fixed steps; edge cells (zero step, non-finite input, negative input) in
  one wavefront with ordinary cells (the substep log, the step hint, the
  per-call totals and the retry ladder's status 1 are checked in every
  layout by tests/test_boundary_gpu.py);
* the 23-species network in 32-lane groups inside a several-network launch
  with graph replay;
* the layout's limits: more species than a group holds are refused.
"""
import numpy as np
import pytest

import synthetic as sy
from tests.test_parity_gpu import assert_parity, run_gpu, run_oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _kr():
    import paper_2504_04941_amd as kr
    return kr


def _layout(kr, G):
    return kr.build_options(layout=kr.KR_LAYOUT_GROUP16 if G == 16 else kr.KR_LAYOUT_GROUP32)


def _case(which, ncell):
    if which == "h_he":
        desc = sy.network_h_he(0)
        cs = sy.cells_h_he(desc, ncell, 0)
    elif which == "h_o_n":
        desc = sy.network_h_o_n(1)
        cs = sy.cells_h_o_n(desc, ncell, 1)
    else:
        desc = sy.network_astro23(2)
        cs = sy.cells_astro23(desc, ncell, 2)
    return desc, cs


def _steps(oracle_lib, desc, cs, factor=20.0, cap=1e-5):
    """per-cell steps of a few fastest timescales (up to ~200 substeps)"""
    on = oracle_lib.OracleNet(desc)
    tau = np.array([on.fastest_timescale(np.r_[cs.n[:, c], cs.T[c]]) for c in range(cs.n_cells)])
    return np.minimum(factor * tau, cap)


@pytest.mark.parametrize("which,G,ncell", [("astro23", 32, 1), ("astro23", 32, 77), ("astro23", 32, 301),
                                           ("h_o_n", 16, 97), ("h_o_n", 32, 64), ("h_he", 16, 130)])
@pytest.mark.parametrize("prec,tol", [(0, 1e-8), (1, 1e-6)])
def test_group_layout_matches_oracle(oracle_lib, which, G, ncell, prec, tol):
    kr = _kr()
    desc, cs = _case(which, ncell)
    dt = _steps(oracle_lib, desc, cs)
    print(f"{which} G={G} ncell={ncell} prec={prec}", flush=True)
    gpu = run_gpu(desc, cs, dt=dt, build=_layout(kr, G), precision=prec)
    orc = run_oracle(oracle_lib, desc, cs, dt=dt)
    assert_parity(gpu, orc, cs, tol, f"{which} G{G} prec {prec}", desc=desc)
    if prec == 0:
        assert np.mean(np.all(gpu[3] == orc[3], axis=1)) > 0.95


def test_group_layout_tcv_tables(oracle_lib):
    kr = _kr()
    desc = sy.network_h_o_n_tcv()
    cs = sy.cells_h_o_n(desc, 90, 1)
    print("h_o_n_tcv G=16", flush=True)
    gpu = run_gpu(desc, cs, dt_scalar=1e-6, build=_layout(kr, 16))
    orc = run_oracle(oracle_lib, desc, cs, dt_scalar=1e-6)
    assert_parity(gpu, orc, cs, 1e-8, "tcv G16", desc=desc)
    assert np.mean(np.all(gpu[3] == orc[3], axis=1)) > 0.95


def test_group_layout_fixed_steps(oracle_lib):
    kr = _kr()
    desc, cs = _case("astro23", 45)
    dt = _steps(oracle_lib, desc, cs, factor=2.0)
    print("astro23 G=32 fixed steps", flush=True)
    gpu = run_gpu(desc, cs, dt=dt, build=_layout(kr, 32), mode=kr.KR_FIXED_STEP, n_fixed=3)
    orc = run_oracle(oracle_lib, desc, cs, dt=dt, mode="fixed", n_fixed=3)
    assert_parity(gpu, orc, cs, 1e-8, "astro23 G32 fixed", desc=desc)
    assert np.all(gpu[3][:, 0][gpu[2] != 2] == 3)


@pytest.mark.parametrize("G", [16, 32])
def test_group_layout_edge_cells(oracle_lib, G):
    """zero step, a non-finite input (reverted, untouched), negative input
    abundances (clipped), beside ordinary cells of the same wavefront."""
    kr = _kr()
    desc, cs = _case("h_o_n", 9)
    dt = _steps(oracle_lib, desc, cs)
    cs.n[:, 1] *= -1.0
    cs.n[3, 2] = np.nan
    dt[0] = 0.0
    print(f"edge cells G={G}", flush=True)
    gpu = run_gpu(desc, cs, dt=dt, build=_layout(kr, G))
    orc = run_oracle(oracle_lib, desc, cs, dt=dt)
    np.testing.assert_array_equal(gpu[2], orc[2])
    assert gpu[2][2] == 2 and np.isnan(gpu[0][3, 2])
    np.testing.assert_array_equal(gpu[0][:, 2], cs.n[:, 2])
    # every abundance negative: clipped to nothing, which the oracle reverts
    # too (input untouched)
    assert gpu[2][1] == 2
    np.testing.assert_array_equal(gpu[0][:, 1], cs.n[:, 1])
    # the zero-step cell and the ordinary cells, at the parity gate
    keep = np.array([c for c in range(cs.n_cells) if c not in (1, 2)])
    sub = sy.CellStates(cs.n[:, keep], cs.T[keep], cs.rho[keep], None)
    n_g, T_g, st_g, stats_g, resid_g = gpu
    n_o, T_o, st_o, stats_o = orc
    assert_parity((n_g[:, keep], T_g[keep], st_g[keep], stats_g[keep], resid_g[keep]),
                  (n_o[:, keep], T_o[keep], st_o[keep], stats_o[keep]), sub, 1e-8, f"edge G{G}", desc=desc)


def test_group_layout_in_several_network_launch(oracle_lib):
    """The 23-species network in 32-lane groups beside two lane-layout
    networks in one launch: each network's cells against the oracle, graph
    replays equal to the eager launch bit for bit."""
    kr = _kr()
    cases = [("h_he", 200), ("h_o_n", 130), ("astro23", 157)]
    descs, cells, dts = [], [], []
    for which, m in cases:
        d, cs = _case(which, m)
        descs.append(d)
        cells.append(cs)
        dts.append(_steps(oracle_lib, d, cs))
    nets = [kr.Network(descs[0]), kr.Network(descs[1]), kr.Network(descs[2], _layout(kr, 32))]
    assert nets[2].group == 32
    multi = kr.Multi(nets)

    def bufs():
        return [{"states": torch.tensor(cs.n, device="cuda"), "T": torch.tensor(cs.T, device="cuda"),
                 "dt": torch.tensor(dt, device="cuda"),
                 "status": torch.full((cs.n_cells,), -7, dtype=torch.int32, device="cuda"),
                 "cell_stats": torch.zeros((cs.n_cells, 4), dtype=torch.int32, device="cuda")}
                for cs, dt in zip(cells, dts)]
    for prec, tol in ((kr.KR_FP64, 1e-8), (kr.KR_FP32LU_REFINE, 1e-6)):
        print(f"multi with G=32 network, precision {prec}", flush=True)
        eager = bufs()
        multi.integrate(eager, rtol=1e-6, opts=kr.default_options(precision=prec), use_graph=False)
        torch.cuda.synchronize()
        for d, cs, dt, b in zip(descs, cells, dts, eager):
            orc = oracle_lib.OracleNet(d).integrate(cs.n, cs.T, dt=dt)
            gpu = (b["states"].cpu().numpy(), b["T"].cpu().numpy(), b["status"].cpu().numpy(),
                   b["cell_stats"].cpu().numpy(), np.zeros(cs.n_cells))
            assert_parity(gpu, orc, cs, tol, f"multi {d.name}", desc=d)
        for rep in range(2):
            g = bufs()
            multi.integrate(g, rtol=1e-6, opts=kr.default_options(precision=prec), use_graph=True)
            torch.cuda.synchronize()
            for a, b in zip(eager, g):
                for key in ("states", "T", "status", "cell_stats"):
                    assert torch.equal(a[key], b[key]), (prec, rep, key)
            torch.ones(1000, device="cuda").sum().item()
    multi.close()
    for n in nets:
        n.close()
