"""Several networks in one persistent launch (and its hipGraph replay),
checked against the oracle network by network; the timescale kernel
against the oracle's."""
import numpy as np
import pytest

import synthetic as sy
from tests.test_parity_gpu import assert_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _kr():
    import paper_2504_04941_amd as kr
    return kr


def _dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=dtype)


@pytest.mark.parametrize("which", ["h_he", "h_o_n", "astro23"])
def test_timescale_matches_oracle(oracle_lib, which):
    kr = _kr()
    desc = {"h_he": sy.network_h_he(0), "h_o_n": sy.network_h_o_n(1),
            "astro23": sy.network_astro23(2)}[which]
    cs = {"h_he": lambda: sy.cells_h_he(desc, 300, 0), "h_o_n": lambda: sy.cells_h_o_n(desc, 300, 1),
          "astro23": lambda: sy.cells_astro23(desc, 300, 2)}[which]()
    net = kr.Network(desc)
    tau = kr.fastest_timescale(net, _dev(cs.n), _dev(cs.T)).cpu().numpy()
    on = oracle_lib.OracleNet(desc)
    ref = np.array([on.fastest_timescale(np.r_[cs.n[:, c], cs.T[c]]) for c in range(300)])
    np.testing.assert_allclose(tau, ref, rtol=1e-11)
    net.close()


def _batches():
    """Three networks' cells, each with steps of a few fastest timescales."""
    out = []
    for desc, cs in ((sy.network_h_he(0), None), (sy.network_h_o_n(1), None),
                     (sy.network_astro23(2), None)):
        if desc.name.startswith("h_he"):
            cs = sy.cells_h_he(desc, 333, 0)
        elif desc.name.startswith("h_o_n"):
            cs = sy.cells_h_o_n(desc, 190, 1)
        else:
            cs = sy.cells_astro23(desc, 257, 2)
        out.append((desc, cs))
    return out


def _buffers(batches, dts):
    return [{"states": _dev(cs.n), "T": _dev(cs.T), "dt": _dev(dt),
             "status": torch.full((cs.n.shape[1],), -7, dtype=torch.int32, device="cuda"),
             "cell_stats": torch.zeros((cs.n.shape[1], 4), dtype=torch.int32, device="cuda")}
            for (desc, cs), dt in zip(batches, dts)]


def _run_multi(kr, multi, batches, dts, use_graph, bufs=None):
    """Integrates from the initial states; with `bufs` the same device
    buffers are refilled and reused (as a simulation loop would)."""
    if bufs is None:
        bufs = _buffers(batches, dts)
    else:
        for (desc, cs), b in zip(batches, bufs):
            b["states"].copy_(_dev(cs.n))
            b["T"].copy_(_dev(cs.T))
            b["status"].fill_(-7)
            b["cell_stats"].zero_()
    multi.integrate(bufs, rtol=1e-6, use_graph=use_graph)
    torch.cuda.synchronize()
    return [{k: v.clone() for k, v in b.items()} for b in bufs]


def test_multi_network_parity_and_graph_replay(oracle_lib):
    kr = _kr()
    batches = _batches()
    nets = [kr.Network(d) for d, _ in batches]
    multi = kr.Multi(nets)
    dts = []
    for (desc, cs), net in zip(batches, nets):
        tau = kr.fastest_timescale(net, _dev(cs.n), _dev(cs.T)).cpu().numpy()
        dts.append(np.minimum(20.0 * tau, 1e-4))
    eager = _run_multi(kr, multi, batches, dts, use_graph=False)
    # each network's cells against the oracle
    for (desc, cs), dt, t in zip(batches, dts, eager):
        orc = oracle_lib.OracleNet(desc).integrate(cs.n, cs.T, dt=dt)
        gpu = (t["states"].cpu().numpy(), t["T"].cpu().numpy(), t["status"].cpu().numpy(),
               t["cell_stats"].cpu().numpy(), np.zeros(cs.n.shape[1]))
        assert_parity(gpu, orc, cs, 1e-8, desc.name, desc=desc)
    # graph: captured once, replayed with eager work and synchronisation in
    # between; every replay equals the eager result bit for bit
    bufs = _buffers(batches, dts)
    for rep in range(3):
        g = _run_multi(kr, multi, batches, dts, use_graph=True, bufs=bufs)
        for a, b in zip(eager, g):
            for key in ("states", "T", "status", "cell_stats"):
                assert torch.equal(a[key], b[key]), (rep, key)
        torch.ones(1000, device="cuda").sum().item()
    launches, captures = multi.graph_stats()
    assert (launches, captures) == (3, 1)
    multi.close()
    for n in nets:
        n.close()


def test_occupancy_groups_give_the_same_results():
    """Automatic occupancy target (lane-layout networks in one kernel at one
    wave per SIMD, the 23-species network in a second at two) against one
    kernel for all three at one wave per SIMD: bitwise the same per-cell
    results in both precisions, eager and graph-replayed."""
    kr = _kr()
    batches = _batches()
    descs = [d for d, _ in batches]
    assert "kr_integrate_multi_fp64_1" in kr.multi_check(descs)          # two kernels
    assert "kr_integrate_multi_fp64_1" not in kr.multi_check(descs[:2])  # lane networks only: one
    nets = [kr.Network(d) for d in descs]
    split = kr.Multi(nets)
    one = kr.Multi(nets, kr.build_options(waves_per_eu=1))
    dts = [np.minimum(20.0 * kr.fastest_timescale(net, _dev(cs.n), _dev(cs.T)).cpu().numpy(), 1e-4)
           for (_, cs), net in zip(batches, nets)]
    for prec in ("fp64", "fp32lu"):
        opts = kr.default_options(precision=prec)
        res = []
        for multi, graph in ((one, False), (split, False), (split, True)):
            bufs = _buffers(batches, dts)
            multi.integrate(bufs, rtol=1e-6, opts=opts, use_graph=graph)
            torch.cuda.synchronize()
            res.append([{k: v.cpu() for k, v in b.items()} for b in bufs])
        for got in res[1:]:
            for a, b, (desc, _) in zip(res[0], got, batches):
                for key in ("states", "T", "status", "cell_stats"):
                    assert torch.equal(a[key], b[key]), (prec, desc.name, key)
        assert all((b["status"] != -7).all() for b in res[0])
    split.close()
    one.close()
    for n in nets:
        n.close()
