"""The project's autotuner on small samples: per-network layout choice among
the lane-group shapes the network fits (timed on the network's own cells) and the module build options, without the
on-disk cache; the chosen configuration still matches the oracle."""
import numpy as np
import pytest

import synthetic as sy
from tests.test_parity_gpu import assert_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _batch(cs, dt):
    n = cs.n.shape[1]
    return {"states": torch.tensor(cs.n, device="cuda"), "T": torch.tensor(cs.T, device="cuda"),
            "dt": torch.tensor(dt, device="cuda"),
            "status": torch.empty(n, dtype=torch.int32, device="cuda"),
            "cell_stats": torch.empty((n, 4), dtype=torch.int32, device="cuda")}


def test_tune_layout_and_multi(oracle_lib):
    import paper_2504_04941_amd as kr
    from paper_2504_04941_amd import autotune
    descs = [sy.network_h_he(0), sy.network_astro23(2)]
    css = [sy.cells_h_he(descs[0], 300, 0), sy.cells_astro23(descs[1], 200, 2)]
    dts = []
    for d, cs in zip(descs, css):
        on = oracle_lib.OracleNet(d)
        dts.append(np.array([1e-2 * on.fastest_timescale(np.r_[cs.n[:, c], cs.T[c]])
                             for c in range(cs.n_cells)]))
    L, rep = autotune.tune_layout(descs[1], _batch(css[1], dts[1]), use_cache=False)
    # the lane-group shapes the 23-species network fits: 1, 32 and 64 lanes
    assert [c["layout"] for c in rep["candidates"]] == [kr.KR_LAYOUT_LANE, kr.KR_LAYOUT_GROUP32, kr.KR_LAYOUT_WAVE]
    assert L == min(rep["candidates"], key=lambda c: c["ms"])["layout"]
    bo, layouts, report = autotune.tune_multi(descs, [_batch(c, d) for c, d in zip(css, dts)],
                                              candidates=[(1, 0.1)], use_cache=False)
    assert len(layouts) == 2 and report["best"] == [1, 0.1]
    assert report["order"] in (kr.KR_ORDER_INPUT, kr.KR_ORDER_WORK) and len(report["candidates"]) == 2
    nets = [kr.Network(d, kr.build_options(layout=L)) for d, L in zip(descs, layouts)]
    multi = kr.Multi(nets, bo)
    bufs = [_batch(c, d) for c, d in zip(css, dts)]
    multi.integrate(bufs, rtol=1e-6, opts=kr.default_options(order=report["order"]))
    torch.cuda.synchronize()
    for d, cs, dt, b in zip(descs, css, dts, bufs):
        orc = oracle_lib.OracleNet(d).integrate(cs.n, cs.T, dt=dt)
        gpu = (b["states"].cpu().numpy(), b["T"].cpu().numpy(), b["status"].cpu().numpy(),
               b["cell_stats"].cpu().numpy(), np.zeros(cs.n_cells))
        assert_parity(gpu, orc, cs, 1e-8, d.name, desc=d)
    multi.close()
    for n in nets:
        n.close()


def test_tune_order():
    import paper_2504_04941_amd as kr
    from paper_2504_04941_amd import autotune
    desc = sy.network_h_o_n(1)
    cs = sy.cells_h_o_n(desc, 700, 1)
    net = kr.Network(desc)
    batch = _batch(cs, np.full(700, 1e-6))
    order, rep = autotune.tune_order(net, batch)
    assert order in (kr.KR_ORDER_INPUT, kr.KR_ORDER_WORK)
    assert [c["order"] for c in rep["candidates"]] == [kr.KR_ORDER_INPUT, kr.KR_ORDER_WORK]
    assert all(c["ms"] > 0 for c in rep["candidates"])
    net.close()
