"""kr_chem_integrate_noalloc (no allocation; a static per-GPU workspace)
against kr_chem_integrate on the same inputs, through the C ABI: two calls
in a row, the second with a smaller batch, both layouts, input and
largest-work-first order, with the per-call totals and the substep log.  The
two entry points run the same kernels, so every cell's result is bitwise the
same."""
import numpy as np
import pytest

import synthetic as sy

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _kr():
    import paper_2504_04941_amd as kr
    return kr


def _run(kr, net, cs, idx, dt_scalar, noalloc, **opt):
    n = torch.tensor(np.ascontiguousarray(cs.n[:, idx]), device="cuda")
    T = torch.tensor(np.ascontiguousarray(cs.T[idx]), device="cuda")
    m = idx.size
    status = torch.full((m,), -7, dtype=torch.int32, device="cuda")
    cst = torch.zeros((m, 4), dtype=torch.int32, device="cuda")
    h_log = torch.zeros((64, m), dtype=torch.float64, device="cuda")
    h_log_n = torch.zeros(m, dtype=torch.int32, device="cuda")
    tot = kr.chem_integrate(net, n, T, dt_scalar=dt_scalar, rtol=1e-6, opts=kr.default_options(**opt),
                            status=status, cell_stats=cst, h_log=h_log, h_log_n=h_log_n, stats=True,
                            noalloc=noalloc)
    torch.cuda.synchronize()
    return (n.cpu().numpy(), T.cpu().numpy(), status.cpu().numpy(), cst.cpu().numpy(),
            h_log.cpu().numpy(), h_log_n.cpu().numpy(), tot)


@pytest.mark.parametrize("which", ["h_o_n_lane", "astro23_wave"])
@pytest.mark.parametrize("order", [0, 1])
def test_noalloc_matches_allocating_entry(which, order):
    kr = _kr()
    if which == "h_o_n_lane":
        desc = sy.network_h_o_n(1)
        cs = sy.cells_h_o_n(desc, 1500, 1)
        dts, sizes = 1e-6, (1500, 333)
        build = None
    else:
        desc = sy.network_astro23(2)
        cs = sy.cells_astro23(desc, 400, 2)
        dts, sizes = 1e2, (400, 97)
        build = kr.build_options(layout=kr.KR_LAYOUT_WAVE)
    net = kr.Network(desc, build)
    rng = np.random.default_rng(3 + order)
    for m in sizes:                      # two calls in a row, the second smaller
        idx = np.sort(rng.choice(cs.n_cells, size=m, replace=False))
        a = _run(kr, net, cs, idx, dts, False, order=order)
        b = _run(kr, net, cs, idx, dts, True, order=order)
        for x, y in zip(a[:6], b[:6]):
            np.testing.assert_array_equal(x, y)
        assert a[6] == b[6]
        assert b[6]["cells"] == m
    net.close()


def test_noalloc_rejects_ordered_batch_beyond_scratch():
    kr = _kr()
    desc = sy.network_h_he(0)
    net = kr.Network(desc)
    m = kr.KR_NOALLOC_MAX_ORDER_CELLS + 1
    n = torch.ones((5, m), dtype=torch.float64, device="cuda")
    T = torch.full((m,), 100.0, dtype=torch.float64, device="cuda")
    with pytest.raises(kr.KrError) as e:
        kr.chem_integrate(net, n, T, dt_scalar=1.0, opts=kr.default_options(order=kr.KR_ORDER_WORK),
                          noalloc=True)
    assert e.value.code == kr.KR_EINVAL
    # in input order the size is not limited: a quick fixed-step call
    kr.chem_integrate(net, n, T, dt_scalar=1e-12, opts=kr.default_options(mode=kr.KR_FIXED_STEP, n_fixed=1),
                      noalloc=True)
    torch.cuda.synchronize()
    net.close()
