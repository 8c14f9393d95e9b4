"""Largest-expected-work-first cell order (KR_ORDER_WORK): the
order the library computes is a permutation of the batch sorted by the work
estimate dt (sum_s |f_s| / sum_s n_s + |Q| / eps), which the oracle's rate
function evaluates independently; and integrating in that order gives
bit-identical per-cell results to the input order (lane and wavefront
layouts, several networks in one launch)."""
import numpy as np
import pytest

import synthetic as sy

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _kr():
    import paper_2504_04941_amd as kr
    return kr


def _dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=dtype)


def _oracle_buckets(oracle, desc, cs, dt):
    """Bucket floor(2 log2 w) + 128 in [0, 255] per cell from the oracle's
    rates at the pre-processed input (negatives to zero, T clamped), and
    whether 2 log2 w lies within 1e-9 of a bucket edge (either side is then
    a correct rounding of the same real number)."""
    on = oracle.OracleNet(desc)
    n = cs.T.shape[0]
    b = np.zeros(n, int)
    edge = np.zeros(n, bool)
    cv = np.asarray(desc.cv, float)
    for c in range(n):
        y = np.maximum(cs.n[:, c], 0.0)
        T = min(max(cs.T[c], desc.T_min), desc.T_max)
        f, Q = on.rhs(np.r_[y, T])
        w = dt[c] * (np.abs(f).sum() / y.sum() + abs(Q) / (T * np.dot(cv, y)))
        if w > 0:
            x = 2.0 * np.log2(w)
            b[c] = int(np.clip(np.floor(x) + 128, 0, 255))
            edge[c] = abs(x - np.round(x)) < 1e-9
    return b, edge


def _assert_sorted(order, b, edge):
    n = len(b)
    assert np.array_equal(np.sort(order), np.arange(n)), "not a permutation"
    cur = 10 ** 9
    for c in order:   # greedy: some admissible bucket per cell, non-increasing
        lo, hi = b[c] - int(edge[c]), b[c] + int(edge[c])
        a = min(hi, cur)
        assert a >= lo, f"cell {c} (bucket {b[c]}) after bucket {cur}"
        cur = a


@pytest.mark.parametrize("which", ["h_o_n", "large48"])
def test_work_order_is_sorted_by_oracle_work(oracle_lib, which):
    kr = _kr()
    if which == "h_o_n":
        desc = sy.network_h_o_n(1)
        cs = sy.cells_h_o_n(desc, 3001, 1)
        dt = np.full(3001, cs.dt_scalar)
        dtt, dts = None, cs.dt_scalar
    else:
        desc = sy.network_large48(3)
        cs = sy.cells_large48(desc, 151, 3)
        dt = cs.dt
        dtt, dts = _dev(cs.dt), 0.0
    net = kr.Network(desc)
    order = kr.work_order(net, _dev(cs.n), _dev(cs.T), dt=dtt, dt_scalar=dts).cpu().numpy().astype(np.int64)
    torch.cuda.synchronize()
    b, edge = _oracle_buckets(oracle_lib, desc, cs, dt)
    assert len(np.unique(b)) > 5          # the estimate does spread the cells
    _assert_sorted(order, b, edge)
    net.close()


def _integrate(kr, net, cs, order, dt=None, dt_scalar=0.0, **opt):
    n = _dev(cs.n)
    T = _dev(cs.T)
    ncell = cs.T.shape[0]
    status = torch.full((ncell,), -7, dtype=torch.int32, device="cuda")
    stats = torch.zeros((ncell, 4), dtype=torch.int32, device="cuda")
    kr.chem_integrate(net, n, T, dt=None if dt is None else _dev(dt), dt_scalar=dt_scalar, rtol=1e-6,
                      opts=kr.default_options(order=order, **opt), status=status, cell_stats=stats)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (n, T, status, stats)]


@pytest.mark.parametrize("which", ["h_he", "h_o_n", "large48"])
def test_order_does_not_change_results(which):
    kr = _kr()
    if which == "h_he":
        desc = sy.network_h_he(0)
        cs = sy.cells_h_he(desc, 4097, 0)
    elif which == "h_o_n":
        desc = sy.network_h_o_n(1)
        cs = sy.cells_h_o_n(desc, 2000, 1)
        args = dict(dt_scalar=1e-5)
    else:
        desc = sy.network_large48(3)
        cs = sy.cells_large48(desc, 70, 3)
        args = dict(dt=np.minimum(cs.dt, 1e-6))
    net = kr.Network(desc)
    if which == "h_he":   # one step of 1e3 fastest timescales per cell
        args = dict(dt=1e3 * kr.fastest_timescale(net, _dev(cs.n), _dev(cs.T)).cpu().numpy())
    for prec in ("fp64", "fp32lu"):
        a = _integrate(kr, net, cs, kr.KR_ORDER_INPUT, precision=prec, **args)
        b = _integrate(kr, net, cs, kr.KR_ORDER_WORK, precision=prec, **args)
        for x, y, name in zip(a, b, ("states", "T", "status", "cell_stats")):
            assert np.array_equal(x, y, equal_nan=True), (which, prec, name)
        assert (a[2] != -7).all()
    net.close()


def test_order_in_multi_network_launch():
    """Three networks in one launch: ordered and input-order launches, eager
    and graph-replayed, give the same per-cell results."""
    kr = _kr()
    sets = [(sy.network_h_he(0), lambda d: sy.cells_h_he(d, 333, 0)),
            (sy.network_h_o_n(1), lambda d: sy.cells_h_o_n(d, 190, 1)),
            (sy.network_astro23(2), lambda d: sy.cells_astro23(d, 257, 2))]
    descs = [d for d, _ in sets]
    css = [mk(d) for d, mk in sets]
    nets = [kr.Network(d) for d in descs]
    multi = kr.Multi(nets)
    dts = [np.minimum(20.0 * kr.fastest_timescale(net, _dev(cs.n), _dev(cs.T)).cpu().numpy(), 1e-4)
           for net, cs in zip(nets, css)]

    def run(order, use_graph):
        bufs = [{"states": _dev(cs.n), "T": _dev(cs.T), "dt": _dev(dt),
                 "status": torch.full((cs.T.shape[0],), -7, dtype=torch.int32, device="cuda"),
                 "cell_stats": torch.zeros((cs.T.shape[0], 4), dtype=torch.int32, device="cuda")}
                for cs, dt in zip(css, dts)]
        multi.integrate(bufs, rtol=1e-6, opts=kr.default_options(order=order), use_graph=use_graph)
        torch.cuda.synchronize()
        return [[b[k].cpu().numpy() for k in ("states", "T", "status", "cell_stats")] for b in bufs]

    ref = run(kr.KR_ORDER_INPUT, False)
    for order, graph in ((kr.KR_ORDER_WORK, False), (kr.KR_ORDER_WORK, True), (kr.KR_ORDER_WORK, True)):
        got = run(order, graph)
        for k, (r, g) in enumerate(zip(ref, got)):
            for x, y, name in zip(r, g, ("states", "T", "status", "cell_stats")):
                assert np.array_equal(x, y, equal_nan=True), (k, order, graph, name)
    multi.close()
    for n in nets:
        n.close()


def test_work_order_invalid_arguments():
    kr = _kr()
    desc = sy.network_h_he(0)
    cs = sy.cells_h_he(desc, 100, 0)
    net = kr.Network(desc)
    n, T = _dev(cs.n), _dev(cs.T)
    with pytest.raises(kr.KrError):      # no step given: dt_scalar must be finite and >= 0
        kr.work_order(net, n, T, dt_scalar=float("nan"))
    with pytest.raises(kr.KrError):
        kr.chem_integrate(net, n, T, dt_scalar=1.0, opts=kr.default_options(order=7))
    out = kr.work_order(net, n[:, :0], T[:0], dt_scalar=1.0)   # empty batch: nothing to do
    assert out.numel() == 0
    net.close()
