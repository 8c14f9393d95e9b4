"""Parity at the full workload sizes, in the launch configuration the
benchmark times: the whole batch runs on the GPU, and the oracle integrates a
seeded sample of its cells one by one (the oracle cannot afford the whole
batch: 4096 cells of the small networks, 512 of the 48-species network,
whose cells cost the oracle ~0.1 s each).  Gates as for the small batches on
the sample; on the whole batch, every status is valid, reverted cells are
rare, and the element residual of every cell not reverted is below 1e-12."""
import numpy as np
import pytest

import synthetic as sy
from tests.test_parity_gpu import assert_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SAMPLE = 4096
SAMPLE_LARGE = 512


def _kr():
    import paper_2504_04941_amd as kr
    return kr


def _sub(cs, idx, dt=None):
    return sy.CellStates(cs.n[:, idx].copy(), cs.T[idx].copy(), cs.rho[idx].copy(),
                         None if dt is None else dt[idx].copy(), cs.dt_scalar)


def _sample(n, seed, size=SAMPLE):
    return np.sort(np.random.default_rng(seed).choice(n, size=min(size, n), replace=False))


def _whole_batch(kr, net, cs, n_dev, st, label):
    """Every status valid, reverted cells rare, element residual of every
    cell not reverted below 1e-12 (kr_element_residual on the whole batch)."""
    resid = torch.empty(cs.n_cells, dtype=torch.float64, device="cuda")
    kr.element_residual(net, torch.tensor(cs.n, device="cuda"), n_dev, resid=resid)
    torch.cuda.synchronize()
    r = resid.cpu().numpy()
    hist = np.bincount(st, minlength=3)
    print(f"{label}: status histogram {hist.tolist()}", flush=True)
    assert hist.size == 3 and hist.sum() == cs.n_cells
    assert hist[2] <= 1e-4 * cs.n_cells, hist
    ok = st != 2
    assert np.all(r[ok] < 1e-12), f"{label}: element residual {r[ok].max():.3e}"
    return r


def _check(oracle_lib, desc, cs, idx, n_g, T_g, st_g, stats_g, tol, label, dt=None, dt_scalar=0.0,
           resid=None):
    sub = _sub(cs, idx, dt)
    orc = oracle_lib.OracleNet(desc).integrate(sub.n, sub.T, sub.rho, dt=None if dt is None else dt[idx],
                                               dt_scalar=dt_scalar)
    gpu = (n_g[:, idx], T_g[idx], st_g[idx], stats_g[idx],
           np.zeros(len(idx)) if resid is None else resid[idx])
    return assert_parity(gpu, orc, sub, tol, label, desc=desc)


@pytest.mark.parametrize("prec,tol", [(0, 1e-8), (1, 1e-6)])
def test_h_o_n_2e20_cells(oracle_lib, prec, tol):
    """9-species network, 2^20 cells, dt = 1e-4 s (the benchmark workload)."""
    kr = _kr()
    desc = sy.network_h_o_n(1)
    cs = sy.cells_h_o_n(desc, 1 << 20, 1)
    net = kr.Network(desc)
    n = torch.tensor(cs.n, device="cuda")
    T = torch.tensor(cs.T, device="cuda")
    st = torch.empty(1 << 20, dtype=torch.int32, device="cuda")
    stats = torch.empty((1 << 20, 4), dtype=torch.int32, device="cuda")
    kr.chem_integrate(net, n, T, dt_scalar=cs.dt_scalar, rtol=1e-6,
                      opts=kr.default_options(precision=prec, order=kr.KR_ORDER_WORK),
                      status=st, cell_stats=stats)
    torch.cuda.synchronize()
    stn = st.cpu().numpy()
    r = _whole_batch(kr, net, cs, n, stn, f"h_o_n 2^20 prec {prec}")
    _check(oracle_lib, desc, cs, _sample(1 << 20, 5), n.cpu().numpy(), T.cpu().numpy(), stn,
           stats.cpu().numpy(), tol, f"h_o_n 2^20 prec {prec}", dt_scalar=cs.dt_scalar, resid=r)
    net.close()


def test_learned_guess_2e20_cells(oracle_lib):
    """The FP32 LU form started from a (briefly trained) learned guess on all
    2^20 cells: the sampled cells equal the oracle's plain results."""
    kr = _kr()
    from paper_2504_04941_amd import learned
    desc = sy.network_h_o_n(1)
    net = kr.Network(desc)
    model = kr.GuessModel(net, hidden=256, layers=3, seed=1)
    X, Y, _ = learned.single_step_pairs(net, model, desc, 1 << 16, salt=1000)
    learned.train(model, X, Y, steps=100, batch=4096, lr=1e-3, lr_min=1e-4)
    cs = sy.cells_h_o_n(desc, 1 << 20, 1)
    n = torch.tensor(cs.n, device="cuda")
    T = torch.tensor(cs.T, device="cuda")
    guess = model.predict(n, T, dt_scalar=cs.dt_scalar)
    counters = torch.zeros(8, dtype=torch.int64, device="cuda")
    st = torch.empty(1 << 20, dtype=torch.int32, device="cuda")
    stats = torch.empty((1 << 20, 4), dtype=torch.int32, device="cuda")
    kr.chem_integrate(net, n, T, dt_scalar=cs.dt_scalar, rtol=1e-6,
                      opts=kr.guess_options(guess, counters, precision=kr.KR_FP32LU_REFINE),
                      status=st, cell_stats=stats)
    torch.cuda.synchronize()
    assert counters[0].item() == 1 << 20
    stn = st.cpu().numpy()
    r = _whole_batch(kr, net, cs, n, stn, "h_o_n 2^20 fp32lu+guess")
    _check(oracle_lib, desc, cs, _sample(1 << 20, 6), n.cpu().numpy(), T.cpu().numpy(), stn,
           stats.cpu().numpy(), 1e-6, "h_o_n 2^20 fp32lu+guess", dt_scalar=cs.dt_scalar, resid=r)
    model.close()
    net.close()


def test_uneven_batch_2e22_cells(oracle_lib):
    """Three networks, 2^22 cells, one graph-replayed persistent launch (the
    uneven-batch benchmark), FP32 LU form."""
    kr = _kr()
    import bench
    descs = bench._mix_descs()
    counts = [int((1 << 22) * f) for f in bench.MIX_FRACTIONS]
    counts[0] += (1 << 22) - sum(counts)
    nets = [kr.Network(d) for d in descs]
    bufs, css, dts = [], [], []
    for k, (d, mk, n) in enumerate(zip(descs, bench._MIX_MAKERS, counts)):
        cs = mk(d, n)
        n0 = torch.tensor(cs.n, device="cuda")
        T0 = torch.tensor(cs.T, device="cuda")
        tau = kr.fastest_timescale(nets[k], n0, T0)
        lo, hi = bench.MIX_U_RANGES[k]
        dt = tau * torch.tensor(sy.log_uniform(n, 10 ** lo, 10 ** hi, 2, 300 + k), device="cuda")
        bufs.append({"states": n0, "T": T0, "dt": dt, "status": torch.empty(n, dtype=torch.int32, device="cuda"),
                     "cell_stats": torch.empty((n, 4), dtype=torch.int32, device="cuda")})
        css.append(cs)
        dts.append(dt.cpu().numpy())
    multi = kr.Multi(nets)
    multi.integrate(bufs, rtol=1e-6, opts=kr.default_options(precision=kr.KR_FP32LU_REFINE), use_graph=True)
    torch.cuda.synchronize()
    for k, (d, cs, dt, b) in enumerate(zip(descs, css, dts, bufs)):
        stn = b["status"].cpu().numpy()
        r = _whole_batch(kr, nets[k], cs, b["states"], stn, f"uneven {d.name}")
        _check(oracle_lib, d, cs, _sample(cs.n_cells, 7 + k), b["states"].cpu().numpy(), b["T"].cpu().numpy(),
               stn, b["cell_stats"].cpu().numpy(), 1e-6, f"uneven {d.name}", dt=dt, resid=r)
    multi.close()
    for n in nets:
        n.close()


@pytest.mark.parametrize("prec,tol", [(0, 1e-8), (1, 1e-6)])
def test_large48_2e18_cells(oracle_lib, prec, tol):
    """48 species, 2^18 cells, per-cell steps log-uniform in [1e-8, 1e-2] s,
    one cell per wavefront, plain FP64 and the FP32 LU form (the
    configuration's stated form)."""
    kr = _kr()
    desc = sy.network_large48(3)
    cs = sy.cells_large48(desc, 1 << 18, 3)
    net = kr.Network(desc)
    assert net.wide
    n = torch.tensor(cs.n, device="cuda")
    T = torch.tensor(cs.T, device="cuda")
    st = torch.empty(1 << 18, dtype=torch.int32, device="cuda")
    stats = torch.empty((1 << 18, 4), dtype=torch.int32, device="cuda")
    kr.chem_integrate(net, n, T, dt=torch.tensor(cs.dt, device="cuda"), rtol=1e-6,
                      opts=kr.default_options(precision=prec, order=kr.KR_ORDER_WORK),
                      status=st, cell_stats=stats)
    torch.cuda.synchronize()
    stn = st.cpu().numpy()
    r = _whole_batch(kr, net, cs, n, stn, f"large48 2^18 prec {prec}")
    _check(oracle_lib, desc, cs, _sample(1 << 18, 8, SAMPLE_LARGE), n.cpu().numpy(), T.cpu().numpy(), stn,
           stats.cpu().numpy(), tol, f"large48 2^18 prec {prec}", dt=cs.dt, resid=r)
    net.close()
