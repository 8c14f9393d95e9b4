"""GPU checks of the boundary's per-cell extras against the oracle:

* the substep log: the oracle replays each cell's logged sequence of
  accepted lengths (no error control) and must land on the GPU's result --
  the controller's sequence is pinned by self-consistency, both layouts;
* the caller's first-substep hint and the proposed next length, against the
  oracle run with the same hint;
* the per-call totals (kr_stats) against the per-cell statistics;
* post-processing alone (kr_postprocess, Sec. 2.2.3) in full waves of cells
  built so that stages 1-3 act, against the oracle's stages and flags;
* the retry ladder's successful branch (status 1) in every layout on cells
  chosen with the oracle (the lane-group layout in 16- and 32-lane groups
  wherever the network fits)."""
import numpy as np
import pytest

import synthetic as sy
from tests.test_parity_gpu import FLOOR, assert_parity, reservoir_slack, run_oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _kr():
    import paper_2504_04941_amd as kr
    return kr


def _dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=dtype)


def _layout(kr, wave):
    """False: one cell per lane, True: per wavefront, "group16" / "group32":
    per lane group"""
    return kr.build_options(layout={False: kr.KR_LAYOUT_LANE, True: kr.KR_LAYOUT_WAVE,
                                    "group16": kr.KR_LAYOUT_GROUP16, "group32": kr.KR_LAYOUT_GROUP32}[wave])


def _run(desc, cs, build, dt=None, dt_scalar=0.0, cap=0, hint=None, stats=False, **opt):
    kr = _kr()
    net = kr.Network(desc, build)
    ncell = cs.T.shape[0]
    n, T = _dev(cs.n), _dev(cs.T)
    status = torch.full((ncell,), -7, dtype=torch.int32, device="cuda")
    cst = torch.zeros((ncell, 4), dtype=torch.int32, device="cuda")
    h_log = torch.full((max(cap, 1), ncell), -1.0, dtype=torch.float64, device="cuda") if cap else None
    h_log_n = torch.full((ncell,), -7, dtype=torch.int32, device="cuda") if cap else None
    h_hint = _dev(hint) if hint is not None else None
    tot = kr.chem_integrate(net, n, T, dt=None if dt is None else _dev(dt), dt_scalar=dt_scalar,
                            rtol=1e-6, opts=kr.default_options(**opt), status=status,
                            cell_stats=cst, h_hint=h_hint, h_log=h_log, h_log_n=h_log_n,
                            stats=stats)
    torch.cuda.synchronize()
    resid = torch.zeros(ncell, dtype=torch.float64, device="cuda")
    kr.element_residual(net, _dev(cs.n), n, resid=resid)
    out = dict(n=n.cpu().numpy(), T=T.cpu().numpy(), status=status.cpu().numpy(),
               stats=cst.cpu().numpy(), resid=resid.cpu().numpy(), totals=tot,
               h_log=None if h_log is None else h_log.cpu().numpy(),
               h_log_n=None if h_log_n is None else h_log_n.cpu().numpy(),
               h_hint=None if h_hint is None else h_hint.cpu().numpy())
    net.close()
    return out


def _gpu_tuple(g):
    return g["n"], g["T"], g["status"], g["stats"], g["resid"]


CASES = [("h_o_n", False), ("h_o_n", True), ("astro23", True), ("h_o_n", "group16"), ("astro23", "group32")]


def _inputs(oracle, which, ncell):
    if which == "h_o_n":
        desc = sy.network_h_o_n(1)
        return desc, sy.cells_h_o_n(desc, ncell, 1), None, 1e-4
    desc = sy.network_astro23(2)
    cs = sy.cells_astro23(desc, ncell, 2)
    on = oracle.OracleNet(desc)
    dt = np.array([10.0 ** (-3 + 3 * (c % 7) / 6) * on.fastest_timescale(np.r_[cs.n[:, c], cs.T[c]])
                   for c in range(ncell)])
    return desc, cs, dt, 0.0


@pytest.mark.parametrize("which,wave", CASES)
def test_substep_log_replayed_by_oracle(oracle_lib, which, wave):
    """The oracle, replaying each cell's logged lengths, lands on the GPU's
    adaptive result (1e-8); the log is what the controller accepted."""
    kr = _kr()
    desc, cs, dt, dts = _inputs(oracle_lib, which, 130)
    cap = 30000
    g = _run(desc, cs, _layout(kr, wave), dt=dt, dt_scalar=dts, cap=cap)
    ok = g["status"] == 0
    assert ok.mean() > 0.95
    # the count equals the accepted substeps, the lengths add up to dt
    np.testing.assert_array_equal(g["h_log_n"][ok], g["stats"][ok, 0])
    np.testing.assert_array_equal(g["h_log_n"][~ok], 0)
    assert g["h_log_n"].max() <= cap
    stepv = dt if dt is not None else np.full(130, dts)
    for c in np.where(ok)[0]:
        L = g["h_log"][:g["h_log_n"][c], c]
        assert np.all(L > 0)
        assert L.sum() == pytest.approx(stepv[c], rel=1e-12)
    on = oracle_lib.OracleNet(desc)
    o = oracle_lib.default_opts()
    o.mode = oracle_lib.REPLAY
    idx = np.where(ok)[0]
    log = np.ascontiguousarray(g["h_log"][:, idx])
    r = on.integrate_ex(cs.n[:, idx], cs.T[idx], dt=stepv[idx], opts=o, replay=log,
                        replay_n=g["h_log_n"][idx])
    np.testing.assert_array_equal(r["status"], 0)
    sub = sy.CellStates(cs.n[:, idx], cs.T[idx], cs.rho[idx], None)
    assert_parity((g["n"][:, idx], g["T"][idx], g["status"][idx], g["stats"][idx], g["resid"][idx]),
                  (r["n"], r["T"], r["status"], r["stats"]), sub, 1e-8,
                  f"{which} replay", desc=desc)


@pytest.mark.parametrize("wave", [False, True, "group16", "group32"])
def test_h_hint_in_and_out(oracle_lib, wave):
    """A positive hint is the first substep of the first attempt; zero or NaN
    hints are ignored; the proposal out matches the oracle's where the two
    took the same substep sequence."""
    kr = _kr()
    desc = sy.network_h_o_n(1)
    cs = sy.cells_h_o_n(desc, 128, 1)
    rng = np.random.default_rng(17)
    hint = 10.0 ** rng.uniform(-9, -5, 128)
    hint[::9] = 0.0
    hint[4::9] = np.nan
    g = _run(desc, cs, _layout(kr, wave), dt_scalar=1e-4, cap=20000, hint=hint)
    on = oracle_lib.OracleNet(desc)
    a = on.integrate_ex(cs.n, cs.T, dt_scalar=1e-4, h_hint=hint.copy(), log_cap=20000)
    assert_parity(_gpu_tuple(g), (a["n"], a["T"], a["status"], a["stats"]), cs, 1e-8,
                  "hint", desc=desc)
    same = (g["h_log_n"] == a["h_log_n"]) & (g["status"] != 2)
    assert same.mean() > 0.95
    for c in np.where(same)[0]:
        n = g["h_log_n"][c]
        # the first accepted length: the hint itself when accepted at once
        if a["h_log"][0, c] == hint[c]:
            assert g["h_log"][0, c] == hint[c]
        # each length is the previous one times a factor of the error
        # estimate, (h/2)|g(y_new) - g(y_old)|: a difference of rates that can
        # cancel to a few digits, so the two sides' lengths agree to ~1e-9
        # and drift further along a sequence; the last one, dt - t, also
        # carries the rounding of t, a sum of n lengths (n eps dt)
        at = 2.0 * n * np.finfo(float).eps * 1e-4
        np.testing.assert_allclose(g["h_log"][:n, c], a["h_log"][:n, c], rtol=1e-6, atol=at)
        assert g["h_hint"][c] == pytest.approx(a["h_hint"][c], rel=1e-6, abs=at)
    # unusable hints act as no hint: the first attempted length is dt
    b = on.integrate_ex(cs.n, cs.T, dt_scalar=1e-4, log_cap=20000)
    for c in list(range(0, 128, 9)) + list(range(4, 128, 9)):
        if same[c]:
            m = g["h_log_n"][c]
            np.testing.assert_allclose(g["h_log"][:m, c], b["h_log"][:b["h_log_n"][c], c],
                                       rtol=1e-6, atol=2.0 * m * np.finfo(float).eps * 1e-4)


def test_h_hint_fixed_mode_untouched():
    kr = _kr()
    desc = sy.network_h_o_n(1)
    cs = sy.cells_h_o_n(desc, 70, 1)
    hint = np.full(70, 3.5e-8)
    g = _run(desc, cs, None, dt_scalar=1e-9, hint=hint, mode=1, n_fixed=3)
    np.testing.assert_array_equal(g["h_hint"], hint)


@pytest.mark.parametrize("which,wave", CASES)
def test_stats_totals(oracle_lib, which, wave):
    kr = _kr()
    desc, cs, dt, dts = _inputs(oracle_lib, which, 100)
    cs.n[:, 3] = np.nan                       # one reverted cell
    g = _run(desc, cs, _layout(kr, wave), dt=dt, dt_scalar=dts, stats=True,
             precision=kr.KR_FP32LU_REFINE)
    t = g["totals"]
    st = g["stats"].astype(np.int64)
    assert t["cells"] == 100
    assert t["substeps"] == st[:, 0].sum() and t["newton_iterations"] == st[:, 1].sum()
    assert t["rejected"] == st[:, 2].sum() and t["newton_failures"] == st[:, 3].sum()
    assert t["retried"] == np.sum(g["status"] == 1) and t["reverted"] == np.sum(g["status"] == 2)
    assert t["reverted"] >= 1
    assert t["refinement_sweeps"] >= t["newton_iterations"] - t["fp64_fallbacks"]
    ok = g["status"] != 2
    assert 0.0 <= t["max_element_residual"] < 1e-12
    assert t["max_element_residual"] == pytest.approx(g["resid"][ok].max(), rel=1e-6, abs=1e-30)


def test_stats_accumulate_caller_counters():
    """With stats requested, the caller's own counters still accumulate."""
    kr = _kr()
    desc = sy.network_h_o_n(1)
    cs = sy.cells_h_o_n(desc, 64, 1)
    net = kr.Network(desc)
    counters = torch.zeros(8, dtype=torch.int64, device="cuda")
    tots = []
    for _ in range(2):
        n, T = _dev(cs.n), _dev(cs.T)
        o = kr.default_options(precision=kr.KR_FP32LU_REFINE)
        o.counters = counters.data_ptr()
        tots.append(kr.chem_integrate(net, n, T, dt_scalar=1e-5, opts=o, stats=True))
    torch.cuda.synchronize()
    c = counters.cpu().numpy()
    assert c[3] == tots[0]["refinement_sweeps"] + tots[1]["refinement_sweeps"] > 0
    assert tots[0] == tots[1]
    net.close()


# --------------------------------------------------------------------------
# post-processing alone
# --------------------------------------------------------------------------

def _post_inputs(desc, cs, seed):
    """after = before, perturbed per cell: tiny negatives (stage 1), excess
    of a row carried by a non-reservoir species so that stage 2 drives the
    row's reservoir negative (stage 3), or both; every fourth cell is left
    alone."""
    rng = np.random.default_rng(seed)
    comp = np.asarray(desc.composition)
    res = np.asarray(desc.reservoir)
    before = cs.n.copy()
    after = before * (1.0 + 1e-13 * rng.standard_normal(before.shape))
    S, nc = before.shape
    for c in range(nc):
        kind = c % 4
        if kind in (1, 3):
            s = rng.integers(S)
            after[s, c] = -1e-12 * before[:, c].sum()
        if kind in (2, 3):
            v = rng.integers(comp.shape[0])
            r = res[v]
            sign = np.sign(comp[v, r])
            carriers = [s for s in range(S) if s != r and comp[v, s] * sign > 0]
            if not carriers:
                continue
            s = carriers[rng.integers(len(carriers))]
            # stage 2 takes 1.5 x the reservoir away: it ends negative
            after[s, c] += 1.5 * before[r, c] * abs(comp[v, r]) / abs(comp[v, s]) + 1e-9 * before[s, c]
    return before, after


POST_CASES = [("h_he", False), ("h_o_n", False), ("h_o_n", True), ("large48", True)]


@pytest.mark.parametrize("which,wave", POST_CASES)
def test_postprocess_matches_oracle(oracle_lib, which, wave):
    kr = _kr()
    ci = {"h_he": 0, "h_o_n": 1, "large48": 3}[which]
    desc = sy.network_for(ci)
    cs = sy.cells_for(ci, desc, 128)
    before, after = _post_inputs(desc, cs, 40 + ci)
    net = kr.Network(desc, _layout(kr, wave))
    a_dev = _dev(after)
    flags = torch.full((128,), -1, dtype=torch.int32, device="cuda")
    kr.postprocess(net, _dev(before), a_dev, flags=flags)
    torch.cuda.synchronize()
    got, gfl = a_dev.cpu().numpy(), flags.cpu().numpy()
    net.close()
    on = oracle_lib.OracleNet(desc)
    comp = np.asarray(desc.composition, float)
    want = np.empty_like(after)
    wfl = np.empty(128, np.int32)
    for c in range(128):
        E0 = comp @ np.maximum(before[:, c], 0.0)
        want[:, c], wfl[c] = on.postprocess_flags(E0, after[:, c].copy())
    np.testing.assert_array_equal(gfl, wfl)
    assert np.sum(wfl & 2) >= 20 and np.sum(wfl & 1) >= 20     # stages 1 and 3 exercised
    nnuc = np.abs(comp[:desc.n_elem]).sum(axis=0) @ before
    # the same operations in the same order as the oracle's stages, up to
    # contraction into fused multiply-adds (lane layout) and the order of the
    # wave sums (wavefront layout): a few ulp of the row totals
    tol = 64 * np.finfo(float).eps
    err = np.abs(got - want) / nnuc[None, :]
    assert err.max() <= tol, (err.max(), np.unravel_index(np.argmax(err), err.shape))
    assert np.all(got >= 0.0)
    # conservation: the after totals equal the before totals
    E0 = comp @ np.maximum(before, 0.0)
    assert np.max(np.abs(comp @ got - E0) / nnuc[None, :]) < 1e-13


# --------------------------------------------------------------------------
# the retry ladder's successful branch
# --------------------------------------------------------------------------

# seeded 9-species combustion batch (1024 cells): with two Newton iterations
# per substep and 8000 substep attempts, attempt 0 of these cells runs out of
# attempts (it needs 8233-9904) and the retry succeeds (5359-7832 attempts),
# as the oracle finds
STATUS1_CELLS = [34, 475, 496, 576, 651]


@pytest.mark.parametrize("wave", [False, True, "group16", "group32"])
def test_retry_success_status_1(oracle_lib, wave):
    kr = _kr()
    desc = sy.network_h_o_n(1)
    cs_all = sy.cells_h_o_n(desc, 1024, 1)
    on = oracle_lib.OracleNet(desc)
    loose = on.integrate_ex(cs_all.n, cs_all.T, dt_scalar=1e-4, log_cap=1,
                            opts=oracle_lib.default_opts(max_newton=2, max_substeps=100000))
    tries0 = loose["stats"][:, 0] + loose["stats"][:, 2] + loose["stats"][:, 3]
    # the rest of two full waves: cells far from the attempt limit either way
    easy = [c for c in np.where(tries0 < 6000)[0] if c not in STATUS1_CELLS][:100]
    hard = [c for c in np.where(tries0 > 14000)[0]][:23]
    idx = np.array(sorted(STATUS1_CELLS + easy + hard))
    assert idx.size == 128
    cs = sy.CellStates(cs_all.n[:, idx], cs_all.T[idx], cs_all.rho[idx], None)
    g = _run(desc, cs, _layout(kr, wave), dt_scalar=1e-4, cap=9000, max_newton=2, max_substeps=8000)
    a = on.integrate_ex(cs.n, cs.T, dt_scalar=1e-4, log_cap=9000,
                        opts=oracle_lib.default_opts(max_newton=2, max_substeps=8000))
    np.testing.assert_array_equal(g["status"], a["status"])
    s1 = np.isin(idx, STATUS1_CELLS)
    np.testing.assert_array_equal(g["status"][s1], 1)
    assert np.all(g["status"][~s1] != 1)
    assert_parity(_gpu_tuple(g), (a["n"], a["T"], a["status"], a["stats"]), cs, 1e-8,
                  "status 1", desc=desc)
    # the retry's controller: first substep at most dt/100, growth at most 2
    for c in np.where(s1)[0]:
        L = g["h_log"][:g["h_log_n"][c], c]
        assert L[0] <= 1e-6 * (1 + 1e-12)
        assert np.max(L[1:] / L[:-1]) <= 2.0 + 1e-12
        assert L.sum() == pytest.approx(1e-4, rel=1e-12)
