"""More pins of the FP64 oracle against values fixed by the paper's
definitions and by mathematics (no GPU):

* the per-cell element residual (Sec. 2.1, eq. method-const-elem taken per
  cell) on hand-worked cells: a multi-atom species, the charge row normalised
  by the nuclei density, NaN propagation;
* the fastest self-coupling timescale against closed forms (an isomer pair,
  a thermal mode, no reaction at all);
* the analytic Jacobian (Sec. 2.2.1, eq. method-jacobian) against an exact
  symbolic derivative of the mass-action right-hand side, evaluated in
  40-digit arithmetic;
* the substep log and its replay: the replayed sequence reproduces the
  adaptive result bit for bit, and on the isomer pair equals the discrete
  closed form of backward Euler with those lengths;
* the caller's first-substep hint (h_hint) and the proposed next length;
* the retry ladder's successful branch (status 1, Sec. 2.2.3) on a cell
  chosen with the oracle: attempt 0 runs out of substeps, the retry (first
  substep dt/100, growth at most 2) succeeds;
* post-processing flags (stage 1 clip, stage 3 break-up, Sec. 2.2.3).
"""
import math

import numpy as np
import pytest

import synthetic as sy
from tests.nets import isomer_pair, make_net


# --------------------------------------------------------------------------
# element residual
# --------------------------------------------------------------------------

def test_element_residual_hand_worked(oracle_lib):
    """Rows H (H, H2, H+), He, charge (H+ - e-); before = (1, 2, 0.5, 0.5,
    0.3): H nuclei 1 + 2*2 + 0.5 = 5.5, He 0.3, nuclei density 5.8."""
    net = sy.network_h_he(0)
    on = oracle_lib.OracleNet(net)
    before = np.array([1.0, 2.0, 0.5, 0.5, 0.3])
    cases = [
        # H2 up by 0.01: the H row changes by 2 * 0.01, normalised by the
        # row's own total 5.5 (a multi-atom species counts twice)
        (np.array([1.0, 2.01, 0.5, 0.5, 0.3]), 0.02 / 5.5),
        # e- down by 0.001: charge +0.001, normalised by the nuclei density
        (np.array([1.0, 2.0, 0.5, 0.499, 0.3]), 0.001 / 5.8),
        # He up by 0.003: the He row, 0.003 / 0.3
        (np.array([1.0, 2.0, 0.5, 0.5, 0.303]), 0.003 / 0.3),
        # H2 -> 2 H exchange conserves every row
        (np.array([1.2, 1.9, 0.5, 0.5, 0.3]), 0.0),
        # two rows off: the larger one counts (H: 0.5/5.5 beats charge 0.5/5.8)
        (np.array([1.0, 2.0, 1.0, 0.5, 0.3]), 0.5 / 5.5),
    ]
    b = np.stack([before] * len(cases), axis=1)
    a = np.stack([c[0] for c in cases], axis=1)
    res = on.element_residual(b, a)
    for k, (_, want) in enumerate(cases):
        assert res[k] == pytest.approx(want, rel=1e-12, abs=1e-16), k
    # a NaN in the after state propagates (it must not pass a < threshold test)
    a_nan = before.copy()
    a_nan[1] = np.nan
    assert np.isnan(on.element_residual(before[:, None], a_nan[:, None])[0])


# --------------------------------------------------------------------------
# fastest timescale
# --------------------------------------------------------------------------

def test_fastest_timescale_isomer_closed_form(oracle_lib):
    """A <=> B with k_f = 2 and k_r = k_f e^{-ds} (no energy change):
    df_A/dA = -k_f, df_B/dB = -k_r, the thermal mode is zero, so
    tau = 1 / max(k_f, k_r)."""
    for kf, ds in ((2.0, 0.7), (2.0, -0.7), (5e3, 0.0)):
        on = oracle_lib.OracleNet(isomer_pair(kf, ds))
        kr = kf * math.exp(-ds)
        tau = on.fastest_timescale(np.array([3.0, 0.25, 400.0]))
        assert tau == pytest.approx(1.0 / max(kf, kr), rel=1e-14)


def _decay_net(A, E, q, cv=1.5):
    """Irreversible A -> B (explicit zero reverse), k = A exp(-E/T), heat
    release q per event (h_A - h_B = q)."""
    return make_net("decay", ["A", "B"], ["X"], 1, [[1, 1]], [0], [cv, cv], [q, 0.0], [0.0, 0.0],
                    [(["A"], ["B"], (A, 0.0, E))], arr_r=[[0.0, 0.0, 0.0]])


def test_fastest_timescale_thermal_mode(oracle_lib):
    """A -> B with k = k0 e^{-E/T}: f_A = -k A, Q = q k A, so |df_A/dA| = k and
    |dQ/dT| / c_V = q k A E / (T^2 c_V).  With A = 1, B = 0, T = 1000 K,
    E = 1e4 K, q = 1e5 K, c = 1.5: the thermal rate is 1e5 * 1e4 / (1e6 *
    1.5) = 666.67 times k, so it decides."""
    k0, E, q, T = 3.0, 1e4, 1e5, 1000.0
    on = oracle_lib.OracleNet(_decay_net(k0, E, q))
    k = k0 * math.exp(-E / T)
    tau = on.fastest_timescale(np.array([1.0, 0.0, T]))
    assert tau == pytest.approx(1.0 / (k * q * E / (T * T * 1.5)), rel=1e-13)
    # without heat release the species mode decides: tau = 1/k
    on0 = oracle_lib.OracleNet(_decay_net(k0, E, 0.0))
    assert on0.fastest_timescale(np.array([1.0, 0.0, T])) == pytest.approx(1.0 / k, rel=1e-14)


def test_fastest_timescale_cap(oracle_lib):
    """No reaction proceeds (A = 0): the timescale is undefined and capped at
    1e7 s; a very slow one is capped too."""
    on = oracle_lib.OracleNet(_decay_net(0.0, 0.0, 0.0))
    assert on.fastest_timescale(np.array([1.0, 1.0, 300.0])) == 1e7
    on = oracle_lib.OracleNet(_decay_net(1e-9, 0.0, 0.0))
    assert on.fastest_timescale(np.array([1.0, 1.0, 300.0])) == 1e7


# --------------------------------------------------------------------------
# Jacobian against an exact symbolic derivative
# --------------------------------------------------------------------------

def _symbolic_rhs(desc, arr):
    """(symbols, [f_0..f_{S-1}, Q]) of the mass-action right-hand side with
    rate parameters arr [R][2][3] (forward, reverse), built from the
    description's integer stoichiometry with sympy."""
    import sympy
    S = desc.n_species
    n = sympy.symbols(f"n0:{S}", positive=True)
    T = sympy.Symbol("T", positive=True)
    nu = desc.stoich()
    qhat = -(nu @ np.asarray(desc.h_form))
    f = [sympy.Integer(0)] * S
    Q = sympy.Integer(0)
    for r in range(desc.n_reactions):
        w = []
        for side, (A, b, E) in ((desc.reac[r], arr[r, 0]), (desc.prod[r], arr[r, 1])):
            term = sympy.Float(A, 40) * T ** sympy.Float(b, 40) * sympy.exp(-sympy.Float(E, 40) / T)
            for s in side:
                if s >= 0:
                    term = term * n[s]
            w.append(term)
        wr = w[0] - w[1]
        for s in range(S):
            if nu[r, s]:
                f[s] = f[s] + int(nu[r, s]) * wr
        Q = Q + sympy.Float(float(qhat[r]), 40) * wr
    return list(n) + [T], f + [Q]


@pytest.mark.parametrize("ci", [0, 1])
def test_jacobian_exact_symbolic(oracle_lib, ci):
    import sympy
    net = sy.network_for(ci)
    cs = sy.cells_for(ci, net, 16)
    on = oracle_lib.OracleNet(net)
    syms, g = _symbolic_rhs(net, on.arrhenius())
    N = len(syms)
    Jsym = [[sympy.diff(g[i], syms[m]) for m in range(N)] for i in range(N)]
    fJ = sympy.lambdify(syms, Jsym, modules="mpmath")
    fg = sympy.lambdify(syms, g, modules="mpmath")
    import mpmath
    mpmath.mp.dps = 40
    for c in (0, 5, 11):
        y = np.r_[cs.n[:, c], cs.T[c] if ci else 3000.0 + 100 * c]
        args = [mpmath.mpf(float(v)) for v in y]
        Jx = np.array([[float(v) for v in row] for row in fJ(*args)])
        gx = np.array([float(v) for v in fg(*args)])
        J = on.jacobian(y)
        f, Q = on.rhs(y)
        # the right-hand side itself, against the row's largest term scale
        # (cancellation between directions limits plain FP64 agreement)
        scale_g = np.maximum(np.abs(Jx * y[None, :]).max(axis=1), np.abs(gx)) + 1e-300
        assert np.max(np.abs(np.r_[f, Q] - gx) / scale_g) < 1e-12, c
        # the sensitivities J_im y_m, row by row against the row's scale
        err = np.abs(J * y[None, :] - Jx * y[None, :]) / scale_g[:, None]
        assert err.max() < 1e-12, (c, err.max())


# --------------------------------------------------------------------------
# substep log, replay, hint
# --------------------------------------------------------------------------

def test_replay_reproduces_adaptive_bitwise(oracle_lib):
    net = sy.network_h_o_n(1)
    cs = sy.cells_h_o_n(net, 32, 1)
    on = oracle_lib.OracleNet(net)
    a = on.integrate_ex(cs.n, cs.T, dt_scalar=1e-4, log_cap=60000)
    ok = a["status"] != 2
    assert ok.all()
    # the accepted lengths of every cell add up to dt
    for c in range(32):
        L = a["h_log"][:a["h_log_n"][c], c]
        assert L.sum() == pytest.approx(1e-4, rel=1e-12)
        assert np.all(L > 0)
    np.testing.assert_array_equal(a["h_log_n"], a["stats"][:, 0])
    r = on.integrate_ex(cs.n, cs.T, dt_scalar=1e-4, replay=a["h_log"], replay_n=a["h_log_n"])
    np.testing.assert_array_equal(r["n"], a["n"])
    np.testing.assert_array_equal(r["T"], a["T"])
    np.testing.assert_array_equal(r["status"], 0)
    np.testing.assert_array_equal(r["stats"][:, 0], a["h_log_n"])


def test_replay_isomer_discrete_closed_form(oracle_lib):
    """A <=> B over a given sequence of lengths h_k: backward Euler gives
    A_{k+1} - A_eq = (A_k - A_eq) / (1 + (k_f + k_r) h_k)."""
    kf, ds = 2.0, 0.7
    on = oracle_lib.OracleNet(isomer_pair(kf, ds))
    kr = kf * math.exp(-ds)
    A0, B0 = 3.0, 0.25
    Aeq = kr * (A0 + B0) / (kf + kr)
    seqs = [[0.1, 0.2, 0.05], [1e-3] * 7 + [2.5], [4.0]]
    cap = max(len(s) for s in seqs)
    log = np.zeros((cap, len(seqs)))
    for c, s in enumerate(seqs):
        log[:len(s), c] = s
    n = np.array([[A0] * len(seqs), [B0] * len(seqs)])
    T = np.full(len(seqs), 500.0)
    r = on.integrate_ex(n, T, dt_scalar=0.0 + 1.0, replay=log, replay_n=[len(s) for s in seqs])
    for c, s in enumerate(seqs):
        A = A0
        for h in s:
            A = Aeq + (A - Aeq) / (1 + (kf + kr) * h)
        assert r["status"][c] == 0
        assert r["n"][0, c] == pytest.approx(A, rel=1e-13)
        assert r["n"][1, c] == pytest.approx(A0 + B0 - A, rel=1e-13)


def test_h_hint_first_substep_and_proposal(oracle_lib):
    kf, ds = 2.0, 0.7
    on = oracle_lib.OracleNet(isomer_pair(kf, ds))
    n = np.array([[3.0] * 3, [0.25] * 3])
    T = np.full(3, 500.0)
    hint = np.array([1e-4, 0.0, np.nan])           # positive, zero (ignored), NaN (ignored)
    a = on.integrate_ex(n, T, dt_scalar=2.0, h_hint=hint, log_cap=10000)
    assert np.all(a["status"] == 0)
    assert a["h_log"][0, 0] == 1e-4                  # the hint, accepted (tiny)
    b = on.integrate_ex(n, T, dt_scalar=2.0, log_cap=10000)
    for c in (1, 2):                                 # no usable hint: as without one
        np.testing.assert_array_equal(a["h_log"][:, c], b["h_log"][:, c])
        np.testing.assert_array_equal(a["n"][:, c], b["n"][:, c])
    # the proposal is positive and at least the last accepted length's share
    # of the controller's range [0.2, 5] (growth) times that length
    for c in range(3):
        L = a["h_log"][:a["h_log_n"][c], c]
        assert 0.2 * L[-1] <= a["h_hint"][c] <= max(5.0 * L[-1], L[-2] * 5.0)
    # a continuation that starts from the proposal takes it as its first
    # substep when the error control accepts it
    c2 = on.integrate_ex(a["n"], a["T"], dt_scalar=1e3, h_hint=a["h_hint"], log_cap=10000)
    acc = c2["h_log"][0] == a["h_hint"]
    assert acc.any()
    # fixed mode keeps the hint as it was
    f = on.integrate_ex(n, T, dt_scalar=2.0, h_hint=hint,
                        opts=oracle_lib.default_opts(mode=oracle_lib.FIXED, n_fixed=3))
    np.testing.assert_array_equal(f["h_hint"][:1], hint[:1])


# --------------------------------------------------------------------------
# the retry ladder's successful branch
# --------------------------------------------------------------------------

# cells of the seeded 9-species combustion batch (1024 cells) for which two
# Newton iterations per substep and 8000 substep attempts are too few for
# attempt 0 but enough for the retry (found by scanning the batch with the
# oracle)
STATUS1_CELLS = (34, 475, 496, 576, 651)


def test_retry_success_status_1(oracle_lib):
    net = sy.network_h_o_n(1)
    cs = sy.cells_h_o_n(net, 1024, 1)
    idx = list(STATUS1_CELLS)
    on = oracle_lib.OracleNet(net)
    n, T = cs.n[:, idx], cs.T[idx]
    tight = oracle_lib.default_opts(max_newton=2, max_substeps=8000)
    a = on.integrate_ex(n, T, dt_scalar=1e-4, opts=tight, log_cap=20000)
    np.testing.assert_array_equal(a["status"], 1)
    # attempt 0 alone needs more than 8000 substep attempts: with room it
    # finishes on its first attempt after that many
    loose = on.integrate_ex(n, T, dt_scalar=1e-4, log_cap=20000,
                            opts=oracle_lib.default_opts(max_newton=2, max_substeps=100000))
    np.testing.assert_array_equal(loose["status"], 0)
    tries0 = loose["stats"][:, 0] + loose["stats"][:, 2] + loose["stats"][:, 3]
    assert np.all(tries0 > 8000)
    for k in range(len(idx)):
        L = a["h_log"][:a["h_log_n"][k], k]
        assert L.sum() == pytest.approx(1e-4, rel=1e-12)
        # the retry's step control: growth at most 2 per accepted substep
        # (attempt 0 grows up to 5: the unlimited run shows larger ratios)
        assert np.max(L[1:] / L[:-1]) <= 2.0 + 1e-12
        L0 = loose["h_log"][:loose["h_log_n"][k], k]
        assert np.max(L0[1:] / L0[:-1]) > 2.0
        # the retry's first substep is dt/100 cut by Newton failures (1/4)
        # and rejections (factor in [0.2, 1)): never above dt/100
        assert L[0] <= 1e-6 * (1 + 1e-12)
    # the result is the backward-Euler composition over the logged lengths
    r = on.integrate_ex(n, T, dt_scalar=1e-4, replay=a["h_log"], replay_n=a["h_log_n"],
                        opts=oracle_lib.default_opts(max_newton=2))
    np.testing.assert_array_equal(r["n"], a["n"])
    np.testing.assert_array_equal(r["T"], a["T"])
    assert np.max(on.element_residual(n, a["n"])) < 1e-12


# --------------------------------------------------------------------------
# post-processing flags
# --------------------------------------------------------------------------

def test_postprocess_flags(oracle_lib):
    net = sy.network_h_he(0)
    on = oracle_lib.OracleNet(net)
    comp = net.composition.astype(float)
    n0 = np.array([1.0, 2.0, 0.5, 0.5, 0.3])
    E0 = comp @ n0
    out, fl = on.postprocess_flags(E0, n0)
    assert fl == 0
    np.testing.assert_array_equal(out, n0)
    out, fl = on.postprocess_flags(E0, np.array([1.0, 2.0, 0.5, 0.5 - 1e-12, 0.3]))
    assert fl == 0                     # stage 2 only (e- takes the charge difference)
    out, fl = on.postprocess_flags(E0, np.array([1.0, 2.0, -1e-9, 0.5, 0.3]))
    assert fl & oracle_lib.POST_CLIPPED and not fl & oracle_lib.POST_BROKEN_UP
    # the H reservoir must give 0.2 nuclei it does not have: H2 breaks up
    E0b = comp @ np.array([0.0, 1.9, 0.5, 0.5, 0.3])
    out, fl = on.postprocess_flags(E0b, np.array([0.0, 2.0, 0.5, 0.5, 0.3]))
    assert fl & oracle_lib.POST_BROKEN_UP
    assert out[0] == 0.0 and out[1] == pytest.approx(1.9, rel=1e-15)
