"""Pins of the oracle's temperature-dependent heat capacities and tabulated
rate factors (no GPU), against what the mathematics fixes:

* e_s(T) is the integral of c_V,s from 0 (numpy's polynomial antiderivative,
  an independent construction), continuous at the breakpoint T_mid, and its
  derivative is c_V,s (central differences);
* the adiabatic equilibrium of an exothermic isomer pair A <=> B with
  T-dependent c_V: the oracle's long-time state equals the root of energy
  conservation plus detailed balance, solved here by bisection with the
  antiderivative above; with c_V frozen at its initial value the equilibrium
  comes out hotter (the sign of the paper's Sec. 4.2 control run, where a
  frozen c_V over-predicts the equilibrium temperature);
* constant-coefficient polynomials reproduce the constant-c_V network;
* U = sum_s n_s (e_s(T) + h_s) is conserved by adiabatic integration;
* a table sampled from A T^b reproduces the Arrhenius coefficient (A, b, 0)
  everywhere (log-log interpolation is exact on power laws), so the two
  networks integrate alike; a table returns its node values at the nodes;
* the analytic Jacobian with tables and T-dependent c_V against Richardson
  differences of the right-hand side and of the residual.
"""
import numpy as np
import pytest
from numpy.polynomial import polynomial as P
from scipy.optimize import brentq

import synthetic as sy
from tests.nets import make_net


def _energy_ref(a_lo, a_hi, T_mid, T):
    """Antiderivative of the piecewise c_V, zero at T = 0, continuous."""
    lo = P.polyint(a_lo)
    hi = P.polyint(a_hi)
    if T < T_mid:
        return P.polyval(T, lo)
    return P.polyval(T, hi) - P.polyval(T_mid, hi) + P.polyval(T_mid, lo)


def test_energy_is_integral_of_heat_capacity(oracle_lib):
    net = sy.network_h_o_n_tcv()
    on = oracle_lib.OracleNet(net)
    for T in (250.0, 700.0, 999.5, 1000.0, 1000.5, 1800.0, 3500.0):
        e, c = on.species_thermo(T)
        for s in range(net.n_species):
            piece = net.cv_poly[s, int(T >= net.T_mid)]
            assert abs(c[s] - P.polyval(T, piece)) <= 1e-14 * abs(c[s])
            ref = _energy_ref(net.cv_poly[s, 0], net.cv_poly[s, 1], net.T_mid, T)
            assert abs(e[s] - ref) <= 1e-13 * abs(ref), (T, s)
    # continuity at the breakpoint and de/dT = c away from it
    eb, _ = on.species_thermo(net.T_mid * (1 - 1e-15))
    ea, _ = on.species_thermo(net.T_mid)
    np.testing.assert_allclose(eb, ea, rtol=1e-12)
    for T in (600.0, 2200.0):
        d = 1e-5 * T
        ep, _ = on.species_thermo(T + d)
        em, _ = on.species_thermo(T - d)
        _, c = on.species_thermo(T)
        np.testing.assert_allclose((ep - em) / (2 * d), c, rtol=1e-8)


def _exo_pair(cvB, dH=-2.0e4, dS=0.5, frozen_T=None):
    """A <=> B with B lower in energy by |dH|; A monatomic-like (c_V 1.5),
    B with the polynomial cvB = [a0..a4] on both pieces (or frozen at its
    value at frozen_T)."""
    net = make_net("exo_pair", ["A", "B"], ["X"], 1, [[1, 1]], [0], [1.5, 1.5],
                   [0.0, dH], [0.0, dS], [(["A"], ["B"], (5.0e3, 0.0, 0.0))], T_min=10.0)
    cvA = np.array([1.5, 0, 0, 0, 0])
    if frozen_T is not None:
        cvB = np.array([P.polyval(frozen_T, cvB), 0, 0, 0, 0])
    net.cv_poly = np.stack([np.stack([cvA, cvA]), np.stack([cvB, cvB])])
    net.T_mid = 1000.0
    return net


def _equilibrium(net, T0, n0):
    """Root of energy conservation with the equilibrium ratio
    n_B / n_A = exp(dS - dH / T) (no change in particle number)."""
    cvA, cvB = net.cv_poly[0, 0], net.cv_poly[1, 0]
    dH = net.h_form[1] - net.h_form[0]
    dS = net.s_form[1] - net.s_form[0]

    def e(a, T):
        return _energy_ref(a, a, net.T_mid, T)
    U0 = n0 * e(cvA, T0)

    def f(T):
        x = 1.0 / (1.0 + np.exp(-(dS - dH / T)))
        return n0 * ((1 - x) * e(cvA, T) + x * (e(cvB, T) + dH)) - U0
    T = brentq(f, T0, 100 * T0, xtol=1e-13, rtol=1e-15)
    x = 1.0 / (1.0 + np.exp(-(dS - dH / T)))
    return T, x


def test_adiabatic_equilibrium_with_t_dependent_cv(oracle_lib):
    cvB = np.array([1.5, 1.0e-3, 0.0, 0.0, 0.0])
    T0, n0 = 400.0, 1.0e10
    out = {}
    for frozen in (None, T0):
        net = _exo_pair(cvB, frozen_T=frozen)
        on = oracle_lib.OracleNet(net)
        n = np.array([[n0], [0.0]])
        nf, Tf, st, _ = on.integrate(n, np.array([T0]), dt_scalar=1.0)
        assert st[0] == 0
        T_ref, x_ref = _equilibrium(net, T0, n0)
        # the backward-Euler fixed point is the exact equilibrium
        assert abs(Tf[0] - T_ref) <= 1e-10 * T_ref, (frozen, Tf[0], T_ref)
        assert abs(nf[1, 0] / n0 - x_ref) <= 1e-10, (frozen, nf[1, 0] / n0, x_ref)
        out[frozen] = Tf[0]
    # c_V rising with T takes up more of the released heat: cooler equilibrium
    assert out[T0] > 1.05 * out[None], out


def test_constant_polynomials_equal_constant_cv(oracle_lib):
    base = sy.network_h_o_n(1)
    poly = sy.network_h_o_n(1)
    poly.cv_poly = np.zeros((base.n_species, 2, 5))
    poly.cv_poly[:, :, 0] = base.cv[:, None]
    cs = sy.cells_h_o_n(base, 24, 1)
    a = oracle_lib.OracleNet(base).integrate(cs.n, cs.T, dt_scalar=1e-5)
    b = oracle_lib.OracleNet(poly).integrate(cs.n, cs.T, dt_scalar=1e-5)
    np.testing.assert_array_equal(a[2], b[2])
    # the same roots, written with T sum c_s n_s or sum n_s (c_s T): they
    # differ by roundings, which the Newton tolerance (1e-3 of rtol 1e-6)
    # may carry to ~1e-9
    nnuc = cs.n.sum(axis=0)
    assert np.max(np.abs(a[0] - b[0]) / np.maximum(np.abs(a[0]), 1e-20 * nnuc)) <= 1e-8
    np.testing.assert_allclose(a[1], b[1], rtol=1e-10)


def test_total_energy_conserved(oracle_lib):
    net = sy.network_h_o_n_tcv()
    cs = sy.cells_h_o_n(net, 32, 1)
    on = oracle_lib.OracleNet(net)
    n, T, st, _ = on.integrate(cs.n, cs.T, dt_scalar=1e-3)
    assert np.all(st == 0)
    for c in range(32):
        e0, _ = on.species_thermo(cs.T[c])
        e1, _ = on.species_thermo(T[c])
        U0 = cs.n[:, c] @ (e0 + net.h_form)
        U1 = n[:, c] @ (e1 + net.h_form)
        scale = np.abs(cs.n[:, c]) @ (np.abs(e0) + np.abs(net.h_form))
        assert abs(U1 - U0) <= 1e-12 * scale, c


def _power_law_pair():
    """h_o_n with four reactions set to (A, b, 0), and the same network with
    those coefficients given as tables sampled from A T^b."""
    ref = sy.network_h_o_n(1)
    picks = [1, 5, 11, 20]
    arr = ref.arr_f.copy()
    arr[picks, 2] = 0.0
    ref.arr_f = arr
    tab = sy.network_h_o_n(1)
    tarr = arr.copy()
    K = 33
    x0, dx = np.log2(300.0), (np.log2(8000.0) - np.log2(300.0)) / (K - 1)
    Tn = 2.0 ** (x0 + dx * np.arange(K))
    tab.tab_of = np.full(ref.n_reactions, -1, np.int32)
    tab.tab_log2k = np.zeros((len(picks), K))
    for t, r in enumerate(picks):
        A, b, _ = arr[r]
        tab.tab_log2k[t] = np.log2(A) + b * np.log2(Tn)
        tarr[r] = (1.0, 0.0, 0.0)
        tab.tab_of[r] = t
    tab.arr_f = tarr
    tab.tab_log2T0, tab.tab_dlog2T = float(x0), float(dx)
    return ref, tab, picks, Tn


def test_tables_exact_on_power_laws(oracle_lib):
    ref, tab, picks, Tn = _power_law_pair()
    a, b = oracle_lib.OracleNet(ref), oracle_lib.OracleNet(tab)
    # between nodes, at nodes, and outside the tabulated range (extended)
    for T in (150.0, 300.0, Tn[7], 777.7, 1234.5, 2999.0, 8000.0, 12000.0):
        kf_a, kr_a = a.rate_coeffs(T)
        kf_b, kr_b = b.rate_coeffs(T)
        np.testing.assert_allclose(kf_b, kf_a, rtol=5e-14)
        np.testing.assert_allclose(kr_b, kr_a, rtol=5e-14)
    cs = sy.cells_h_o_n(ref, 24, 1)
    ra = a.integrate(cs.n, cs.T, dt_scalar=1e-5)
    rb = b.integrate(cs.n, cs.T, dt_scalar=1e-5)
    np.testing.assert_array_equal(ra[2], rb[2])
    nnuc = cs.n.sum(axis=0)
    assert np.max(np.abs(ra[0] - rb[0]) / np.maximum(np.abs(ra[0]), 1e-20 * nnuc)) <= 1e-9
    np.testing.assert_allclose(ra[1], rb[1], rtol=1e-12)


def test_table_node_values(oracle_lib):
    net = sy.network_h_o_n_tcv()
    on = oracle_lib.OracleNet(net)
    K = net.tab_log2k.shape[1]
    for i in (0, 5, K // 2, K - 1):
        T = 2.0 ** (net.tab_log2T0 + i * net.tab_dlog2T)
        kf, _ = on.rate_coeffs(T)
        for r in np.where(net.tab_of >= 0)[0]:
            want = 2.0 ** net.tab_log2k[net.tab_of[r], i]
            assert abs(kf[r] / want - 1.0) <= 1e-12, (i, r)


def _richardson(fun, x, h):
    d1 = (fun(x + h) - fun(x - h)) / (2 * h)
    d2 = (fun(x + h / 2) - fun(x - h / 2)) / h
    return (4 * d2 - d1) / 3


@pytest.mark.parametrize("cell", [0, 3, 9])
def test_jacobian_with_tables_and_tcv(oracle_lib, cell):
    net = sy.network_h_o_n_tcv()
    on = oracle_lib.OracleNet(net)
    cs = sy.cells_h_o_n(net, 16, 1)
    y = np.r_[cs.n[:, cell], cs.T[cell]]
    N = y.size
    J = on.jacobian(y)

    def rhs(v):
        f, Q = on.rhs(v)
        return np.r_[f, Q]
    for m in range(N):
        h = 1e-4 * max(abs(y[m]), 1e-3 * y[:-1].max() if m < N - 1 else 1.0)

        def col(t, m=m):
            v = y.copy()
            v[m] = t
            return rhs(v)
        fd = _richardson(col, y[m], h)
        # rows that do not depend on y_m at all are exact zeros on both sides
        scale = np.maximum(np.abs(J[:, m]), 1e-8 * np.abs(J).max(axis=1))
        live = scale > 0
        np.testing.assert_array_equal(fd[~live], 0.0)
        assert np.max(np.abs(fd - J[:, m])[live] / scale[live]) <= 1e-5, m
    # the energy row of the Newton matrix: d eps / d y by differences
    hstep = 1e-9
    M = on.newton_matrix(y, hstep)
    yn = y.copy()

    def res(v):
        return on.residual(v, yn, hstep)
    for m in range(N):
        h = 1e-4 * max(abs(y[m]), 1e-3 * y[:-1].max() if m < N - 1 else 1.0)

        def col(t, m=m):
            v = y.copy()
            v[m] = t
            return res(v)[-1]
        fd = _richardson(col, y[m], h)
        assert abs(fd - M[-1, m]) <= 1e-6 * max(abs(M[-1, m]), 1e-8 * np.abs(M[-1]).max()), m
