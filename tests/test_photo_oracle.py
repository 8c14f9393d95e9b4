"""Pins of the oracle's photoreactions and radiative heat terms (no GPU),
against what the paper and the mathematics fix, on the hydrogen chemistry of
the paper's Stromgren-sphere test (Sec. 4.3, eq. strom-chem, with the rate
coefficients and the recombination cooling of eq. thermo-strom as printed,
tests/golden/cie_paper_constants.json):

* the effective flux of a photoreaction is the path average of the
  attenuated flux over the cell (eq. method-rad-equiv-flux), checked against
  numerical quadrature of F exp(-s / lambda) over the path, and its
  derivative against differences of that quadrature;
* isothermal photo-ionisation equilibrium: the oracle's long-time state
  solves the ionisation balance of eq. strom-equil (optically thin: the
  closed-form root of its quadratic; with self-shielding: a root found
  here by bisection);
* thermal plus ionisation equilibrium (eq. strom-equil, the balance of
  photo-heating against recombination and collisional-ionisation cooling):
  the long-time state against an independent two-level root;
* the recombination cooling per event equals lambda_rec of eq.
  thermo-strom;
* the analytic Jacobian: exact (Richardson differences) with one absorber;
  with two absorbers the flux derivative carries the paper's cutoff
  min{1, n_i sigma_i lambda} exactly (Sec. 2.2.1).
"""
import json
import os

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.optimize import brentq

import synthetic as sy

HERE = os.path.dirname(os.path.abspath(__file__))
G = json.load(open(os.path.join(HERE, "golden", "cie_paper_constants.json")))
I_H = G["I_H_eV"] * G["eV_erg"] / G["k_B_erg_per_K"]          # K
PC = 3.0857e18


def _k_ci(T):
    return G["k_ci_coeff_cm3_s"] * (T / G["T_ref_K"]) ** G["k_ci_T_exponent"] * np.exp(-I_H / T)


def _alpha(T):
    return G["alpha_coeff_cm3_s"] * (T / G["T_ref_K"]) ** G["alpha_T_exponent"]


def _lambda_rec(T):
    """eq. thermo-strom, in K (energy / k_B)"""
    return (0.684 - 0.0416 * np.log(T / 1.0e4)) * T


def _feff(F, L, linv):
    """path average of F exp(-s linv) over s in [0, L], by quadrature"""
    if L == 0.0:
        return F
    v, _ = quad(lambda s: np.exp(-s * linv), 0.0, L, epsabs=0.0, epsrel=1e-13, limit=200)
    return F * v / L


def test_effective_flux_is_path_average(oracle_lib):
    net = sy.network_stromgren(isothermal=True)
    on = oracle_lib.OracleNet(net)
    sig = sy.SIGMA_H
    F = 3.0e11
    for tau in (1e-7, 1e-5, 3e-4, 0.02, 0.7, 4.0, 45.0):
        nH = 100.0
        L = tau / (sig * nH)
        # only H present: the collisional and recombination rates vanish
        y = np.array([nH, 0.0, 0.0, 1.0e4])
        f, _ = on.rhs_photo(y, F, L)
        feff = -f[0] / (sig * nH)
        ref = _feff(F, L, sig * nH)
        assert abs(feff / ref - 1.0) <= 1e-12, (tau, feff, ref)
        # d f_H / d n_H = -sigma (F_eff + n_H dF_eff/dn_H), one absorber
        J = on.jacobian_photo(y, F, L)
        d = 1e-4 * nH
        dref = (_feff(F, L, sig * (nH + d)) * (nH + d) - _feff(F, L, sig * (nH - d)) * (nH - d)) / (2 * d)
        # (at large tau F_eff n_H saturates: compare on the scale of F_eff)
        assert abs(-J[0, 0] / sig - dref) <= 1e-7 * max(abs(dref), ref), (tau, -J[0, 0] / sig, dref)


def _x_thin(T, n, F):
    """root in (0, 1) of alpha n x^2 - k_ci n x (1 - x) - F sigma (1 - x) = 0
    (eq. strom-equil divided by n)"""
    a, k, p = _alpha(T) * n, _k_ci(T) * n, F * sy.SIGMA_H
    A, B, C = a + k, p - k, -p
    return (-B + np.sqrt(B * B - 4 * A * C)) / (2 * A)


@pytest.mark.parametrize("F,L", [(1e9, 0.0), (3e11, 0.0), (0.0, 0.0), (1e10, 3e18), (1e12, 1e19)])
def test_isothermal_photoionisation_equilibrium(oracle_lib, F, L):
    net = sy.network_stromgren(isothermal=True)
    on = oracle_lib.OracleNet(net)
    T, n = 1.0e4, 130.0
    if L == 0.0:
        x = _x_thin(T, n, F)
    else:
        def bal(u):            # in the neutral fraction u = 1 - x
            x = 1.0 - u
            feff = _feff(F, L, sy.SIGMA_H * n * u)
            return _alpha(T) * n * x * x - _k_ci(T) * n * x * u - feff * sy.SIGMA_H * u
        x = 1.0 - brentq(bal, 1e-15, 1.0 - 1e-12, xtol=1e-30, rtol=1e-15)
    # start 10 % off in the minority fraction, integrate for many relaxation
    # times (collisional equilibrium relaxes over ~2e12 s at this density)
    x0 = 0.9 * x if x < 0.5 else 1.0 - 1.1 * (1.0 - x)
    y = np.array([[n * (1 - x0)], [n * x0], [n * x0]])
    r = on.integrate_ex(y, np.array([T]), dt_scalar=1e16 if F == 0.0 else 1e13, photo_flux=F, photo_length=L)
    assert r["status"][0] == 0
    assert abs(r["T"][0] / T - 1.0) <= 1e-13
    got = r["n"][1, 0] / n
    # the backward-Euler fixed point is the exact balance
    assert abs(got - x) <= 1e-10 * max(x, 1e-3), (got, x)
    assert abs((1 - got) - (1 - x)) <= 1e-9 * (1 - x) + 1e-14


def test_thermal_and_ionisation_equilibrium(oracle_lib):
    """An isochoric cell 1 pc from the fiducial source (Phi = 1e49 s^-1,
    n_H = 130 cm^-3, optically thin): eq. strom-equil's ionisation and
    energy balances, solved here as x(T) from the quadratic and a root in T
    of photo-heating (h nu - I_H) F sigma n (1 - x) against lambda_rec
    alpha n^2 x^2 + I_H k_ci n^2 x (1 - x)."""
    net = sy.network_stromgren()
    on = oracle_lib.OracleNet(net)
    n = 130.0
    F = 1.0e49 / (4 * np.pi * PC ** 2)
    h_nu = sy.H_NU_EV * G["eV_erg"] / G["k_B_erg_per_K"]

    def heat(T):
        x = _x_thin(T, n, F)
        return ((h_nu - I_H) * F * sy.SIGMA_H * n * (1 - x)
                - _lambda_rec(T) * _alpha(T) * n * n * x * x - I_H * _k_ci(T) * n * n * x * (1 - x))
    T_eq = brentq(heat, 5e3, 2e5, xtol=1e-12, rtol=1e-15)
    x_eq = _x_thin(T_eq, n, F)
    y = np.array([[n * 1e-5], [n * (1 - 1e-5)], [n * (1 - 1e-5)]])
    r = on.integrate_ex(y, np.array([3.0e4]), dt_scalar=1e14, photo_flux=F, photo_length=0.0)
    assert r["status"][0] == 0
    assert abs(r["T"][0] / T_eq - 1.0) <= 1e-9, (r["T"][0], T_eq)
    assert abs(r["n"][0, 0] / n / (1 - x_eq) - 1.0) <= 1e-8, (r["n"][0, 0] / n, 1 - x_eq)


def test_recombination_cooling_is_lambda_rec(oracle_lib):
    net = sy.network_stromgren()
    on = oracle_lib.OracleNet(net)
    for T in (3e3, 1e4, 2.5e4, 8e4):
        ne = 50.0
        y = np.array([0.0, ne, ne, T])        # no H: only recombination acts
        f, Q = on.rhs_photo(y, 0.0, 0.0)
        rate = _alpha(T) * ne * ne
        assert abs(f[0] / rate - 1.0) <= 1e-13
        assert abs(Q / (-_lambda_rec(T) * rate) - 1.0) <= 1e-12, (T, Q, -_lambda_rec(T) * rate)
    # collisional ionisation cools by I_H per event, photo-ionisation heats
    # by h nu - I_H
    T = 2.0e4
    y = np.array([80.0, 0.0, 20.0, T])
    f, Q = on.rhs_photo(y, 0.0, 0.0)
    ci = _k_ci(T) * 80.0 * 20.0
    assert abs(Q / (-I_H * ci) - 1.0) <= 1e-12
    y = np.array([80.0, 0.0, 0.0, T])
    f, Q = on.rhs_photo(y, 1e10, 0.0)
    h_nu = sy.H_NU_EV * G["eV_erg"] / G["k_B_erg_per_K"]
    assert abs(Q / ((h_nu - I_H) * 1e10 * sy.SIGMA_H * 80.0) - 1.0) <= 1e-12


def _richardson(fun, x, h):
    d1 = (fun(x + h) - fun(x - h)) / (2 * h)
    d2 = (fun(x + h / 2) - fun(x - h / 2)) / h
    return (4 * d2 - d1) / 3


def _fd_jacobian(on, y, F, L):
    N = y.size
    out = np.zeros((N, N))
    for m in range(N):
        h = 1e-4 * abs(y[m]) if y[m] != 0 else 1e-6

        def col(t, m=m):
            v = y.copy()
            v[m] = t
            f, Q = on.rhs_photo(v, F, L)
            return np.r_[f, Q]
        out[:, m] = _richardson(col, y[m], h)
    return out


def test_jacobian_single_absorber_exact(oracle_lib):
    on = oracle_lib.OracleNet(sy.network_stromgren())
    for (F, L) in ((1e11, 0.0), (1e11, 2e18), (5e12, 4e19)):
        y = np.array([40.0, 90.0, 90.0, 1.2e4])
        J = on.jacobian_photo(y, F, L)
        fd = _fd_jacobian(on, y, F, L)
        scale = np.maximum(np.abs(J), 1e-10 * np.abs(J).max())
        assert np.max(np.abs(fd - J) / scale) <= 1e-6, (F, L)


def test_jacobian_cutoff_with_two_absorbers(oracle_lib):
    """With H+ given a cross-section too, the derivative of the
    photoreaction's coefficient in n_i is the exact one times min{1, n_i
    sigma_i / lambda^-1}: the difference to exact differences is
    (1 - cutoff_i) times the exact flux term, column by column."""
    net = sy.network_stromgren(isothermal=True)
    sig = np.array([sy.SIGMA_H, 2.0e-18, 0.0])
    net.sigma_abs = sig
    on = oracle_lib.OracleNet(net)
    F, L = 2e11, 5e18
    y = np.array([40.0, 90.0, 90.0, 1.0e4])
    linv = sig @ y[:3]
    J = on.jacobian_photo(y, F, L)
    fd = _fd_jacobian(on, y, F, L)
    # exact flux term of f_H in column i: -sigma_H n_H dF_eff/dlinv sigma_i
    d = 1e-6 * linv
    dF = (_feff(F, L, linv + d) - _feff(F, L, linv - d)) / (2 * d)
    for i in (0, 1):
        cut = min(1.0, y[i] * sig[i] / linv)
        flux_term = -sy.SIGMA_H * y[0] * dF * sig[i]
        assert cut < 1.0
        np.testing.assert_allclose(fd[0, i] - J[0, i], (1.0 - cut) * flux_term, rtol=1e-6,
                                   atol=1e-9 * abs(flux_term))
    np.testing.assert_allclose(J[:, 2], fd[:, 2], rtol=1e-6, atol=1e-12 * np.abs(J).max())
