"""The FP64 base-2 exponential and logarithm of the rate coefficients
(csrc/kr_math.h), built for the host with g++ and checked against 50-digit
references: relative error bounds, special arguments, and the Arrhenius form
k = 2^(log2 A + b log2 T - C log2(e) / T) against A T^b exp(-C/T) (paper
Sec. 2.1) over the parameter ranges of the synthetic networks."""
import ctypes as C
import os
import subprocess

import mpmath as mp
import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("krmath") / "libkrmath.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-shared", "-fPIC", "-o", out,
                    os.path.join(HERE, "kr_math_host.cpp")], check=True)
    L = C.CDLL(out)
    for f in (L.kr_exp2_host, L.kr_log2_host):
        f.argtypes = [C.c_void_p, C.c_void_p, C.c_long]
        f.restype = None
    return L


def _call(f, x):
    x = np.ascontiguousarray(x, np.float64)
    y = np.empty_like(x)
    f(x.ctypes.data, y.ctypes.data, len(x))
    return y


def test_exp2_relative_error(lib):
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.uniform(-60, 60, 3000), rng.uniform(-0.5, 0.5, 1000),
                        np.arange(-40, 41, dtype=float), np.arange(-40, 41) + 0.5])
    y = _call(lib.kr_exp2_host, x)
    mp.mp.dps = 40
    ref = np.array([float(mp.power(2, mp.mpf(float(v)))) for v in x])
    rel = np.abs(y - ref) / ref
    assert rel.max() < 6e-16, rel.max()
    # integers are exact: the polynomial's value at f = 0 is exactly 1
    xi = np.arange(-1000, 1001, dtype=float)
    assert np.array_equal(_call(lib.kr_exp2_host, xi), np.ldexp(1.0, xi.astype(int)))


def test_exp2_range_ends(lib):
    y = _call(lib.kr_exp2_host, np.array([-1074.0, -1075.5, -3000.0, -1e300, 1023.5, 1024.0, 3000.0, 1e300,
                                          -np.inf, np.inf]))
    assert y[0] == 2.0 ** -1074
    assert y[1] == 0.0 and y[2] == 0.0 and y[3] == 0.0 and y[8] == 0.0
    assert abs(y[4] / (2.0 ** 1023 * np.sqrt(2.0)) - 1.0) < 1e-15
    assert np.isinf(y[5]) and np.isinf(y[6]) and np.isinf(y[7]) and np.isinf(y[9])
    # subnormal results are rounded from the scaled polynomial value
    xs = -1060.0 + np.linspace(-10, 10, 41)
    ys = _call(lib.kr_exp2_host, xs)
    ref = np.array([float(mp.power(2, mp.mpf(float(v)))) for v in xs])
    assert np.all(np.abs(ys - ref) <= 2.0 ** -1074)


def test_log2_relative_error(lib):
    rng = np.random.default_rng(6)
    x = np.concatenate([10.0 ** rng.uniform(-300, 300, 3000), rng.uniform(0.5, 2.0, 2000),
                        1.0 + rng.uniform(-1e-6, 1e-6, 200), [2.0 ** -1074, 2.0 ** -1030, 1.7e308]])
    y = _call(lib.kr_log2_host, x)
    mp.mp.dps = 40
    ref = np.array([float(mp.log(mp.mpf(float(v)), 2)) for v in x])
    err = np.abs(y - ref)
    big = np.abs(ref) > 1e-3
    assert (err[big] / np.abs(ref[big])).max() < 5e-16
    assert err[~big].max() < 1e-18
    # powers of two are exact
    e = np.arange(-1074, 1024)
    assert np.array_equal(_call(lib.kr_log2_host, np.ldexp(1.0, e)), e.astype(float))


def test_log2_invalid_arguments(lib):
    y = _call(lib.kr_log2_host, np.array([0.0, -0.0, -1.0, -np.inf, np.nan, np.inf]))
    assert np.all(np.isnan(y))


def test_arrhenius_form_matches_natural_form(lib):
    """k = A T^b exp(-C/T) from the base-2 form, with log2 A and C log2(e) rounded
    once (as the network compiler writes them), against a 40-digit reference,
    for log10 A ~ U[-12, -8] cm^3/s units, b ~ U[-1, 1], C ~ U[0, 5e4] K and T
    from 10 K to 1e4 K: relative agreement 2e-13 (the same order as the rounding
    of the exponent itself)."""
    rng = np.random.default_rng(7)
    n = 3000
    A = 10.0 ** rng.uniform(-12, -8, n)
    b = rng.uniform(-1, 1, n)
    Cc = rng.uniform(0, 5e4, n)
    T = 10.0 ** rng.uniform(1, 4, n)
    mp.mp.dps = 40
    a2 = np.array([float(mp.log(mp.mpf(float(v)), 2)) for v in A])
    c2 = np.array([float(mp.mpf(float(v)) / mp.log(2)) for v in Cc])
    l2T = _call(lib.kr_log2_host, T)
    iT = 1.0 / T
    x = c2 * 0.0
    for i in range(n):   # the two FMAs of the generated code
        x[i] = float(mp.mpf(float(-c2[i])) * mp.mpf(float(iT[i])) +
                     mp.mpf(float(mp.mpf(float(b[i])) * mp.mpf(float(l2T[i])) + mp.mpf(float(a2[i])))))
    k = _call(lib.kr_exp2_host, x)
    ref = np.array([float(mp.mpf(float(A[i])) * mp.power(mp.mpf(float(T[i])), mp.mpf(float(b[i]))) *
                          mp.exp(-mp.mpf(float(Cc[i])) / mp.mpf(float(T[i])))) for i in range(n)])
    ok = ref > 1e-300
    rel = np.abs(k[ok] - ref[ok]) / ref[ok]
    assert rel.max() < 2e-13, rel.max()
