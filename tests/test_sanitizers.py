"""Sanitizer builds of the host code (no GPU): the FP64 oracle (with its
stand-alone driver oracle/kr_oracle_check.c) and the host build of the
rate-coefficient math, compiled with AddressSanitizer and
UndefinedBehaviorSanitizer (-fno-sanitize-recover: any finding stops the
run), run on the synthetic networks, and their results compared with the
ordinary builds."""
import os
import subprocess

import numpy as np
import pytest

import synthetic as sy

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")
ENV.pop("LD_PRELOAD", None)


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("san") / "kr_oracle_check")
    subprocess.run(["gcc", "-O1", "-std=c11", *SAN, "-o", exe,
                    os.path.join(ROOT, "oracle", "kr_oracle.c"),
                    os.path.join(ROOT, "oracle", "kr_oracle_check.c"), "-lm"], check=True)
    return exe


def _write(path, desc, n, T, dt):
    S, R = desc.n_species, desc.n_reactions
    with open(path, "wb") as f:
        np.array([S, desc.n_rows, desc.n_elem, R, T.shape[0], desc.arr_r is not None],
                 np.int32).tofile(f)
        for a in (desc.composition, desc.reservoir, desc.reac, desc.prod):
            np.ascontiguousarray(a, np.int32).tofile(f)
        for a in (desc.cv, desc.h_form, desc.s_form, desc.arr_f):
            np.ascontiguousarray(a, np.float64).tofile(f)
        if desc.arr_r is not None:
            np.ascontiguousarray(desc.arr_r, np.float64).tofile(f)
        np.array([desc.p_ref, desc.T_min, desc.T_max], np.float64).tofile(f)
        for a in (n, T, dt):
            np.ascontiguousarray(a, np.float64).tofile(f)


CASES = {
    "h_he": (lambda: sy.network_h_he(0), lambda d: sy.cells_h_he(d, 48, 0), 1e-9),
    "h_o_n": (lambda: sy.network_h_o_n(1), lambda d: sy.cells_h_o_n(d, 12, 1), 2e-8),
    "astro23": (lambda: sy.network_astro23(2), lambda d: sy.cells_astro23(d, 8, 2), 1e3),
    "large48": (lambda: sy.network_large48(3), lambda d: sy.cells_large48(d, 4, 3), 1e-9),
}


@pytest.mark.parametrize("name", list(CASES))
def test_oracle_under_sanitizers(oracle_lib, checker, tmp_path, name):
    mk_net, mk_cells, dt_s = CASES[name]
    desc = mk_net()
    cs = mk_cells(desc)
    nc = cs.T.shape[0]
    dt = np.full(nc, dt_s)
    inp, out = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    _write(inp, desc, cs.n, cs.T, dt)
    r = subprocess.run([checker, inp, out], env=ENV, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    S = desc.n_species
    raw = open(out, "rb").read()
    got_n = np.frombuffer(raw, np.float64, S * nc).reshape(S, nc)
    got_T = np.frombuffer(raw, np.float64, nc, offset=8 * S * nc)
    off = 8 * (S * nc + 3 * nc)
    got_st = np.frombuffer(raw, np.int32, nc, offset=off)
    # the sanitized build computes the same results as the ordinary one
    on = oracle_lib.OracleNet(desc)
    ref = on.integrate_ex(cs.n, cs.T, dt=dt, nthreads=1)
    np.testing.assert_array_equal(got_st, ref["status"])
    np.testing.assert_array_equal(got_n, ref["n"])
    np.testing.assert_array_equal(got_T, ref["T"])


def test_rate_math_under_sanitizers(tmp_path):
    main = tmp_path / "main.cpp"
    main.write_text(
        '#include "' + os.path.join(ROOT, "tests", "kr_math_host.cpp") + '"\n'
        "#include <cstdio>\n#include <cmath>\n"
        "int main() {\n  double x[4001], y[4001], z[4001];\n"
        "  for (int i = 0; i <= 4000; ++i) x[i] = -1100.0 + 0.55 * i;\n"
        "  kr_exp2_host(x, y, 4001);\n"
        "  for (int i = 0; i <= 4000; ++i) x[i] = std::ldexp(1.0 + 0.00025 * i, i % 200 - 100);\n"
        "  kr_log2_host(x, z, 4001);\n"
        "  double s = 0; for (int i = 0; i <= 4000; ++i) s += std::isfinite(y[i]) ? y[i] * 1e-300 : 0.0;\n"
        "  for (int i = 0; i <= 4000; ++i) s += z[i];\n"
        "  std::printf(\"%.17g\\n\", s);\n  return 0;\n}\n")
    exe = str(tmp_path / "math")
    subprocess.run(["g++", "-O1", "-std=c++17", "-ffp-contract=off", *SAN, "-o", exe, str(main)], check=True)
    r = subprocess.run([exe], env=ENV, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "runtime error" not in r.stderr, r.stderr[-3000:]
    assert np.isfinite(float(r.stdout.strip()))
