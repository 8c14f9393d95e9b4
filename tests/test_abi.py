"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/kr.h declares, validates descriptions, generates the
network code and compiles it for gfx950 with hipRTC."""
import ctypes
import os
import re

import numpy as np
import pytest

import synthetic as sy

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _kr():
    import paper_2504_04941_amd as kr
    kr.lib()
    return kr


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "kr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(kr_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    kr = _kr()
    names = _declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(kr.lib(), name), name
    assert set(kr.EXPORTED) <= set(names)


def test_defaults():
    kr = _kr()
    o = kr.default_options()
    assert (o.precision, o.mode, o.max_newton, o.max_substeps) == (0, 0, 10, 100000)
    assert o.floor == 1e-20 and o.newton_tol == 1e-3


def test_validation_errors():
    kr = _kr()
    bad = sy.network_h_o_n(1)
    bad.reac = bad.reac.copy()
    bad.reac[3, 0] = bad.reac[3, 1]             # no longer conserves rows
    with pytest.raises(kr.KrError) as e:
        kr.network_check(bad)
    assert e.value.code == kr.KR_EINVAL and "conserve" in str(e.value)
    bad = sy.network_h_he(0)
    bad.reservoir = np.array([1, 4, 3], np.int32)   # H2 carries H but is not single-row? it is; use e-
    bad.reservoir = np.array([3, 4, 3], np.int32)   # e- does not carry the H row
    with pytest.raises(kr.KrError):
        kr.network_check(bad)
    bad = sy.network_h_he(0)
    bad.p_ref = 0.0
    with pytest.raises(kr.KrError):
        kr.network_check(bad)
    bad = sy.network_h_he(0)
    bad.reac = bad.reac.copy()
    bad.reac[0, 0] = 17
    with pytest.raises(kr.KrError):
        kr.network_check(bad)


def test_generated_code_is_straight_line():
    kr = _kr()
    src = kr.network_check(sy.network_h_o_n(1), compile=False)
    assert "#define KR_S 9" in src and "kr_eval" in src
    # one block per reaction, only compile-time indices into the matrix
    assert src.count("/* reaction ") == 24
    body = src.split("const R T = y[KR_S];")[1].split("kr_device.h")[0]
    assert re.search(r"(J|g|y)\[[a-zA-Z_]", body) is None


@pytest.mark.parametrize("ci", [0, 1])
def test_hiprtc_compile_gfx950(ci):
    kr = _kr()
    kr.network_check(sy.network_for(ci), compile=True)


def test_derived_reverse_parameters_match_oracle(oracle_lib):
    """The library and the oracle derive the same reverse Arrhenius table
    (each by its own code) -- checked through the source literal values."""
    kr = _kr()
    desc = sy.network_h_o_n(1)
    src = kr.network_check(desc)
    par = oracle_lib.OracleNet(desc).arrhenius()
    # k = 2^(log2 A + b log2 T - C log2(e) / T): literals -C log2(e), b, log2 A
    lits = re.findall(r"const R kr = kr_exp2\(fma\(R\((\S+)\), iT, fma\(R\((\S+)\), l2T, R\((\S+)\)\)\)\);", src)
    assert len(lits) == desc.n_reactions
    for r, (mc2, b, a2) in enumerate(lits):
        # log2 A is rounded once: A carries ~|log2 A| ulp of relative error
        a2 = float.fromhex(a2)
        assert abs(2.0 ** a2 / par[r, 1, 0] - 1.0) <= 2.5e-16 * (abs(a2) + 1.0)
        assert float.fromhex(b) == par[r, 1, 1]
        np.testing.assert_allclose(-float.fromhex(mc2) / np.log2(np.e), par[r, 1, 2], rtol=1e-15)


def _literals(src, name):
    body = src.split(f"kr_{name}[")[1].split("= {", 1)[1].split("};", 1)[0]
    return np.array([float.fromhex(x) for x in re.findall(r"-?0x[0-9a-fp.+-]+", body)])


def test_generated_heat_capacity_and_table_data():
    """The network compiler carries c_V(T) and the tables into the device
    source: the c_V coefficients as given, the energy's a_k / (k + 1), its
    upper-piece constant making e_s continuous at T_mid, and the table values
    as given (checked on the generated literals, no device needed)."""
    kr = _kr()
    desc = sy.network_h_o_n_tcv()
    src = kr.network_check(desc)
    assert "#define KR_CV_POLY 1" in src and "#define KR_NTAB 4" in src
    S = desc.n_species
    cvp = _literals(src, "cvp").reshape(S, 2, 5)
    np.testing.assert_array_equal(cvp, desc.cv_poly)
    evp = _literals(src, "evp").reshape(S, 2, 6)
    k1 = np.arange(1, 6)
    np.testing.assert_allclose(evp[:, :, :5], desc.cv_poly / k1, rtol=1e-15)
    assert np.all(evp[:, 0, 5] == 0.0)
    Tm = desc.T_mid
    for s in range(S):
        lo = Tm * np.polyval(evp[s, 0, 4::-1], Tm)
        hi = Tm * np.polyval(evp[s, 1, 4::-1], Tm) + evp[s, 1, 5]
        assert abs(lo - hi) <= 1e-12 * abs(lo)
    tab = _literals(src, "tab").reshape(desc.tab_log2k.shape)
    np.testing.assert_array_equal(tab, desc.tab_log2k)
    # a network without them generates neither
    plain = kr.network_check(sy.network_h_o_n(1))
    assert "KR_CV_POLY 1" not in plain and "#define KR_NTAB 0" in plain


def test_invalid_heat_capacity_and_tables_rejected():
    kr = _kr()
    for mutate in (lambda d: setattr(d, "T_mid", 0.0),
                   lambda d: d.cv_poly.__setitem__((0, 0, 0), np.nan),
                   lambda d: d.tab_of.__setitem__(3, 9),
                   lambda d: d.tab_log2k.__setitem__((0, 0), np.inf),
                   lambda d: setattr(d, "tab_dlog2T", -1.0)):
        desc = sy.network_h_o_n_tcv()
        mutate(desc)
        with pytest.raises(kr.KrError) as e:
            kr.network_check(desc)
        assert e.value.code == kr.KR_EINVAL


def test_photoreaction_code_and_validation():
    """The network compiler emits the effective-flux evaluation, one cutoff
    per absorber and the photoreaction's coefficient A F_eff (no reverse
    direction), and refuses inconsistent photoreaction data."""
    kr = _kr()
    desc = sy.network_stromgren()
    src = kr.network_check(desc)
    assert "#define KR_PHOTO 1" in src and "kr_photo_flux(phF, phL, linv, Fe, dFe);" in src
    assert src.count("const R cut") == 1                  # H is the only absorber
    block = src.split("/* reaction 0 */")[1].split("/* reaction 1 */")[0]
    assert "* Fe;" in block and "const R kr " not in block
    assert float.fromhex(re.search(r"const R kf = R\((\S+)\) \* Fe;", block).group(1)) == sy.SIGMA_H
    # extra heat: reaction 2 carries q0 + q1 T + q2 T ln T
    assert "const R qx" in src.split("/* reaction 2 */")[1]
    plain = kr.network_check(sy.network_h_o_n(1))
    assert "KR_PHOTO 1" not in plain
    for mutate in (lambda d: setattr(d, "sigma_abs", None),
                   lambda d: d.arr_f.__setitem__((0, 1), 0.5),
                   lambda d: d.photo.__setitem__(1, 2),
                   lambda d: d.heat_extra.__setitem__((2, 0), np.inf)):
        bad = sy.network_stromgren()
        bad.arr_f = bad.arr_f.copy()
        mutate(bad)
        with pytest.raises(kr.KrError) as e:
            kr.network_check(bad)
        assert e.value.code == kr.KR_EINVAL


def test_automatic_layout_keeps_lane_only_terms_in_the_lane_layout():
    """Photoreactions and extra heat terms exist in the lane layout only: the
    automatic layout keeps such a network one cell per lane at any size (a
    23-species network with extra heat compiles there), while the same
    network without them goes to 32-lane groups; forcing another layout is
    refused."""
    kr = _kr()
    desc = sy.network_astro23(2)
    assert "one cell per lane group" in kr.network_check(desc)
    desc.heat_extra = np.zeros((desc.n_reactions, 3))
    desc.heat_extra[0] = (10.0, 0.0, 0.0)
    src = kr.network_check(desc)
    assert "network-specialised device code" in src and "const R qx" in src
    for L in (kr.KR_LAYOUT_WAVE, kr.KR_LAYOUT_GROUP32):
        with pytest.raises(kr.KrError) as e:
            kr.network_check(desc, build=kr.build_options(layout=L))
        assert e.value.code == kr.KR_EINVAL
