"""Host-side checks of the wavefront and lane-group layouts' generated
tables (no GPU):
the per-lane contribution lists rebuild exactly the rate-Jacobian terms the
network implies, every destination entry is owned by one lane and closed by
a flush mark, and the direction tables hold the derived Arrhenius
parameters of every reaction direction."""
import re
from collections import defaultdict

import numpy as np
import pytest

import synthetic as sy


def _kr():
    import paper_2504_04941_amd as kr
    kr.lib()
    return kr


def _tables(src):
    def arr(name, conv):
        m = re.search(r"kr_%s\[(\d+)\] = \{([^}]*)\}" % name, src)
        return [conv(x) for x in m.group(2).split(",")]
    defs = {k: int(v) for k, v in re.findall(r"#define KR_(S|LDJ|NDR|NC|NF) (\d+)", src)}
    u = lambda x: int(x.rstrip("u"))
    return defs, {n: arr(n, u) for n in ("dr", "wc", "wf")}, {n: arr(n, float.fromhex) for n in ("da2", "db", "dE")}


def _expected(desc, par, S, LDJ):
    """(destination -> sorted list of (source, nu)) from the network."""
    full, fonly = defaultdict(list), defaultdict(list)
    dirs = []
    for r in range(desc.n_reactions):
        for d, (re_, pr_) in enumerate(((desc.reac[r], desc.prod[r]), (desc.prod[r], desc.reac[r]))):
            if par[r, d, 0] == 0.0:
                continue
            dirs.append((r, d, [int(x) for x in re_], [int(x) for x in pr_]))
    for i, (r, d, re_, pr_) in enumerate(dirs):
        nu = np.zeros(S, int)
        for s in re_:
            if s >= 0:
                nu[s] -= 1
        for s in pr_:
            if s >= 0:
                nu[s] += 1
        for s in np.nonzero(nu)[0]:
            full[s * LDJ + S + 1].append((5 * i, int(nu[s])))
            fonly[s * LDJ + S + 1].append((5 * i, int(nu[s])))
            full[s * LDJ + S].append((5 * i + 1, int(nu[s])))
            for k, m in enumerate(re_):
                if m >= 0:
                    full[s * LDJ + m].append((5 * i + 2 + k, int(nu[s])))
    return dirs, full, fonly


def _decode(tab, length, lanes=64):
    got, owner = defaultdict(list), {}
    for lane in range(lanes):
        open_dst = None
        for i in range(length):
            e = tab[i * lanes + lane]
            src, dst, nu, fl = e & 4095, (e >> 12) & 8191, ((e >> 25) & 7) - 4, e >> 28
            if nu == 0 and not fl:
                continue                       # padding
            assert owner.setdefault(dst, lane) == lane, "destination split over lanes"
            assert open_dst in (None, dst)
            got[dst].append((src, nu))
            open_dst = None if fl else dst
        assert open_dst is None, "list ends without a flush"
    return got


@pytest.mark.parametrize("make", [lambda: sy.network_h_o_n(1), lambda: sy.network_astro23(2),
                                  lambda: sy.network_large48(3)])
def test_contribution_lists_rebuild_the_jacobian_terms(oracle_lib, make):
    kr = _kr()
    desc = make()
    src = kr.network_check(desc, build=kr.build_options(layout=kr.KR_LAYOUT_WAVE))
    defs, ut, dt = _tables(src)
    S, LDJ = defs["S"], defs["LDJ"]
    assert LDJ % 2 == 1 and LDJ >= S + 2
    par = oracle_lib.OracleNet(desc).arrhenius()
    dirs, full, fonly = _expected(desc, par, S, LDJ)
    assert defs["NDR"] == (len(dirs) + 63) // 64
    got = _decode(ut["wc"], defs["NC"])
    assert {k: sorted(v) for k, v in got.items()} == {k: sorted(v) for k, v in full.items()}
    gotf = _decode(ut["wf"], defs["NF"])
    assert {k: sorted(v) for k, v in gotf.items()} == {k: sorted(v) for k, v in fonly.items()}
    # lists are balanced: no lane longer than the largest entry or the mean,
    # rounded up to the gather's chunk of eight entries
    terms = sum(len(v) for v in full.values())
    bound = max(max(len(v) for v in full.values()), -(-terms // 64) + 8)
    assert defs["NC"] % 8 == 0 and defs["NF"] % 8 == 0
    assert defs["NC"] <= -(-bound // 8) * 8
    # direction tables: derived (log2 A, b, E) and reactant slots, padding
    # inert (log2 A = -4096, i.e. k = 0)
    for i, (r, d, re_, _) in enumerate(dirs):
        a2 = dt["da2"][i]
        assert abs(2.0 ** a2 / par[r, d, 0] - 1.0) <= 2.5e-16 * (abs(a2) + 1.0)
        np.testing.assert_allclose([dt["db"][i], dt["dE"][i]], par[r, d, 1:], rtol=1e-15)
        slots = [(ut["dr"][i] >> (8 * k)) & 255 for k in range(3)]
        assert slots == [m if m >= 0 else 63 for m in re_]   # 63: an empty slot (reads 1.0)
    assert all(a == -4096.0 for a in dt["da2"][len(dirs):])


@pytest.mark.parametrize("make,G", [(lambda: sy.network_h_o_n(1), 16), (lambda: sy.network_h_o_n(1), 32),
                                    (lambda: sy.network_astro23(2), 32), (lambda: sy.network_h_he(0), 16)])
def test_group_lists_rebuild_the_jacobian_terms(oracle_lib, make, G):
    """Lane-group layout: contribution lists balanced over G lanes rebuild
    the same Jacobian terms; reactant slots with the empty slot at the
    group's spare lane G - 1; direction rounds of G."""
    kr = _kr()
    desc = make()
    src = kr.network_check(desc, build=kr.build_options(layout=kr.KR_LAYOUT_GROUP16 if G == 16
                                                              else kr.KR_LAYOUT_GROUP32))
    defs = {k: int(v) for k, v in re.findall(r"#define KR_(S|LDJ|G|GNDR|GNC|GNF) (\d+)", src)}
    assert defs["G"] == G and defs["S"] + 2 <= G

    def arr(name):
        m = re.search(r"kr_%s\[(\d+)\] = \{([^}]*)\}" % name, src)
        return [int(x.rstrip("u")) for x in m.group(2).split(",")]
    S, LDJ = defs["S"], defs["LDJ"]
    par = oracle_lib.OracleNet(desc).arrhenius()
    dirs, full, fonly = _expected(desc, par, S, LDJ)
    assert defs["GNDR"] == max(1, -(-len(dirs) // G))
    got = _decode(arr("gc"), defs["GNC"], G)
    assert {k: sorted(v) for k, v in got.items()} == {k: sorted(v) for k, v in full.items()}
    gotf = _decode(arr("gf"), defs["GNF"], G)
    assert {k: sorted(v) for k, v in gotf.items()} == {k: sorted(v) for k, v in fonly.items()}
    assert max(full) < (S + 1) * LDJ               # destinations inside the block's Jacobian
    gdr = arr("gdr")
    assert len(gdr) == defs["GNDR"] * G
    for i in range(len(gdr)):
        re_ = dirs[i][2] if i < len(dirs) else [-1, -1, -1]
        assert [(gdr[i] >> (8 * k)) & 255 for k in range(3)] == [m if m >= 0 else G - 1 for m in re_]


def test_group_layout_limits_and_compiles():
    kr = _kr()
    for G, L in ((16, kr.KR_LAYOUT_GROUP16), (32, kr.KR_LAYOUT_GROUP32)):
        with pytest.raises(kr.KrError) as e:
            kr.network_check(sy.network_large48(3) if G == 32 else sy.network_astro23(2),
                             build=kr.build_options(layout=L))
        assert e.value.code == kr.KR_EINVAL
    src = kr.network_check(sy.network_astro23(2), compile=True, build=kr.build_options(layout=kr.KR_LAYOUT_GROUP32))
    assert "one cell per lane group" in src
    with pytest.raises(kr.KrError):
        kr.network_check(sy.network_h_he(0), build=kr.build_options(layout=5))


def test_wave_layout_compiles_for_gfx950():
    kr = _kr()
    kr.network_check(sy.network_h_o_n(1), compile=True, build=kr.build_options(layout=kr.KR_LAYOUT_WAVE))


def test_wave_layout_limits():
    kr = _kr()
    with pytest.raises(kr.KrError):
        kr.network_check(sy.network_h_o_n(1), build=kr.build_options(layout=7))


def test_automatic_occupancy_target():
    """waves_per_eu = 0: one wave per SIMD for the lane layout, two for a
    wavefront network whose LDS block leaves room for them (23 species,
    11 KB), one where it does not (48 species, 39 KB of the 40 KB share of
    a SIMD); an explicit value is kept."""
    kr = _kr()

    def waves(desc, **kw):
        src = kr.network_check(desc, build=kr.build_options(**kw))
        return int(re.search(r"#define KR_WAVES_PER_EU (\d+)", src).group(1))

    assert kr.build_options().waves_per_eu == 0
    assert waves(sy.network_h_o_n(1)) == 1
    assert waves(sy.network_astro23(2)) == 2
    assert waves(sy.network_large48(3)) == 1
    assert waves(sy.network_h_o_n(1), layout=kr.KR_LAYOUT_WAVE) == 2
    assert waves(sy.network_astro23(2), waves_per_eu=3) == 3
    assert waves(sy.network_astro23(2), layout=kr.KR_LAYOUT_LANE) == 1
    # one kernel for several networks takes the smallest choice
    src = kr.multi_check([sy.network_astro23(2), sy.network_large48(3)])
    assert "#define KR_WAVES_PER_EU 1" in src
    with pytest.raises(kr.KrError):
        kr.network_check(sy.network_h_o_n(1), build=kr.build_options(waves_per_eu=9))


def test_multi_kernels_grouped_by_occupancy_target():
    """Several networks: lane- and wavefront-layout networks with different
    automatic targets get a kernel each; networks that share a target, one."""
    kr = _kr()

    def kernels(descs):
        src = kr.multi_check(descs)
        return re.findall(r"__launch_bounds__\(64, (\d+)\) kr_integrate_multi_fp64_(\d+)", src)

    assert kernels([sy.network_h_he(0), sy.network_h_o_n(1), sy.network_astro23(2)]) == [("1", "0"), ("2", "1")]
    assert kernels([sy.network_h_he(0), sy.network_h_o_n(1)]) == [("1", "0")]
    assert kernels([sy.network_astro23(2), sy.network_large48(3)]) == [("1", "0")]
    assert kernels([sy.network_astro23(2)]) == [("2", "0")]


def test_fp32_math_overloads_outside_network_namespaces():
    """The FP32 overloads of kr_exp2 / kr_log2 are declared once, at global
    scope beside the FP64 ones: declared inside a network's namespace of a
    several-network source, they would hide the FP64 overloads there and turn
    every FP64 rate coefficient into an FP32 one."""
    kr = _kr()
    descs = [sy.network_h_he(0), sy.network_h_o_n_tcv(), sy.network_astro23(2)]
    for src in (kr.multi_check(descs), kr.network_check(descs[1])):
        first_ns = src.find("namespace kr_m")
        for f in ("float kr_exp2(float", "float kr_log2(float"):
            assert src.count(f) == 1, f
            assert first_ns < 0 or src.index(f) < first_ns, f
        assert src.index("double kr_exp2(double") < src.index("float kr_exp2(float")


def test_blocked_lu_build_option():
    """lu_mfma=1 selects the blocked FP32 LU (MFMA trailing updates) where it
    applies -- the 48-species network in the wavefront layout -- and is
    ignored elsewhere; the blocked source compiles for gfx950."""
    kr = _kr()
    src = kr.network_check(sy.network_large48(3), compile=True, build=kr.build_options(lu_mfma=1))
    assert "#define KR_LU_MFMA 1" in src
    assert "#define KR_LU_MFMA 1" not in kr.network_check(sy.network_large48(3))
    assert "#define KR_LU_MFMA 1" not in kr.network_check(sy.network_astro23(2),
                                                          build=kr.build_options(lu_mfma=1))
    with pytest.raises(kr.KrError):
        kr.network_check(sy.network_large48(3), build=kr.build_options(lu_mfma=2))
