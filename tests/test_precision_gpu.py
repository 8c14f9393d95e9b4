"""GPU checks of the paper's single- and mixed-precision modes (Sec. 2: the
thermochemistry module runs in full single, full double, or mixed precision,
the latter using FP64 only for the final abundance update of each call),
through the C ABI, against the FP64 oracle.

The FP32 integration takes its own adaptive substep sequence (its error
estimates carry FP32 noise), so each result is compared with the oracle
replaying that cell's logged substep lengths in FP64: the difference is then
the FP32 arithmetic alone.  Its size follows from the arithmetic (unit
roundoff u = 2^-24): (i) each substep rounds the state to FP32 and a stiff
trajectory carries those perturbations forward, at most ~u per substep;
(ii) a rate coefficient 2^x is evaluated from an FP32 exponent x, whose
rounding of ~u |x| is a relative error of ln2 u |x| in the coefficient, and
where a reaction is near balance the abundances follow the ratio of its two
coefficients, off by up to ln2 u (|x_f| + |x_r|).  So per cell
L = max over reactions of |log2 k_f| + |log2 k_r| (the oracle's coefficients
at the cell's initial and final temperatures) and m its accepted substeps
bound the error by a multiple of u (m + L).  Measured on these batches
(major species and T, in units of u (m + L)): at most 4.5 on the
combustion network at dt = 1e-4 s, 0.35 at 1e-7 s; 284 on the astro H/He
network, whose cells reach 10 K and take steps of 1e3 times their fastest
timescale: there coefficients beyond FP32's exponent range (2^-126) vanish
that FP64 keeps, which the model does not count.  Gates:

* species above 1e-4 of the nuclei density, and T: relative error
  <= K_REL u (m + L), K_REL = 16 (combustion) and 1024 (astro H/He);
* every species: absolute error <= K_ABS u (m + L) n_nuc (the roundings of
  the major species and rates reach every species through the coupled
  solve);
* status 0 everywhere; element residual after post-processing <= 1e-12
  (post-processing runs in FP64 in both modes);
* mixed precision adds the FP32 change of the call to the FP64 input: over a
  short step, where most changes are below an FP32 ulp of the abundance, its
  median error on the major species is far below the single mode's (which
  rounds every abundance to FP32 on the way in).

The paper's own check of the mixed mode (the H2/O2 burning test against an
external solver, Sec. 4.2) finds ~1e-3 on the major species and 1e-4 on T;
the FP32 modes here stay within those on the combustion-shaped network.
"""
import numpy as np
import pytest

import synthetic as sy

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
K_REL = {"h_o_n": 16.0, "h_he": 1024.0}
K_ABS = 16.0
MAJOR = 1e-4


def _kr():
    import paper_2504_04941_amd as kr
    return kr


def _dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=dtype)


def _nnuc(desc, n):
    return np.abs(np.asarray(desc.composition)[:desc.n_elem]).sum(axis=0) @ n


def _gpu(desc, cs, precision, dt=None, dt_scalar=0.0, cap=40000, **opt):
    kr = _kr()
    net = kr.Network(desc)
    m = cs.T.shape[0]
    n, T = _dev(cs.n), _dev(cs.T)
    status = torch.full((m,), -7, dtype=torch.int32, device="cuda")
    stats = torch.zeros((m, 4), dtype=torch.int32, device="cuda")
    h_log = torch.zeros((cap, m), dtype=torch.float64, device="cuda")
    h_log_n = torch.zeros(m, dtype=torch.int32, device="cuda")
    kr.chem_integrate(net, n, T, dt=None if dt is None else _dev(dt), dt_scalar=dt_scalar, rtol=1e-6,
                      opts=kr.default_options(precision=precision, **opt), status=status, cell_stats=stats,
                      h_log=h_log, h_log_n=h_log_n)
    torch.cuda.synchronize()
    resid = torch.zeros(m, dtype=torch.float64, device="cuda")
    kr.element_residual(net, _dev(cs.n), n, resid=resid)
    torch.cuda.synchronize()
    out = dict(n=n.cpu().numpy(), T=T.cpu().numpy(), status=status.cpu().numpy(), stats=stats.cpu().numpy(),
               h_log=h_log.cpu().numpy(), h_log_n=h_log_n.cpu().numpy(), resid=resid.cpu().numpy())
    net.close()
    return out


def _replay(oracle, desc, cs, g, dt=None, dt_scalar=0.0):
    on = oracle.OracleNet(desc)
    return on.integrate_ex(cs.n, cs.T, dt=dt, dt_scalar=dt_scalar, opts=oracle.default_opts(rtol=1e-6),
                           replay=np.ascontiguousarray(g["h_log"]), replay_n=g["h_log_n"])


def _rate_exponents(oracle, desc, T0, T1):
    """L per cell: the largest |log2 k_f| + |log2 k_r| over the reactions,
    at the initial and at the final temperature (coefficients that are 0 in
    FP64 count 0)."""
    on = oracle.OracleNet(desc)
    out = np.zeros(T0.size)
    for c in range(T0.size):
        for T in (T0[c], T1[c]):
            kf, kr = on.rate_coeffs(T)
            with np.errstate(divide="ignore"):
                x = np.abs(np.log2(kf)) + np.abs(np.log2(kr))
            x[~np.isfinite(x)] = 0.0
            out[c] = max(out[c], x.max())
    return out


def _errors(oracle, desc, cs, g, r):
    """Per species and cell: relative error (over |replay|) and absolute
    error over n_nuc, both divided by u (m + L); T relative over u (m + L)."""
    nnuc = _nnuc(desc, cs.n)
    L = _rate_exponents(oracle, desc, cs.T, r["T"])
    um = U32 * (np.maximum(g["stats"][:, 0], 1).astype(float) + L)
    d = np.abs(g["n"] - r["n"])
    rel = d / np.maximum(np.abs(r["n"]), 1e-300) / um[None, :]
    ab = d / nnuc[None, :] / um[None, :]
    major = np.abs(r["n"]) > MAJOR * nnuc[None, :]
    trel = np.abs(g["T"] - r["T"]) / r["T"] / um
    return rel, ab, major, trel


def _case(which, ncell):
    if which == "h_he":
        desc = sy.network_h_he(0)
        cs = sy.cells_h_he(desc, ncell, 0)
        return desc, cs, "tau", 0.0
    desc = sy.network_h_o_n(1)
    cs = sy.cells_h_o_n(desc, ncell, 1)
    return desc, cs, None, {"h_o_n_1e-7": 1e-7, "h_o_n_1e-4": 1e-4}[which]


@pytest.mark.parametrize("mode", ["single", "mixed"])
@pytest.mark.parametrize("which", ["h_he", "h_o_n_1e-7", "h_o_n_1e-4"])
def test_fp32_modes_against_fp64_replay(oracle_lib, which, mode):
    kr = _kr()
    ncell = 320
    desc, cs, dt, dts = _case(which, ncell)
    if dt == "tau":
        on = oracle_lib.OracleNet(desc)
        dt = np.array([1e3 * on.fastest_timescale(np.r_[cs.n[:, c], cs.T[c]]) for c in range(ncell)])
    prec = {"single": kr.KR_SINGLE, "mixed": kr.KR_MIXED}[mode]
    g = _gpu(desc, cs, prec, dt=dt, dt_scalar=dts)
    np.testing.assert_array_equal(g["status"], 0)
    np.testing.assert_array_equal(g["h_log_n"], g["stats"][:, 0])
    assert g["resid"].max() <= 1e-12, g["resid"].max()
    r = _replay(oracle_lib, desc, cs, g, dt=dt, dt_scalar=dts)
    np.testing.assert_array_equal(r["status"], 0)
    rel, ab, major, trel = _errors(oracle_lib, desc, cs, g, r)
    worst_rel = max(rel[major].max(), trel.max())
    worst_abs = ab.max()
    print(f"{which} {mode}: major-species/T error {worst_rel:.3g} u (m + L), any species "
          f"{worst_abs:.3g} u (m + L) n_nuc; "
          f"substeps per cell {g['stats'][:, 0].mean():.0f} (max {g['stats'][:, 0].max()})")
    assert worst_rel <= K_REL[which.split("_1e")[0]], worst_rel
    assert worst_abs <= K_ABS, worst_abs


def test_mixed_final_update_keeps_fp64_input(oracle_lib):
    """Short step (1e-10 s, a few substeps): the major species change by
    less than an FP32 ulp in most cells; the mixed mode keeps their FP64
    input values there, the single mode rounds them to FP32."""
    kr = _kr()
    desc = sy.network_h_o_n(1)
    cs = sy.cells_h_o_n(desc, 1000, 1)
    med = {}
    for mode, prec in (("single", kr.KR_SINGLE), ("mixed", kr.KR_MIXED)):
        g = _gpu(desc, cs, prec, dt_scalar=1e-10)
        np.testing.assert_array_equal(g["status"], 0)
        r = _replay(oracle_lib, desc, cs, g, dt_scalar=1e-10)
        nnuc = _nnuc(desc, cs.n)
        major = np.abs(r["n"]) > MAJOR * nnuc[None, :]
        e = np.abs(g["n"] - r["n"])[major] / np.abs(r["n"])[major]
        med[mode] = float(np.median(e))
        L = _rate_exponents(oracle_lib, desc, cs.T, r["T"]).max()
        assert e.max() <= K_REL["h_o_n"] * U32 * (max(int(g["stats"][:, 0].max()), 1) + L)
    print(f"median relative error of the major species: single {med['single']:.3g}, mixed {med['mixed']:.3g}")
    # single: about a quarter of an FP32 ulp (rounding to nearest); mixed:
    # the lost sub-ulp changes, orders of magnitude smaller
    assert med["single"] > 0.05 * U32
    assert med["mixed"] <= 1e-2 * med["single"]


def test_fp32_modes_fixed_steps(oracle_lib):
    """Fixed substep sequence (no error control): both sides take the same
    substeps by construction; same gates.  With no step cut to fall back
    on, an FP32 Newton iteration that stalls above its tolerance fails the
    cell (status 2, input untouched): measured 7 of these 200 cells; the
    others must converge and match."""
    kr = _kr()
    desc = sy.network_h_o_n(1)
    cs = sy.cells_h_o_n(desc, 200, 1)
    for prec in (kr.KR_SINGLE, kr.KR_MIXED):
        g = _gpu(desc, cs, prec, dt_scalar=1e-7, mode=kr.KR_FIXED_STEP, n_fixed=16)
        ok = g["status"] == 0
        assert ok.mean() >= 0.9, np.bincount(g["status"], minlength=3)
        assert np.all(g["status"][~ok] == 2)
        np.testing.assert_array_equal(g["n"][:, ~ok], cs.n[:, ~ok])
        np.testing.assert_array_equal(g["stats"][ok, 0], 16)
        on = oracle_lib.OracleNet(desc)
        o = oracle_lib.default_opts(rtol=1e-6)
        o.mode = oracle_lib.FIXED
        o.n_fixed = 16
        r = on.integrate_ex(cs.n, cs.T, dt_scalar=1e-7, opts=o)
        rel, ab, major, trel = _errors(oracle_lib, desc, cs, g, r)
        assert max(rel[:, ok][major[:, ok]].max(), trel[ok].max()) <= K_REL["h_o_n"]
        assert ab[:, ok].max() <= K_ABS


def test_fp32_modes_rejected_where_unsupported():
    """The FP32 modes run in the lane layout only, and not in several-network
    launches: both are refused with KR_EINVAL before any launch."""
    kr = _kr()
    desc = sy.network_h_o_n(1)
    cs = sy.cells_h_o_n(desc, 8, 1)
    net = kr.Network(desc, kr.build_options(layout=kr.KR_LAYOUT_WAVE))
    n, T = _dev(cs.n), _dev(cs.T)
    for prec in (kr.KR_SINGLE, kr.KR_MIXED):
        with pytest.raises(kr.KrError) as e:
            kr.chem_integrate(net, n, T, dt_scalar=1e-7, rtol=1e-6, opts=kr.default_options(precision=prec))
        assert e.value.code == kr.KR_EINVAL
    net.close()
    np.testing.assert_array_equal(n.cpu().numpy(), cs.n)
    lane = kr.Network(desc)
    with pytest.raises(kr.KrError) as e:
        kr.chem_integrate(lane, n, T, dt_scalar=1e-7, rtol=1e-6, opts=kr.default_options(precision=7))
    assert e.value.code == kr.KR_EINVAL
    lane.close()
