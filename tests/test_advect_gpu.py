"""GPU parity of the stoichiometry-compatible PLM advection (kr_advect_plm)
against the FP64 reference (oracle/plm.py), through the C ABI:

* one stage, every mode (projected PLM, plain PLM, donor cell), on seeded
  lines of three networks (4, 9 and 48 species), non-uniform grids, varying
  density, both flow directions, lines of 128 cells and a ragged 77-cell
  line (partial chunk), with a line stride and leading dimension larger than
  the batch: element by element within 1e-13 of the largest abundance of the
  line (the same arithmetic up to fused multiply-adds and the association of
  dt / dx);
* the advection test of Sec. 4.1 on the GPU (one period, SSP-RK2 from two
  stages per step): the element abundances of every cell stay at their exact
  values to machine precision with the projection (<= 1e-14; the paper
  reports <~1e-15), drift by ~1e-3 without it, and the profiles equal the
  oracle's run;
* the element fluxes of the projected stage are proportional to the mass
  flux: the stage leaves each cell's element abundances per mass unchanged;
* the fused SSP-RK2 step (kr_advect_plm_ssprk2), register and LDS forms,
  bit for bit against the two stage calls and within 1e-13 of the oracle's
  step, the test of Sec. 4.1 with it, and its refusals.
"""
import numpy as np
import pytest

import synthetic as sy
from oracle import plm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _kr():
    import paper_2504_04941_amd as kr
    return kr


_NETS = {}


def _net(which):
    """One network per description for the whole module (creating one
    compiles its module); closed when the module's tests end."""
    if which not in _NETS:
        desc = {"e1": sy.network_e1(), "h_he": sy.network_h_he(0), "h_o_n": sy.network_h_o_n(1),
                "astro23": sy.network_astro23(2), "large48": sy.network_large48(3)}[which]
        _NETS[which] = (_kr().Network(desc), desc)
    return _NETS[which]


@pytest.fixture(scope="module", autouse=True)
def _close_networks():
    yield
    for net, _ in _NETS.values():
        net.close()
    _NETS.clear()


def _dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=torch.float64)


def _face_flux(rho, v, n_lines, n_cells):
    """Mass flux through each cell's left face: upwind density times v."""
    F = np.empty(n_lines * n_cells)
    for l in range(n_lines):
        r = rho[l * n_cells:(l + 1) * n_cells]
        F[l * n_cells:(l + 1) * n_cells] = (np.roll(r, 1) if v[l] > 0 else r) * v[l]
    return F


MODES = [(1, "projected"), (0, "plain"), (2, "donor")]


@pytest.mark.parametrize("which", ["e1", "h_o_n", "large48"])
@pytest.mark.parametrize("n_cells", [128, 77])
@pytest.mark.parametrize("mode,label", MODES)
def test_stage_matches_oracle(which, n_cells, mode, label):
    kr = _kr()
    net, desc = _net(which)
    n_lines = 6
    n, rho, xc, xf, v = sy.advection_lines(desc, n_lines, n_cells)
    F = _face_flux(rho, v, n_lines, n_cells)
    dt = 0.3 * np.min(np.diff(xf))
    S = desc.n_species
    stride, ld = n_cells + 5, n_lines * (n_cells + 5) + 3
    n_in = np.zeros((S, ld))
    base = np.zeros((S, ld))
    rho_p, F_p = np.ones(ld), np.zeros(ld)
    rng = np.random.default_rng(3)
    for l in range(n_lines):
        sl = slice(l * n_cells, (l + 1) * n_cells)
        dl = slice(l * stride, l * stride + n_cells)
        n_in[:, dl] = n[:, sl]
        base[:, dl] = n[:, sl] * rng.uniform(0.9, 1.1, (S, n_cells))
        rho_p[dl] = rho[sl]
        F_p[dl] = F[sl]
    out = torch.full((S, ld), -9.0, dtype=torch.float64, device="cuda")
    kr.advect_plm(net, _dev(n_in), out, _dev(rho_p), _dev(F_p), _dev(xc), _dev(xf), dt, n_lines=n_lines,
                  line_stride=stride, base=_dev(base), alpha=0.25, beta=0.75, mode=mode)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    P = plm.projector_svd(desc.composition) if mode == 1 else None
    for l in range(n_lines):
        sl = slice(l * n_cells, (l + 1) * n_cells)
        dl = slice(l * stride, l * stride + n_cells)
        ref, _ = plm.stage(n[:, sl], rho[sl], F[sl], xc, xf, dt, P, limit=mode != 2)
        want = 0.25 * base[:, dl] + 0.75 * ref
        scale = np.abs(n[:, sl]).max()
        err = np.abs(got[:, dl] - want).max() / scale
        assert err <= 1e-13, (l, err)
        # cells outside the lines are not written
        if l + 1 < n_lines:
            assert np.all(got[:, l * stride + n_cells:(l + 1) * stride] == -9.0)


def _gpu_e1(kr, net, n_cells, mode):
    xc, xf = sy.uniform_grid(n_cells)
    n0 = sy.e1_initial(xc)
    dt = 0.4 * (xf[1] - xf[0])
    steps = int(round(1.0 / dt))
    dt = 1.0 / steps
    u0 = _dev(n0)
    u1 = torch.empty_like(u0)
    rho = torch.ones(n_cells, dtype=torch.float64, device="cuda")
    F = torch.ones(n_cells, dtype=torch.float64, device="cuda")
    xcd, xfd = _dev(xc), _dev(xf)
    u = u0.clone()
    for _ in range(steps):
        kr.advect_plm(net, u, u1, rho, F, xcd, xfd, dt, mode=mode)
        kr.advect_plm(net, u1, u0, rho, F, xcd, xfd, dt, base=u, alpha=0.5, beta=0.5, mode=mode)
        u, u0 = u0, u
    torch.cuda.synchronize()
    return n0, u.cpu().numpy(), steps


def test_e1_advection_test_on_gpu():
    kr = _kr()
    net, _ = _net("e1")
    comp = plm.E1_COMP
    n0, u, steps = _gpu_e1(kr, net, 128, kr.ADVECT_PROJECTED)
    E0 = comp @ n0
    err = np.max(np.abs(comp @ u - E0) / E0)
    assert err <= 1e-14, err
    # the oracle's run of the same test
    xc, xf = sy.uniform_grid(128)
    s, r = n0.copy(), np.ones(128)
    P = plm.projector_svd(comp)
    for _ in range(steps):
        s, r = plm.ssp_rk2(s, r, 1.0, xc, xf, 1.0 / steps, P)
    assert np.max(np.abs(u - s)) <= 1e-12
    # without the projection element A drifts (paper: ~1e-3)
    _, u_plain, _ = _gpu_e1(kr, net, 128, kr.ADVECT_PLAIN)
    drift = np.max(np.abs(comp @ u_plain - E0)[0] / E0[0])
    assert 1e-4 < drift < 3e-2, drift


@pytest.mark.parametrize("which", ["h_o_n", "large48"])
def test_projected_stage_keeps_element_abundances(which):
    """With uniform element abundances per mass along each line, a projected
    stage keeps every cell's element abundances per mass (the fluxes carry
    elements in proportion to mass) to rounding."""
    kr = _kr()
    net, desc = _net(which)
    n_lines, n_cells = 8, 256
    n, rho, xc, xf, v = sy.advection_lines(desc, n_lines, n_cells)
    F = _face_flux(rho, v, n_lines, n_cells)
    dt = 0.4 * np.min(np.diff(xf))
    out = torch.empty((desc.n_species, n_lines * n_cells), dtype=torch.float64, device="cuda")
    kr.advect_plm(net, _dev(n), out, _dev(rho), _dev(F), _dev(xc), _dev(xf), dt, n_lines=n_lines)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    comp = np.asarray(desc.composition, np.float64)
    # the density after the same mass fluxes
    rho2 = np.empty_like(rho)
    dx = np.diff(xf)
    for l in range(n_lines):
        sl = slice(l * n_cells, (l + 1) * n_cells)
        Fl = F[sl]
        rho2[sl] = rho[sl] - dt / dx * (np.roll(Fl, -1) - Fl)
    e_before = comp @ (n / rho[None, :])
    e_after = comp @ (got / rho2[None, :])
    assert np.max(np.abs(e_after - e_before) / np.abs(e_before).max(axis=1, keepdims=True)) <= 1e-13


def _stage_density(rho, F, xf, n_lines, n_cells, dt):
    """The first stage's density (the caller's update by the same mass
    fluxes), line by line."""
    dx = np.diff(xf)
    out = np.empty_like(rho)
    for l in range(n_lines):
        sl = slice(l * n_cells, (l + 1) * n_cells)
        out[sl] = rho[sl] - dt / dx * (np.roll(F[sl], -1) - F[sl])
    return out


FUSED_CASES = [(w, n, False) for w in ("e1", "h_he", "h_o_n") for n in (128, 77, 56, 57, 4)] + \
    [("h_o_n", 128, True), ("e1", 57, True), ("h_he", 4, True)] + \
    [(w, n, False) for w in ("astro23", "large48") for n in (128, 77, 64, 65, 4)] + \
    [("astro23", 128, True), ("large48", 65, True)]


@pytest.mark.parametrize("which,n_cells,flip", FUSED_CASES)
@pytest.mark.parametrize("mode,label", MODES)
def test_fused_step_matches_two_stages_and_oracle(which, n_cells, flip, mode, label):
    """kr_advect_plm_ssprk2 against the two kr_advect_plm stages it fuses
    (bit for bit) and the oracle's SSP-RK2 step (within 1e-13 of the line's
    largest abundance), with the density evolving through the step, lines
    one chunk long, one cell over, ragged and of the minimum 4 cells, a line
    stride and leading dimension larger than the batch; the register form
    (4, 5, 9 and 23 species: 56-cell chunks) and the LDS form (48 species:
    64-cell chunks); flip: the second stage's mass flux reversed at
    a random third of the faces (the upwind cell, hence the face geometry,
    changes between the stages)."""
    kr = _kr()
    net, desc = _net(which)
    n_lines = 5
    n, rho, xc, xf, v = sy.advection_lines(desc, n_lines, n_cells)
    dt = 0.3 * np.min(np.diff(xf))
    F0 = _face_flux(rho, v, n_lines, n_cells)
    rho1 = _stage_density(rho, F0, xf, n_lines, n_cells, dt)
    F1 = _face_flux(rho1, v, n_lines, n_cells)
    if flip:
        F1 = np.where(np.random.default_rng(11).uniform(size=F1.size) < 1 / 3, -F1, F1)
    S = desc.n_species
    stride, ld = n_cells + 3, n_lines * (n_cells + 3) + 5

    def spread(a, fill):
        out = np.full(a.shape[:-1] + (ld,), fill)
        for l in range(n_lines):
            out[..., l * stride:l * stride + n_cells] = a[..., l * n_cells:(l + 1) * n_cells]
        return out
    print(f"fused advection {which} n_cells={n_cells} flip={flip} mode={label}", flush=True)
    n_d = _dev(spread(n, 0.0))
    r0, f0, r1, f1 = (_dev(spread(a, 1.0 if i % 2 == 0 else 0.0)) for i, a in enumerate((rho, F0, rho1, F1)))
    xcd, xfd = _dev(xc), _dev(xf)
    fused = torch.full((S, ld), -9.0, dtype=torch.float64, device="cuda")
    kr.advect_plm_ssprk2(net, n_d, fused, r0, f0, r1, f1, xcd, xfd, dt, n_lines=n_lines, line_stride=stride,
                         mode=mode)
    u1 = torch.full_like(fused, -9.0)
    two = torch.full_like(fused, -9.0)
    kr.advect_plm(net, n_d, u1, r0, f0, xcd, xfd, dt, n_lines=n_lines, line_stride=stride, mode=mode)
    kr.advect_plm(net, u1, two, r1, f1, xcd, xfd, dt, n_lines=n_lines, line_stride=stride, base=n_d, alpha=0.5,
                  beta=0.5, mode=mode)
    torch.cuda.synchronize()
    got = fused.cpu().numpy()
    P = plm.projector_svd(desc.composition) if mode == 1 else None
    for l in range(n_lines):
        sl = slice(l * n_cells, (l + 1) * n_cells)
        dl = slice(l * stride, l * stride + n_cells)
        a1, _ = plm.stage(n[:, sl], rho[sl], F0[sl], xc, xf, dt, P, limit=mode != 2)
        a2, _ = plm.stage(a1, rho1[sl], F1[sl], xc, xf, dt, P, limit=mode != 2)
        want = 0.5 * (n[:, sl] + a2)
        err = np.abs(got[:, dl] - want).max() / np.abs(n[:, sl]).max()
        assert err <= 1e-13, (l, err)
        # cells outside the lines are not written
        assert np.all(got[:, l * stride + n_cells:(l + 1) * stride] == -9.0)
    assert np.all(got[:, n_lines * stride:] == -9.0)
    diff = np.abs(got - two.cpu().numpy())
    assert torch.equal(fused, two), (int(np.count_nonzero(diff)), float(diff.max()))


def test_fused_step_e1_advection_test():
    """The test of Sec. 4.1 with the fused step: the same profiles as two
    stages per step bit for bit, element abundances exact to <= 1e-14."""
    kr = _kr()
    net, _ = _net("e1")
    n0, u_two, steps = _gpu_e1(kr, net, 128, kr.ADVECT_PROJECTED)
    xc, xf = sy.uniform_grid(128)
    a, b = _dev(n0), torch.empty_like(_dev(n0))
    rho = torch.ones(128, dtype=torch.float64, device="cuda")
    F = torch.ones(128, dtype=torch.float64, device="cuda")
    for _ in range(steps):
        kr.advect_plm_ssprk2(net, a, b, rho, F, rho, F, _dev(xc), _dev(xf), 1.0 / steps)
        a, b = b, a
    torch.cuda.synchronize()
    u = a.cpu().numpy()
    np.testing.assert_array_equal(u, u_two)
    E0 = plm.E1_COMP @ n0
    assert np.max(np.abs(plm.E1_COMP @ u - E0) / E0) <= 1e-14


def test_fused_step_refusals():
    """Lines under 4 cells, aliasing, a bad mode, a non-finite step: the
    host refuses them before any launch; empty batches are no-ops."""
    kr = _kr()
    r = torch.ones(64, dtype=torch.float64, device="cuda")
    xc, xf = _dev(np.linspace(0.5 / 64, 1 - 0.5 / 64, 64)), _dev(np.linspace(0, 1, 65))
    net, _ = _net("h_o_n")
    d = torch.ones((9, 64), dtype=torch.float64, device="cuda")
    o = torch.full_like(d, -9.0)
    for args, kw in (((d, o, r[:3], r[:3], r[:3], r[:3], xc[:3], xf[:4], 1e-3), {}),
                     ((d, d, r, r, r, r, xc, xf, 1e-3), {}),
                     ((d, o, r, r, r, r, xc, xf, 1e-3), {"mode": 3}),
                     ((d, o, r, r, r, r, xc, xf, float("nan")), {})):
        with pytest.raises(kr.KrError) as e:
            kr.advect_plm_ssprk2(net, *args, **kw)
        assert e.value.code == kr.KR_EINVAL
    kr.advect_plm_ssprk2(net, d, o, r, r, r, r, xc, xf, 1e-3, n_lines=0)
    torch.cuda.synchronize()
    assert torch.all(o == -9.0)
