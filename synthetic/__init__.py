"""Seeded synthetic reaction networks and cell states.

This module only *describes* inputs: species, their element/charge
composition, reaction lists with forward Arrhenius parameters, species
thermodynamic data and per-cell initial states.  It contains none of the
integration method's arithmetic (no rate evaluation, no reverse-rate
derivation, no Jacobians); both the CPU oracle and the HIP library receive
the same description and derive everything else themselves.

The networks stand in for the paper's workloads (a 12-species/116-reaction
H2/O2 combustion network, astro H/He/e- chemistry and "10-30 species per
cell", Sec. 2.3.2): the paper's own mechanism data (GRI-Mech, UMIST) are not
available, so shapes and value ranges follow the benchmark recipe documented
alongside the benchmark, and every draw is seeded.

Conventions (cgs, energies divided by k_B so they are in K):
  * composition[nu][s]   atoms of element row nu in species s; the rows after
                         ``n_elem`` are charge-like rows (+1 per positive
                         charge, -1 for the electron).
  * reservoir[nu]        the single-row species that absorbs element/charge
                         corrections for row nu (post-processing stage 2).
  * reac/prod[r][3]      species indices of the reactant/product multisets of
                         reaction r, padded with -1 (at most 3 per side).
  * arr_f[r] = (A, b, E) forward rate coefficient k = A T^b exp(-E/T).
  * h_form, s_form       per-species formation energy [K] and entropy [k_B]
                         at the standard-state pressure p_ref (reference
                         density p_ref / (k_B T)), from which detailed balance
                         fixes the reverse rate.
  * cv                   per-particle heat capacity at constant volume [k_B].
  * cv_poly, T_mid       optional temperature-dependent heat capacities:
                         cv_poly[s][piece][k], c_V/k_B = sum_k a_k T^k on
                         T < T_mid (piece 0) and T >= T_mid (piece 1).
  * sigma_abs, photo,    optional photoreactions: photo[r] = 1 makes the
    heat_extra           forward coefficient A F_eff (A the reaction's
                         cross-section) with no reverse; heat_extra[r] =
                         (q0, q1, q2) adds q0 + q1 T + q2 T ln T of gas
                         heating per net event (K), besides -dH.
  * tab_of, tab_log2k,   optional tabulated rate factors: reaction r with
    tab_log2T0,          tab_of[r] = t >= 0 has its coefficient multiplied by
    tab_dlog2T           the factor whose log2 is tab_log2k[t][i] at
                         log2 T = tab_log2T0 + i tab_dlog2T.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 2504_04941
K_BOLTZ = 1.380649e-16      # erg / K
ATM = 1.01325e6             # dyn / cm^2


def rng_for(config_index: int, salt: int = 0) -> np.random.Generator:
    """The seeded generator for one workload: Philox keyed on the config."""
    return np.random.Generator(np.random.Philox(key=SEED_BASE + config_index + (salt << 32)))


@dataclass
class NetworkDesc:
    name: str
    species: list
    rows: list                 # element rows then charge rows
    n_elem: int
    composition: np.ndarray    # int32 [n_rows, S]
    reservoir: np.ndarray      # int32 [n_rows]
    cv: np.ndarray             # float64 [S]
    h_form: np.ndarray         # float64 [S]  (K)
    s_form: np.ndarray         # float64 [S]  (k_B)
    reac: np.ndarray           # int32 [R, 3]
    prod: np.ndarray           # int32 [R, 3]
    arr_f: np.ndarray          # float64 [R, 3]
    arr_r: np.ndarray | None = None   # explicit reverse (A, b, E) or None
    p_ref: float = ATM         # standard-state pressure of the thermo data (dyn cm^-2)
    T_min: float = 1.0
    T_max: float = 1.0e5
    meta: dict = field(default_factory=dict)
    cv_poly: np.ndarray | None = None        # float64 [S, 2, 5]
    T_mid: float = 1000.0
    tab_of: np.ndarray | None = None         # int32 [R]
    tab_log2k: np.ndarray | None = None      # float64 [n_tables, n_nodes]
    tab_log2T0: float = 0.0
    tab_dlog2T: float = 1.0
    sigma_abs: np.ndarray | None = None      # float64 [S] photo-absorption cross-sections (cm^2)
    photo: np.ndarray | None = None          # int32 [R] 1: photoreaction
    heat_extra: np.ndarray | None = None     # float64 [R, 3] extra heat q0 + q1 T + q2 T ln T (K)

    @property
    def n_species(self) -> int:
        return len(self.species)

    @property
    def n_rows(self) -> int:
        return len(self.rows)

    @property
    def n_reactions(self) -> int:
        return int(self.reac.shape[0])

    @property
    def n_unknowns(self) -> int:
        return self.n_species + 1

    def stoich(self) -> np.ndarray:
        """Net stoichiometric matrix nu[r][s] = (#s in prod) - (#s in reac).

        Pure bookkeeping of the description (integer counts)."""
        nu = np.zeros((self.n_reactions, self.n_species), dtype=np.int64)
        for r in range(self.n_reactions):
            for s in self.reac[r]:
                if s >= 0:
                    nu[r, s] -= 1
            for s in self.prod[r]:
                if s >= 0:
                    nu[r, s] += 1
        return nu


# ----------------------------------------------------------------------------
# helpers
# ----------------------------------------------------------------------------

def _heat_capacity(atoms: int, linear: bool) -> float:
    """Per-particle c_V/k_B by rigid-rotor counting: 3/2 monatomic (and the
    electron), 5/2 linear, 3 non-linear."""
    if atoms <= 1:
        return 1.5
    return 2.5 if linear else 3.0


def _thermo(rng, comp: np.ndarray, n_elem: int):
    """Species formation energy and entropy (standard state p_ref).

    Bond-counting model: every bond of a tree-shaped molecule lowers the
    formation energy by a bond energy ~U[4e4, 6e4] K, every positive charge
    raises it by an ionisation energy ~U[1.2e5, 1.6e5] K, plus U[-5e3, 5e3] K
    of noise; entropy is ~12 k_B per particle (translation) with U[-2, 2]
    noise.  This keeps detailed-balance reverse rates near gas-kinetic values
    (dissociation endothermic, recombination exothermic), as for real
    combustion and astro networks."""
    S = comp.shape[1]
    atoms = comp[:n_elem].sum(axis=0)
    charge = comp[n_elem:].sum(axis=0) if comp.shape[0] > n_elem else np.zeros(S, int)
    bonds = np.maximum(atoms - 1, 0)
    h = (-bonds * rng.uniform(4e4, 6e4, size=S)
         + np.maximum(charge, 0) * rng.uniform(1.2e5, 1.6e5, size=S)
         + rng.uniform(-5e3, 5e3, size=S))
    s = 12.0 + rng.uniform(-2.0, 2.0, size=S)
    return h, s


def _pad3(ms):
    out = [-1, -1, -1]
    for i, s in enumerate(ms):
        out[i] = s
    return out


def enumerate_reactions(comp: np.ndarray, max_small: int, max_large: int,
                        max_common: int = 1, spectator_only=()):
    """All element- and charge-conserving reaction candidates between species
    multisets.  One side has at most ``max_small`` species, the other at most
    ``max_large``; sides share at most ``max_common`` distinct species (a
    catalyst/third body); species in ``spectator_only`` may appear only as a
    shared species.  Each unordered pair appears once, as (small, large)."""
    S = comp.shape[1]
    groups: dict = {}
    for k in range(1, max_large + 1):
        for m in itertools.combinations_with_replacement(range(S), k):
            v = tuple(int(x) for x in comp[:, list(m)].sum(axis=1))
            groups.setdefault(v, []).append(m)
    out = []
    for v, ms in groups.items():
        for a, b in itertools.combinations(ms, 2):
            if len(a) > len(b):
                a, b = b, a
            if len(a) > max_small:
                continue
            common = set(a) & set(b)
            if len(common) > max_common:
                continue
            sa, sb = set(a) - common, set(b) - common
            if any(s in sa or s in sb for s in spectator_only):
                continue
            # the net change must be nonzero
            if sorted(a) == sorted(b):
                continue
            out.append((a, b))
    return out


def _span_ok(comp: np.ndarray, picks) -> bool:
    S = comp.shape[1]
    nu = np.zeros((len(picks), S))
    for i, (a, b) in enumerate(picks):
        for s in a:
            nu[i, s] -= 1
        for s in b:
            nu[i, s] += 1
    null_dim = S - np.linalg.matrix_rank(comp.astype(float))
    return np.linalg.matrix_rank(nu) == null_dim


def _choose_reactions(rng, comp, cands, n_react, must_touch=None, tries=2000):
    """Seeded choice of ``n_react`` candidates whose net stoichiometry spans
    the null space of the composition matrix (so every conserved-quantity
    preserving direction can be reached)."""
    S = comp.shape[1]
    touch = set(range(S)) if must_touch is None else set(must_touch)
    for _ in range(tries):
        idx = rng.choice(len(cands), size=n_react, replace=False)
        picks = [cands[i] for i in sorted(idx)]
        used = set()
        for a, b in picks:
            used |= set(a) | set(b)
        if not touch <= used:
            continue
        if _span_ok(comp, picks):
            return picks
    raise RuntimeError("could not draw a spanning reaction set")


def _choose_by_shape(rng, comp, cands, quotas, tries=2000):
    """Like _choose_reactions, with a quota of reactions per side-size shape
    (len(small side), len(large side)): e.g. {(2, 2): 120, (1, 2): 40}."""
    by_shape: dict = {}
    for c in cands:
        by_shape.setdefault((len(c[0]), len(c[1])), []).append(c)
    S = comp.shape[1]
    for _ in range(tries):
        picks = []
        for shape, k in sorted(quotas.items()):
            pool = by_shape[shape]
            idx = rng.choice(len(pool), size=k, replace=False)
            picks += [pool[i] for i in sorted(idx)]
        used = set()
        for a, b in picks:
            used |= set(a) | set(b)
        if used == set(range(S)) and _span_ok(comp, picks):
            return picks
    raise RuntimeError("could not draw a spanning reaction set")


def _orient_and_draw(rng, picks, h_form, logA_of, b_rng, E_max, small_side_forward=True):
    """Arrhenius parameters for each picked reaction.

    The given ("forward") direction is the side with fewer species.  Its
    barrier: the exothermic direction's barrier is drawn from U[0, E_max];
    if the given direction is the endothermic one, its barrier is that draw
    plus the reaction's energy change, so both directions have E >= 0."""
    R = len(picks)
    reac = np.full((R, 3), -1, np.int32)
    prod = np.full((R, 3), -1, np.int32)
    arr = np.zeros((R, 3))
    for r, (a, b) in enumerate(picks):
        reac[r] = _pad3(a)
        prod[r] = _pad3(b)
        dh = sum(h_form[s] for s in b) - sum(h_form[s] for s in a)   # forward energy change
        e_exo = rng.uniform(0.0, E_max)
        E = e_exo if dh <= 0.0 else e_exo + dh
        arr[r] = (10.0 ** logA_of(len(a), rng), rng.uniform(*b_rng), E)
    return reac, prod, arr


# ----------------------------------------------------------------------------
# the workload networks
# ----------------------------------------------------------------------------

def network_h_he(seed_index: int = 0) -> NetworkDesc:
    """5 species H, H2, H+, e-, He over rows H, He and charge; 10 reversible
    reactions with at most 3 species per side (astro H/He/e- chemistry)."""
    rng = rng_for(seed_index, salt=1)
    species = ["H", "H2", "H+", "e-", "He"]
    rows = ["H", "He", "charge"]
    comp = np.array([[1, 2, 1, 0, 0],
                     [0, 0, 0, 0, 1],
                     [0, 0, 1, -1, 0]], np.int32)
    reservoir = np.array([0, 4, 3], np.int32)
    cv = np.array([1.5, 2.5, 1.5, 1.5, 1.5])
    h_form, s_form = _thermo(rng, comp, 2)
    cands = enumerate_reactions(comp, 3, 3, max_common=1)
    picks = _choose_reactions(rng, comp, cands, 10)
    reac, prod, arr = _orient_and_draw(
        rng, picks, h_form, lambda order, g: g.uniform(-12.0, -8.0), (-1.0, 1.0), 5e4)
    return NetworkDesc("h_he_5sp", species, rows, 2, comp, reservoir, cv, h_form, s_form,
                       reac, prod, arr, None, p_ref=ATM, T_min=1.0, T_max=1.0e6,
                       meta={"config_index": 0})


def network_h_o_n(seed_index: int = 1) -> NetworkDesc:
    """9 species H2, O2, H, O, OH, H2O, HO2, H2O2, N2 over rows H, O, N;
    24 reversible reactions with at most 2 species on one side and 3 on the
    other; N2 only as a shared third body (combustion-shaped network)."""
    rng = rng_for(seed_index, salt=1)
    species = ["H2", "O2", "H", "O", "OH", "H2O", "HO2", "H2O2", "N2"]
    rows = ["H", "O", "N"]
    comp = np.array([[2, 0, 1, 0, 1, 2, 1, 2, 0],
                     [0, 2, 0, 1, 1, 1, 2, 2, 0],
                     [0, 0, 0, 0, 0, 0, 0, 0, 2]], np.int32)
    reservoir = np.array([2, 3, 8], np.int32)
    atoms = comp.sum(axis=0)
    linear = [True, True, True, True, True, False, False, False, True]
    cv = np.array([_heat_capacity(int(a), l) for a, l in zip(atoms, linear)])
    h_form, s_form = _thermo(rng, comp, 3)
    cands = enumerate_reactions(comp, 2, 3, max_common=1, spectator_only=(8,))
    picks = _choose_reactions(rng, comp, cands, 24, must_touch=range(8))

    def logA(order, g):
        return g.uniform(6.0, 13.0) if order == 1 else g.uniform(-12.0, -9.0)
    reac, prod, arr = _orient_and_draw(rng, picks, h_form, logA, (-1.0, 1.0), 3e4)
    return NetworkDesc("h_o_n_9sp", species, rows, 3, comp, reservoir, cv, h_form, s_form,
                       reac, prod, arr, None, p_ref=ATM, T_min=50.0, T_max=1.0e5,
                       meta={"config_index": 1})


# ----------------------------------------------------------------------------
# cell states
# ----------------------------------------------------------------------------

@dataclass
class CellStates:
    n: np.ndarray      # float64 [S, n_cells]  (SoA, cm^-3)
    T: np.ndarray      # float64 [n_cells]     (K)
    rho: np.ndarray    # float64 [n_cells]     (g cm^-3, informational / floors)
    dt: np.ndarray | None  # float64 [n_cells] or None when a scalar step applies
    dt_scalar: float = 0.0

    @property
    def n_cells(self) -> int:
        return int(self.T.shape[0])


_AMU = 1.66053906660e-24


def _rho(net: NetworkDesc, n: np.ndarray) -> np.ndarray:
    # mass from nucleon counts (1 amu per H, 4 He, 12 C, 14 N, 16 O)
    amu = {"H": 1.0, "He": 4.0, "C": 12.0, "N": 14.0, "O": 16.0}
    m = np.zeros(net.n_species)
    for nu, row in enumerate(net.rows[:net.n_elem]):
        m += amu.get(row, 1.0) * net.composition[nu]
    return (m[:, None] * n).sum(axis=0) * _AMU


def cells_h_he(net: NetworkDesc, n_cells: int, seed_index: int = 0) -> CellStates:
    """T log-uniform [10, 1e4] K, hydrogen nuclei log-uniform [1, 1e6] cm^-3,
    He = 0.1 n_H, hydrogen split H : 2 H2 : H+ by Dirichlet(1,1,1), n_e = n_H+.
    The step is set later from the cells' fastest timescale."""
    rng = rng_for(seed_index, salt=2)
    T = 10.0 ** rng.uniform(1.0, 4.0, size=n_cells)
    nH = 10.0 ** rng.uniform(0.0, 6.0, size=n_cells)
    f = rng.dirichlet((1.0, 1.0, 1.0), size=n_cells)
    n = np.zeros((5, n_cells))
    n[0] = f[:, 0] * nH
    n[1] = 0.5 * f[:, 1] * nH
    n[2] = f[:, 2] * nH
    n[3] = n[2]
    n[4] = 0.1 * nH
    return CellStates(n, T, _rho(net, n), None, 0.0)


def cells_h_o_n(net: NetworkDesc, n_cells: int, seed_index: int = 1,
                dt: float = 1e-4, salt: int = 2) -> CellStates:
    """T ~ U[900, 2500] K at p = 1 atm; majors H2, O2, H2O, N2 ~
    Dirichlet(2,1,1,4); radicals H, O, OH, HO2, H2O2 each 10^U[-12,-4];
    renormalised mole fractions times n_tot = p / (k_B T).  Different salts
    give independent sets (e.g. training and held-out cells)."""
    rng = rng_for(seed_index, salt=salt)
    T = rng.uniform(900.0, 2500.0, size=n_cells)
    ntot = ATM / (K_BOLTZ * T)
    x = np.zeros((9, n_cells))
    maj = rng.dirichlet((2.0, 1.0, 1.0, 4.0), size=n_cells)
    for j, s in enumerate((0, 1, 5, 8)):
        x[s] = maj[:, j]
    for s in (2, 3, 4, 6, 7):
        x[s] = 10.0 ** rng.uniform(-12.0, -4.0, size=n_cells)
    x /= x.sum(axis=0, keepdims=True)
    n = x * ntot[None, :]
    return CellStates(n, T, _rho(net, n), None, dt)


def _einstein(T: np.ndarray, thetas: np.ndarray) -> np.ndarray:
    """Heat capacity [k_B] of harmonic modes with vibrational temperatures
    thetas at temperatures T (the Einstein function, summed over modes)."""
    x = thetas[None, :] / T[:, None]
    q = np.exp(-x)
    return (x * x * q / (1.0 - q) ** 2).sum(axis=1)


def heat_capacity_polys(cv0: np.ndarray, n_modes, rng, T_mid: float = 1000.0,
                        pieces=((200.0, 1000.0), (1000.0, 6000.0))) -> np.ndarray:
    """Synthetic NASA-style c_V(T) data (the paper's mechanism data are not
    available): per species the rigid-rotor value cv0 plus n_modes harmonic
    vibrational modes with vibrational temperatures ~U[800, 6000] K, fitted
    by a quartic in T (least squares on 200 points) on each piece.  Returns
    [S, 2, 5] ascending-power coefficients."""
    S = len(cv0)
    out = np.zeros((S, 2, 5))
    for s in range(S):
        thetas = rng.uniform(800.0, 6000.0, int(n_modes[s]))
        for piece, (lo, hi) in enumerate(pieces):
            T = np.linspace(lo, hi, 200)
            c = cv0[s] + (_einstein(T, thetas) if thetas.size else 0.0)
            if thetas.size == 0:
                out[s, piece, 0] = cv0[s]
                continue
            coef = np.polynomial.polynomial.Polynomial.fit(T, c, 4).convert().coef
            out[s, piece, :coef.size] = coef
    return out


def network_h_o_n_tcv(seed_index: int = 1, n_tables: int = 4, n_nodes: int = 48) -> NetworkDesc:
    """The 9-species combustion network with temperature-dependent heat
    capacities (vibrational modes: 3 atoms - 5 linear, 3 atoms - 6 otherwise)
    and n_tables reactions whose forward coefficient is tabulated: a second,
    lower-barrier channel A2 T^b2 exp(-E2/T) added to the drawn Arrhenius
    one and sampled at n_nodes nodes uniform in log2 T over [200, 1e4] K
    (arr_f of those reactions becomes (1, 0, 0): the table is the whole
    forward coefficient).  E2 is at least the reaction's energy change, so
    the detailed-balance reverse of the extra channel has no negative
    barrier."""
    net = network_h_o_n(seed_index)
    rng = rng_for(seed_index, salt=7)
    atoms = net.composition.sum(axis=0)
    linear = [True, True, True, True, True, False, False, False, True]
    modes = [0 if a <= 1 else (3 * a - 5 if l else 3 * a - 6) for a, l in zip(atoms, linear)]
    net.cv_poly = heat_capacity_polys(net.cv, modes, rng)
    net.T_mid = 1000.0
    R = net.n_reactions
    x0, x1 = np.log2(200.0), np.log2(1.0e4)
    dx = (x1 - x0) / (n_nodes - 1)
    Tn = 2.0 ** (x0 + dx * np.arange(n_nodes))
    nu = net.stoich()
    picks = np.sort(rng.choice(R, n_tables, replace=False))
    tab_of = np.full(R, -1, np.int32)
    tab = np.zeros((n_tables, n_nodes))
    arr = net.arr_f.copy()
    for t, r in enumerate(picks):
        A, b, E = arr[r]
        dH = float(nu[r] @ net.h_form)
        A2 = A * 10.0 ** rng.uniform(-2.0, 0.0)
        b2 = b + rng.uniform(-1.0, 1.0)
        E2 = max(E * rng.uniform(0.2, 0.6), dH, 0.0)
        # log of the two-channel sum, in log space (no underflow)
        tab[t] = np.logaddexp(np.log(A) + b * np.log(Tn) - E / Tn,
                              np.log(A2) + b2 * np.log(Tn) - E2 / Tn) / np.log(2.0)
        arr[r] = (1.0, 0.0, 0.0)
        tab_of[r] = t
    net.arr_f = arr
    net.tab_of, net.tab_log2k = tab_of, tab
    net.tab_log2T0, net.tab_dlog2T = float(x0), float(dx)
    net.name = "h_o_n_tcv_9sp"
    net.meta = dict(net.meta, tabulated=picks.tolist())
    return net


E_V = 1.602176634e-12        # erg
I_H_K = 13.6 * E_V / K_BOLTZ   # hydrogen ionisation energy / k_B (K)
SIGMA_H = 6.3e-18            # H photo-ionisation cross-section at threshold (cm^2)
H_NU_EV = 16.0               # photon energy of the monochromatic field (eV)


def network_stromgren(isothermal: bool = False) -> NetworkDesc:
    """The hydrogen chemistry of the paper's Stromgren-sphere test (Sec. 4.3,
    eq. strom-chem): H + photon -> H+ + e- (photoreaction, cross-section
    6.3e-18 cm^2), H + e- -> H+ + 2 e- (collisional ionisation, k_ci of
    eq. thermo-strom: 1.05e-9 (T/300)^0.5 exp(-I_H/k_B T) cm^3 s^-1) and
    H+ + e- -> H + photon (case-B recombination alpha = 3.5e-12 (T/300)^-0.75
    cm^3 s^-1), all irreversible.  Energies: H+ lies I_H = 13.6 eV above H
    (formation energies), the photoreaction adds the absorbed photon's
    h nu = 16 eV, the recombination removes the radiated I_H + lambda_rec,
    lambda_rec = [0.684 - 0.0416 ln(T / 1e4 K)] k_B T (eq. thermo-strom).
    isothermal=True drops every energy term and gives the electron no heat
    capacity, so that c_V does not change with ionisation: Q = 0 and T stays
    put."""
    species = ["H", "H+", "e-"]
    rows = ["H", "charge"]
    comp = np.array([[1, 1, 0], [0, 1, -1]], np.int32)
    reservoir = np.array([0, 2], np.int32)
    cv = np.array([1.5, 1.5, 0.0 if isothermal else 1.5])
    h_form = np.array([0.0, 0.0 if isothermal else I_H_K, 0.0])
    s_form = np.zeros(3)
    reac = np.array([[0, -1, -1], [0, 2, -1], [1, 2, -1]], np.int32)
    prod = np.array([[1, 2, -1], [1, 2, 2], [0, -1, -1]], np.int32)
    arr_f = np.array([[SIGMA_H, 0.0, 0.0],
                      [1.05e-9 * 300.0 ** -0.5, 0.5, I_H_K],
                      [3.5e-12 * 300.0 ** 0.75, -0.75, 0.0]])
    arr_r = np.zeros((3, 3))
    heat = np.zeros((3, 3))
    if not isothermal:
        heat[0] = (H_NU_EV * E_V / K_BOLTZ, 0.0, 0.0)
        heat[2] = (-I_H_K, -(0.684 + 0.0416 * np.log(1.0e4)), 0.0416)
    net = NetworkDesc("stromgren_h" + ("_iso" if isothermal else ""), species, rows, 1, comp, reservoir, cv,
                      h_form, s_form, reac, prod, arr_f, arr_r, p_ref=ATM, T_min=10.0, T_max=1.0e6,
                      meta={"h_nu_eV": H_NU_EV})
    net.sigma_abs = np.array([SIGMA_H, 0.0, 0.0])
    net.photo = np.array([1, 0, 0], np.int32)
    net.heat_extra = heat
    return net


PARSEC = 3.0857e18          # cm


def cells_stromgren(net: NetworkDesc, n_cells: int, seed_index: int = 6):
    """Cells of an H II region around the paper's fiducial source (Sec. 4.3:
    Phi = 1e49 photons/s, cells of 1/4 pc): radius log-uniform [0.1, 16] pc,
    optical depth to the source log-uniform [1e-4, 30], so F = Phi / (4 pi
    r^2) e^-tau; n_H log-uniform [10, 1e4] cm^-3, ionised fraction x with
    log10(x / (1 - x)) ~ U[-4, 4], T log-uniform [3e3, 5e4] K; path length
    L = 1/4 pc; per-cell step log-uniform [1e8, 1e12] s.  Returns
    (CellStates, photo_flux, photo_length)."""
    rng = rng_for(seed_index, salt=3)
    r = PARSEC * 10.0 ** rng.uniform(-1.0, np.log10(16.0), n_cells)
    tau = 10.0 ** rng.uniform(-4.0, np.log10(30.0), n_cells)
    F = 1.0e49 / (4.0 * np.pi * r * r) * np.exp(-tau)
    nH = 10.0 ** rng.uniform(1.0, 4.0, n_cells)
    lx = rng.uniform(-4.0, 4.0, n_cells)
    x = 1.0 / (1.0 + 10.0 ** -lx)
    T = 10.0 ** rng.uniform(np.log10(3e3), np.log10(5e4), n_cells)
    n = np.vstack([nH * (1.0 - x), nH * x, nH * x])
    dt = 10.0 ** rng.uniform(8.0, 12.0, n_cells)
    L = np.full(n_cells, 0.25 * PARSEC)
    return CellStates(n, T, _rho(net, n), dt), F, L


def network_astro23(seed_index: int = 2) -> NetworkDesc:
    """23 species over rows H, He, C, O and charge (an astrochemistry-shaped
    ion-molecule network); 64 reversible reactions with at most 3 species
    per side, spanning the null space of the composition (dimension 18)."""
    rng = rng_for(seed_index, salt=1)
    # (name, H, He, C, O, charge)
    table = [("H", 1, 0, 0, 0, 0), ("H2", 2, 0, 0, 0, 0), ("H+", 1, 0, 0, 0, 1),
             ("H2+", 2, 0, 0, 0, 1), ("H3+", 3, 0, 0, 0, 1), ("e-", 0, 0, 0, 0, -1),
             ("He", 0, 1, 0, 0, 0), ("He+", 0, 1, 0, 0, 1), ("C", 0, 0, 1, 0, 0),
             ("C+", 0, 0, 1, 0, 1), ("CH", 1, 0, 1, 0, 0), ("CH+", 1, 0, 1, 0, 1),
             ("CH2", 2, 0, 1, 0, 0), ("O", 0, 0, 0, 1, 0), ("O+", 0, 0, 0, 1, 1),
             ("OH", 1, 0, 0, 1, 0), ("OH+", 1, 0, 0, 1, 1), ("H2O", 2, 0, 0, 1, 0),
             ("H2O+", 2, 0, 0, 1, 1), ("H3O+", 3, 0, 0, 1, 1), ("CO", 0, 0, 1, 1, 0),
             ("CO+", 0, 0, 1, 1, 1), ("O2", 0, 0, 0, 2, 0)]
    species = [t[0] for t in table]
    comp = np.array([[t[k] for t in table] for k in range(1, 6)], np.int32)
    reservoir = np.array([0, 6, 8, 13, 5], np.int32)
    atoms = comp[:4].sum(axis=0)
    linear = {"H2", "H2+", "CH", "CH+", "OH", "OH+", "CO", "CO+", "O2"}
    cv = np.array([1.5 if s == "e-" else _heat_capacity(int(a), s in linear)
                   for s, a in zip(species, atoms)])
    h_form, s_form = _thermo(rng, comp, 4)
    cands = enumerate_reactions(comp, 3, 3, max_common=1)
    picks = _choose_reactions(rng, comp, cands, 64)
    reac, prod, arr = _orient_and_draw(
        rng, picks, h_form, lambda order, g: g.uniform(-12.0, -8.0), (-1.0, 1.0), 5e4)
    return NetworkDesc("astro_23sp", species, ["H", "He", "C", "O", "charge"], 4, comp,
                       reservoir, cv, h_form, s_form, reac, prod, arr, None, p_ref=ATM,
                       T_min=1.0, T_max=1.0e6, meta={"config_index": 2})


def cells_astro23(net: NetworkDesc, n_cells: int, seed_index: int = 2, salt: int = 2) -> CellStates:
    """T log-uniform [10, 3000] K, hydrogen nuclei log-uniform [1, 1e6]
    cm^-3 split H : 2 H2 : H+ by Dirichlet(1,1,1) with n_e balancing the
    charge, He = 0.1 n_H, C = 1e-4 n_H (as C+), O = 3e-4 n_H (as O),
    other species 10^U[-12,-6] n_H."""
    rng = rng_for(seed_index, salt=salt)
    S = net.n_species
    idx = {s: i for i, s in enumerate(net.species)}
    T = 10.0 ** rng.uniform(1.0, np.log10(3000.0), size=n_cells)
    nH = 10.0 ** rng.uniform(0.0, 6.0, size=n_cells)
    f = rng.dirichlet((1.0, 1.0, 1.0), size=n_cells)
    n = 10.0 ** rng.uniform(-12.0, -6.0, size=(S, n_cells)) * nH[None, :]
    n[idx["H"]] = f[:, 0] * nH
    n[idx["H2"]] = 0.5 * f[:, 1] * nH
    n[idx["H+"]] = f[:, 2] * nH
    n[idx["He"]] = 0.1 * nH
    n[idx["C+"]] = 1e-4 * nH
    n[idx["O"]] = 3e-4 * nH
    charge = net.composition[4].astype(float)
    n[idx["e-"]] = 0.0
    n[idx["e-"]] = np.maximum(charge @ n, 0.0)
    return CellStates(n, T, _rho(net, n), None, 0.0)


# (name, H, C, N, O, linear) of the 43 molecules of the large network
_LARGE48_MOLECULES = [
    ("H2", 2, 0, 0, 0, 1), ("C2", 0, 2, 0, 0, 1), ("N2", 0, 0, 2, 0, 1), ("O2", 0, 0, 0, 2, 1),
    ("CH", 1, 1, 0, 0, 1), ("NH", 1, 0, 1, 0, 1), ("OH", 1, 0, 0, 1, 1), ("CN", 0, 1, 1, 0, 1),
    ("CO", 0, 1, 0, 1, 1), ("NO", 0, 0, 1, 1, 1),
    ("H2O", 2, 0, 0, 1, 0), ("CH2", 2, 1, 0, 0, 0), ("NH2", 2, 0, 1, 0, 0), ("HCN", 1, 1, 1, 0, 1),
    ("HCO", 1, 1, 0, 1, 0), ("HNO", 1, 0, 1, 1, 0), ("CO2", 0, 1, 0, 2, 1), ("N2O", 0, 0, 2, 1, 1),
    ("NO2", 0, 0, 1, 2, 0), ("O3", 0, 0, 0, 3, 0), ("C2H", 1, 2, 0, 0, 1), ("C3", 0, 3, 0, 0, 1),
    ("HO2", 1, 0, 0, 2, 0), ("NCO", 0, 1, 1, 1, 1), ("C2O", 0, 2, 0, 1, 1), ("C2N", 0, 2, 1, 0, 1),
    ("CH3", 3, 1, 0, 0, 0), ("NH3", 3, 0, 1, 0, 0), ("H2CO", 2, 1, 0, 1, 0), ("C2H2", 2, 2, 0, 0, 1),
    ("HNCO", 1, 1, 1, 1, 0), ("H2O2", 2, 0, 0, 2, 0), ("N2H2", 2, 0, 2, 0, 0), ("HNO2", 1, 0, 1, 2, 0),
    ("C3H", 1, 3, 0, 0, 1),
    ("CH4", 4, 1, 0, 0, 0), ("HCOOH", 2, 1, 0, 2, 0), ("CH2CO", 2, 2, 0, 1, 0), ("NH2OH", 3, 0, 1, 1, 0),
    ("HC3N", 1, 3, 1, 0, 1), ("CH3O", 3, 1, 0, 1, 0),
    ("CH3OH", 4, 1, 0, 1, 0), ("C2H4", 4, 2, 0, 0, 0),
]


def network_large48(seed_index: int = 3) -> NetworkDesc:
    """48 neutral species over rows H, He, C, N, O: the five atoms and 43
    molecules of 2-6 atoms; 200 reversible reactions (120 two-to-two, 50
    one-to-two, 30 two-to-three; at most one species on both sides, e.g. a
    third body), spanning the null space of the composition (dimension 43)."""
    rng = rng_for(seed_index, salt=1)
    atoms_tab = [("H", 1, 0, 0, 0, 0), ("He", 0, 0, 0, 0, 0), ("C", 0, 1, 0, 0, 0),
                 ("N", 0, 0, 1, 0, 0), ("O", 0, 0, 0, 1, 0)]
    table = atoms_tab + _LARGE48_MOLECULES
    species = [t[0] for t in table]
    S = len(species)
    comp = np.zeros((5, S), np.int32)
    for j, t in enumerate(table):
        comp[0, j], comp[2, j], comp[3, j], comp[4, j] = t[1], t[2], t[3], t[4]
    comp[1, 1] = 1                                     # He
    reservoir = np.array([0, 1, 2, 3, 4], np.int32)
    atoms = comp.sum(axis=0)
    cv = np.array([_heat_capacity(int(a), bool(t[5])) for a, t in zip(atoms, table)])
    h_form, s_form = _thermo(rng, comp, 5)
    cands = enumerate_reactions(comp, 2, 3, max_common=1)
    # mostly bimolecular exchange, plus dissociation/association and
    # third-body (3-species side) reactions
    picks = _choose_by_shape(rng, comp, cands, {(2, 2): 120, (1, 2): 50, (2, 3): 30})

    # slower than the combustion network (log10 A one to five decades lower,
    # barriers up to 5e4 K) so that steps up to 1e-2 s at up to 5000 K stay
    # within a few hundred substeps for most cells
    def logA(order, g):
        return {1: g.uniform(2.0, 8.0), 2: g.uniform(-13.0, -10.0)}.get(order, g.uniform(-35.0, -32.0))
    reac, prod, arr = _orient_and_draw(rng, picks, h_form, logA, (-1.0, 1.0), 5e4)
    return NetworkDesc("large_48sp", species, ["H", "He", "C", "N", "O"], 5, comp, reservoir, cv,
                       h_form, s_form, reac, prod, arr, None, p_ref=ATM, T_min=10.0, T_max=1.0e5,
                       meta={"config_index": 3})


def cells_large48(net: NetworkDesc, n_cells: int, seed_index: int = 3, salt: int = 2) -> CellStates:
    """T log-uniform [50, 5000] K; hydrogen nuclei log-uniform [1, 1e8]
    cm^-3 split H : 2 H2 by Dirichlet(1,1); He = 0.1 n_H, C = 1e-4 n_H (as
    CO), N = 5e-5 n_H (as N2), O = 3e-4 n_H (CO, the rest as H2O and O),
    every other species 10^U[-12,-6] n_H; per-cell step log-uniform in
    [1e-8, 1e-2] s."""
    rng = rng_for(seed_index, salt=salt)
    S = net.n_species
    idx = {s: i for i, s in enumerate(net.species)}
    T = 10.0 ** rng.uniform(np.log10(50.0), np.log10(5000.0), size=n_cells)
    nH = 10.0 ** rng.uniform(0.0, 8.0, size=n_cells)
    f = rng.dirichlet((1.0, 1.0), size=n_cells)
    n = 10.0 ** rng.uniform(-12.0, -6.0, size=(S, n_cells)) * nH[None, :]
    n[idx["H"]] = f[:, 0] * nH
    n[idx["H2"]] = 0.5 * f[:, 1] * nH
    n[idx["He"]] = 0.1 * nH
    n[idx["CO"]] = 1e-4 * nH
    n[idx["N2"]] = 2.5e-5 * nH
    n[idx["H2O"]] = 1.5e-4 * nH
    n[idx["O"]] = 0.5e-4 * nH
    dt = 10.0 ** rng.uniform(-8.0, -2.0, size=n_cells)
    return CellStates(n, T, _rho(net, n), dt, 0.0)


def log_uniform(n: int, lo: float, hi: float, config_index: int, salt: int) -> np.ndarray:
    """n values log-uniform in [lo, hi] from the seeded stream (config, salt)."""
    rng = rng_for(config_index, salt=salt)
    return 10.0 ** rng.uniform(np.log10(lo), np.log10(hi), size=n)


# ----------------------------------------------------------------------------
# species advection (Sec. 2.1 and the advection test of Sec. 4.1)
# ----------------------------------------------------------------------------

def network_e1() -> NetworkDesc:
    """Passive species A, A2, AB, B over elements A and B (the advection
    test's species); two reversible reactions 2 A <=> A2 and A + B <=> AB make
    it a complete description (advection does not use them)."""
    species = ["A", "A2", "AB", "B"]
    comp = np.array([[1, 2, 1, 0],
                     [0, 0, 1, 1]], np.int32)
    reac = np.array([[0, 0, -1], [0, 3, -1]], np.int32)
    prod = np.array([[1, -1, -1], [2, -1, -1]], np.int32)
    arr = np.array([[1e-12, 0.0, 0.0], [1e-12, 0.0, 0.0]])
    return NetworkDesc("e1_4sp", species, ["A", "B"], 2, comp, np.array([0, 3], np.int32),
                       np.array([1.5, 2.5, 2.5, 1.5]), np.array([0.0, -1e4, -1e4, 0.0]),
                       np.zeros(4), reac, prod, arr, None, p_ref=ATM, T_min=1.0, T_max=1.0e6)


def uniform_grid(n: int, lo: float = -0.5, hi: float = 0.5):
    """Cell centres [n] and faces [n + 1] of a uniform 1-D grid."""
    xf = np.linspace(lo, hi, n + 1)
    return 0.5 * (xf[:-1] + xf[1:]), xf


def e1_initial(xc) -> np.ndarray:
    """Abundances [4, n] of A, A2, AB, B at the cell centres xc in [-0.5, 0.5]
    (the advection test's initial profiles: steps at x = 0 plus linear
    parts; element abundances 0.9 and 0.1 everywhere)."""
    x = np.asarray(xc, np.float64)
    h = (x > 0).astype(float)
    hm = 1.0 - h
    return np.vstack([0.49 * hm + 0.05 * h + 0.2 * x,
                      0.20 * hm + 0.40 * h - 0.1 * x,
                      0.01 * hm + 0.05 * h,
                      0.09 * hm + 0.05 * h])


def advection_lines(net: NetworkDesc, n_lines: int, n_cells: int, seed_index: int = 5):
    """Seeded lines for the advection kernel: per line, the cells of a
    random composition of the network's own cell recipe mixed along the line
    with a smooth wave and a step (element abundances vary per line, not
    along it: each cell is a mixture of the line's two end states moved
    along reaction directions); a non-uniform grid (faces jittered by up to
    30 % of the spacing); density 1 + 0.5 sin; velocity +1 or -1 per line.
    Returns (n [S, n_lines * n_cells], rho, xc [n_cells], xf [n_cells + 1],
    v [n_lines])."""
    rng = rng_for(seed_index, salt=77)
    S = net.n_species
    # reaction directions (net stoichiometry of the network's reactions)
    null = np.asarray(net.stoich(), np.float64)
    xf = np.linspace(0.0, 1.0, n_cells + 1)
    h = 1.0 / n_cells
    xf[1:-1] += rng.uniform(-0.3, 0.3, n_cells - 1) * h
    xc = 0.5 * (xf[:-1] + xf[1:])
    n = np.empty((S, n_lines * n_cells))
    rho = np.empty(n_lines * n_cells)
    v = np.where(rng.uniform(size=n_lines) < 0.5, -1.0, 1.0)
    for line in range(n_lines):
        base = rng.uniform(0.2, 1.0, S)
        amp = rng.uniform(-1.0, 1.0, null.shape[0])
        d = null.T @ amp
        scale = 0.15 / max(np.abs(d / base).max(), 1e-30)
        wave = np.sin(2 * np.pi * (xc + rng.uniform())) + (xc > rng.uniform(0.2, 0.8))
        cells = base[:, None] + scale * d[:, None] * wave[None, :] * 0.5
        r = 1.0 + 0.5 * np.sin(2 * np.pi * (xc + rng.uniform()))
        n[:, line * n_cells:(line + 1) * n_cells] = cells * r[None, :]
        rho[line * n_cells:(line + 1) * n_cells] = r
    return n, rho, xc, xf, v


def network_for(config_index: int) -> NetworkDesc:
    if config_index == 0:
        return network_h_he(0)
    if config_index == 1:
        return network_h_o_n(1)
    if config_index == 2:
        return network_astro23(2)
    if config_index == 3:
        return network_large48(3)
    raise ValueError(f"no network for config {config_index}")


def cells_for(config_index: int, net: NetworkDesc, n_cells: int) -> CellStates:
    if config_index == 0:
        return cells_h_he(net, n_cells, 0)
    if config_index == 1:
        return cells_h_o_n(net, n_cells, 1)
    if config_index == 2:
        return cells_astro23(net, n_cells, 2)
    if config_index == 3:
        return cells_large48(net, n_cells, 3)
    raise ValueError(f"no cells for config {config_index}")
