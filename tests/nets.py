"""Small hand-made networks used by the tests (descriptions only)."""
import numpy as np

from synthetic import ATM, NetworkDesc


def make_net(name, species, rows, n_elem, comp, reservoir, cv, h, s, reactions,
             arr_r=None, p_ref=ATM, T_min=1.0, T_max=1e6):
    """reactions: list of (reactants, products, (A, b, E)) with species names."""
    idx = {sp: i for i, sp in enumerate(species)}
    R = len(reactions)
    reac = np.full((R, 3), -1, np.int32)
    prod = np.full((R, 3), -1, np.int32)
    arr = np.zeros((R, 3))
    for r, (a, b, par) in enumerate(reactions):
        for k, sp in enumerate(a):
            reac[r, k] = idx[sp]
        for k, sp in enumerate(b):
            prod[r, k] = idx[sp]
        arr[r] = par
    return NetworkDesc(name, list(species), list(rows), n_elem,
                       np.array(comp, np.int32), np.array(reservoir, np.int32),
                       np.array(cv, float), np.array(h, float), np.array(s, float),
                       reac, prod, arr, None if arr_r is None else np.array(arr_r, float),
                       p_ref=p_ref, T_min=T_min, T_max=T_max)


def isomer_pair(kf=2.0, ds=0.7):
    """A <=> B, same composition, no energy change, equal heat capacity:
    isothermal with k_r = k_f exp(-ds)."""
    return make_net("isomers", ["A", "B"], ["X"], 1, [[1, 1]], [0], [1.5, 1.5],
                    [0.0, 0.0], [0.0, ds], [(["A"], ["B"], (kf, 0.0, 0.0))])


def linear_three(ks=(3.0, 0.5, 1.2), ds=(0.3, -0.4)):
    """A <=> B, B <=> C, A <=> C (all first order), isothermal."""
    s = [0.0, ds[0], ds[1]]
    reacts = [(["A"], ["B"], (ks[0], 0.0, 0.0)),
              (["B"], ["C"], (ks[1], 0.0, 0.0)),
              (["A"], ["C"], (ks[2], 0.0, 0.0))]
    # a single-atom "element" shared by all three isomers: A is the reservoir
    return make_net("linear3", ["A", "B", "C"], ["X"], 1, [[1, 1, 1]], [0],
                    [1.5, 1.5, 1.5], [0.0, 0.0, 0.0], s, reacts)
