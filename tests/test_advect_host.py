"""Host checks of the projector tables the network compiler generates for
the advection kernels (no GPU): the dense kr_proj and the orthonormal basis
kr_projq of the conserved rows' span, read back from the generated source,
against the oracle's projector (oracle/plm.py: P = V V^T from the SVD of the
element-species matrix, Sec. 2.1, eq. method-sto-plm-proj)."""
import re

import numpy as np
import pytest

import synthetic as sy
from oracle import plm

NETS = {"e1": sy.network_e1, "h_he": lambda: sy.network_h_he(0), "h_o_n": lambda: sy.network_h_o_n(1),
        "stromgren": sy.network_stromgren, "astro23": lambda: sy.network_astro23(2),
        "large48": lambda: sy.network_large48(3)}


def _table(src, name):
    m = re.search(name + r"\[(\d+)\]\[(\d+)\] = \{(.*?)\};", src, re.S)
    rows, cols = int(m.group(1)), int(m.group(2))
    vals = [float.fromhex(v) for v in re.findall(r"-?0x[0-9a-fp.+-]+", m.group(3))]
    return np.array(vals).reshape(rows, cols)


@pytest.mark.parametrize("which", list(NETS))
def test_generated_projector_tables_match_the_oracle(which):
    import paper_2504_04941_amd as kr
    desc = NETS[which]()
    src = kr.network_check(desc)
    S = desc.n_species
    N = np.asarray(desc.composition, np.float64)
    R = int(re.search(r"#define KR_PROJ_R (\d+)", src).group(1))
    assert R == np.linalg.matrix_rank(N)
    P_oracle = plm.projector_svd(desc.composition)
    P = _table(src, "kr_proj")
    assert P.shape == (S, S)
    np.testing.assert_allclose(P, P_oracle, rtol=0, atol=1e-15)
    Q = _table(src, "kr_projq")
    assert Q.shape == (max(R, 1), S)
    if R:
        # orthonormal rows spanning the conserved rows: Q Q^T = I, N (I - Q^T Q) = 0
        np.testing.assert_allclose(Q @ Q.T, np.eye(R), rtol=0, atol=4e-16 * S)
        np.testing.assert_allclose(np.eye(S) - Q.T @ Q, P_oracle, rtol=0, atol=2e-15)
        assert np.abs(N @ (np.eye(S) - Q.T @ Q)).max() <= 1e-14 * np.abs(N).max()
    # the kernels take the low-rank form where it is cheaper
    assert (2 * R * S < S * S) == {"e1": False, "h_he": False, "h_o_n": True, "stromgren": False,
                                   "astro23": True, "large48": True}[which]
