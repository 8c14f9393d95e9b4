"""Host logic of bench.py (no GPU): the parity summary it prints beside the
CPU baseline, and the refusal of more than one GPU."""
import os
import subprocess
import sys

import numpy as np

import bench
import synthetic as sy

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _case():
    desc = sy.network_h_o_n(1)
    cs = sy.cells_h_o_n(desc, 6, 1)
    idx = np.arange(6)
    n_o = cs.n.copy() * 1.01
    T_o = cs.T * 1.02
    return desc, cs, idx, n_o, T_o


def test_parity_compares_cells_both_sides_integrated():
    desc, cs, idx, n_o, T_o = _case()
    gpu_n, gpu_T = n_o.copy(), T_o.copy()
    gpu_n[0, 1] *= 1.0 + 3e-7                 # a non-reservoir species of cell 1
    gpu_T[4] *= 1.0 + 2e-9
    st = np.zeros(6, dtype=np.int32)
    iters = np.full(6, 10)
    assert 0 not in list(desc.reservoir)
    p = bench.parity(desc, cs, idx, gpu_n, gpu_T, st, (n_o, T_o, st), iters)
    assert abs(p["max_rel_err"] - 3e-7) < 1e-12
    assert p["status_agree"] == 1.0 and p["cells_compared"] == 6
    nnuc = np.abs(np.asarray(desc.composition)[:desc.n_elem]).sum(axis=0) @ cs.n
    major0 = abs(n_o[0, 1]) > 1e-4 * nnuc[1]
    assert abs(p["max_rel_err_major"] - (3e-7 if major0 else 2e-9)) < 1e-12
    # a trace species far off leaves the major-species figure alone
    trace = np.argmin(np.abs(n_o[:, 3]) / nnuc[3])
    assert abs(n_o[trace, 3]) < 1e-4 * nnuc[3] and trace not in list(desc.reservoir)
    g2 = gpu_n.copy()
    g2[trace, 3] *= 2.0
    p2 = bench.parity(desc, cs, idx, g2, gpu_T, st, (n_o, T_o, st), iters)
    assert p2["max_rel_err"] >= 0.99 and p2["max_rel_err_major"] == p["max_rel_err_major"]
    # a reverted cell (status 2, input kept) leaves the error statistics and
    # shows in the status agreement only
    gpu_st = st.copy()
    gpu_st[1] = 2
    gpu_n[:, 1] = cs.n[:, 1]
    p = bench.parity(desc, cs, idx, gpu_n, gpu_T, gpu_st, (n_o, T_o, st), iters)
    assert abs(p["max_rel_err"] - 2e-9) < 1e-14
    assert p["cells_compared"] == 5 and abs(p["status_agree"] - 5 / 6) < 1e-15
    # nothing integrated on both sides: no error statistics
    p = bench.parity(desc, cs, idx, gpu_n, gpu_T, np.full(6, 2, np.int32), (n_o, T_o, st), iters)
    assert p["max_rel_err"] is None and p["cells_compared"] == 0


def test_parity_reservoir_slack():
    """A reservoir species differing by less than 4 sqrt(iterations) eps n_nuc
    counts as equal (the rounding drift of its row's total); above that the
    excess counts."""
    desc, cs, idx, n_o, T_o = _case()
    rs = int(np.asarray(desc.reservoir)[0])
    nnuc = np.abs(np.asarray(desc.composition)[:desc.n_elem]).sum(axis=0) @ cs.n
    iters = np.full(6, 16)
    walk = 4.0 * bench.EPS * 4.0 * nnuc
    st = np.zeros(6, dtype=np.int32)
    gpu_n = n_o.copy()
    gpu_n[rs] += 0.9 * walk
    p = bench.parity(desc, cs, idx, gpu_n, T_o, st, (n_o, T_o, st), iters)
    assert p["max_rel_err"] == 0.0
    gpu_n = n_o.copy()
    gpu_n[rs, 0] += 2.0 * walk[0]
    p = bench.parity(desc, cs, idx, gpu_n, T_o, st, (n_o, T_o, st), iters)
    ref = walk[0] / max(abs(n_o[rs, 0]), bench.FLOOR * nnuc[0])
    assert abs(p["max_rel_err"] / ref - 1.0) < 1e-9


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=ROOT)
    assert r.returncode != 0
    assert "single-GPU" in r.stderr
