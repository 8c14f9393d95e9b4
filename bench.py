#!/usr/bin/env python3
"""Benchmark: cell-steps/s of the implicit thermochemistry update on one GPU.

Workload: 2^20 cells of the 9-species / 3-row / 24-reversible-reaction
combustion-shaped network (energy equation, 10 unknowns per cell), T ~
U[900, 2500] K at 1 atm, each cell integrated over dt = 1e-4 s with adaptive
backward-Euler substeps at rtol 1e-6 (synthetic, seeded inputs).  A step is
one kr_chem_integrate call over all cells from the same initial batch (the
initial state is restored on the device before each step, a copy of ~100 MB
that is <0.1% of a step).

Variants: plain FP64 (the headline), the FP32 LU form with FP64
refinement, the same with the learned Newton guess, and the paper's single-
and mixed-precision modes (FP32 integration; the latter with the final
abundance update in FP64).

Prints one JSON line (metric, value, configuration and variants), with a
roofline object for the integrator kernel (FP64 VALU bound, algorithmic
flops from the per-cell Newton/substep counts the kernel returns, timed with
HIP events on the launch stream) and the CPU oracle timed on a bounded
sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6e12          # MI355X FP64 vector, flop/s
PEAK_FP32 = 157.3e12         # MI355X FP32 vector, flop/s
SHORT_DT = 1e-7              # the learned guess's short-step leg (s)
C_EXP = 27.0                 # FP64 exp / log counted as 27 flops each (range
                             # reduction + degree-11 polynomial + scaling)


def flops_per_unit(desc):
    """Algorithmic FP64 flops of one Newton iteration and of one right-hand
    side evaluation (the error estimate), from the network's structure.

    Per direction d with m reactant slots: rate argument and coefficient
    (4 + exp), slot products (m), d/dT (3), d/dn by the product rule
    (m (m - 1) + m); per reaction: w and dw (1 + #columns), scatter into g
    and J (2 flops per touched entry, energy row included).  Per iteration:
    assembly 2 N^2 + residual 3 N, LU 2N^3/3, solve 2 N^2, update and
    convergence 4 N.  Plus log T and 1/T."""
    S = desc.n_species
    N = S + 1
    nu = desc.stoich()
    f_eval = 2 * C_EXP
    f_rhs = 2 * C_EXP
    for r in range(desc.n_reactions):
        cols = set()
        for side in (desc.reac[r], desc.prod[r]):
            sl = [s for s in side if s >= 0]
            m = len(sl)
            f_eval += 4 + C_EXP + m + 3 + m * (m - 1) + m
            f_rhs += 4 + C_EXP + m
            cols |= set(sl)
        nnz = int(np.count_nonzero(nu[r])) + 1          # species rows + energy row
        f_eval += 2 + len(cols) + 2 * nnz * (len(cols) + 1) + 2 * nnz
        f_rhs += 1 + 2 * nnz
    # temperature-dependent heat capacities: per species c_V and e (two
    # degree-4/5 Horner chains) and the two sums; tabulated factors: the
    # lookup (index, fraction, interpolation, slope) per tabulated reaction
    if getattr(desc, "cv_poly", None) is not None:
        f_eval += S * (8 + 10 + 4)
        f_rhs += S * (8 + 10 + 4)
    if getattr(desc, "tab_of", None) is not None:
        n_tab = int(np.count_nonzero(np.asarray(desc.tab_of) >= 0))
        f_eval += 8 * n_tab
        f_rhs += 8 * n_tab
    f_it = f_eval + 2 * N * N + 3 * N + (2.0 / 3.0) * N ** 3 + 2 * N * N + 4 * N
    return f_it, f_rhs


PROFILE = os.path.join(ROOT, "profiles", "kr_integrate_fp64_h_o_n_1M.md")
PROFILE_ADVECT = os.path.join(ROOT, "profiles", "kr_advect_h_o_n_1M.md")


def measured_traffic(kernel_source, profile=PROFILE, key="traffic_bytes"):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on this exact kernel (hash of the generated device source); else
    None."""
    import hashlib
    import re
    try:
        text = open(profile).read()
        rec = json.loads(re.search(r"```json\n(.*?)```", text, re.S).group(1))
    except (OSError, AttributeError, ValueError):
        return None
    if rec.get("source_sha256") != hashlib.sha256(kernel_source.encode()).hexdigest():
        return None
    return rec.get(key)


EPS = float(np.finfo(np.float64).eps)
FLOOR = 1e-20


def parity(desc, cs, idx, gpu_n, gpu_T, gpu_status, orc, iters):
    """Relative error of GPU results on the sampled cells against the
    oracle's: abundances over max(|oracle|, 1e-20 n_nuc), T over T; the
    reservoir species of each conserved row first get the stage-2 rounding
    drift of the row totals, 4 sqrt(Newton iterations) eps n_nuc (the parity
    tests' gate).  The errors cover the cells both sides integrated (status
    0): a reverted cell keeps its input by design, which status agreement
    reports.  Returns max and 99.9th percentile, the max over species above
    1e-4 of the nuclei density and T, status agreement and the number of
    cells compared."""
    n_o, T_o, st_o = orc
    ok = (np.asarray(gpu_status) == 0) & (np.asarray(st_o) == 0)
    out = {"status_agree": float(np.mean(gpu_status == st_o)), "cells": int(idx.size),
           "cells_compared": int(ok.sum())}
    if not ok.any():
        return {"max_rel_err": None, "p99.9_rel_err": None, "max_rel_err_major": None, **out}
    sub_n = cs.n[:, idx][:, ok]
    nnuc = np.abs(np.asarray(desc.composition)[:desc.n_elem]).sum(axis=0) @ sub_n
    n_o, gpu_n = n_o[:, ok], gpu_n[:, ok]
    slack = np.zeros_like(n_o)
    walk = 4.0 * EPS * np.sqrt(np.maximum(iters[ok], 1).astype(float)) * nnuc
    for rs in np.unique(np.asarray(desc.reservoir)):
        slack[rs] = walk
    err = np.maximum(np.abs(gpu_n - n_o) - slack, 0.0) / np.maximum(np.abs(n_o), FLOOR * nnuc[None, :])
    terr = np.abs(gpu_T[ok] - T_o[ok]) / np.abs(T_o[ok])
    both = np.concatenate([err.ravel(), terr])
    # the species above 1e-4 of the nuclei density and T: the accuracy the
    # FP32 modes can hold (an FP32 ulp of the nuclei density is far above the
    # FP64 floor, so trace species say nothing about them)
    major = np.concatenate([err[np.abs(n_o) > 1e-4 * nnuc[None, :]], terr])
    return {"max_rel_err": float(both.max()), "p99.9_rel_err": float(np.percentile(both, 99.9)),
            "max_rel_err_major": float(major.max()), **out}


def cpu_baseline(desc, cs, dt_scalar, sample, seed=7, dt=None, gpu=None, one_core=256):
    """The oracle on a seeded sample of the batch, on every host core and on
    one; with gpu = {variant: (n [S, sample], T, status, newton iterations)}
    of the same sampled cells, also the parity of each variant against the
    oracle's results."""
    import oracle
    oracle.build(force=False)
    rng = np.random.default_rng(seed)
    idx = np.sort(rng.choice(cs.n.shape[1], size=sample, replace=False))
    on = oracle.OracleNet(desc)
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    n_o, T_o, st_o, stats_o = on.integrate(cs.n[:, idx], cs.T[idx], cs.rho[idx],
                                           dt=None if dt is None else dt[idx],
                                           dt_scalar=dt_scalar, nthreads=cores)
    el = time.perf_counter() - t0
    k1 = min(one_core, sample)
    t0 = time.perf_counter()
    on.integrate(cs.n[:, idx[:k1]], cs.T[idx[:k1]], cs.rho[idx[:k1]],
                 dt=None if dt is None else dt[idx[:k1]], dt_scalar=dt_scalar, nthreads=1)
    el1 = time.perf_counter() - t0
    out = {"value": sample / el, "unit": "cell-steps/s", "cores": cores, "kind": "oracle",
           "sample": f"{sample} cells drawn uniformly (seed {seed}) from the same {cs.n.shape[1]}-cell "
                     f"batch, FP64 C oracle, OpenMP over {cores} threads, {el:.1f} s; the first {k1} "
                     f"of them on 1 thread, {el1:.1f} s",
           "value_1_core": k1 / el1}
    if gpu:
        out["parity"] = {v: parity(desc, cs, idx, g[0][:, idx], g[1][idx], g[2][idx], (n_o, T_o, st_o),
                                   stats_o[:, 1])
                         for v, g in gpu.items()}
    return out


MIX_FRACTIONS = (0.5, 0.3, 0.2)
# per-network step ranges, dt = tau_fast * 10^U[lo, hi], read off the
# calibration table (bench.py --workload calibrate, 16384 cells per network)
# so that the largest substep count of each network stays near 200
MIX_U_RANGES = ((-4.0, -1.0), (-5.5, -4.0), (-4.0, -2.0))


def _mix_descs():
    import synthetic as sy
    return [sy.network_h_he(0), sy.network_h_o_n(1), sy.network_astro23(2)]


def _cells(name):
    def make(d, n):
        import synthetic as sy
        return getattr(sy, name)(d, n, {"cells_h_he": 0, "cells_h_o_n": 1, "cells_astro23": 2}[name])
    return make


_MIX_MAKERS = [_cells("cells_h_he"), _cells("cells_h_o_n"), _cells("cells_astro23")]


def run_mixed(args):
    """Uneven batch in one persistent launch: 2^22 cells mixing the 6-, 10-
    and 24-unknown networks (50/30/20%), each cell's step a seeded multiple
    10^U[lo, hi] (per network, MIX_U_RANGES) of its own fastest timescale,
    FP32 LU with FP64 refinement, one hipGraph-replayed launch per step; the
    5- and 9-species networks run one cell per lane, the 23-species one one
    cell per wavefront (or as the autotuner picks)."""
    import torch
    import paper_2504_04941_amd as kr
    import synthetic as sy
    from paper_2504_04941_amd import autotune

    dev = torch.device("cuda", 0)
    descs = _mix_descs()
    makers = _MIX_MAKERS
    counts = [int(args.cells * f) for f in MIX_FRACTIONS]
    counts[0] += args.cells - sum(counts)
    bo = kr.build_options()
    t0 = time.perf_counter()
    base_nets = [kr.Network(d) for d in descs]
    init, bufs = [], []
    for k, (d, mk, n) in enumerate(zip(descs, makers, counts)):
        cs = mk(d, n)
        n0 = torch.tensor(cs.n, device=dev)
        T0 = torch.tensor(cs.T, device=dev)
        tau = kr.fastest_timescale(base_nets[k], n0, T0)
        lo, hi = MIX_U_RANGES[k]
        dt = tau * torch.tensor(sy.log_uniform(n, 10 ** lo, 10 ** hi, 2, 300 + k), device=dev)
        init.append((n0, T0))
        bufs.append({"states": n0.clone(), "T": T0.clone(), "dt": dt,
                     "status": torch.empty(n, dtype=torch.int32, device=dev),
                     "cell_stats": torch.empty((n, 4), dtype=torch.int32, device=dev)})
    setup_s = time.perf_counter() - t0
    report = None
    layouts = [_layout_code(kr, L) for L in args.mix_layouts.split(",")]
    if len(layouts) != len(descs):
        raise SystemExit(f"--mix-layouts needs {len(descs)} entries")
    if args.autotune:
        # tuned on the whole batch: the layouts' relative speed depends on how
        # many cells each lane or wavefront gets (a 1/64 sample picked the
        # wavefront layout for the 9-species network, which is slower at size)
        bo, layouts, report = autotune.tune_multi(descs, bufs, precision=kr.KR_FP32LU_REFINE,
                                                  candidates=[(0, 0.1), (1, 0.1)],
                                                  log=lambda s: print("# " + s, file=sys.stderr, flush=True))
    nets = [kr.Network(d, kr.build_options(waves_per_eu=bo.waves_per_eu, pivot_tau=bo.pivot_tau, layout=L))
            for d, L in zip(descs, layouts)]
    multi = kr.Multi(nets, bo)
    order = _order(args)
    if report is not None and args.order == _ORDER_DEFAULT["mixed"]:
        order = report["order"]          # the tuner's choice unless --order was given
        args.order = "work" if order == kr.KR_ORDER_WORK else "input"
    opts = kr.default_options(precision=kr.KR_FP32LU_REFINE, order=order)
    stream = torch.cuda.current_stream()

    def step():
        for (n0, T0), b in zip(init, bufs):
            b["states"].copy_(n0)
            b["T"].copy_(T0)
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        multi.integrate(bufs, rtol=1e-6, opts=opts, use_graph=True, stream=stream)
        ev1.record(stream)
        return ev0, ev1

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_s = np.mean([a.elapsed_time(b) for a, b in evs]) * 1e-3
    flops, per_net = 0.0, {}
    for d, b in zip(descs, bufs):
        st = b["cell_stats"].cpu().numpy().astype(np.int64)
        f_it, f_rhs = flops_per_unit(d)
        flops += st[:, 1].sum() * f_it + (st[:, 0] + st[:, 2]).sum() * f_rhs
        acc = st[:, 0]
        per_net[d.name] = {"cells": int(acc.size), "newton_per_cell": float(st[:, 1].mean()),
                           "substep_histogram": {"1": int((acc <= 1).sum()),
                                                 "2-10": int(((acc > 1) & (acc <= 10)).sum()),
                                                 "11-50": int(((acc > 10) & (acc <= 50)).sum()),
                                                 "51-200": int(((acc > 50) & (acc <= 200)).sum()),
                                                 ">200": int((acc > 200).sum())},
                           "status_counts": np.bincount(b["status"].cpu().numpy(), minlength=3).tolist()}
    launches, captures = multi.graph_stats()
    out = {"metric": "cell-steps/s implicit chem update, uneven multi-network batch, 1 GPU",
           "value": args.cells * args.steps / wall, "unit": "cell-steps/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64+f32lu",
           "data": "synthetic",
           "config": {"workload": f"mixed: {args.cells} cells, 5/9/23-species networks 50/30/20%, "
                                  f"dt = tau_fast*10^U[range] per network {list(MIX_U_RANGES)}, FP32 LU + "
                                  "FP64 refinement, one hipGraph launch (one persistent kernel per occupancy group)",
                      "build": [bo.waves_per_eu, bo.pivot_tau], "cell_order": args.order,
                      "layouts": [{1: "lane", 16: "group16", 32: "group32", 64: "wave"}[n.group] for n in nets]},
           "per_network": per_net, "graph": {"launches": launches, "captures": captures},
           "autotune": report, "setup_s": setup_s,
           "roofline": {"bound": "alu", "achieved": flops / kernel_s / 1e12, "peak": PEAK_FP64 / 1e12,
                        "unit": "TFLOP/s", "frac": flops / kernel_s / PEAK_FP64, "traffic": None,
                        "kernel": "kr_integrate_multi_fp32lu_*"}}
    print(json.dumps(out), flush=True)


def run_large(args):
    """Large network: 48 species / 200 reversible reactions / 5 element rows
    + energy (49x49 LU), one cell per wavefront; per-cell steps log-uniform
    in [1e-8, 1e-2] s; plain FP64 and the FP32 LU form."""
    import torch
    import paper_2504_04941_amd as kr
    import synthetic as sy

    dev = torch.device("cuda", 0)
    desc = sy.network_large48(3)
    cs = sy.cells_large48(desc, args.cells, 3)
    t0 = time.perf_counter()
    net = kr.Network(desc)
    setup_s = time.perf_counter() - t0
    n0 = torch.tensor(cs.n, device=dev)
    T0 = torch.tensor(cs.T, device=dev)
    dt = torch.tensor(cs.dt, device=dev)
    n, T = torch.empty_like(n0), torch.empty_like(T0)
    status = torch.empty(args.cells, dtype=torch.int32, device=dev)
    stats = torch.empty((args.cells, 4), dtype=torch.int32, device=dev)
    counters = torch.zeros(8, dtype=torch.int64, device=dev)
    f_it, f_rhs = flops_per_unit(desc)
    stream = torch.cuda.current_stream()
    results, gpu_out = {}, {}
    net_mfma = None
    for variant in args.variants.split(","):
        prec = {"fp64": kr.KR_FP64, "fp32lu": kr.KR_FP32LU_REFINE, "fp32lu+mfma": kr.KR_FP32LU_REFINE}.get(variant)
        if prec is None:
            continue
        vnet = net
        if variant == "fp32lu+mfma":
            # the FP32 LU blocked, its trailing updates on MFMA tiles
            net_mfma = net_mfma or kr.Network(desc, kr.build_options(lu_mfma=1))
            vnet = net_mfma
        opts = kr.default_options(precision=prec, order=_order(args))
        opts.counters = counters.data_ptr()

        def step():
            n.copy_(n0)
            T.copy_(T0)
            counters.zero_()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            kr.chem_integrate(vnet, n, T, dt=dt, rtol=1e-6, opts=opts, status=status, cell_stats=stats,
                              stream=stream)
            ev1.record(stream)
            return ev0, ev1

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        evs = [step() for _ in range(args.steps)]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kernel_s = np.mean([a.elapsed_time(b) for a, b in evs]) * 1e-3
        st = stats.cpu().numpy().astype(np.int64)
        acc = st[:, 0]
        flops = st[:, 1].sum() * f_it + (st[:, 0] + st[:, 2]).sum() * f_rhs
        gpu_out[variant] = (n.cpu().numpy(), T.cpu().numpy(), status.cpu().numpy(), st[:, 1])
        results[variant] = {
            "ms_per_step": wall / args.steps * 1e3, "value": args.cells * args.steps / wall,
            "kernel_ms": kernel_s * 1e3, "flops_per_launch": float(flops),
            "achieved_tflops": flops / kernel_s / 1e12,
            "newton_iters_per_cell": float(st[:, 1].mean()), "substeps_per_cell": float(acc.mean()),
            "max_substeps": int(acc.max()),
            "substep_histogram": {"1": int((acc <= 1).sum()), "2-10": int(((acc > 1) & (acc <= 10)).sum()),
                                  "11-200": int(((acc > 10) & (acc <= 200)).sum()),
                                  "201-10^4": int(((acc > 200) & (acc <= 10000)).sum()),
                                  ">10^4": int((acc > 10000).sum())},
            "status_counts": np.bincount(status.cpu().numpy(), minlength=3).tolist(),
            "counters_last_step": dict(zip(("guess_starts", "guess_fallbacks", "row_exchanges",
                                            "fp32_solves", "fp64_fallbacks"),
                                           counters.cpu().numpy()[:5].tolist()))}
        print(f"# {variant}: {results[variant]}", file=sys.stderr, flush=True)
    head = results.get("fp64") or next(iter(results.values()))
    out = {"metric": "cell-steps/s implicit chem update, 48-species network, 1 GPU",
           "value": head["value"], "unit": "cell-steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"large_48sp: {args.cells} cells, 48 species / 200 reversible reactions / "
                                  "5 element rows + energy (49x49 LU), dt log-uniform [1e-8, 1e-2] s, rtol 1e-6, "
                                  "one cell per wavefront",
                      "layout": "wave" if net.wide else "lane", "cell_order": args.order},
           "variants": results, "setup_s": setup_s,
           "roofline": {"bound": "alu", "achieved": head["achieved_tflops"], "peak": PEAK_FP64 / 1e12,
                        "unit": "TFLOP/s", "frac": head["achieved_tflops"] * 1e12 / PEAK_FP64, "traffic": None,
                        "kernel": "kr_integrate_fp64", "flops_per_newton_iteration": f_it,
                        "flops_per_error_estimate": f_rhs}}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(desc, cs, 0.0, min(args.cpu_sample, args.cells), dt=cs.dt, gpu=gpu_out,
                                           one_core=4)
    print(json.dumps(out), flush=True)
    net.close()


LAYOUT_NAMES = ["auto", "lane", "wave", "group16", "group32"]


def _layout_code(kr, name):
    return {"auto": kr.KR_LAYOUT_AUTO, "lane": kr.KR_LAYOUT_LANE, "wave": kr.KR_LAYOUT_WAVE,
            "group16": kr.KR_LAYOUT_GROUP16, "group32": kr.KR_LAYOUT_GROUP32}[name]


def run_h_he(args):
    """Small case: 4096 cells of the 5-species H/He/charge network (10
    reversible reactions, 6 unknowns), each cell's step 1e3 times its own
    fastest timescale, adaptive, rtol 1e-6; plain FP64, the FP32 LU form
    and the paper's single- and mixed-precision modes."""
    import torch
    import paper_2504_04941_amd as kr
    import synthetic as sy

    dev = torch.device("cuda", 0)
    desc = sy.network_h_he(0)
    cs = sy.cells_h_he(desc, args.cells, 0)
    net = kr.Network(desc, kr.build_options(layout=_layout_code(kr, args.layout)))
    n0 = torch.tensor(cs.n, device=dev)
    T0 = torch.tensor(cs.T, device=dev)
    dt = 1e3 * kr.fastest_timescale(net, n0, T0)
    n, T = torch.empty_like(n0), torch.empty_like(T0)
    status = torch.empty(args.cells, dtype=torch.int32, device=dev)
    stats = torch.empty((args.cells, 4), dtype=torch.int32, device=dev)
    f_it, f_rhs = flops_per_unit(desc)
    stream = torch.cuda.current_stream()
    results, gpu_out = {}, {}
    for variant in args.variants.split(","):
        if net.wide and variant in ("single", "mixed"):
            continue                      # the FP32 modes run in the lane layout only
        opts = kr.default_options(precision=variant)

        def step():
            n.copy_(n0)
            T.copy_(T0)
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            kr.chem_integrate(net, n, T, dt=dt, rtol=1e-6, opts=opts, status=status, cell_stats=stats,
                              stream=stream)
            ev1.record(stream)
            return ev0, ev1

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        evs = [step() for _ in range(args.steps)]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kernel_s = np.mean([a.elapsed_time(b) for a, b in evs]) * 1e-3
        st = stats.cpu().numpy().astype(np.int64)
        flops = st[:, 1].sum() * f_it + (st[:, 0] + st[:, 2]).sum() * f_rhs
        resid = torch.empty(args.cells, dtype=torch.float64, device=dev)
        kr.element_residual(net, n0, n, resid=resid)
        gpu_out[variant] = (n.cpu().numpy(), T.cpu().numpy(), status.cpu().numpy(), st[:, 1])
        results[variant] = {"ms_per_step": wall / args.steps * 1e3, "value": args.cells * args.steps / wall,
                            "kernel_ms": kernel_s * 1e3, "achieved_tflops": flops / kernel_s / 1e12,
                            "newton_iters_per_cell": float(st[:, 1].mean()),
                            "max_newton_iters": int(st[:, 1].max()),
                            "substeps_per_cell": float(st[:, 0].mean()),
                            "status_counts": np.bincount(status.cpu().numpy(), minlength=3).tolist(),
                            "max_element_residual": float(resid.max().item())}
        print(f"# {variant}: {results[variant]}", file=sys.stderr, flush=True)
    head = results["fp64"]
    out = {"metric": "cell-steps/s implicit chem update, 5-species H/He network, 1 GPU",
           "value": head["value"], "unit": "cell-steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"h_he_5sp: {args.cells} cells, 5 species / 10 reversible reactions / "
                                  "H, He, charge rows + energy (6x6 LU), dt = 1e3 tau_fast per cell, "
                                  "adaptive, rtol 1e-6, one cell per " + ("wavefront" if net.wide else "lane")},
           "variants": results,
           "roofline": {"bound": "alu", "achieved": head["achieved_tflops"], "peak": PEAK_FP64 / 1e12,
                        "unit": "TFLOP/s", "frac": head["achieved_tflops"] * 1e12 / PEAK_FP64, "traffic": None,
                        "kernel": "kr_integrate_fp64", "flops_per_newton_iteration": f_it,
                        "flops_per_error_estimate": f_rhs}}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(desc, cs, 0.0, args.cells, dt=dt.cpu().numpy(), gpu=gpu_out,
                                           one_core=args.cells)
    print(json.dumps(out), flush=True)
    net.close()


def run_stromgren(args):
    """Photo-ionisation chemistry (Sec. 4.3's hydrogen network: photo- and
    collisional ionisation, case-B recombination, photo-heating and
    recombination cooling) on 2^20 cells of an H II region around the
    fiducial source (synthetic.cells_stromgren: per-cell flux, path length,
    density, ionised fraction, temperature and step), one cell per lane."""
    import torch
    import paper_2504_04941_amd as kr
    import synthetic as sy

    dev = torch.device("cuda", 0)
    desc = sy.network_stromgren()
    cs, F_h, L_h = sy.cells_stromgren(desc, args.cells)
    net = kr.Network(desc)
    n0 = torch.tensor(cs.n, device=dev)
    T0 = torch.tensor(cs.T, device=dev)
    dt = torch.tensor(cs.dt, device=dev)
    F = torch.tensor(F_h, device=dev)
    L = torch.tensor(L_h, device=dev)
    n, T = torch.empty_like(n0), torch.empty_like(T0)
    status = torch.empty(args.cells, dtype=torch.int32, device=dev)
    stats = torch.empty((args.cells, 4), dtype=torch.int32, device=dev)
    f_it, f_rhs = flops_per_unit(desc)
    stream = torch.cuda.current_stream()
    results, gpu_out = {}, {}
    for variant in args.variants.split(","):
        opts = kr.default_options(precision=variant, order=_order(args))

        def step():
            n.copy_(n0)
            T.copy_(T0)
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            kr.chem_integrate(net, n, T, dt=dt, rtol=1e-6, opts=opts, status=status, cell_stats=stats,
                              stream=stream, photo_flux=F, photo_length=L)
            ev1.record(stream)
            return ev0, ev1

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        evs = [step() for _ in range(args.steps)]
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kernel_s = np.mean([a.elapsed_time(b) for a, b in evs]) * 1e-3
        st = stats.cpu().numpy().astype(np.int64)
        flops = st[:, 1].sum() * f_it + (st[:, 0] + st[:, 2]).sum() * f_rhs
        resid = torch.empty(args.cells, dtype=torch.float64, device=dev)
        kr.element_residual(net, n0, n, resid=resid)
        gpu_out[variant] = (n.cpu().numpy(), T.cpu().numpy(), status.cpu().numpy(), st[:, 1])
        results[variant] = {"ms_per_step": wall / args.steps * 1e3, "value": args.cells * args.steps / wall,
                            "kernel_ms": kernel_s * 1e3, "achieved_tflops": flops / kernel_s / 1e12,
                            "newton_iters_per_cell": float(st[:, 1].mean()),
                            "substeps_per_cell": float(st[:, 0].mean()), "max_substeps": int(st[:, 0].max()),
                            "status_counts": np.bincount(status.cpu().numpy(), minlength=3).tolist(),
                            "max_element_residual": float(resid.max().item())}
        print(f"# {variant}: {results[variant]}", file=sys.stderr, flush=True)
    head_name = "fp64" if "fp64" in results else next(iter(results))
    head = results[head_name]
    peak = PEAK_FP32 if head_name in ("single", "mixed") else PEAK_FP64
    out = {"metric": "cell-steps/s implicit chem update, photo-ionisation (Stromgren) network, 1 GPU",
           "value": head["value"], "unit": "cell-steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32" if peak == PEAK_FP32 else "f64",
           "data": "synthetic",
           "config": {"workload": f"stromgren: {args.cells} cells, H/H+/e- with photo- and collisional ionisation, "
                                  "recombination, photo-heating and recombination cooling, per-cell flux and path "
                                  "length (Phi = 1e49 s^-1 source, 1/4 pc cells), dt log-uniform [1e8, 1e12] s, "
                                  "rtol 1e-6, one cell per lane", "cell_order": args.order},
           "variants": results,
           "roofline": {"bound": "alu", "achieved": head["achieved_tflops"], "peak": peak / 1e12,
                        "unit": "TFLOP/s", "frac": head["achieved_tflops"] * 1e12 / peak, "traffic": None,
                        "kernel": "kr_integrate_" + head_name, "flops_per_newton_iteration": f_it,
                        "flops_per_error_estimate": f_rhs}}
    if not args.no_cpu_baseline:
        import oracle
        oracle.build(force=False)
        # these cells cost the oracle about a quarter of a combustion cell:
        # four times the sample keeps the CPU leg at several seconds
        k = min(4 * args.cpu_sample, args.cells)
        rng = np.random.default_rng(7)
        idx = np.sort(rng.choice(args.cells, size=k, replace=False))
        on = oracle.OracleNet(desc)
        cores = len(os.sched_getaffinity(0))
        t1 = time.perf_counter()
        r = on.integrate_ex(cs.n[:, idx], cs.T[idx], dt=cs.dt[idx], nthreads=cores, photo_flux=F_h[idx],
                            photo_length=L_h[idx])
        el = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": k / el, "unit": "cell-steps/s", "cores": cores, "kind": "oracle",
                               "sample": f"{k} cells drawn uniformly (seed 7) from the same batch, FP64 C oracle, "
                                         f"OpenMP over {cores} threads, {el:.1f} s",
                               "parity": {v: parity(desc, cs, idx, g[0][:, idx], g[1][idx], g[2][idx],
                                                    (r["n"], r["T"], r["status"]), r["stats"][:, 1])
                                          for v, g in gpu_out.items()}}
    print(json.dumps(out), flush=True)
    net.close()


def run_advect(args):
    """Species advection (Sec. 2.1): one SSP-RK2 step of the
    stoichiometry-compatible PLM over lines of cells with periodic ends,
    9-species combustion network, non-uniform grid, density and velocity per
    line as synthetic.advection_lines draws them.  HBM bound.  Fused form
    (kr_advect_plm_ssprk2, the default): per cell and step the algorithmic
    traffic is (2 S + 4) 8 bytes (n in and out, both stages' density and
    face flux).  Two-stage form (--advect-form stages, two kr_advect_plm
    calls): (5 S + 4) 8 bytes (stage 1 reads n, rho, the face flux and
    writes n; stage 2 also reads the step's initial state)."""
    import torch
    import paper_2504_04941_amd as kr
    import synthetic as sy

    dev = torch.device("cuda", 0)
    desc = {"h_o_n": lambda: sy.network_h_o_n(1), "astro23": lambda: sy.network_astro23(2),
            "large48": lambda: sy.network_large48(3)}[args.advect_net]()
    S = desc.n_species
    n_cells = 256
    n_lines = max(1, args.cells // n_cells)
    t0 = time.perf_counter()
    n_h, rho_h, xc_h, xf_h, v = sy.advection_lines(desc, n_lines, n_cells)
    F_h = np.empty_like(rho_h)
    for l in range(n_lines):
        r = rho_h[l * n_cells:(l + 1) * n_cells]
        F_h[l * n_cells:(l + 1) * n_cells] = (np.roll(r, 1) if v[l] > 0 else r) * v[l]
    setup_s = time.perf_counter() - t0
    net = kr.Network(desc)
    u0 = torch.tensor(n_h, device=dev)
    u = u0.clone()
    u1 = torch.empty_like(u0)
    u2 = torch.empty_like(u0)
    rho = torch.tensor(rho_h, device=dev)
    F = torch.tensor(F_h, device=dev)
    # the second stage's density and fluxes in buffers of their own (equal
    # values: see the note in step())
    rho1, F1 = rho.clone(), F.clone()
    fused = args.advect_form == "fused"
    xc, xf = torch.tensor(xc_h, device=dev), torch.tensor(xf_h, device=dev)
    dt = 0.4 * float(np.min(np.diff(xf_h)))
    stream = torch.cuda.current_stream()

    def step():
        # the density is held fixed across the step: a stage's fluxes move
        # mass as the density's own update would, whose effect on the species
        # per mass the test of the kernel covers; the work per cell is the same
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        if fused:
            kr.advect_plm_ssprk2(net, u, u2, rho, F, rho1, F1, xc, xf, dt, n_lines=n_lines, stream=stream)
        else:
            kr.advect_plm(net, u, u1, rho, F, xc, xf, dt, n_lines=n_lines, stream=stream)
            kr.advect_plm(net, u1, u2, rho1, F1, xc, xf, dt, n_lines=n_lines, base=u, alpha=0.5, beta=0.5,
                          stream=stream)
        ev1.record(stream)
        return ev0, ev1

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    evs = [step() for _ in range(args.steps)]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_s = float(np.mean([a.elapsed_time(b) for a, b in evs])) * 1e-3
    cells = n_lines * n_cells
    per_cell = (2 * S + 4) * 8 if fused else (5 * S + 4) * 8
    bytes_step = cells * float(per_cell)
    out = {"metric": "cell-steps/s species advection (projected PLM, SSP-RK2), 1 GPU",
           "value": cells * args.steps / wall, "unit": "cell-steps/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"advect: {n_lines} periodic lines x {n_cells} cells, {desc.name}, "
                                  "non-uniform grid, projected PLM, SSP-RK2 "
                                  + ("(both stages in one kernel)" if fused else "(2 stage kernels)")},
           "kernel_ms_per_step": kernel_s * 1e3, "setup_s": setup_s,
           "roofline": {"bound": "hbm", "achieved": bytes_step / kernel_s / 1e9, "peak": 8000.0, "unit": "GB/s",
                        "frac": bytes_step / kernel_s / 8e12,
                        "traffic": (measured_traffic(kr.network_check(desc), PROFILE_ADVECT, "traffic_bytes_per_step")
                                    if fused else None),
                        "kernel": "kr_advect2" if fused else "kr_advect", "bytes_per_cell_step": per_cell}}
    if not args.no_cpu_baseline:
        from oracle import plm
        P = plm.projector_svd(desc.composition)
        k = n_lines
        got = u2.cpu().numpy()
        cores = len(os.sched_getaffinity(0))
        t1 = time.perf_counter()
        worst = 0.0
        for l in range(k):
            sl = slice(l * n_cells, (l + 1) * n_cells)
            n1, _ = plm.stage(n_h[:, sl], rho_h[sl], F_h[sl], xc_h, xf_h, dt, P)
            n2, _ = plm.stage(n1, rho_h[sl], F_h[sl], xc_h, xf_h, dt, P)
            ref = 0.5 * (n_h[:, sl] + n2)
            worst = max(worst, float(np.abs(got[:, sl] - ref).max() / np.abs(n_h[:, sl]).max()))
        el = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": k * n_cells / el, "unit": "cell-steps/s", "cores": 1, "kind": "oracle",
                               "sample": f"{k} lines of {n_cells} cells, numpy FP64 reference (one thread), "
                                         f"{el:.2f} s",
                               "parity": {"max_rel_err": worst, "cells": k * n_cells}}
    print(json.dumps(out), flush=True)
    net.close()


def calibrate_mixed(args):
    """Substep-count distribution of each network of the uneven batch for
    steps dt = tau_fast * 10^u over a grid of u (16384 cells per network,
    same seeded cell recipe as the batch): the table the per-network step
    ranges of the uneven batch were read from."""
    import torch
    import paper_2504_04941_amd as kr
    import synthetic as sy

    dev = torch.device("cuda", 0)
    n_cells = 16384
    grid = [float(u) for u in np.arange(-6.0, -0.99, 0.5)]
    out = {}
    for k, (d, mk) in enumerate(zip(_mix_descs(), _MIX_MAKERS)):
        cs = mk(d, n_cells)
        net = kr.Network(d)
        n0 = torch.tensor(cs.n, device=dev)
        T0 = torch.tensor(cs.T, device=dev)
        tau = kr.fastest_timescale(net, n0, T0)
        rows = {}
        for u in grid:
            n = n0.clone()
            T = T0.clone()
            st = torch.empty((n_cells, 4), dtype=torch.int32, device=dev)
            status = torch.empty(n_cells, dtype=torch.int32, device=dev)
            kr.chem_integrate(net, n, T, dt=tau * 10.0 ** u, rtol=1e-6,
                              opts=kr.default_options(precision=kr.KR_FP32LU_REFINE),
                              status=status, cell_stats=st)
            a = st[:, 0].cpu().numpy()
            rows[f"{u:+.1f}"] = {"p50": float(np.median(a)), "p90": float(np.percentile(a, 90)),
                                 "p99": float(np.percentile(a, 99)), "max": int(a.max()),
                                 "newton_per_cell": float(st[:, 1].float().mean()),
                                 "status_counts": np.bincount(status.cpu().numpy(), minlength=3).tolist()}
            print(f"# {d.name} u={u:+.1f}: {rows[f'{u:+.1f}']}", file=sys.stderr, flush=True)
        out[d.name] = rows
        net.close()
    print(json.dumps({"calibration": out, "cells_per_network": n_cells}), flush=True)


# cell order per workload (measured on MI355X): largest expected work first
# for the long, uneven cells of the combustion and 48-species batches; input
# order (coalesced state accesses, no extra rate evaluation) for the mixed
# batch, whose cells mostly take one substep
_ORDER_DEFAULT = {"h_o_n": "work", "h_o_n_tcv": "work", "stromgren": "work", "large48": "work", "mixed": "input", "calibrate": "input",
                  "h_he": "input", "advect": "input"}


def _order(args):
    import paper_2504_04941_amd as kr
    if args.order == "default":
        args.order = _ORDER_DEFAULT[args.workload]
    return kr.KR_ORDER_WORK if args.order == "work" else kr.KR_ORDER_INPUT


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="h_o_n",
                    choices=["h_o_n", "h_o_n_tcv", "h_he", "mixed", "large48", "calibrate", "advect",
                             "stromgren"])
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--mix-layouts", default="auto,auto,auto",
                    help="per-network layouts of the uneven batch (5, 9, 23 species), from " + ",".join(LAYOUT_NAMES))
    ap.add_argument("--layout", default="auto", choices=LAYOUT_NAMES,
                    help="h_he workload: the integrator layout")
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--cells", type=int, default=1 << 20)
    ap.add_argument("--variants", default="fp64,fp32lu,fp32lu+mlp,single,mixed")
    ap.add_argument("--train-pairs", type=int, default=1 << 24)
    ap.add_argument("--train-steps", type=int, default=4000)
    ap.add_argument("--cpu-sample", type=int, default=8192)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--advect-net", default="h_o_n", choices=["h_o_n", "astro23", "large48"],
                    help="advect workload: the network whose species are advected")
    ap.add_argument("--advect-form", default="fused", choices=["fused", "stages"],
                    help="advect workload: both SSP-RK2 stages in one kernel, or two stage kernels")
    ap.add_argument("--order", default="default", choices=["default", "work", "input"],
                    help="order in which the persistent kernel hands out cells: largest expected "
                         "work first or input order (default: the faster one for the workload)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the per-cell integration needs no communication "
              "between GPUs, and only the single-GPU path is implemented (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    if args.workload == "calibrate":
        calibrate_mixed(args)
        return
    if args.workload == "advect":
        run_advect(args)
        return
    if args.workload == "stromgren":
        if args.variants == ap.get_default("variants"):
            args.variants = "fp64,fp32lu,single,mixed"
        if args.cpu_sample == 8192:
            args.cpu_sample = 4096
        run_stromgren(args)
        return
    if args.workload == "h_he":
        if args.cells == 1 << 20:
            args.cells = 4096
        if args.variants == ap.get_default("variants"):
            args.variants = "fp64,fp32lu,single,mixed"
        run_h_he(args)
        return
    if args.workload == "large48":
        if args.cells == 1 << 20:
            args.cells = 1 << 18
        if args.variants == ap.get_default("variants"):
            args.variants = "fp64,fp32lu"
        if args.cpu_sample == 8192:
            args.cpu_sample = 48
        run_large(args)
        return
    if args.workload == "mixed":
        if args.cells == 1 << 20:
            args.cells = 1 << 22
        run_mixed(args)
        return

    import torch
    import paper_2504_04941_amd as kr
    import synthetic as sy

    tcv = args.workload == "h_o_n_tcv"
    if tcv and args.variants == ap.get_default("variants"):
        args.variants = "fp64,fp32lu,single,mixed"
    desc = sy.network_h_o_n_tcv() if tcv else sy.network_h_o_n(1)
    cs = sy.cells_h_o_n(desc, args.cells, 1)
    dt_scalar = cs.dt_scalar
    net = kr.Network(desc)
    dev = torch.device("cuda", 0)
    n0 = torch.tensor(cs.n, device=dev)
    T0 = torch.tensor(cs.T, device=dev)
    n = torch.empty_like(n0)
    T = torch.empty_like(T0)
    status = torch.empty(args.cells, dtype=torch.int32, device=dev)
    stats = torch.empty((args.cells, 4), dtype=torch.int32, device=dev)
    f_it, f_rhs = flops_per_unit(desc)
    stream = torch.cuda.current_stream()

    results = {}
    learned_info = None
    model = None
    if any("mlp" in v for v in args.variants.split(",")):
        from paper_2504_04941_amd import learned
        t0 = time.perf_counter()
        model = kr.GuessModel(net, hidden=256, layers=3, seed=1)
        X, Y, _ = learned.single_step_pairs(net, model, desc, args.train_pairs, salt=1000)
        hist = learned.train(model, X, Y, steps=args.train_steps, batch=4096, lr=1e-3, lr_min=1e-5,
                             log=lambda s: print("# " + s, file=sys.stderr, flush=True))
        del X, Y
        torch.cuda.synchronize()
        train_s = time.perf_counter() - t0
        # held-out single substeps (h log-uniform in [1e-10, 1e-4] s): Newton
        # iterations from the plain start and from the learned start
        evals = {}
        for use in (False, True):
            r = learned.newton_counts(net, model if use else None, desc, 1 << 20, salt=99,
                                      precision=kr.KR_FP32LU_REFINE)
            st_ = r["cell_stats"].cpu().numpy()
            hl = np.floor(np.log10(r["h"].cpu().numpy())).astype(int)
            evals["guess" if use else "plain"] = {
                "newton_per_cell": float(st_[:, 1].mean()),
                "newton_per_cell_by_h_decade": {f"1e{d}": float(st_[hl == d, 1].mean())
                                                for d in range(-10, -4) if np.any(hl == d)},
                "newton_failures": int(st_[:, 3].sum()),
                "status_counts": np.bincount(r["status"].cpu().numpy(), minlength=3).tolist(),
                "guess_starts_fallbacks": r["counters"].cpu().numpy()[:2].tolist()}
        # a short adaptive step (few substeps per cell), where the learned
        # first substep is a large share of the work
        short = {}
        for use in (False, True):
            ns, Ts = n0.clone(), T0.clone()
            st_s = torch.empty((args.cells, 4), dtype=torch.int32, device=dev)
            cnt = torch.zeros(8, dtype=torch.int64, device=dev)
            guess_s = torch.empty((desc.n_unknowns, args.cells), dtype=torch.float64, device=dev)
            o_ = (kr.guess_options(guess_s, cnt, precision=kr.KR_FP32LU_REFINE) if use
                  else kr.default_options(precision=kr.KR_FP32LU_REFINE))
            o_.counters = cnt.data_ptr()
            ts = []
            for rep_ in range(3):
                ns.copy_(n0)
                Ts.copy_(T0)
                cnt.zero_()
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                if use:
                    model.predict(ns, Ts, dt_scalar=SHORT_DT, guess=guess_s, stream=stream)
                kr.chem_integrate(net, ns, Ts, dt_scalar=SHORT_DT, rtol=1e-6, opts=o_, cell_stats=st_s,
                                  stream=stream)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t1)
            sts = st_s.cpu().numpy().astype(np.int64)
            short["guess" if use else "plain"] = {
                "ms": float(np.min(ts) * 1e3), "cell_steps_per_s": args.cells / float(np.min(ts)),
                "newton_per_cell": float(sts[:, 1].mean()), "substeps_per_cell": float(sts[:, 0].mean()),
                "guess_starts_fallbacks": cnt.cpu().numpy()[:2].tolist()}
        learned_info = {"training_pairs": args.train_pairs, "training_steps": args.train_steps,
                        "final_batch_loss": hist[-1][1], "setup_s": train_s,
                        "single_substep_eval_2^20_cells_fp32lu": evals,
                        f"short_step_dt_{SHORT_DT:g}_fp32lu": short}
        print(f"# learned guess: {learned_info}", file=sys.stderr, flush=True)

    guess = torch.empty((desc.n_unknowns, args.cells), dtype=torch.float64, device=dev)
    counters = torch.zeros(8, dtype=torch.int64, device=dev)
    gpu_out = {}
    xs = torch.empty((args.cells, desc.n_species + 2), dtype=torch.float32, device=dev)
    for variant in args.variants.split(","):
        prec = {"fp64": kr.KR_FP64, "fp32lu": kr.KR_FP32LU_REFINE,
                "fp32lu+mlp": kr.KR_FP32LU_REFINE, "fp64+mlp": kr.KR_FP64,
                "single": kr.KR_SINGLE, "mixed": kr.KR_MIXED}[variant]
        use_guess = "mlp" in variant
        opts = (kr.guess_options(guess, precision=prec, order=_order(args)) if use_guess
                else kr.default_options(precision=prec, order=_order(args)))
        opts.counters = counters.data_ptr()

        def step():
            n.copy_(n0)
            T.copy_(T0)
            counters.zero_()
            if use_guess:   # the inference pre-pass is part of the step
                model.predict(n, T, dt_scalar=dt_scalar, guess=guess, X_scratch=xs, stream=stream)
            ev0 = torch.cuda.Event(enable_timing=True)
            ev1 = torch.cuda.Event(enable_timing=True)
            ev0.record(stream)
            kr.chem_integrate(net, n, T, dt_scalar=dt_scalar, rtol=1e-6, opts=opts,
                              status=status, cell_stats=stats, stream=stream)
            ev1.record(stream)
            return ev0, ev1

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        events = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            events.append(step())
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kernel_s = np.mean([a.elapsed_time(b) for a, b in events]) * 1e-3
        st = stats.cpu().numpy().astype(np.int64)
        stat_codes = np.bincount(status.cpu().numpy(), minlength=3)
        iters, acc, rej = st[:, 1].sum(), st[:, 0].sum(), st[:, 2].sum()
        flops = iters * f_it + (acc + rej) * f_rhs
        gpu_out[variant] = (n.cpu().numpy(), T.cpu().numpy(), status.cpu().numpy(), st[:, 1])
        resid = torch.empty(args.cells, dtype=torch.float64, device=dev)
        kr.element_residual(net, n0, n, resid=resid)
        ok = status != 2
        max_resid = float(resid[ok].max().item()) if bool(ok.any()) else 0.0
        results[variant] = {
            "ms_per_step": wall / args.steps * 1e3,
            "value": args.cells * args.steps / wall,
            "kernel_ms": kernel_s * 1e3,
            "flops_per_launch": float(flops),
            "achieved_tflops": flops / kernel_s / 1e12,
            "newton_iters_per_cell": float(iters) / args.cells,
            "substeps_per_cell": float(acc) / args.cells,
            "status_counts": stat_codes.tolist(),
            "max_element_residual": max_resid,
            "counters_last_step": dict(zip(("guess_starts", "guess_fallbacks", "row_exchanges",
                                            "fp32_solves", "fp64_fallbacks"),
                                           counters.cpu().numpy()[:5].tolist())),
        }
        print(f"# {variant}: {results[variant]}", file=sys.stderr, flush=True)

    head_name = "fp64" if "fp64" in results else next(iter(results))
    head = results[head_name]
    # the FP32 modes run their arithmetic on the FP32 vector ALUs
    fp32_head = head_name in ("single", "mixed")
    peak = PEAK_FP32 if fp32_head else PEAK_FP64
    kernel_name = {"fp64": "kr_integrate_fp64", "single": "kr_integrate_single",
                   "mixed": "kr_integrate_mixed"}.get(head_name, "kr_integrate_fp32lu")
    out = {
        "metric": ("cell-steps/s implicit chem update, c_V(T) and tabulated rates, 1 GPU" if tcv else
                   "cell-steps/s implicit chem update @1e-6 rel: plain FP64 vs mixed+MLP, 1 GPU"),
        "value": head["value"],
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if fp32_head else "f64",
        "data": "synthetic",
        "config": {"workload": ("h_o_n 9-species/24-reaction network + energy (10x10 LU), "
                                + ("NASA-style piecewise-polynomial c_V(T), 4 tabulated reactions (48 nodes), "
                                   if tcv else "")
                                + f"{args.cells} cells, T~U[900,2500] K, 1 atm, dt=1e-4 s adaptive BE, rtol 1e-6"),
                   "cells": args.cells, "unknowns": desc.n_unknowns, "reactions": desc.n_reactions,
                   "variant": "fp64" if "fp64" in results else args.variants, "cell_order": args.order},
        "variants": results,
        "learned_guess": learned_info,
        "roofline": {"bound": "alu", "achieved": head["achieved_tflops"], "peak": peak / 1e12,
                     "unit": "TFLOP/s", "frac": head["achieved_tflops"] * 1e12 / peak,
                     "traffic": (measured_traffic(kr.network_check(desc))
                                 if head_name == "fp64" and not tcv else None),
                     "kernel": kernel_name, "flops_per_newton_iteration": f_it,
                     "flops_per_error_estimate": f_rhs, "exp_log_flops": C_EXP},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(desc, cs, dt_scalar, min(args.cpu_sample, args.cells), gpu=gpu_out)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
