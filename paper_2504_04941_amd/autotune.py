"""Autotuner for the generated integrator kernels.

Tunables (compile-time, `kr_build_opts`): per network, the layout (one cell
per lane; one cell per group of 16 or 32 lanes, or per wavefront, with the
Newton matrix one row per lane: the lane-group shapes G = 1, 16, 32, 64
that the network fits); for the module, the occupancy target the register allocator budgets
for (waves per SIMD, or 0 for the library's per-layout choice; the lane's
Newton matrix lives in VGPRs, so a higher target trades registers for
scratch spills) and the threshold of the LU's
partial pivoting (a smaller threshold takes fewer row exchanges, which
execute wave-wide when any lane needs one).  Run-time tunable
(`kr_options.order`): the order in which cells are handed out (input order,
or largest expected work first, which pays for long uneven cells and costs
more than it saves on cheap ones).  Each candidate
is compiled, run on a sample of the caller's own cells (fresh copies per
timing) and timed with HIP events on the launch stream; the fastest wins.
Choices are cached in a JSON file keyed by the generated source (which
encodes the network and the kernel template), the device name, the
precision and the batch size class (log2 of the cell count: the layouts'
relative speed depends on the cells per lane or wavefront), so a network is
tuned once per machine and size class.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

from . import (KR_LAYOUT_GROUP16, KR_LAYOUT_GROUP32, KR_LAYOUT_LANE, KR_LAYOUT_WAVE, KR_ORDER_INPUT,
               KR_ORDER_WORK, BuildOpts, KrError, Multi, Network, build_options, chem_integrate,
               default_options, multi_check, network_check)

CACHE = os.environ.get("KR_AUTOTUNE_CACHE",
                       os.path.join(os.path.expanduser("~"), ".cache", "kr_autotune.json"))
CANDIDATES = [(0, 0.1), (1, 0.1), (1, 0.01), (2, 0.1)]   # (waves_per_eu, pivot_tau); 0 = automatic
LAYOUTS = (KR_LAYOUT_LANE, KR_LAYOUT_GROUP16, KR_LAYOUT_GROUP32, KR_LAYOUT_WAVE)
LAYOUT_NAMES = {KR_LAYOUT_LANE: "lane", KR_LAYOUT_GROUP16: "group16", KR_LAYOUT_GROUP32: "group32",
                KR_LAYOUT_WAVE: "wave"}


def layout_candidates(desc):
    """The layouts (lane-group shapes) the network fits, with their sources."""
    out = []
    for L in LAYOUTS:
        try:
            out.append((L, network_check(desc, build=build_options(layout=L))))
        except KrError:
            pass
    return out


def _key(sources, precision):
    import torch
    h = hashlib.sha256()
    for s in sources:
        h.update(s.encode())
    h.update(torch.cuda.get_device_name(0).encode())
    h.update(str(precision).encode())
    return h.hexdigest()[:32]


def _load():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(db):
    os.makedirs(os.path.dirname(CACHE), exist_ok=True)
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def _time_call(fn, reps):
    import torch
    stream = torch.cuda.current_stream()
    best = float("inf")
    for _ in range(reps):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        prep = fn(None)           # copies the inputs (not timed)
        ev0.record(stream)
        fn(prep)
        ev1.record(stream)
        torch.cuda.synchronize()
        best = min(best, ev0.elapsed_time(ev1))
    return best


def tune_layout(desc, batch, precision=0, rtol=1e-6, reps=2, use_cache=True, log=None):
    """Fastest layout (lane, 16- or 32-lane groups, wavefront: those the
    network fits) of one network on a sample of its cells (batch: dict as
    for Multi.integrate, copied before every timed run).  Returns (layout,
    report)."""
    import torch
    cands = layout_candidates(desc)
    srcs = [src for _, src in cands]
    # the answer depends on how many cells there are per lane or wavefront
    size_class = int(batch["T"].numel()).bit_length()
    key = "layout-" + _key(srcs + [str(size_class)], precision)
    db = _load() if use_cache else {}
    if key in db:
        return int(db[key]["best"]), db[key]
    opts = default_options(precision=precision)
    report = {"candidates": [], "sample_cells": int(batch["T"].numel())}
    best, best_t = None, float("inf")
    for L, _ in cands:
        t0 = time.time()
        net = Network(desc, build_options(layout=L))
        compile_s = time.time() - t0

        def run(prep):
            if prep is None:
                return {k: (v.clone() if torch.is_tensor(v) else v) for k, v in batch.items()}
            chem_integrate(net, prep["states"], prep["T"], rho=prep.get("rho"), dt=prep.get("dt"),
                           dt_scalar=prep.get("dt_scalar", 0.0), rtol=rtol, opts=opts,
                           status=prep.get("status"), cell_stats=prep.get("cell_stats"))
            return None

        ms = _time_call(run, reps)
        net.close()
        report["candidates"].append({"layout": L, "ms": ms, "compile_s": compile_s})
        if log:
            log(f"autotune layout={LAYOUT_NAMES[L]}: {ms:.2f} ms "
                f"(compile {compile_s:.1f} s)")
        if ms < best_t:
            best, best_t = L, ms
    report["best"] = best
    if use_cache:
        db = _load()
        db[key] = report
        _store(db)
    return best, report


def tune_order(net, batch, precision=0, rtol=1e-6, reps=2, log=None):
    """Faster cell order (KR_ORDER_INPUT or KR_ORDER_WORK) for one network's
    batch (dict as for Multi.integrate, copied before every timed run).
    Not cached: the answer depends on the cells, not only on the network.
    Returns (order, report)."""
    import torch
    report = {"candidates": [], "cells": int(batch["T"].numel())}
    best, best_t = None, float("inf")
    for order in (KR_ORDER_INPUT, KR_ORDER_WORK):
        opts = default_options(precision=precision, order=order)

        def run(prep):
            if prep is None:
                return {k: (v.clone() if torch.is_tensor(v) else v) for k, v in batch.items()}
            chem_integrate(net, prep["states"], prep["T"], rho=prep.get("rho"), dt=prep.get("dt"),
                           dt_scalar=prep.get("dt_scalar", 0.0), rtol=rtol, opts=opts,
                           status=prep.get("status"), cell_stats=prep.get("cell_stats"))
            return None

        ms = _time_call(run, reps)
        report["candidates"].append({"order": order, "ms": ms})
        if log:
            log(f"autotune order={'work' if order == KR_ORDER_WORK else 'input'}: {ms:.2f} ms")
        if ms < best_t:
            best, best_t = order, ms
    report["best"] = best
    return best, report


def tune_multi(descs, batches, precision=0, rtol=1e-6, candidates=CANDIDATES, reps=2,
               use_cache=True, log=None):
    """Best layout per network (tune_layout on its own sample), best module
    build options for the networks integrated together and, with those, the
    faster cell order (report["order"]).

    batches: list of dicts as for Multi.integrate (a sample of the cells;
    they are copied before every timed run and left untouched).  Returns
    (BuildOpts, layouts, report)."""
    import torch
    layouts, lay_reports = [], []
    for d, b in zip(descs, batches):
        L, r = tune_layout(d, b, precision, rtol, reps, use_cache, log)
        layouts.append(L)
        lay_reports.append(r)
    key = _key([multi_check(descs)] + [str(layouts)] + [str(int(b["T"].numel()).bit_length()) for b in batches],
               precision)
    db = _load() if use_cache else {}
    if key in db and "order" in db[key]:
        w, tau = db[key]["best"]
        return build_options(waves_per_eu=int(w), pivot_tau=float(tau)), layouts, db[key]
    nets_cache = {}
    report = {"candidates": [], "sample_cells": [int(b["T"].numel()) for b in batches],
              "layouts": [LAYOUT_NAMES[L] for L in layouts],
              "layout_timings": lay_reports}
    best, best_t = None, float("inf")
    for w, tau in candidates:
        bo = build_options(waves_per_eu=w, pivot_tau=tau)
        t0 = time.time()
        nets = [Network(d, build_options(waves_per_eu=w, pivot_tau=tau, layout=L))
                for d, L in zip(descs, layouts)]
        multi = Multi(nets, bo)
        compile_s = time.time() - t0

        for order in (KR_ORDER_INPUT, KR_ORDER_WORK):
            opts = default_options(precision=precision, order=order)

            def run(prep):
                if prep is None:
                    return [{k: (v.clone() if torch.is_tensor(v) else v) for k, v in b.items()}
                            for b in batches]
                multi.integrate(prep, rtol=rtol, opts=opts)
                return None

            ms = _time_call(run, reps)
            report["candidates"].append({"waves_per_eu": w, "pivot_tau": tau, "order": order, "ms": ms,
                                         "compile_s": compile_s})
            if log:
                log(f"autotune waves_per_eu={w} pivot_tau={tau} order={'work' if order else 'input'}: "
                    f"{ms:.1f} ms (compile {compile_s:.1f} s)")
            if ms < best_t:
                best, best_t = (w, tau, order), ms
        multi.close()
        for n in nets:
            n.close()
        nets_cache.clear()
    report["best"] = list(best[:2])
    report["order"] = best[2]
    if use_cache:
        db = _load()
        db[key] = report
        _store(db)
    return build_options(waves_per_eu=best[0], pivot_tau=best[1]), layouts, report
