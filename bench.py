"""Benchmark of the coupled bubble-column step on one MI355X.

A step is one pass of the whole hot path of Algorithm 1 over the lattice: the bubble kernel
(forward coupling, bubble ODE, backward coupling) followed by the fused liquid step. The
default workload is the single-bubble FP32 column, 128 x 128 x 512 (8.4 M sites), omega = 1.6,
bounce-back walls, one bubble of diameter 4 at the bottom centre.

Prints one JSON line: whole-job throughput in MLUPS (lattice-site updates per second), the
roofline of the dominant kernel (the fused liquid step, HBM-bound; its per-launch duration comes
from HIP events recorded around each launch on the library's stream in the timed region), and the
CPU oracle timed on a bounded sample of the same workload on the host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import re
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("MLUPS and % HBM peak of fused step; batched and adjoint vs plain FP64 at stated error")
HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = ["paper_1710_07073_amd/csrc/step.hip", "paper_1710_07073_amd/csrc/lattice.hpp",
                  "paper_1710_07073_amd/csrc/internal.hpp", "paper_1710_07073_amd/csrc/collide.hpp",
                  "paper_1710_07073_amd/csrc/step_cell.hpp"]


def code_text(src):
    """Source text without comments and blank-space differences: what the compiler sees."""
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def kernel_source_sha():
    """Hash of the fused step's code (comments and spacing ignored): counter summaries taken on
    other code are not used."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p)) as f:
            h.update(code_text(f.read()).encode())
    return h.hexdigest()[:16]


def read_traffic(workload, elem_bytes):
    """HBM bytes per launch of the liquid step from the committed counter summary, if it was
    taken on the current kernel source; else None."""
    path = os.path.join(PROFILES, f"k_step_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha") != kernel_source_sha():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(w, budget_s=12.0):
    """The oracle (plain FP64 C++, OpenMP over cells) on the same lattice and bubble, timed for
    whole method steps until about budget_s of wall time has passed."""
    import oracle as O

    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    lat = O.Lattice(*w.shape, w.omega, w.bc)
    bub = O.Bubbles(pos=w.pos.copy(), d=w.d.copy())
    P = O.bubble_params(**w.params)
    O.method_step(lat, P, bub, threads)  # warm-up (first touch of the arrays)
    n = 0
    t0 = time.perf_counter()
    while True:
        O.method_step(lat, P, bub, threads)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= 1000:
            break
    return {"value": round(w.cells * n / el / 1e6, 2), "unit": "MLUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"{n} full method steps of the same {w.shape[0]}x{w.shape[1]}x{w.shape[2]} "
                      f"lattice and bubble, FP64, {threads} OpenMP threads, {el:.1f} s"}


def leg_batched(args, steps):
    """64 uneven columns stepped together (FP32, graph replays), against the same columns run one
    at a time as plain single-lattice FP64 simulations (also replayed from graphs); error of the
    FP32 batch against FP64 single-column runs of the same number of steps on four of the columns;
    and the time of the same steps as persistent launches."""
    import torch
    import workloads as W
    from paper_1710_07073_amd import autotune
    from paper_1710_07073_amd import lbm as L
    from paper_1710_07073_amd import sim as S

    ws = W.batched()
    cols = [dict(shape=w.shape, omega=w.omega, bc=w.bc, pos=w.pos, d=w.d) for w in ws]
    stream = torch.cuda.current_stream()
    cells = sum(w.cells for w in ws)
    gsteps = args.graph_steps or 100
    batch = S.Batch(cols, S.bubble_params(**ws[0].params), precision="f32", stream=stream)
    items = occ = None
    if not args.no_autotune:
        items, sweep = autotune.tune_batch(batch, steps=3)
        for k, cand, ms in sweep:
            print(f"[autotune] class {k} item {cand}: {ms:.3f} ms/step", file=sys.stderr, flush=True)
        occ, osweep = autotune.tune_batch_occupancy(batch, steps=3)
        for o, ms in osweep:
            print(f"[autotune] batch occupancy {o}: {ms:.3f} ms/step", file=sys.stderr, flush=True)
    batch.close()
    # tuning stepped the columns; time a fresh batch with the tuned items and occupancy
    batch = S.Batch(cols, S.bubble_params(**ws[0].params), precision="f32", stream=stream)
    if items is not None:
        L.lbm_batch_set_items(batch.handle, items)
        L.lbm_batch_set_step_occupancy(batch.handle, occ)
    wgs = L.lbm_batch_get_step_occupancy(batch.handle)
    warm = args.warmup + (-args.warmup) % gsteps
    batch.run(warm, graph_steps=gsteps)
    stream.synchronize()
    K = max(gsteps, steps - steps % gsteps)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    batch.run(K, graph_steps=gsteps)
    e1.record(stream)
    stream.synchronize()
    elapsed = time.perf_counter() - t0
    ev_s = e0.elapsed_time(e1) * 1e-3
    batch.check()
    total = warm + K
    # plain single-lattice FP64 form: every column on its own, its steps replayed from a HIP graph
    # as the batch's are (the graph captured and replayed once before the timed replays)
    ks = 2 * gsteps
    t_single = 0.0
    for w in ws:
        sim = S.Simulation(w.shape, w.omega, precision="f64", bc=w.bc, stream=stream)
        sim.add_bubbles(w.pos, w.d, S.bubble_params(**w.params))
        sim.run(gsteps, graph_steps=gsteps)
        stream.synchronize()
        a = time.perf_counter()
        sim.run(ks, graph_steps=gsteps)
        stream.synchronize()
        t_single += time.perf_counter() - a
        sim.close()
    # error of the FP32 batch against FP64 single-column runs over the same steps
    err_g, err_x = 0.0, 0.0
    for c in (0, 17, 40, 63):
        w = ws[c]
        sim = S.Simulation(w.shape, w.omega, precision="f64", bc=w.bc, stream=stream)
        sim.add_bubbles(w.pos, w.d, S.bubble_params(**w.params))
        sim.run(total, graph_steps=gsteps)
        g64 = sim.populations()
        x64 = sim.bubbles.positions()
        sim.close()
        g32 = batch.populations(c)
        b0, b1 = batch.bubble_range(c)
        x32 = batch.bubbles.positions()[:, b0:b1]
        err_g = max(err_g, float(((g32.double() - g64).norm() / g64.norm()).item()))
        err_x = max(err_x, float(np.abs(x32 - x64).max()))
    # the same steps as persistent launches (one kernel of gsteps steps per graph), for comparison
    L.lbm_batch_set_persistent(batch.handle, True)
    batch.run(gsteps, graph_steps=gsteps)
    stream.synchronize()
    p0, p1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    p0.record(stream)
    batch.run(K, graph_steps=gsteps)
    p1.record(stream)
    stream.synchronize()
    batch.check()
    persistent_ms = p0.elapsed_time(p1) / K
    persistent_grid = L.lbm_batch_get_persistent(batch.handle)[1]
    batch.close()
    mlups = cells * K / elapsed / 1e6
    fp64 = cells * ks / t_single / 1e6
    return {"columns": len(ws), "cells": cells, "bubbles": int(sum(w.nb for w in ws)),
            "steps": K, "graph_steps": gsteps, "item_cells": items, "workgroups_per_cu": wgs,
            "batched_f32_mlups": round(mlups, 1), "ms_per_step": round(elapsed / K * 1e3, 5),
            "event_ms_per_step": round(ev_s / K * 1e3, 5),
            "plain_fp64_single_mlups": round(fp64, 1), "ratio_vs_plain_fp64": round(mlups / fp64, 3),
            "persistent_ms_per_step": round(persistent_ms, 5), "persistent_grid": persistent_grid,
            "error_vs_fp64": {"after_steps": total, "columns_checked": [0, 17, 40, 63],
                              "populations_rel_l2_max": err_g,
                              "bubble_pos_max_abs": err_x}}


def time_steps(sim, K, stream):
    """Runs K method steps of a single-lattice simulation; returns the wall time, the mean duration
    of the fused step's launch that updates the lattice away from the bubbles (recorded by the
    library on the stream it runs on: the side stream when the step is overlapped), the number of
    launches timed and the region of the last overlapped step (sites)."""
    import torch
    from paper_1710_07073_amd import lbm as L

    # every EVERY-th launch is timed (a timing event record costs several microseconds of the
    # queue), at least five launches of a short run; the steps run through lbm_run in runs of
    # EVERY, the first of which is timed
    EVERY = max(4, min(64, K // 16))
    nt = (K + EVERY - 1) // EVERY
    ev0 = [torch.cuda.Event(enable_timing=True) for _ in range(nt)]
    ev1 = [torch.cuda.Event(enable_timing=True) for _ in range(nt)]
    for e in ev0 + ev1:
        e.record(stream)  # creates the underlying HIP event
    bub = sim.bubbles
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(0, K, EVERY):
        L.lbm_time_next_step(sim.ctx, ev0[k // EVERY], ev1[k // EVERY])
        L.lbm_run(sim.ctx, sim.params, bub.soa, bub.nb, min(EVERY, K - k), 0)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kern_s = float(np.mean([a.elapsed_time(b) for a, b in zip(ev0, ev1)])) * 1e-3
    return elapsed, kern_s, nt, L.lbm_region_cells(sim.ctx)


def leg_dense(args, steps):
    """The dense dispersed column (256 x 256 x 768, 20 000 bubbles, FP32) for its stated number of
    whole method steps, the liquid launch tuned as for the headline column and the step overlapped
    or serial, whichever the tuning timed faster; then a shorter run of the serial step for the
    fused kernel's rate when it has the chip alone, and the bubble half timed alone."""
    import torch
    import workloads as W
    from paper_1710_07073_amd import autotune
    from paper_1710_07073_amd import lbm as L
    from paper_1710_07073_amd import sim as S

    w = W.dense()
    stream = torch.cuda.current_stream()
    sim = S.Simulation(w.shape, w.omega, precision=w.dtype, bc=w.bc, stream=stream)
    if not args.no_autotune:
        autotune.tune(sim, use_cache=False)
    vec, bx = L.lbm_get_launch(sim.ctx)
    sim.add_bubbles(w.pos, w.d, S.bubble_params(**w.params))
    if not args.no_autotune:
        autotune.tune_method_occupancy(sim)
    for _ in range(10):
        sim.step(1)
    overlapped, _ = L.lbm_get_overlap(sim.ctx)
    elapsed, kern_s, nt, region = time_steps(sim, steps, stream)
    _, _, sums = sim.moments(fields=False)
    sim.check()
    alg = 38 * 4 * (w.cells - region)
    out = {"workload": w.name, "cells": w.cells, "bubbles": w.nb, "omega": w.omega,
           "steps": steps, "mlups": round(w.cells * steps / elapsed / 1e6, 1),
           "ms_per_step": round(elapsed / steps * 1e3, 5),
           "overlapped": overlapped,
           "roofline": {"bound": "hbm", "kernel": "k_step_bb (bulk launch of the overlapped step)"
                        if region else "k_step_bb (whole lattice, serial step)",
                        "sites_per_launch": w.cells - region, "alg_bytes_per_launch": alg,
                        "avg_launch_ms": round(kern_s * 1e3, 5), "launches_timed": nt,
                        "achieved": round(alg / kern_s / 1e9, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(alg / kern_s / 1e9 / HBM_PEAK_GBS, 4)},
           "launch": {"vec": vec, "bx": bx, "workgroups_per_cu": L.lbm_get_step_occupancy(sim.ctx)},
           "mass_drift": sums[0] - w.cells}
    # the same column with the bubble half and the liquid step one after the other: the fused
    # step then updates the whole lattice alone on the chip (its 152 B per site are a lower bound
    # of what it moves: forced tiles add 36 B per site)
    L.lbm_set_overlap(sim.ctx, False)
    for _ in range(4):
        sim.step(1)
    ks = min(steps, 256)
    s_el, s_kern, s_nt, _ = time_steps(sim, ks, stream)
    sim.check()
    alg_full = 38 * 4 * w.cells
    out["serial"] = {"steps": ks, "ms_per_step": round(s_el / ks * 1e3, 5),
                     "roofline": {"bound": "hbm", "kernel": "k_step_bb (whole lattice, alone)",
                                  "sites_per_launch": w.cells, "alg_bytes_per_launch": alg_full,
                                  "avg_launch_ms": round(s_kern * 1e3, 5), "launches_timed": s_nt,
                                  "achieved": round(alg_full / s_kern / 1e9, 1),
                                  "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                  "frac": round(alg_full / s_kern / 1e9 / HBM_PEAK_GBS, 4)}}
    # the bubble half alone (serial step: its kernels on the caller's stream), events around it
    out["bubbles"] = time_bubble_half(sim, stream, 32)
    sim.close()
    return out


def window_cells(pos, d, shape, kernel_factor):
    """Cells of the bubbles' kernel windows (eq. (18)-(19): the cells whose extent overlaps
    [x - n, x + n], n = kernel_factor d), clipped to a lattice with walls on every face."""
    n = kernel_factor * np.asarray(d)
    cells = np.ones(len(n))
    for a, ext in enumerate(shape):
        lo = np.maximum(np.floor(pos[a] - n - 0.5) + 1, 0)
        hi = np.minimum(np.ceil(pos[a] + n + 0.5) - 1, ext - 1)
        cells *= np.maximum(hi - lo + 1, 0)
    return int(cells.sum())


def time_bubble_half(sim, stream, k):
    """Median over k serial method steps of the bubble half's GPU time (events on the caller's
    stream around bubbles_step; each step's liquid update follows), and the window cells it
    touches per second."""
    import torch
    from paper_1710_07073_amd import lbm as L
    bub = sim.bubbles
    touches = window_cells(bub.positions(), bub.t["d"].cpu().numpy(), sim.shape,
                           sim.params.kernel_factor)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(k)]
    for a, b in evs:
        a.record(stream)
        L.bubbles_step(sim.ctx, sim.params, bub.soa, bub.nb)
        b.record(stream)
        L.lbm_step(sim.ctx, 1)
    torch.cuda.synchronize()
    t = sorted(a.elapsed_time(b) for a, b in evs)[k // 2] / 1e3
    return {"kernels": "k_interp, k_ode, k_spread_gather (serial step)", "steps_timed": k,
            "us_per_step_median": round(t * 1e6, 1), "window_cells_per_step": touches,
            "cell_touches_per_s": round(touches / t, 1)}


def copy_calibration():
    """One device copy of 1 GiB (torch copy_): the HBM counters of the same run read it as a
    reference for the scale of the kernels' counters."""
    import torch
    a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)  # 1 GiB read + 1 GiB write
    torch.cuda.synchronize()


def bench_batched(args):
    if args.copy_calibration:
        copy_calibration()
    leg = leg_batched(args, args.steps)
    out = {
        "metric": METRIC, "value": leg["batched_f32_mlups"], "unit": "MLUPS", "n_gpus": 1,
        "steps": leg["steps"], "warmup": args.warmup, "ms_per_step": leg["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic", "config": {"workload": "batched_64_columns", "parallelism": "single GPU"},
        "batched": leg,
    }
    print(json.dumps(out), flush=True)


def bench_stability(args):
    """Stability sweep (Sec. 4.3): the App. A column (30 x 30 x 90, 4 mm bubble, d = 0.8) at 16
    values of omega from 1.90 to 1.9999 in one batch, FP32, graph replays of 500 steps; after each
    chunk the per-column sums tell which columns went unstable."""
    import torch
    import workloads as W
    from paper_1710_07073_amd import sim as S

    ws = W.stability(steps=args.steps)
    cols = [dict(shape=w.shape, omega=w.omega, bc=w.bc, pos=w.pos, d=w.d) for w in ws]
    stream = torch.cuda.current_stream()
    batch = S.Batch(cols, S.bubble_params(**ws[0].params), precision="f32", stream=stream)
    chunk = 500
    first = [None] * len(ws)
    t0 = time.perf_counter()
    done = 0
    while done < args.steps:
        n = min(chunk, args.steps - done)
        batch.run(n, graph_steps=chunk if n == chunk else 0)
        done += n
        _, diverged = batch.sums()
        for k, dv in enumerate(diverged):
            if dv and first[k] is None:
                first[k] = done
        print(f"[stability] {done} steps, unstable: {[w.omega for w, f in zip(ws, first) if f]}",
              file=sys.stderr, flush=True)
    elapsed = time.perf_counter() - t0
    z = batch.bubbles.positions()[2]
    batch.close()
    cells = sum(w.cells for w in ws)
    stable = [w.omega for w, f in zip(ws, first) if f is None]
    swarm = swarm_map(stream)
    out = {
        "metric": METRIC, "value": round(cells * args.steps / elapsed / 1e6, 1), "unit": "MLUPS",
        "n_gpus": 1, "steps": args.steps, "warmup": 0,
        "ms_per_step": round(elapsed / args.steps * 1e3, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "stability_sweep_30x30x90_x16", "columns": len(ws),
                   "parallelism": "single GPU"},
        "stability": {"omega": [w.omega for w in ws], "first_unstable_step": first,
                      "bubble_z_end": [None if not np.isfinite(v) else round(float(v), 3) for v in z],
                      "max_stable_omega": max(stable) if stable else None,
                      "check_every_steps": chunk},
        "swarm_map": swarm,
    }
    print(json.dumps(out), flush=True)


def swarm_map(stream, steps=3000, chunk=250):
    """Stability map over omega and forcing (Sec. 4.3 with the forcing made strong): the App. A
    column (30 x 30 x 90, free-slip top) holding swarms of 16 to 768 bubbles at g = 3e-2, one
    column per (omega, swarm size), 64 columns in one batch, FP32; a column is unstable once its
    FP64 sums are not finite (checked every `chunk` steps)."""
    import workloads as W
    from paper_1710_07073_amd import sim as S

    ws = W.stability_swarm(steps=steps)
    cols = [dict(shape=w.shape, omega=w.omega, bc=w.bc, pos=w.pos, d=w.d) for w in ws]
    batch = S.Batch(cols, S.bubble_params(**ws[0].params), precision="f32", stream=stream)
    first = [None] * len(ws)
    t0 = time.perf_counter()
    for done in range(chunk, steps + 1, chunk):
        batch.run(chunk, graph_steps=chunk // 5 * 2)
        _, diverged = batch.sums()
        for k, dv in enumerate(diverged):
            if dv and first[k] is None:
                first[k] = done
    elapsed = time.perf_counter() - t0
    batch.close()
    rows = {}
    for w, f in zip(ws, first):
        r = rows.setdefault(w.meta["nb"], {"stable": [], "unstable": {}})
        if f is None:
            r["stable"].append(w.omega)
        else:
            r["unstable"][str(w.omega)] = f
    summary = {str(nb): {"max_stable_omega": max(r["stable"]) if r["stable"] else None,
                         "min_unstable_omega": min(float(o) for o in r["unstable"]) if r["unstable"] else None,
                         "first_unstable_step": r["unstable"]} for nb, r in rows.items()}
    print(f"[stability] swarm map: {summary}", file=sys.stderr, flush=True)
    return {"columns": len(ws), "lattice": [30, 30, 90], "g": W.SWARM_G, "steps": steps,
            "check_every_steps": chunk, "omegas": list(W.SWARM_OMEGAS),
            "swarm_sizes": list(W.SWARM_COUNTS), "by_swarm_size": summary,
            "mlups": round(sum(w.cells for w in ws) * steps / elapsed / 1e6, 1)}


# Table 6: the paper's terminal velocity (m/s), identical at all three aspect ratios
PAPER_VT = {4: 0.2383, 8: 0.2411, 10: 0.2538}


def physical_rise(w, steps, chunk=100, params=None):
    """One physical-unit column (a workload of grid_independence) for `steps` steps, FP32, graph
    replays of `chunk` steps; the bubble's rise velocity read after every chunk. The terminal
    velocity is its mean over 0.5 to 0.9 s in m/s (the second half of the run if shorter); the
    slip velocity the same mean of u_b - u_l, u_l the liquid velocity interpolated at the bubble.
    Returns (row, seconds of GPU stepping)."""
    import torch
    import workloads as W
    from paper_1710_07073_amd import sim as S
    from paper_1710_07073_amd import units as U

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    u = U.column_units(w.meta["d_mm"] * 1e-3, w.meta["aspect"])
    sim = S.Simulation(w.shape, w.omega, precision="f32", bc=w.bc, device=dev, stream=stream)
    sim.add_bubbles(w.pos, w.d, S.bubble_params(**(params or w.params)))
    t_s, z_m, v_ms, ul_ms = [], [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps // chunk):
        sim.run(chunk, graph_steps=chunk)
        x, v, ul = sim.bubbles.positions(), sim.bubbles.velocities(), sim.bubbles.liquid_velocity()
        t_s.append((k + 1) * chunk * u.dt)
        z_m.append(float(x[2, 0]) * u.dx)
        v_ms.append(u.velocity_pu(float(v[2, 0])))
        ul_ms.append(u.velocity_pu(float(ul[2, 0])))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    state = int(sim.bubbles.state()[0])
    sim.check()
    sim.close()
    t_s, v_ms, ul_ms = np.array(t_s), np.array(v_ms), np.array(ul_ms)
    window = (t_s >= 0.5 - 1e-9) & (t_s <= 0.9 + 1e-9)
    if not window.any():
        window = t_s >= t_s[-1] / 2
    vt = float(v_ms[window].mean())
    marks = {f"{t:.2f}": round(z_m[int(round(t / (chunk * u.dt))) - 1], 5)
             for t in (0.25, 0.5, 0.75, 1.0) if int(round(t / (chunk * u.dt))) <= len(z_m)}
    row = dict(case=w.name, d_mm=w.meta["d_mm"], aspect=w.meta["aspect"], grid=list(w.shape),
               d_lu=float(w.d[0]), omega=w.omega, vT_ms=round(vt, 5),
               vT_spread_ms=round(float(np.ptp(v_ms[window])), 6),
               ul_at_bubble_ms=round(float(ul_ms[window].mean()), 5),
               slip_ms=round(float((v_ms - ul_ms)[window].mean()), 5),
               re_end=round(v_ms[-1] * w.meta["d_mm"] * 1e-3 / W.WATER_NU, 1),
               z_m=marks, active=state)
    return row, elapsed


def physical_rise_batch(ws, steps, chunk=100):
    """physical_rise for several physical-unit columns at once: one batch (FP32, graph replays of
    `chunk` steps) whose columns carry their own lattice-unit g and sigma (the grid spacing sets
    them, App. A); each column's bubble is read after every chunk. Returns (rows, seconds of GPU
    stepping); the rows are those of physical_rise."""
    import torch
    import workloads as W
    from paper_1710_07073_amd import sim as S
    from paper_1710_07073_amd import units as U

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    cols = [dict(shape=w.shape, omega=w.omega, bc=w.bc, pos=w.pos, d=w.d, g=w.params["g"],
                 sigma=w.params["sigma"]) for w in ws]
    batch = S.Batch(cols, S.bubble_params(**ws[0].params), precision="f32", stream=stream)
    units = [U.column_units(w.meta["d_mm"] * 1e-3, w.meta["aspect"]) for w in ws]
    first = [batch.bubble_range(c)[0] for c in range(len(ws))]
    t_s, z_m, v_ms, ul_ms = [], [], [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps // chunk):
        batch.run(chunk, graph_steps=chunk)
        x, v = batch.bubbles.positions(), batch.bubbles.velocities()
        ul = batch.bubbles.liquid_velocity()
        t_s.append((k + 1) * chunk * units[0].dt)
        z_m.append([float(x[2, b]) * u.dx for b, u in zip(first, units)])
        v_ms.append([u.velocity_pu(float(v[2, b])) for b, u in zip(first, units)])
        ul_ms.append([u.velocity_pu(float(ul[2, b])) for b, u in zip(first, units)])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    state = batch.bubbles.state()
    batch.check()
    batch.close()
    t_s, z_m, v_ms, ul_ms = np.array(t_s), np.array(z_m), np.array(v_ms), np.array(ul_ms)
    window = (t_s >= 0.5 - 1e-9) & (t_s <= 0.9 + 1e-9)
    if not window.any():
        window = t_s >= t_s[-1] / 2
    rows = []
    for c, w in enumerate(ws):
        marks = {f"{t:.2f}": round(z_m[int(round(t / (chunk * units[c].dt))) - 1, c], 5)
                 for t in (0.25, 0.5, 0.75, 1.0) if int(round(t / (chunk * units[c].dt))) <= len(z_m)}
        rows.append(dict(case=w.name, d_mm=w.meta["d_mm"], aspect=w.meta["aspect"],
                         grid=list(w.shape), d_lu=float(w.d[0]), omega=w.omega,
                         vT_ms=round(float(v_ms[window, c].mean()), 5),
                         vT_spread_ms=round(float(np.ptp(v_ms[window, c])), 6),
                         ul_at_bubble_ms=round(float(ul_ms[window, c].mean()), 5),
                         slip_ms=round(float((v_ms[:, c] - ul_ms[:, c])[window].mean()), 5),
                         re_end=round(v_ms[-1, c] * w.meta["d_mm"] * 1e-3 / W.WATER_NU, 1),
                         z_m=marks, active=int(state[first[c]])))
    return rows, elapsed


def bench_grid(args):
    """Grid-independence study (Sec. 4.2, Tables 5 and 6): the nine columns of Table 5 (4, 8 and
    10 mm bubbles at aspect ratios 1.25, 0.625, 0.3125) in physical units, FP32, stepped together
    as one batch (physical_rise_batch)."""
    import workloads as W

    chunk = 100
    steps = max(args.steps - args.steps % chunk, 2 * chunk)
    ws = W.grid_independence(steps=steps)
    rows, elapsed = physical_rise_batch(ws, steps, chunk)
    cells = sum(w.cells for w in ws)
    for w, row in zip(ws, rows):
        row["paper_vT_ms"] = PAPER_VT[int(w.meta["d_mm"])]
        print(f"[grid] {w.name} {w.shape} omega {w.omega:.6f}: v_T {row['vT_ms']:.4f} m/s "
              f"(paper {row['paper_vT_ms']})", file=sys.stderr, flush=True)

    def spread(key):
        by_d = {}
        for r in rows:
            by_d.setdefault(r["d_mm"], []).append(r[key])
        return {f"{int(d)}mm": round((max(v) - min(v)) / np.mean(v), 6) for d, v in by_d.items()}
    out = {
        "metric": METRIC, "value": round(cells * steps / elapsed / 1e6, 1), "unit": "MLUPS",
        "n_gpus": 1, "steps": steps, "warmup": 0, "ms_per_step": round(elapsed / steps * 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "grid_independence_table5_x9", "columns": len(ws),
                   "parallelism": "single GPU, one batch"},
        "grid": {"cases": rows, "vT_relative_spread_over_aspect": spread("vT_ms"),
                 "slip_relative_spread_over_aspect": spread("slip_ms"),
                 "vT_window_s": [0.5, 0.9], "sample_every_steps": chunk},
    }
    print(json.dumps(out), flush=True)


# Table 4: the paper's simulated terminal velocity (m/s) per bubble diameter (mm)
PAPER_VT_T4 = {2: 0.2898, 3: 0.2533, 4: 0.2383, 5: 0.2331, 6: 0.2332, 7: 0.2363, 8: 0.2411,
               9: 0.2471, 10: 0.2538}


def bench_terminal(args):
    """Terminal-velocity sweep (Sec. 4.1, Table 4): 2 to 10 mm bubbles in the water tank at aspect
    ratio 1.25, coupled runs in physical units stepped together as one batch
    (physical_rise_batch), against the paper's simulated column."""
    import workloads as W

    chunk = 100
    steps = max(args.steps - args.steps % chunk, 2 * chunk)
    ws = W.terminal_sweep(steps=steps)
    rows, elapsed = physical_rise_batch(ws, steps, chunk)
    cells = sum(w.cells for w in ws)
    for w, row in zip(ws, rows):
        row["paper_simulated_vT_ms"] = PAPER_VT_T4[int(round(w.meta["d_mm"]))]
        print(f"[terminal] {w.name} {w.shape}: v_T {row['vT_ms']:.4f} slip {row['slip_ms']:.4f} m/s "
              f"(paper {row['paper_simulated_vT_ms']})", file=sys.stderr, flush=True)
    out = {
        "metric": METRIC, "value": round(cells * steps / elapsed / 1e6, 1), "unit": "MLUPS",
        "n_gpus": 1, "steps": steps, "warmup": 0, "ms_per_step": round(elapsed / steps * 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "terminal_velocity_2_10mm_ar1.25", "columns": len(ws),
                   "parallelism": "single GPU, one batch"},
        "terminal": {"cases": rows, "vT_window_s": [0.5, 0.9], "sample_every_steps": chunk},
    }
    print(json.dumps(out), flush=True)


# coupling variants measured by bench_coupling: name -> bubble_params.coupling
COUPLINGS = {"default": 0, "substep_mean_reaction": 1, "net_force_reaction": 2,
             "point_kernel": 4, "exact_time": 8, "substep_point_exact": 13}


def bench_coupling(args):
    """Coupling variants against the default (the readings of the reaction, the kernel weights
    and the coupling time level): the 4 mm bubble of Table 5 on the 60 x 60 x 180 column
    (aspect ratio 0.625) in physical units for 1 s, each variant's rise, slip and height at 1 s
    against the default's; and the whole method step of the 128 x 128 x 512 FP32 column under
    each variant (cost)."""
    import torch
    import workloads as W
    from paper_1710_07073_amd import lbm as L
    from paper_1710_07073_amd import sim as S

    chunk = 100
    steps = max(args.steps - args.steps % chunk, 2 * chunk)
    w = [c for c in W.grid_independence(steps=steps) if c.name == "grid_4mm_ar0.625"][0]
    rows = {}
    for name, coupling in COUPLINGS.items():
        p = dict(w.params, coupling=coupling)
        row, sec = physical_rise(w, steps, chunk, params=p)
        row["ms_per_step"] = round(sec / steps * 1e3, 5)
        rows[name] = row
        print(f"[coupling] {name}: v_T {row['vT_ms']:.5f} slip {row['slip_ms']:.5f} m/s",
              file=sys.stderr, flush=True)
    base = rows["default"]
    for name, row in rows.items():
        row["vT_rel_vs_default"] = round(row["vT_ms"] / base["vT_ms"] - 1.0, 6)
        row["slip_rel_vs_default"] = round(row["slip_ms"] / base["slip_ms"] - 1.0, 6)
        row["z_1s_diff_m"] = round(row["z_m"].get("1.00", float("nan")) - base["z_m"].get("1.00", float("nan")), 6)
    # cost on the timed column
    t = W.single_fp32()
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    cost = {}
    for name, coupling in COUPLINGS.items():
        sim = S.Simulation(t.shape, t.omega, precision="f32", bc=t.bc, device=dev, stream=stream)
        sim.add_bubbles(t.pos, t.d, S.bubble_params(**dict(t.params, coupling=coupling)))
        sim.run(50)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(0, 800, 8):
            L.lbm_run(sim.ctx, sim.params, sim.bubbles.soa, sim.bubbles.nb, 8, 0)
        torch.cuda.synchronize()
        cost[name] = round((time.perf_counter() - t0) / 800 * 1e3, 5)
        sim.check()
        sim.close()
        print(f"[coupling] {name}: {cost[name]} ms per step on {t.name}", file=sys.stderr, flush=True)
    out = {
        "metric": METRIC, "value": round(t.cells / (cost["default"] * 1e-3) / 1e6, 1), "unit": "MLUPS",
        "n_gpus": 1, "steps": steps, "warmup": 0, "ms_per_step": cost["default"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "coupling_variants_4mm_60x60x180", "parallelism": "single GPU"},
        "coupling": {"column": w.name, "steps": steps, "variants": rows,
                     "ms_per_step_single_fp32_128x128x512": cost},
    }
    print(json.dumps(out), flush=True)


ADJOINT_GOLDEN = os.path.join(ROOT, "tests", "golden", "adjoint_64x64x192_oracle_gradient.json")


def leg_adjoint(args):
    """Gradient of the trajectory loss (drag scale, lift scale, omega) on the 64 x 64 x 192 FP32
    column with 4 bubbles, 2000 steps, checkpoints every 100 steps: throughput of the whole gradient
    pass (forward with checkpoints, segment recompute, reverse sweep) in lattice-site updates of
    the simulated steps per second, against the plain FP64 forward of the same column; gradient
    error against the oracle's central differences (h = 1e-3)."""
    import torch
    import workloads as W
    from paper_1710_07073_amd import adjoint as A
    from paper_1710_07073_amd import sim as S

    w = W.adjoint()
    stream = torch.cuda.current_stream()
    prob = A.TrajectoryProblem(w.shape, w.bc, w.pos, w.d, w.params, w.steps, precision="f32",
                               checkpoint=w.meta["checkpoint"], stream=stream)
    target, sim, _ = prob.forward(w.meta["target"], checkpoints=False)
    sim.close()
    # one untimed gradient pass first: the backward kernels' first launches (code loading) and
    # the allocator's first requests stay out of the timed pass
    warm = torch.tensor(w.meta["theta0"], dtype=torch.float64, requires_grad=True)
    ((A.BubbleTrajectory.apply(warm, prob) - target) ** 2).sum().backward()
    torch.cuda.synchronize()
    prob.liquid_events = []
    theta = torch.tensor(w.meta["theta0"], dtype=torch.float64, requires_grad=True)
    t0 = time.perf_counter()
    traj = A.BubbleTrajectory.apply(theta, prob)
    loss = ((traj - target) ** 2).sum()
    lv = loss.item()
    t1 = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    g = theta.grad.numpy()
    kern_s = float(np.mean([a.elapsed_time(b) for a, b in prob.liquid_events])) * 1e-3
    # plain single-instance FP64 form: the same column forward, graph replays
    sim = S.Simulation(w.shape, w.omega, precision="f64", bc=w.bc, stream=stream)
    sim.add_bubbles(w.pos, w.d, S.bubble_params(**w.params))
    sim.run(20, graph_steps=20)
    torch.cuda.synchronize()
    a = time.perf_counter()
    sim.run(w.steps, graph_steps=20)
    torch.cuda.synchronize()
    t_fp64 = time.perf_counter() - a
    sim.close()
    cells = int(np.prod(w.shape))
    mlups = cells * w.steps / (t2 - t0) / 1e6
    fp64 = cells * w.steps / t_fp64 / 1e6
    # per cell: pulled state 76 B, lambda in 76 B, lambda out 76 B (the adjoint step's own bytes);
    # the force, the velocity adjoint (read and cleared) and dL/dF add 48 B in the flagged tiles
    alg = 228 * cells
    out = {"workload": "adjoint_64x64x192_4b_f32", "steps": w.steps, "checkpoint": w.meta["checkpoint"],
           "gradient_pass_mlups": round(mlups, 1), "forward_s": round(t1 - t0, 4),
           "backward_s": round(t2 - t1, 4), "plain_fp64_forward_mlups": round(fp64, 1),
           "ratio_vs_plain_fp64": round(mlups / fp64, 3), "loss": lv, "gradient": g.tolist(),
           "k_adj_liquid": {"avg_launch_ms": round(kern_s * 1e3, 5), "alg_bytes_per_launch": alg,
                            "achieved_GBs": round(alg / kern_s / 1e9, 1),
                            "frac_hbm": round(alg / kern_s / 1e9 / HBM_PEAK_GBS, 4)}}
    if os.path.exists(ADJOINT_GOLDEN):
        ref = json.load(open(ADJOINT_GOLDEN))
        fd = np.array(ref["gradient"])
        out["error_vs_oracle_fd"] = {"loss_rel": abs(lv - ref["loss"]) / abs(ref["loss"]),
                                     "grad_rel_per_component": (np.abs(g - fd) / np.abs(fd)).tolist(),
                                     "grad_rel_to_max": float(np.abs(g - fd).max() / np.abs(fd).max())}
    return out


def bench_adjoint(args):
    leg = leg_adjoint(args)
    out = {
        "metric": METRIC, "value": leg["gradient_pass_mlups"], "unit": "MLUPS", "n_gpus": 1,
        "steps": leg["steps"], "warmup": 0,
        "ms_per_step": round((leg["forward_s"] + leg["backward_s"]) / leg["steps"] * 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic", "config": {"workload": leg["workload"], "parallelism": "single GPU"},
        "adjoint": leg,
    }
    print(json.dumps(out), flush=True)


def leg_precision(w, sim32, total_steps, gsteps=20):
    """Error of the FP32 shifted path per result: on the 32 x 32 x 64 column (500 steps) against the
    FP64 oracle itself, and on the timed workload against the FP64 GPU path (which matches the
    oracle to 1e-12) after the same number of steps."""
    import torch
    import oracle as O
    import workloads as W
    from paper_1710_07073_amd import sim as S

    def results(u, rho, x, v, sums):
        return dict(u=u, rho=rho, x=x, v=v, sums=sums)

    def compare(a, b):
        return {"u_rel_l2": float(np.linalg.norm(a["u"] - b["u"]) / np.linalg.norm(b["u"])),
                "rho_max_abs": float(np.abs(a["rho"] - b["rho"]).max()),
                "bubble_pos_max_abs": float(np.abs(a["x"] - b["x"]).max()),
                "bubble_vel_rel": float(np.abs(a["v"] - b["v"]).max() / np.abs(b["v"]).max()),
                "mass_sum_abs": float(abs(a["sums"][0] - b["sums"][0])),
                "momentum_sum_abs": float(np.abs(np.asarray(a["sums"][1:]) - np.asarray(b["sums"][1:])).max())}

    def of_sim(sim):
        rho, u, sums = sim.moments()
        b = sim.bubbles
        return results(u.double().cpu().numpy(), rho.double().cpu().numpy(),
                       b.positions(), b.velocities(), list(sums))

    small = W.plain_fp64()
    s32 = S.Simulation(small.shape, small.omega, precision="f32", bc=small.bc)
    s32.add_bubbles(small.pos, small.d, S.bubble_params(**small.params))
    s32.step(small.steps)
    r32 = of_sim(s32)
    s32.close()
    lat = O.Lattice(*small.shape, small.omega, small.bc)
    bub = O.Bubbles(pos=small.pos.copy(), d=small.d.copy())
    O.run(lat, O.bubble_params(**small.params), bub, small.steps)
    rho, u, sums = lat.moments()
    ro = results(u, rho, bub.pos, bub.vel, list(sums))
    out = {"small_vs_oracle": dict(workload="32x32x64 column, one bubble d=3, 500 steps",
                                   **compare(r32, ro))}
    s64 = S.Simulation(w.shape, w.omega, precision="f64", bc=w.bc)
    s64.add_bubbles(w.pos, w.d, S.bubble_params(**w.params))
    s64.run(total_steps - total_steps % gsteps, graph_steps=gsteps)
    s64.step(total_steps % gsteps)
    r64 = of_sim(s64)
    s64.close()
    out["timed_vs_fp64_gpu"] = dict(workload=f"{w.name}, {total_steps} steps", **compare(of_sim(sim32), r64))
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="single_fp32",
                    choices=["single_fp32", "plain_fp64", "dense", "batched", "adjoint", "stability",
                             "grid", "coupling", "terminal"])
    ap.add_argument("--graph-steps", type=int, default=0,
                    help="replay the step loop from a HIP graph of this many steps (even)")
    ap.add_argument("--precision", default=None, choices=[None, "f32", "f64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--launch", default=None,
                    help="vec,block_x[,workgroups_per_cu] of the liquid step (skips tuning)")
    ap.add_argument("--layout", default="plane", choices=["plane", "soa"],
                    help="population buffer layout: plane-blocked (default) or plain structure of arrays")
    ap.add_argument("--top", default="bounce-back", choices=["bounce-back", "free-slip"],
                    help="top face of the single-lattice workloads (free-slip: the paper's face set, "
                         "Sec. 3.3)")
    ap.add_argument("--no-overlap", action="store_true",
                    help="run the bubble kernels and the liquid step one after the other")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the precision, batched, adjoint and dense legs of the default line")
    ap.add_argument("--batched-steps", type=int, default=3000)
    ap.add_argument("--dense-steps", type=int, default=2000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one device copy of known size (for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the method runs on a single MI355X here; "
              "multi-GPU runs (slab decomposition with halo exchange) are not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as W
    from paper_1710_07073_amd import lbm as L
    from paper_1710_07073_amd import sim as S

    if args.workload == "batched":
        return bench_batched(args)
    if args.workload == "adjoint":
        return bench_adjoint(args)
    if args.workload == "stability":
        return bench_stability(args)
    if args.workload == "grid":
        return bench_grid(args)
    if args.workload == "coupling":
        return bench_coupling(args)
    if args.workload == "terminal":
        return bench_terminal(args)
    w = {"single_fp32": W.single_fp32, "plain_fp64": W.plain_fp64, "dense": W.dense}[args.workload]()
    if args.top == "free-slip":
        w = W.Workload(w.name + "_fstop", w.shape, w.omega, tuple(w.bc[:5]) + (W.FS,), w.pos, w.d,
                       w.params, w.steps, w.dtype)
    if args.precision:
        w = W.Workload(w.name.replace("fp32", args.precision).replace("fp64", args.precision),
                       w.shape, w.omega, w.bc, w.pos, w.d, w.params, w.steps, args.precision)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    layout_flags = L.LBM_FLAG_PLAIN_SOA if args.layout == "soa" else 0
    sim = S.Simulation(w.shape, w.omega, precision=w.dtype, bc=w.bc, flags=layout_flags, device=dev,
                       stream=stream)
    launch = {"vec": None, "bx": None, "tuned": False}
    if args.launch:
        parts = [int(v) for v in args.launch.split(",")]
        L.lbm_set_launch(sim.ctx, parts[0], parts[1])
        if len(parts) > 2:
            L.lbm_set_step_occupancy(sim.ctx, parts[2])
        launch.update(vec=parts[0], bx=parts[1])
    elif not args.no_autotune:
        # the liquid is at rest before the bubbles are added: tuning steps leave it unchanged
        from paper_1710_07073_amd import autotune
        vec, bx, entry = autotune.tune(sim, use_cache=False)
        launch.update(vec=vec, bx=bx, tuned=True)
        for v, b, us in entry["sweep"]:
            print(f"[autotune] vec={v} bx={b}: {us:.1f} us", file=sys.stderr, flush=True)
        for o, us in entry["occupancy_sweep"]:
            print(f"[autotune] occupancy {o}: {us:.1f} us", file=sys.stderr, flush=True)
    else:
        vec, bx = L.lbm_get_launch(sim.ctx)
        launch.update(vec=vec, bx=bx)
    launch["workgroups_per_cu"] = L.lbm_get_step_occupancy(sim.ctx)
    sim.add_bubbles(w.pos, w.d, S.bubble_params(**w.params))
    if args.no_overlap:
        L.lbm_set_overlap(sim.ctx, False)
    print(f"[bench] {w.name}: {w.cells} cells, warmup {args.warmup}, steps {args.steps}",
          file=sys.stderr, flush=True)
    tune_steps = 0
    if launch["tuned"] and w.nb:
        # the occupancy caps timed again on the method step itself (bubble kernels beside the
        # liquid step), which can prefer another cap than the liquid step alone
        from paper_1710_07073_amd import autotune
        launch["workgroups_per_cu_liquid_only"] = launch.get("workgroups_per_cu")
        occ, osweep, tune_steps = autotune.tune_method_occupancy(sim)
        for o, us, ov in osweep:
            print(f"[autotune] method-step occupancy {o}, {'overlapped' if ov else 'serial'}: "
                  f"{us:.1f} us", file=sys.stderr, flush=True)
        launch["tuning_method_steps"] = tune_steps
    for _ in range(args.warmup):
        sim.step(1)
    warm_done = tune_steps + args.warmup
    if args.copy_calibration:
        copy_calibration()
    torch.cuda.synchronize()

    K = args.steps
    launch["workgroups_per_cu"] = L.lbm_get_step_occupancy(sim.ctx)
    elapsed, kern_s, nt, region_cells = time_steps(sim, K, stream)
    overlap_on, overlap_avail = L.lbm_get_overlap(sim.ctx)

    # the run stayed finite and conserved mass
    _, _, sums = sim.moments(fields=False)
    sim.check()
    elem = 4 if w.dtype == "f32" else 8
    mlups = w.cells * K / elapsed / 1e6
    # 19 loads + 19 stores per site the launch updates (the bulk: every site outside the region)
    alg_bytes = 38 * elem * (w.cells - region_cells)
    achieved = alg_bytes / kern_s / 1e9
    traffic = read_traffic(w.name, elem) if region_cells else None  # taken on the bulk launch
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / K * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": w.dtype,
        "data": "synthetic",
        "config": {"workload": w.name, "lattice": list(w.shape), "cells": w.cells,
                   "omega": w.omega, "bubbles": w.nb, "bubble_diameter": float(np.median(w.d)),
                   "populations": f"D3Q19 shifted f-w, {w.dtype}",
                   "layout": "plane-blocked (nz,19,ny,nx)" if args.layout == "plane"
                   else "structure of arrays (19,nz,ny,nx)", "parallelism": "single GPU"},
        "roofline": {"bound": "hbm",
                     "kernel": "k_step_bb (fused collide-stream, bulk launch of the overlapped step)"
                     if region_cells else "fused collide-stream step over the whole lattice (serial step)",
                     "sites_per_launch": w.cells - region_cells,
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "alg_bytes_per_launch": alg_bytes,
                     "avg_launch_ms": round(kern_s * 1e3, 5), "launches_timed": nt,
                     "kernel_mlups": round((w.cells - region_cells) / kern_s / 1e6, 1),
                     "launch": launch},
        "overlap": {"enabled": overlap_on and overlap_avail, "region_sites_last_step": region_cells},
        "mass_drift": sums[0] - w.cells,
    }
    legs = (args.workload == "single_fp32" and not args.no_legs and not args.precision
            and args.top == "bounce-back")
    if legs:
        print("[bench] precision leg", file=sys.stderr, flush=True)
        out["precision"] = leg_precision(w, sim, warm_done + K)
    sim.close()
    if legs:
        print("[bench] batched leg", file=sys.stderr, flush=True)
        out["batched"] = leg_batched(args, args.batched_steps)
        print("[bench] adjoint leg", file=sys.stderr, flush=True)
        out["adjoint"] = leg_adjoint(args)
        print("[bench] dense leg", file=sys.stderr, flush=True)
        out["dense"] = leg_dense(args, args.dense_steps)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
