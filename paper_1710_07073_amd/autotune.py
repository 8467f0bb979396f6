"""Launch-shape autotuner of the fused liquid step.

The step kernel has two shape parameters (see lbm_set_launch in include/lbm.h): cells per thread
along x (1, 2, 4) and threads per workgroup along x; and an occupancy cap (lbm_set_step_occupancy:
at most so many of its workgroups per compute unit). Results do not depend on them; speed does,
and the best choice depends on the row length nx, the precision and the machine. The tuner times
every valid shape with HIP events on the simulation's stream, keeps the fastest, then times the
occupancy caps with that shape, and caches the winner per size class (precision, nx, bucketed
ny*nz) in a JSON file.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np
import torch

from . import lbm as L

CACHE = os.environ.get("LBM_AUTOTUNE_CACHE",
                       os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib",
                                    "autotune_cache.json"))


def candidates(nx):
    out = []
    for vec in (1, 2, 4):
        if nx % vec:
            continue
        per_row = nx // vec
        for bx in (16, 32, 64, 128, 256):
            if bx > 16 and bx > per_row and bx // 2 >= per_row:
                continue  # half the workgroup or more would idle past the end of the row
            out.append((vec, bx))
    return out


OCCUPANCY = (0, 3, 4, 5, 6, 7)  # workgroups per compute unit, 0 = no cap


def size_class(shape, precision):
    nx, ny, nz = shape
    plane = ny * nz
    bucket = 1 << max(0, int(plane - 1).bit_length())  # next power of two of ny*nz
    return f"p{precision}_nx{nx}_yz{bucket}"


def _load():
    try:
        with open(CACHE) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save(db):
    os.makedirs(os.path.dirname(CACHE), exist_ok=True)
    tmp = CACHE + ".tmp"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1, sort_keys=True)
    os.replace(tmp, CACHE)


def time_launch(sim, vec, bx, steps=20, warmup=3, occ=None):
    """Average duration (s) of one liquid-step launch with the given shape (and occupancy cap, if
    given)."""
    L.lbm_set_launch(sim.ctx, vec, bx)
    if occ is not None:
        L.lbm_set_step_occupancy(sim.ctx, occ)
    stream = sim.stream
    L.lbm_step(sim.ctx, warmup)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    L.lbm_step(sim.ctx, steps)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / steps


def tune(sim, steps=20, use_cache=True, verbose=False):
    """Pick the fastest launch shape for this simulation's lattice and apply it. The lattice state
    advances by the timing steps (callers tune before loading their initial state, or on a
    scratch simulation of the same shape)."""
    key = size_class(sim.shape, sim.precision)
    db = _load() if use_cache else {}
    if key in db and "occ" in db[key]:
        vec, bx, occ = db[key]["vec"], db[key]["bx"], db[key]["occ"]
        L.lbm_set_launch(sim.ctx, vec, bx)
        L.lbm_set_step_occupancy(sim.ctx, occ)
        return vec, bx, db[key]
    results = []
    for vec, bx in candidates(sim.shape[0]):
        t = time_launch(sim, vec, bx, steps)
        results.append((t, vec, bx))
        if verbose:
            print(f"  vec={vec} bx={bx}: {t * 1e6:.1f} us/step", flush=True)
    results.sort()
    t, vec, bx = results[0]
    occ_results = []
    for occ in OCCUPANCY:
        to = time_launch(sim, vec, bx, steps, occ=occ)
        occ_results.append((to, occ))
        if verbose:
            print(f"  vec={vec} bx={bx} occupancy={occ}: {to * 1e6:.1f} us/step", flush=True)
    occ_results.sort()
    t, occ = occ_results[0]
    L.lbm_set_launch(sim.ctx, vec, bx)
    L.lbm_set_step_occupancy(sim.ctx, occ)
    entry = {"vec": vec, "bx": bx, "occ": occ, "us_per_step": t * 1e6,
             "sweep": [[v, b, r * 1e6] for r, v, b in results],
             "occupancy_sweep": [[o, r * 1e6] for r, o in occ_results], "time": time.time()}
    db[key] = entry
    _save(db)
    return vec, bx, entry


def tune_method_occupancy(sim, steps=8, caps=OCCUPANCY, modes=None):
    """The occupancy cap timed on whole method steps (bubble half and liquid step) rather than on
    the liquid step alone: beside the bubble kernels the best cap can differ. Where the lattice
    can overlap, the overlapped and the serial step are both timed (the same results bit for bit;
    which is faster depends on how long the bubble half is against the liquid step). Applies the
    fastest (cap, overlap) and returns (cap, [[cap, us per step, overlap]], method steps run).
    The simulation advances by len(modes) * len(caps) * (steps + 2) steps (callers count them as
    warm-up)."""
    stream = sim.stream
    bub = sim.bubbles
    on, avail = L.lbm_get_overlap(sim.ctx)
    if modes is None:
        modes = (True, False) if avail else (bool(on),)
    sweep = []
    for ov in modes:
        L.lbm_set_overlap(sim.ctx, ov)
        for occ in caps:
            L.lbm_set_step_occupancy(sim.ctx, occ)
            L.lbm_run(sim.ctx, sim.params, bub.soa, bub.nb, 2, 0)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            L.lbm_run(sim.ctx, sim.params, bub.soa, bub.nb, steps, 0)
            e1.record(stream)
            e1.synchronize()
            sweep.append([occ, e0.elapsed_time(e1) * 1e3 / steps, bool(ov)])
    best = min(sweep, key=lambda r: r[1])
    L.lbm_set_overlap(sim.ctx, best[2])
    L.lbm_set_step_occupancy(sim.ctx, best[0])
    return best[0], sweep, len(modes) * len(caps) * (steps + 2)


# ---------------------------------------------------------------------------------------------
# Batched columns: cells per work item, per column size class
# ---------------------------------------------------------------------------------------------
ITEM_CANDIDATES = (256, 512, 1024, 2048, 4096)


def column_class(shape):
    """Size class of a column for the batch tuner: by cells, in factors of 4."""
    cells = int(np.prod(shape))
    k = 0
    while cells > 65536 and k < 4:
        cells //= 4
        k += 1
    return k


def time_batch(batch, steps=4, warmup=1):
    """Average seconds per liquid+bubble step of the whole batch (eager launches)."""
    batch.step(warmup)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(batch.stream)
    batch.step(steps)
    e1.record(batch.stream)
    e1.synchronize()
    return e0.elapsed_time(e1) * 1e-3 / steps


def tune_batch(batch, steps=4, verbose=False):
    """Coordinate descent over the size classes: for each class in turn, try every candidate item
    size with the other classes fixed, keep the fastest. Applies and returns the per-column item
    sizes and the sweep. The batch state advances by the timing steps."""
    ncols = batch.ncols
    classes = [column_class(c["shape"]) for c in batch.columns]
    items = L.lbm_batch_get_items(batch.handle, ncols)
    sweep = []
    for k in sorted(set(classes)):
        best = None
        for cand in ITEM_CANDIDATES:
            trial = [cand if classes[i] == k else items[i] for i in range(ncols)]
            L.lbm_batch_set_items(batch.handle, trial)
            t = time_batch(batch, steps)
            sweep.append((k, cand, t * 1e3))
            if verbose:
                print(f"  class {k} item {cand}: {t * 1e3:.3f} ms/step", flush=True)
            if best is None or t < best[0]:
                best = (t, cand)
        items = [best[1] if classes[i] == k else items[i] for i in range(ncols)]
    L.lbm_batch_set_items(batch.handle, items)
    return items, sweep


BATCH_OCCUPANCY = (0, 2, 3, 4)  # workgroups per compute unit of the batched step, 0 = no cap


def tune_batch_occupancy(batch, steps=4, verbose=False):
    """Time the occupancy caps of the batched liquid step with the batch's current items; applies
    and returns the fastest and the sweep [(cap, ms/step)]. The batch state advances."""
    sweep = []
    for occ in BATCH_OCCUPANCY:
        L.lbm_batch_set_step_occupancy(batch.handle, occ)
        t = time_batch(batch, steps)
        sweep.append((occ, t * 1e3))
        if verbose:
            print(f"  occupancy {occ}: {t * 1e3:.3f} ms/step", flush=True)
    best = min(sweep, key=lambda e: e[1])[0]
    L.lbm_batch_set_step_occupancy(batch.handle, best)
    return best, sweep
