"""The benchmark workload at its full size — 128 x 128 x 512 FP32 lattice (8.4 M sites), omega 1.6,
bounce-back walls, one bubble of diameter 4 released at the bottom centre — in the launch
configuration the benchmark times (one cell per thread, workgroup x-width 128, overlapped method
step), eager and replayed from a HIP graph, against the oracle on the whole lattice."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_common import gpu_sim, oracle_state, rel_l2
from paper_1710_07073_amd import lbm as L

U_TOL = 2e-5   # FP32 shifted path, relative L2
POS_TOL = 1e-4  # bubble position, lattice units


@pytest.mark.gpu
def test_single_fp32_full_size_matches_oracle():
    w = W.single_fp32(steps=40)
    print(f"[case] {w.name}: {w.cells} sites, 20 eager + 20 graph-replayed steps", flush=True)
    sim = gpu_sim(w)
    L.lbm_set_launch(sim.ctx, 1, 128)
    assert L.lbm_get_overlap(sim.ctx) == (True, True)
    sim.step(20)
    sim.run(20, graph_steps=10)
    assert L.lbm_region_cells(sim.ctx) > 0  # the last steps were overlapped
    _, u, sums = sim.moments()
    g = sim.populations().double().cpu().numpy()
    u = u.double().cpu().numpy()
    x, v = sim.bubbles.positions(), sim.bubbles.velocities()
    sim.check()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    lat, bub, P = oracle_state(w)
    for _ in range(w.steps):
        O.method_step(lat, P, bub)
    _, u_o, sums_o = lat.moments()
    eg, eu = rel_l2(g, lat.g), rel_l2(u, u_o)
    dx = np.abs(x - bub.pos).max()
    print(f"rel-L2 g {eg:.2e}, u {eu:.2e}; |dx_b| {dx:.2e}; bubble z {x[2, 0]:.4f}", flush=True)
    assert eg <= U_TOL and eu <= U_TOL
    assert dx <= POS_TOL
    assert np.abs(v - bub.vel).max() <= 1e-4 * np.abs(bub.vel).max()
    assert abs(sums[0] - sums_o[0]) <= 1e-6 * w.cells
    assert x[2, 0] > w.pos[2, 0]  # the bubble rose


def _gpu_run(w, precision, checkpoints):
    """Coupled method steps of w in the benchmark's launch configuration (one cell per thread,
    x-width 128, overlapped steps replayed from 20-step graphs): the state after each of the
    step counts in checkpoints."""
    import dataclasses
    sim = gpu_sim(dataclasses.replace(w, dtype=precision))
    L.lbm_set_launch(sim.ctx, 1, 128)
    out, done = {}, 0
    for k in checkpoints:
        sim.run(k - done, graph_steps=20)
        done = k
        _, u, sums = sim.moments()
        out[k] = dict(u=u.double().cpu().numpy(), x=sim.bubbles.positions(),
                      v=sim.bubbles.velocities(), sums=np.asarray(sums))
    sim.check()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out


@pytest.fixture(scope="module")
def long_run():
    """FP32 and FP64 GPU runs of the full column (state after 500 and after 1000 steps) and the
    oracle at step 0; the tests advance the oracle in turn, so each reports within about a
    minute."""
    w = W.single_fp32(steps=1000)
    print(f"[case] {w.name}: {w.cells} sites, {w.steps} steps, FP32 and FP64", flush=True)
    runs = {"f32": _gpu_run(w, "f32", (500, 1000)), "f64": _gpu_run(w, "f64", (500, 1000))}
    lat, bub, P = oracle_state(w)
    return dict(w=w, runs=runs, lat=lat, bub=bub, P=P, done=[0])


@pytest.mark.gpu
@pytest.mark.timeout(900)
@pytest.mark.parametrize("upto", [500, 1000])
def test_single_column_1000_steps_fp32_and_fp64_match_oracle(long_run, upto):
    """1000 coupled steps of the full 128 x 128 x 512 column, FP32 and FP64, against one oracle
    run, checked after 500 and after 1000 steps: u relative L2 <= 2e-5 (FP32) and <= 1e-12
    (FP64), bubble position <= 1e-4 lattice units (FP64: 1e-10)."""
    r = long_run
    w, lat, bub, P = r["w"], r["lat"], r["bub"], r["P"]
    for k in range(r["done"][0], upto):
        O.method_step(lat, P, bub)
        if (k + 1) % 100 == 0:
            print(f"  oracle step {k + 1}", flush=True)
    r["done"][0] = upto
    _, u_o, sums_o = lat.moments()
    for name, utol, xtol in (("f32", U_TOL, POS_TOL), ("f64", 1e-12, 1e-10)):
        g = r["runs"][name][upto]
        eu = rel_l2(g["u"], u_o)
        dx = np.abs(g["x"] - bub.pos).max()
        dv = np.abs(g["v"] - bub.vel).max() / np.abs(bub.vel).max()
        dm = abs(g["sums"][0] - sums_o[0])
        print(f"{name} step {upto}: u rel-L2 {eu:.2e}, |dx_b| {dx:.2e}, u_b rel {dv:.2e}, "
              f"mass {dm:.1e}", flush=True)
        assert eu <= utol, (name, eu)
        assert dx <= xtol, (name, dx)
    assert bub.pos[2, 0] > w.pos[2, 0] + 0.005 * upto / 500  # the bubble rose
