"""The dense dispersed-flow workload at its full size (256 x 256 x 768 FP32 lattice, 20 000
bubbles, lognormal diameters around 3, omega drawn in [1.2, 1.8]) as overlapped steps replayed
from HIP graphs (the same bits as the serial step, which the benchmark's tuning may keep): its
first 200 steps compared with the oracle on the whole lattice and every bubble after 100 and
after 200 steps (by then the bubbles have reached their rise velocity and their wakes overlap),
and properties that hold at any size (mass conservation, finiteness) over more steps."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_common import gpu_sim, oracle_state, rel_l2
from paper_1710_07073_amd import lbm as L

POS_TOL = 1e-4
U_TOL = 2e-5


@pytest.fixture(scope="module")
def dense_run():
    """The GPU run of the first 200 steps (state after 100 and after 200) and the oracle's lattice
    and bubbles at step 0; the tests advance the oracle in turn, so that each reports within
    about a minute and a half."""
    w = W.dense(steps=200)
    print(f"[case] {w.name}: {w.cells} cells, {w.nb} bubbles, omega {w.omega:.4f}, "
          f"{w.steps} steps", flush=True)
    sim = gpu_sim(w)
    L.lbm_set_launch(sim.ctx, 1, 256)  # the width the benchmark's tuning keeps on this column
    assert L.lbm_get_overlap(sim.ctx)[0]
    snaps = {}
    for k in (100, 200):
        sim.run(100, graph_steps=20)
        _, u, sums = sim.moments()
        snaps[k] = dict(u=u.double().cpu().numpy(), pos=sim.bubbles.positions(),
                        vel=sim.bubbles.velocities(), st=sim.bubbles.state(), sums=sums)
    sim.check()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    lat, bub, P = oracle_state(w)
    return dict(w=w, snaps=snaps, lat=lat, bub=bub, P=P, done=[0], pos0=w.pos.copy())


@pytest.mark.gpu
@pytest.mark.timeout(900)
@pytest.mark.parametrize("upto", [100, 200])
def test_dense_column_full_size_matches_oracle(dense_run, upto):
    r = dense_run
    w, lat, bub, P = r["w"], r["lat"], r["bub"], r["P"]
    for k in range(r["done"][0], upto):
        O.method_step(lat, P, bub)
        if (k + 1) % 25 == 0:
            print(f"  oracle step {k + 1}", flush=True)
    r["done"][0] = upto
    g = r["snaps"][upto]
    _, u_o, _ = lat.moments()
    eu = rel_l2(g["u"], u_o)
    dx = np.abs(g["pos"] - bub.pos).max()
    ev = rel_l2(g["vel"], bub.vel)
    rise = (bub.pos[2] - r["pos0"][2]).mean()
    print(f"step {upto}: u rel-L2 {eu:.3e}, max |dx_b| {dx:.2e}, u_b rel-L2 {ev:.2e}, "
          f"mean rise {rise:.3f}", flush=True)
    assert np.array_equal(g["st"], bub.state)
    assert dx <= POS_TOL
    assert ev <= U_TOL
    assert eu <= U_TOL
    assert abs(g["sums"][0] - w.cells) < 1e-3
    # the bubbles rose (Stokes rise of a d = 3 bubble: about 0.005 in 100 steps)
    assert rise > 0.002 * upto / 100


@pytest.mark.gpu
def test_dense_column_serial_step_is_the_overlapped_step(dense_run):
    """The serial method step (the benchmark's tuning keeps it when it is the faster) reproduces
    the overlapped run of the first 200 steps bit for bit at full size."""
    w = dense_run["w"]
    sim = gpu_sim(w)
    L.lbm_set_launch(sim.ctx, 1, 256)
    L.lbm_set_overlap(sim.ctx, False)
    sim.run(200, graph_steps=20)
    _, u, _ = sim.moments()
    g = dense_run["snaps"][200]
    assert np.array_equal(u.double().cpu().numpy(), g["u"])
    assert np.array_equal(sim.bubbles.positions(), g["pos"])
    assert np.array_equal(sim.bubbles.velocities(), g["vel"])
    sim.check()
    sim.close()


@pytest.mark.gpu
def test_dense_column_conserves_mass_over_many_steps():
    w = W.dense(steps=200)
    sim = gpu_sim(w)
    _, _, s0 = sim.moments(fields=False)
    sim.step(w.steps)
    _, _, s1 = sim.moments(fields=False)
    sim.check()
    assert np.all(np.isfinite(s1))
    # FP32 storage: each step rounds every population; the total mass still stays at N to ~1e-9
    assert abs(s1[0] - s0[0]) <= 1e-9 * w.cells
    pos = sim.bubbles.positions()
    assert np.all(np.isfinite(pos)) and np.all(pos[2] >= 0)
    sim.close()
