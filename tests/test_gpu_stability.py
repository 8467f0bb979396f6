"""Divergence detection on a real BGK instability (Sec. 4.3): a bubble swarm column that the oracle
shows going non-finite by itself at omega = 1.995 and staying bounded at 1.98
(test_oracle_stability). On the GPU the single-lattice moments() must report LBM_EDIVERGED, and in
a batch only the unstable column may be flagged by lbm_batch_sums."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_common import gpu_sim, oracle_state, rel_l2
from paper_1710_07073_amd import lbm as L
from paper_1710_07073_amd import sim as S


def _first_divergence(sim, steps, chunk=50):
    """Run in chunks; the step count at which moments() first reports LBM_EDIVERGED, else None."""
    done = 0
    while done < steps:
        sim.run(chunk, graph_steps=10)
        done += chunk
        try:
            sim.moments(fields=False)
        except L.LbmError as e:
            assert e.code == L.LBM_EDIVERGED, e
            return done
    return None


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_swarm_lattice_diverges_and_moments_reports_it(precision):
    w = W.swarm(nb=32, omega=1.995, steps=100, dtype=precision)
    print(f"[case] {w.name} {precision}", flush=True)
    sim = gpu_sim(w)
    sim.run(w.steps, graph_steps=10)
    _, u, sums = sim.moments()
    assert np.all(np.isfinite(sums))
    u = u.double().cpu().numpy()
    lat, bub, P = oracle_state(w)
    for _ in range(w.steps):
        O.method_step(lat, P, bub)
    _, u_o, _ = lat.moments()
    err = rel_l2(u, u_o)
    print(f"before the blow-up (step {w.steps}): u rel-L2 {err:.2e}, max |u| {np.abs(u_o).max():.3f}",
          flush=True)
    assert err <= (1e-10 if precision == "f64" else 1e-3)
    first = _first_divergence(sim, 900)
    print(f"moments() reports LBM_EDIVERGED after {first} steps in all", flush=True)
    assert first is not None and first <= w.steps + 900
    sim.close()


@pytest.mark.gpu
def test_swarm_stable_omega_stays_finite():
    w = W.swarm(nb=32, omega=1.98, steps=1000, dtype="f32")
    print(f"[case] {w.name}", flush=True)
    sim = gpu_sim(w)
    assert _first_divergence(sim, w.steps, chunk=100) is None
    _, u, _ = sim.moments()
    assert float(u.abs().max()) < 0.3
    sim.close()


@pytest.mark.gpu
def test_batch_flags_only_the_unstable_swarm_column():
    omegas = (1.9, 1.97, 1.98, 1.995)
    ws = [W.swarm(nb=32, omega=om, dtype="f32") for om in omegas]
    print(f"[case] batch of swarm columns at omega {omegas}", flush=True)
    cols = [dict(shape=w.shape, omega=w.omega, bc=w.bc, pos=w.pos, d=w.d) for w in ws]
    batch = S.Batch(cols, S.bubble_params(**ws[0].params), precision="f32")
    first = [None] * len(ws)
    for done in range(100, 1101, 100):
        batch.run(100, graph_steps=20)
        _, diverged = batch.sums()
        for k, dv in enumerate(diverged):
            if dv and first[k] is None:
                first[k] = done
    print(f"first flagged step per column: {first}", flush=True)
    sums, diverged = batch.sums()
    assert list(diverged) == [False, False, False, True]
    assert np.all(np.abs(sums[:3, 0] - np.array([w.cells for w in ws[:3]])) < 1e-2)
    batch.close()


@pytest.mark.gpu
def test_swarm_of_384_reproduces_the_papers_stability_limit():
    """Sec. 4.3 (Fig. 5): stable up to omega = 1.97, unstable at 1.98. The App. A column (30 x 30 x
    90, free-slip top) with the 384-bubble swarm of the stability map, FP32 batch (bit-reproducible
    spreading): the column at 1.98 diverges within 2000 steps, those at 1.96 and 1.97 do not."""
    omegas = (1.96, 1.97, 1.98)
    ws = [w for w in W.stability_swarm(steps=2000, omegas=omegas, counts=(384,))]
    print(f"[case] 384-bubble swarm, App. A column, omega {omegas}", flush=True)
    cols = [dict(shape=w.shape, omega=w.omega, bc=w.bc, pos=w.pos, d=w.d) for w in ws]
    batch = S.Batch(cols, S.bubble_params(**ws[0].params), precision="f32")
    first = [None] * len(ws)
    for done in range(250, 2001, 250):
        batch.run(250, graph_steps=50)
        _, diverged = batch.sums()
        for k, dv in enumerate(diverged):
            if dv and first[k] is None:
                first[k] = done
    print(f"first flagged step per column: {first}", flush=True)
    assert first[0] is None and first[1] is None and first[2] is not None
    batch.close()
