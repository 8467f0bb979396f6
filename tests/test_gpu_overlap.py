"""Overlapped method step (bubble kernels on the caller's stream while the liquid step updates the
tiles away from the bubbles on a side stream): identical to the serial step bit for bit, eager and
replayed from a HIP graph, and a bubble leaving the step's region is reported."""
import numpy as np
import pytest
import torch

import workloads as W
from paper_1710_07073_amd import lbm as L
from paper_1710_07073_amd import sim as S

BB, FS, PER = 0, 1, 2


def _run(shape, prec, pos, d, overlap, steps, graph_steps=0, vel=None, run=False, bc=(BB,) * 6,
         **pkw):
    """steps method steps: through lbm_run (graph replay if graph_steps) or, unless run is set and
    graph_steps is 0, one bubbles_step + lbm_step pair at a time."""
    sim = S.Simulation(shape, 1.35, precision=prec, bc=bc)
    L.lbm_set_overlap(sim.ctx, overlap)
    sim.add_bubbles(pos, d, S.bubble_params(**pkw), vel=vel)
    if graph_steps or run:
        sim.run(steps, graph_steps=graph_steps)
    else:
        sim.step(steps)
    out = dict(g=sim.populations().cpu().numpy(), U=sim.vel.cpu().numpy(),
               x=sim.bubbles.positions(), v=sim.bubbles.velocities(), st=sim.bubbles.state())
    sim.check()
    sim.close()
    return out


def _same(a, b):
    for k in a:
        assert np.array_equal(a[k], b[k]), k


CASES = [
    # ragged shape (partial tiles), bubbles near the walls and close to each other
    ((37, 29, 45), [[2.0, 18.5, 34.3], [27.2, 14.0, 3.1], [9.0, 30.5, 21.0]], [3.0, 2.5, 4.0]),
    ((64, 64, 96), [[32.0, 31.5, 10.0, 40.0], [32.0, 33.0, 60.0, 12.0], [8.0, 8.0, 8.5, 30.0]],
     [4.0, 4.0, 3.0, 5.0]),
]


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("shape,pos,d", CASES)
def test_overlapped_step_matches_serial_step(prec, shape, pos, d):
    print(f"overlap vs serial {shape} {prec}", flush=True)
    pos = np.array(pos, dtype=np.float64)
    kw = dict(g=1e-4, sigma=1e-4)
    sim = S.Simulation(shape, 1.35, precision=prec, bc=(BB,) * 6)
    assert L.lbm_get_overlap(sim.ctx) == (False, True)  # available; off by default below 2^22 cells
    sim.close()
    a = _run(shape, prec, pos, d, False, 40, **kw)
    b = _run(shape, prec, pos, d, True, 40, **kw)
    _same(a, b)
    c = _run(shape, prec, pos, d, True, 40, run=True, **kw)  # eager lbm_run: marks ahead
    _same(a, c)
    assert np.abs(a["x"][2] - pos[2]).max() > 1e-3  # the bubbles moved


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_overlapped_steps_replayed_from_a_graph(prec):
    shape, pos, d = CASES[1]
    pos = np.array(pos, dtype=np.float64)
    print(f"overlap graph {prec}", flush=True)
    kw = dict(g=1e-4, sigma=1e-4)
    eager = _run(shape, prec, pos, d, False, 26, **kw)
    graph = _run(shape, prec, pos, d, True, 26, graph_steps=4, **kw)
    _same(eager, graph)


@pytest.mark.gpu
@pytest.mark.parametrize("graph_steps", [0, 4])
def test_many_bubbles_overlapped_match_serial(graph_steps):
    """More than 64 bubbles: the region is updated on the caller's stream after the bulk."""
    rng = np.random.default_rng(11)
    nb = 96
    shape = (64, 64, 96)
    pos = np.stack([rng.uniform(6, 58, nb), rng.uniform(6, 58, nb), rng.uniform(6, 70, nb)])
    d = rng.uniform(2.0, 3.5, nb)
    print(f"overlap vs serial, {nb} bubbles, graph_steps {graph_steps}", flush=True)
    kw = dict(g=1e-4, sigma=1e-4)
    a = _run(shape, "f32", pos, d, False, 12, **kw)
    b = _run(shape, "f32", pos, d, True, 12, graph_steps=graph_steps, run=True, **kw)
    _same(a, b)


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_overlap_with_the_papers_faces(prec):
    """Bounce-back walls and bottom with a free-slip top (Sec. 3.3): the wall fast path overlaps
    too, bit for bit the serial step, with bubbles rising into the top layer."""
    shape = (40, 36, 30)
    pos = np.array([[20.0, 8.0, 30.0], [18.0, 27.5, 9.0], [24.0, 28.7, 12.0]])
    d = [3.0, 2.5, 4.0]
    print(f"overlap vs serial, free-slip top {prec}", flush=True)
    kw = dict(g=3e-3, sigma=1e-3)
    bc = (BB, BB, BB, BB, BB, FS)
    sim = S.Simulation(shape, 1.35, precision=prec, bc=bc)
    assert L.lbm_get_overlap(sim.ctx) == (False, True)
    sim.close()
    a = _run(shape, prec, pos, d, False, 60, bc=bc, **kw)
    b = _run(shape, prec, pos, d, True, 60, bc=bc, **kw)
    _same(a, b)
    c = _run(shape, prec, pos, d, True, 60, graph_steps=6, bc=bc, **kw)
    _same(a, c)
    assert (a["st"] == 0).any()  # a bubble reached the top layer


@pytest.mark.gpu
def test_overlap_unavailable_is_the_serial_step():
    """Periodic faces take the general step: no overlap, and asking for it is a no-op."""
    sim = S.Simulation((24, 24, 32), 1.2, precision="f32", bc=(PER, PER, PER, PER, BB, FS))
    L.lbm_set_overlap(sim.ctx, True)
    assert L.lbm_get_overlap(sim.ctx) == (True, False)
    sim.add_bubbles(np.array([[12.0], [12.0], [8.0]]), [3.0], S.bubble_params(g=1e-4, sigma=1e-4))
    sim.step(5)
    sim.check()
    sim.close()


@pytest.mark.gpu
def test_bubble_leaving_the_region_is_reported():
    """A buoyancy kick moving the bubble by several cells in one step takes its next velocity
    window out of the step's region: the step reports it (kernels run to completion). With the
    bubble at z = 16 (d = 3) the region ends at z = 23, a tile boundary; the kick (g = 10) moves it
    by about 3.6 cells, so its next velocity window reaches z = 25."""
    print("region miss", flush=True)
    P = S.bubble_params(g=10.0, sigma=1e-4)
    nu = (1 / 1.2 - 0.5) / 3
    x, _, _ = L.host_bubble_ode(P, nu, 3.0, np.array([12.0, 12.0, 16.0]), np.zeros(3), np.zeros(3),
                                np.zeros(3), np.zeros(3), (24, 24, 96))
    assert x[2] > 19.0
    sim = S.Simulation((24, 24, 96), 1.2, precision="f32", bc=(BB,) * 6)
    L.lbm_set_overlap(sim.ctx, True)
    sim.add_bubbles(np.array([[12.0], [12.0], [16.0]]), [3.0], P)
    sim.step(1)
    with pytest.raises(L.LbmError) as e:
        sim.check()
    assert e.value.code == L.LBM_EUNSUPPORTED
    sim.close()


@pytest.mark.gpu
def test_overlap_is_on_by_default_for_large_lattices():
    sim = S.Simulation((128, 128, 256), 1.6, precision="f32", bc=(BB,) * 6)
    assert L.lbm_get_overlap(sim.ctx) == (True, True)
    sim.close()


def _run_with_moves(overlap, graph_steps, prec="f32"):
    shape, pos, d = CASES[1]
    sim = S.Simulation(shape, 1.35, precision=prec, bc=(BB,) * 6)
    L.lbm_set_overlap(sim.ctx, overlap)
    sim.add_bubbles(np.array(pos, dtype=np.float64), d, S.bubble_params(g=1e-4, sigma=1e-4))
    sim.run(10, graph_steps=graph_steps)
    # the caller moves the bubbles between calls, beyond the region the last step marked ahead
    sim.bubbles.t["z"] += 20.0
    sim.run(10, graph_steps=graph_steps)
    sim.step(3)
    sim.bubbles.t["x"] -= 6.0
    sim.bubbles.t["y"] += 5.0
    sim.run(6, graph_steps=graph_steps)
    out = dict(g=sim.populations().cpu().numpy(), U=sim.vel.cpu().numpy(),
               x=sim.bubbles.positions(), v=sim.bubbles.velocities(), st=sim.bubbles.state())
    sim.check()  # no bubble left its step's region
    sim.close()
    return out


@pytest.mark.gpu
@pytest.mark.parametrize("graph_steps", [0, 2])
def test_bubbles_moved_between_runs_are_marked_afresh(graph_steps):
    """Inside lbm_run each overlapped step marks the next step's region after its bubble update;
    a new call (or a single bubbles_step) marks afresh from the caller's bubble state, and marks
    left over from the previous call only widen the region: identical to the serial step."""
    print(f"overlap with host moves between runs, graph_steps {graph_steps}", flush=True)
    a = _run_with_moves(False, graph_steps)
    b = _run_with_moves(True, graph_steps)
    _same(a, b)


@pytest.mark.gpu
@pytest.mark.parametrize("graph_steps", [0, 4])
def test_region_cells_reports_only_an_overlapped_last_step(graph_steps):
    """lbm_region_cells: the region of the last step if it was overlapped, 0 once a serial step
    (with bubbles, or a liquid step alone) has come after it, eager and through graph replays."""
    shape = (48, 40, 64)
    print(f"[case] {shape}, graph_steps {graph_steps}", flush=True)
    sim = S.Simulation(shape, 1.35, precision="f32")
    sim.add_bubbles([[20.0], [20.0], [12.0]], [3.0], S.bubble_params())
    assert L.lbm_get_overlap(sim.ctx)[1]
    L.lbm_set_overlap(sim.ctx, True)
    sim.run(8, graph_steps=graph_steps)
    overlapped = L.lbm_region_cells(sim.ctx)
    assert 0 < overlapped < sim.cells
    L.lbm_set_overlap(sim.ctx, False)
    sim.run(8, graph_steps=graph_steps)
    assert L.lbm_region_cells(sim.ctx) == 0
    L.lbm_set_overlap(sim.ctx, True)
    sim.run(8, graph_steps=graph_steps)
    assert L.lbm_region_cells(sim.ctx) == overlapped  # the bubble barely moved: the same rows
    sim.liquid_steps(1)
    assert L.lbm_region_cells(sim.ctx) == 0
    sim.check()
    sim.close()


@pytest.mark.gpu
def test_method_step_tuning_keeps_the_results():
    """The method-step tuning (overlapped and serial steps, every occupancy cap) changes how the
    steps run, not what they compute: the tuned run continues bit for bit like an untuned run of
    the same number of steps."""
    from paper_1710_07073_amd import autotune
    shape = (128, 128, 256)  # 2^22 sites: the overlapped step is available and on by default
    rng = np.random.default_rng(11)
    nb = 200
    pos = np.stack([rng.uniform(8, 119, nb), rng.uniform(8, 119, nb), rng.uniform(8, 60, nb)])
    d = rng.uniform(2.0, 4.0, nb)
    print(f"[case] {shape}, {nb} bubbles", flush=True)
    a = S.Simulation(shape, 1.6, precision="f32")
    a.add_bubbles(pos, d, S.bubble_params())
    assert L.lbm_get_overlap(a.ctx) == (True, True)
    cap, sweep, n = autotune.tune_method_occupancy(a, steps=2)
    assert len(sweep) == 2 * len(autotune.OCCUPANCY)
    assert {r[2] for r in sweep} == {True, False}
    best = min(sweep, key=lambda r: r[1])
    assert L.lbm_get_overlap(a.ctx)[0] == best[2] and L.lbm_get_step_occupancy(a.ctx) == cap
    a.run(10, graph_steps=10)
    b = S.Simulation(shape, 1.6, precision="f32")
    b.add_bubbles(pos, d, S.bubble_params())
    b.step(n + 10)
    assert np.array_equal(a.populations().cpu().numpy(), b.populations().cpu().numpy())
    assert np.array_equal(a.bubbles.positions(), b.bubbles.positions())
    for s in (a, b):
        s.check()
        s.close()
