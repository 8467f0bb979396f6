"""Batched columns (many independent lattices of uneven size and relaxation rate stepped by one
launch per kernel, repeated steps replayed from a HIP graph): every column must reproduce its own
single-lattice run, the oracle, and graph replays must reproduce eager launches."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_common import rel_l2
from paper_1710_07073_amd import lbm as L
from paper_1710_07073_amd import sim as S

BB, FS, PER = O.BC_BOUNCE_BACK, O.BC_FREE_SLIP, O.BC_PERIODIC
TOL = {"f64": 1e-12, "f32": 2e-5}


def _columns(seed=21, nb_max=4):
    rng = np.random.default_rng(seed)
    specs = [((24, 30, 50), 0.7, (BB,) * 6), ((37, 25, 61), 1.9, (BB,) * 6),
             ((64, 40, 90), 1.3, (BB,) * 6), ((33, 33, 70), 1.1, (BB, BB, BB, BB, BB, FS)),
             ((20, 28, 44), 1.6, (PER, PER, PER, PER, BB, BB))]
    cols = []
    for shape, omega, bc in specs:
        nb = int(rng.integers(1, nb_max + 1))
        d = rng.uniform(2.0, 4.0, nb)
        n = 1.5 * d
        nx, ny, nz = shape
        pos = np.stack([rng.uniform(n, nx - 1 - n), rng.uniform(n, ny - 1 - n),
                        rng.uniform(n, 0.4 * nz)])
        cols.append(dict(shape=shape, omega=omega, bc=bc, pos=pos, d=d))
    return cols


def _params():
    return W.params(g=1e-4, sigma=W.sigma_for(1e-4, 3.0))


def _single(col, prec, steps):
    sim = S.Simulation(col["shape"], col["omega"], precision=prec, bc=col["bc"])
    sim.add_bubbles(col["pos"], col["d"], S.bubble_params(**_params()))
    sim.step(steps)
    out = sim.populations().double().cpu().numpy(), sim.bubbles.positions()
    sim.close()
    return out


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_columns_match_single_lattice_runs(prec):
    cols = _columns()
    batch = S.Batch(cols, S.bubble_params(**_params()), precision=prec)
    steps = 40
    batch.step(steps)
    pos = batch.bubbles.positions()
    for c, col in enumerate(cols):
        g_ref, pos_ref = _single(col, prec, steps)
        g = batch.populations(c).double().cpu().numpy()
        assert rel_l2(g, g_ref) <= TOL[prec], c
        b0, b1 = batch.bubble_range(c)
        assert np.abs(pos[:, b0:b1] - pos_ref).max() <= 1e-4
    batch.check()
    batch.close()


def _crowded_columns(seed=31, nb=6):
    """Columns whose bubbles sit close together (overlapping windows), one of each face set."""
    rng = np.random.default_rng(seed)
    specs = [((24, 30, 50), 0.9, (BB,) * 6), ((33, 33, 70), 1.5, (BB, BB, BB, BB, BB, FS)),
             ((20, 28, 44), 1.2, (PER, PER, PER, PER, BB, BB))]
    cols = []
    for shape, omega, bc in specs:
        nx, ny, nz = shape
        d = rng.uniform(2.0, 3.5, nb)
        pos = np.stack([rng.uniform(nx / 2 - 3, nx / 2 + 3, nb), rng.uniform(ny / 2 - 3, ny / 2 + 3, nb),
                        rng.uniform(6, 14, nb)])
        cols.append(dict(shape=shape, omega=omega, bc=bc, pos=pos, d=d))
    return cols


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_is_bitwise_identical_to_single_lattice_runs(prec):
    """Each cell sums its bubbles' forces in bubble order in the batch as on a single lattice, so a
    column of crowded bubbles reproduces its own single-lattice run bit for bit."""
    cols = _crowded_columns()
    print(f"[case] crowded batch {prec}", flush=True)
    batch = S.Batch(cols, S.bubble_params(**_params()), precision=prec)
    steps = 30
    batch.step(10)
    batch.run(steps - 10, graph_steps=10)
    pos = batch.bubbles.positions()
    for c, col in enumerate(cols):
        g_ref, pos_ref = _single(col, prec, steps)
        b0, b1 = batch.bubble_range(c)
        assert np.array_equal(batch.populations(c).double().cpu().numpy(), g_ref), c
        assert np.array_equal(pos[:, b0:b1], pos_ref), c
        assert np.abs(pos_ref[2] - col["pos"][2]).max() > 1e-3  # the bubbles moved
    batch.check()
    batch.close()


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_per_column_gravity_and_surface_tension(prec):
    """Columns carrying their own g and sigma (one physical setup at several grid spacings) step
    like single lattices run with those constants, bit for bit; a column without them takes the
    batch's."""
    cols = _crowded_columns()
    consts = [(3e-4, W.sigma_for(3e-4, 2.5)), (0.0, 0.0), (5e-5, W.sigma_for(5e-5, 3.5))]
    for col, (g, sigma) in zip(cols, consts):
        col.update(g=g, sigma=sigma)
    print(f"[case] per-column g, sigma batch {prec}", flush=True)
    batch = S.Batch(cols, S.bubble_params(**_params()), precision=prec)
    steps = 24
    batch.step(8)
    batch.run(steps - 8, graph_steps=8)
    pos = batch.bubbles.positions()
    for c, (col, (g, sigma)) in enumerate(zip(cols, consts)):
        p = _params()
        if g:
            p.update(g=g, sigma=sigma)
        sim = S.Simulation(col["shape"], col["omega"], precision=prec, bc=col["bc"])
        sim.add_bubbles(col["pos"], col["d"], S.bubble_params(**p))
        sim.step(steps)
        b0, b1 = batch.bubble_range(c)
        assert np.array_equal(batch.populations(c).double().cpu().numpy(),
                              sim.populations().double().cpu().numpy()), c
        assert np.array_equal(pos[:, b0:b1], sim.bubbles.positions()), c
        sim.close()
    # the columns with their own constants move otherwise than with the batch's
    for c in (0, 2):
        col = cols[c]
        sim = S.Simulation(col["shape"], col["omega"], precision=prec, bc=col["bc"])
        sim.add_bubbles(col["pos"], col["d"], S.bubble_params(**_params()))
        sim.step(steps)
        assert np.abs(pos[:, slice(*batch.bubble_range(c))] - sim.bubbles.positions()).max() > 1e-4
        sim.close()
    batch.check()
    batch.close()


@pytest.mark.gpu
def test_columns_without_bubbles_and_a_bubble_free_batch():
    """A column holding no bubble (an empty bubble range between two others) steps as a plain
    lattice; a batch with no bubble at all runs the liquid step alone."""
    cols = _crowded_columns(nb=3)
    cols[1] = dict(cols[1], pos=np.zeros((3, 0)), d=np.zeros(0))
    print("[case] batch with an empty middle column", flush=True)
    batch = S.Batch(cols, S.bubble_params(**_params()), precision="f64")
    assert batch.bubble_range(1) == (3, 3)
    batch.step(6)
    batch.run(10, graph_steps=10)
    pos = batch.bubbles.positions()
    for c, col in enumerate(cols):
        g_ref, pos_ref = _single(col, "f64", 16)
        b0, b1 = batch.bubble_range(c)
        assert np.array_equal(batch.populations(c).double().cpu().numpy(), g_ref), c
        assert np.array_equal(pos[:, b0:b1], pos_ref), c
    g1 = batch.populations(1).double().cpu().numpy()
    assert np.abs(g1).max() == 0.0  # no force ever reached the empty column: still at rest
    batch.check()
    batch.close()
    empty = [dict(col, pos=np.zeros((3, 0)), d=np.zeros(0)) for col in cols]
    batch = S.Batch(empty, S.bubble_params(**_params()), precision="f32")
    batch.run(8, graph_steps=4)
    sums, diverged = batch.sums()
    assert not diverged.any()
    assert np.allclose(sums[:, 0], [np.prod(c["shape"]) for c in empty], rtol=0, atol=1e-6)
    batch.check()
    batch.close()


@pytest.mark.gpu
def test_batched_sweep_rerun_is_bitwise_identical():
    """The 64-column sweep (1-8 bubbles per column, 50 M sites) run twice, per-step launches and
    persistent launches: same bits everywhere."""
    ws = W.batched()
    cols = [dict(shape=w.shape, omega=w.omega, bc=w.bc, pos=w.pos, d=w.d) for w in ws]
    print(f"[case] batched sweep rerun: {len(cols)} columns", flush=True)
    runs = []
    for persistent in (False, True):  # the second run as persistent launches
        b = S.Batch(cols, S.bubble_params(**ws[0].params), precision="f32")
        L.lbm_batch_set_persistent(b.handle, persistent)
        b.run(40, graph_steps=20)
        torch.cuda.synchronize()
        runs.append(b)
    a, b = runs
    assert np.array_equal(a.bubbles.positions(), b.bubbles.positions())
    for c in range(len(cols)):
        assert torch.equal(a.populations(c), b.populations(c)), c
    for r in runs:
        r.check()
        r.close()


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_persistent_launch_matches_per_step_launches(prec):
    """The persistent launch (phases of every step in one kernel, grid barriers between them), eager
    and captured in graphs, gives the per-step launches' results bit for bit."""
    cols = _crowded_columns(seed=41)
    print(f"[case] persistent batch {prec}", flush=True)
    out = []
    for persistent, graph in ((False, 0), (True, 0), (True, 6)):
        b = S.Batch(cols, S.bubble_params(**_params()), precision=prec)
        L.lbm_batch_set_persistent(b.handle, persistent)
        if graph:
            b.run(24, graph_steps=graph)
        else:
            b.step(24)
        b.check()
        if persistent:
            assert L.lbm_batch_get_persistent(b.handle)[1] > 0
        out.append(([b.populations(c).cpu().numpy() for c in range(len(cols))],
                    b.bubbles.positions(), b.bubbles.velocities()))
        b.close()
    for o in out[1:]:
        for a, r in zip(o[0], out[0][0]):
            assert np.array_equal(a, r)
        assert np.array_equal(o[1], out[0][1]) and np.array_equal(o[2], out[0][2])


@pytest.mark.gpu
def test_batch_columns_match_oracle():
    cols = _columns(seed=22, nb_max=2)[:3]
    batch = S.Batch(cols, S.bubble_params(**_params()), precision="f64")
    steps = 30
    batch.step(steps)
    pos = batch.bubbles.positions()
    P = O.bubble_params(**_params())
    for c, col in enumerate(cols):
        lat = O.Lattice(*col["shape"], col["omega"], col["bc"])
        bub = O.Bubbles(pos=col["pos"].copy(), d=col["d"].copy())
        O.run(lat, P, bub, steps)
        assert rel_l2(batch.populations(c).cpu().numpy(), lat.g) <= 1e-12
        b0, b1 = batch.bubble_range(c)
        assert np.abs(pos[:, b0:b1] - bub.pos).max() <= 1e-10
    batch.close()


@pytest.mark.gpu
def test_batch_item_sizes_are_bit_identical():
    """Item sizes and the occupancy cap are tuning knobs only."""
    cols = _crowded_columns(seed=23)
    ref = None
    for items, occ in ((256, 3), (1024, 0), (4096, 2), (256, 0)):
        batch = S.Batch(cols, S.bubble_params(**_params()), precision="f32")
        L.lbm_batch_set_items(batch.handle, [items] * len(cols))
        L.lbm_batch_set_step_occupancy(batch.handle, occ)
        assert L.lbm_batch_get_step_occupancy(batch.handle) == occ
        batch.step(12)
        out = [batch.populations(c).cpu().numpy() for c in range(len(cols))]
        batch.close()
        if ref is None:
            ref = out
        else:
            for a, b in zip(out, ref):
                assert np.array_equal(a, b)


@pytest.mark.gpu
def test_batch_graph_replays_match_eager_launches():
    """Each graph replay is checked against eager launches, with eager work and synchronisation
    between the replays."""
    cols = [dict(c, pos=c["pos"][:, :1], d=c["d"][:1]) for c in _columns(seed=24)]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        eager = S.Batch(cols, S.bubble_params(**_params()), precision="f64", stream=stream)
        graph = S.Batch(cols, S.bubble_params(**_params()), precision="f64", stream=stream)
        for rep in range(4):
            eager.step(6)
            graph.run(6, graph_steps=6)
            stream.synchronize()
            for c in range(len(cols)):
                a = graph.populations(c).cpu().numpy()
                b = eager.populations(c).cpu().numpy()
                assert np.array_equal(a, b), (rep, c)
            assert np.array_equal(graph.bubbles.positions(), eager.bubbles.positions())
            _ = torch.ones(1000, device="cuda", dtype=torch.float64).sum().item()  # eager work
        eager.close()
        graph.close()


@pytest.mark.gpu
def test_single_lattice_graph_run_matches_eager():
    w = W.Workload("graph", (40, 36, 64), 1.3, (BB,) * 6, np.array([[19.2], [17.7], [9.0]]),
                   np.array([3.0]), _params(), 0, "f64")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        sims = []
        for _ in range(2):
            sim = S.Simulation(w.shape, w.omega, precision="f64", stream=stream)
            sim.add_bubbles(w.pos, w.d, S.bubble_params(**w.params))
            sims.append(sim)
        for rep in range(3):
            sims[0].step(10)
            sims[1].run(10, graph_steps=4)  # two replays and two eager steps
            stream.synchronize()
            assert np.array_equal(sims[0].populations().cpu().numpy(),
                                  sims[1].populations().cpu().numpy()), rep
            assert np.array_equal(sims[0].bubbles.positions(), sims[1].bubbles.positions())
        for s in sims:
            s.close()


@pytest.mark.gpu
def test_batched_sweep_full_size():
    """The 64-column sweep (cross-sections 24-96, heights 2-4 times the width, omega from 0.6 to
    1.9, 1-8 bubbles each) in the benchmark's launch configuration (graph replays, at most 3
    workgroups per compute unit): every column reproduces its single-lattice run bit for bit
    (forces gathered in bubble order on both), and every column conserves mass."""
    ws = W.batched(steps=20)
    cols = [dict(shape=w.shape, omega=w.omega, bc=w.bc, pos=w.pos, d=w.d) for w in ws]
    print(f"[case] 64-column sweep, 20 steps in graphs of 10, every column against its own run",
          flush=True)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        batch = S.Batch(cols, S.bubble_params(**ws[0].params), precision="f32", stream=stream)
        L.lbm_batch_set_step_occupancy(batch.handle, 3)
        batch.run(20, graph_steps=10)
        stream.synchronize()
        batch.check()
        pos = batch.bubbles.positions()
        for c, w in enumerate(ws):
            sim = S.Simulation(w.shape, w.omega, precision="f32", bc=w.bc, stream=stream)
            sim.add_bubbles(w.pos, w.d, S.bubble_params(**w.params))
            sim.run(20, graph_steps=10)
            b0, b1 = batch.bubble_range(c)
            assert torch.equal(batch.populations(c), sim.populations()), c
            assert np.array_equal(pos[:, b0:b1], sim.bubbles.positions()), c
            sim.close()
            mass = batch.populations(c).double().sum().item()  # sum of g = sum rho - N
            assert abs(mass) < 1e-6 * w.cells
        batch.close()


@pytest.mark.gpu
def test_batch_sums_flag_only_the_diverged_column():
    """Three columns stepped together; in the middle one the host sets a non-finite bubble
    velocity, which makes that column's reaction force and then its populations non-finite (the
    state of a column that went unstable). The per-column sums flag it, and the other two columns'
    sums stay finite and equal those of their single-lattice runs."""
    shape = (20, 20, 40)
    cols = []
    for om, v in ((1.5, 0.0), (1.9999, float("nan")), (1.2, 0.0)):
        cols.append(dict(shape=shape, omega=om, bc=(0,) * 6, pos=np.array([[10.0], [10.0], [12.0]]),
                         d=np.array([3.0]), vel=np.array([[0.0], [0.0], [v]])))
    P = S.bubble_params(g=1e-4, sigma=1e-4)
    b = S.Batch(cols, P, precision="f64")
    b.step(60)
    sums, diverged = b.sums()
    print(f"sums {sums.tolist()}", flush=True)
    b.close()
    assert diverged.tolist() == [False, True, False]
    for k in (0, 2):
        c = cols[k]
        sim = S.Simulation(shape, c["omega"], precision="f64", bc=c["bc"])
        sim.add_bubbles(c["pos"], c["d"], P, vel=c["vel"])
        sim.step(60)
        _, _, s1 = sim.moments(fields=False)
        sim.close()
        assert np.allclose(sums[k], s1, rtol=1e-12, atol=1e-14)
