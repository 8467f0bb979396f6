"""GPU parity of the fused liquid step (Sec. 2.2, eq. (13)-(16); Sec. 3.3 face conditions) against
the CPU oracle, through the C ABI: random non-equilibrium states under a fixed force field, ragged
shapes that do not fill the launch tiles, every face condition, both precisions."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from paper_1710_07073_amd import lbm as L
from gpu_common import rel_l2, set_post_collision_state, gpu_u
from paper_1710_07073_amd import sim as S

BB, FS, PER = O.BC_BOUNCE_BACK, O.BC_FREE_SLIP, O.BC_PERIODIC
FLAGS = L.LBM_FLAG_STATIC_FORCE | L.LBM_FLAG_WRITE_U_ALL

# FP64 path: rounding-order differences only. FP32 path: storage and collision in float, the
# tolerance of the method's stated FP32 target.
TOL = {"f64": 1e-12, "f32": 2e-5}

CASES = [
    ((37, 23, 19), (BB,) * 6),
    ((64, 8, 9), (BB, BB, BB, BB, BB, FS)),
    ((33, 20, 17), (PER, PER, BB, BB, FS, FS)),
    ((16, 16, 16), (PER,) * 6),
    ((1, 12, 10), (PER, PER, BB, FS, BB, BB)),
    ((130, 3, 5), (FS,) * 6),
    ((256, 4, 3), (BB, BB, PER, PER, BB, FS)),
]


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape,bc", CASES)
def test_liquid_steps_match_oracle(prec, shape, bc):
    print(f"[case] liquid {prec} {shape} bc={bc}", flush=True)
    R = W.random_populations(shape, 1e-3, seed=3)
    F = W.random_field(shape, 2e-5, seed=4)
    if prec == "f32":
        R = R.astype(np.float32).astype(np.float64)
        F = F.astype(np.float32).astype(np.float64)
    omega = 1.3
    sim = S.Simulation(shape, omega, precision=prec, bc=bc, flags=FLAGS)
    set_post_collision_state(sim, R)
    sim.force.copy_(torch.from_numpy(F).to(sim.dtype))
    lat = O.Lattice(*shape, omega, bc, g=O.stream(R, bc))
    steps = 12
    for _ in range(steps):
        sim.liquid_steps(1)
        lat.step(F)
    gpu = sim.populations().double().cpu().numpy()
    assert rel_l2(gpu, lat.g) <= TOL[prec]
    U = sim.vel.double().cpu().numpy()
    assert rel_l2(U, lat.U) <= TOL[prec]
    u, sums = gpu_u(sim)
    _, u_o, sums_o = lat.moments()
    assert rel_l2(u, u_o) <= TOL[prec]
    assert abs(sums[0] - sums_o[0]) <= 1e-9 * sums_o[0]
    # the fixed force field is still there (static force is never cleared)
    assert np.array_equal(sim.force.double().cpu().numpy(), F)
    sim.close()


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_rest_state_stays_at_rest(prec):
    sim = S.Simulation((40, 24, 18), 1.7, precision=prec)
    sim.liquid_steps(25)
    g = sim.populations()
    assert torch.count_nonzero(g).item() == 0
    _, _, sums = sim.moments()
    assert sums == [40 * 24 * 18, 0.0, 0.0, 0.0]
    sim.close()


@pytest.mark.gpu
def test_periodic_momentum_balance_on_gpu():
    """Fully periodic FP64 box: total momentum grows by exactly the total force per step."""
    shape = (24, 20, 18)
    R = W.random_populations(shape, 1e-3, seed=5)
    F = W.random_field(shape, 1e-5, seed=6)
    sim = S.Simulation(shape, 1.1, precision="f64", bc=(PER,) * 6, flags=FLAGS)
    set_post_collision_state(sim, R)
    sim.force.copy_(torch.from_numpy(F))
    _, _, s0 = sim.moments(fields=False)
    for k in range(1, 6):
        sim.liquid_steps(1)
        _, _, s1 = sim.moments(fields=False)
        assert np.allclose(np.array(s1[1:]) - np.array(s0[1:]), F.sum(axis=(1, 2, 3)), rtol=0,
                           atol=1e-15)
        assert abs(s1[0] - s0[0]) < 1e-10
        s0 = s1
    sim.close()


@pytest.mark.gpu
def test_poiseuille_on_gpu():
    """Body-force channel between bounce-back walls, FP64: the closed form with the half-way
    bounce-back slip (the same closed form that pins the oracle)."""
    N, Fz, omega = 12, 1e-6, 1.0
    shape = (N, 2, 2)
    sim = S.Simulation(shape, omega, precision="f64", bc=(BB, BB, PER, PER, PER, PER), flags=FLAGS)
    F = np.zeros((3, 2, 2, N))
    F[2] = Fz
    sim.force.copy_(torch.from_numpy(F))
    sim.liquid_steps(8000)
    tau = 1 / omega
    nu = (2 * tau - 1) / 6
    x = np.arange(N)
    ex = Fz / (2 * nu) * (x + 0.5) * (N - 0.5 - x) + Fz * ((2 * tau - 1) ** 2 - 0.75) / (2 * tau - 1)
    U = sim.vel.cpu().numpy()
    assert np.max(np.abs(U[2, 1, 1] - ex)) / ex.max() < 1e-12
    sim.close()


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("shape,bc", [
    ((128, 12, 10), (BB,) * 6),
    ((36, 10, 9), (BB, BB, BB, BB, BB, FS)),
    ((30, 12, 10), (FS, BB, FS, BB, BB, FS)),  # free-slip faces meeting at edges
    ((24, 8, 9), (FS,) * 6),
    ((40, 9, 11), (PER, PER, PER, PER, FS, FS)),
    ((64, 8, 8), (PER,) * 6),
    ((8, 6, 7), (BB, BB, PER, PER, BB, BB)),
])
def test_every_launch_shape_gives_identical_results(prec, shape, bc):
    """The launch shape (cells per thread, workgroup width) and the occupancy cap are tuning knobs
    only: every combination the autotuner may pick reproduces the reference launch bit for bit
    (with walls only, one cell per thread runs the wall fast path, wider launches the general
    kernel)."""
    from paper_1710_07073_amd import autotune
    R = W.random_populations(shape, 1e-3, seed=8)
    F = W.random_field(shape, 2e-5, seed=9)
    ref = None
    for vec, bx, occ in [(v, b, o) for v, b in autotune.candidates(shape[0]) for o in (0, 3, 5)]:
        sim = S.Simulation(shape, 1.45, precision=prec, bc=bc, flags=FLAGS)
        # the default cap: 5 workgroups per compute unit in FP32, 3 in FP64
        assert L.lbm_get_step_occupancy(sim.ctx) == (5 if prec == "f32" else 3)
        L.lbm_set_launch(sim.ctx, vec, bx)
        L.lbm_set_step_occupancy(sim.ctx, occ)
        set_post_collision_state(sim, R)
        sim.force.copy_(torch.from_numpy(F).to(sim.dtype))
        sim.liquid_steps(7)
        out = (sim.populations().cpu().numpy(), sim.vel.cpu().numpy())
        sim.close()
        if ref is None:
            ref = out
            lat = O.Lattice(*shape, 1.45, bc, g=O.stream(R.astype(np.float32).astype(np.float64)
                                                         if prec == "f32" else R, bc))
            Fo = F.astype(np.float32).astype(np.float64) if prec == "f32" else F
            for _ in range(7):
                lat.step(Fo)
            assert rel_l2(out[0], lat.g) <= TOL[prec]
        else:
            assert np.array_equal(out[0], ref[0]), (vec, bx, occ)
            assert np.array_equal(out[1], ref[1]), (vec, bx, occ)


@pytest.mark.gpu
@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("shape,bc", [
    ((37, 23, 19), (BB,) * 6),
    ((33, 20, 17), (PER, PER, BB, BB, FS, FS)),
    ((16, 16, 16), (PER,) * 6),
    ((130, 3, 5), (FS,) * 6),
])
def test_population_layouts_give_identical_results(prec, shape, bc):
    """Plane-blocked and plain structure-of-arrays buffers hold the same numbers in another
    order: liquid steps with a force field, then coupled steps with bubbles, bit for bit."""
    R = W.random_populations(shape, 1e-3, seed=11)
    F = W.random_field(shape, 2e-5, seed=12)
    outs = []
    for flags in (FLAGS, FLAGS | L.LBM_FLAG_PLAIN_SOA):
        print(f"layout flags={flags} shape={shape} bc={bc} {prec}", flush=True)
        sim = S.Simulation(shape, 1.3, precision=prec, bc=bc, flags=flags)
        set_post_collision_state(sim, R)
        sim.force.copy_(torch.from_numpy(F).to(sim.dtype))
        sim.liquid_steps(5)
        outs.append((sim.populations().cpu().numpy(), sim.vel.cpu().numpy()))
        sim.close()
    assert np.array_equal(outs[0][0], outs[1][0]) and np.array_equal(outs[0][1], outs[1][1])
    nx, ny, nz = shape
    pos = np.array([[nx / 2, nx / 3], [ny / 2, ny / 2 + 0.3], [nz / 3, nz / 2]])
    res = []
    for flags in (0, L.LBM_FLAG_PLAIN_SOA):
        sim = S.Simulation(shape, 1.3, precision=prec, bc=bc, flags=flags)
        sim.add_bubbles(pos, [2.5, 3.0], S.bubble_params(g=1e-4, sigma=1e-4))
        sim.step(12)
        res.append((sim.populations().cpu().numpy(), sim.bubbles.positions()))
        sim.check()
        sim.close()
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
