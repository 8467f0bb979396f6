"""Gradient of the bubble-trajectory loss with respect to (drag_scale, lift_scale, omega) through
the hand-written adjoint (checkpointed, torch.autograd.Function), against central finite
differences of the GPU forward and of the FP64 oracle (h = 1e-3)."""
import json
import os

import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from paper_1710_07073_amd import adjoint as A

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "adjoint_64x64x192_oracle_gradient.json")
H = 1e-3


def _small(steps=150):
    pos = np.array([[10.0, 14.0], [11.0, 12.5], [9.0, 14.0]])
    return W.Workload("adjoint_small_24x24x48_2b", (24, 24, 48), 1.4, (0,) * 6, pos,
                      np.array([3.0, 2.5]), W.params(g=1e-4, sigma=1e-4), steps, "f64",
                      meta=dict(target=(1.15, 0.8, 1.5), theta0=(1.0, 1.0, 1.4)))


def _problem(w, precision, K):
    return A.TrajectoryProblem(w.shape, w.bc, w.pos, w.d, w.params, w.steps, precision=precision,
                               checkpoint=K)


def _gpu_loss(problem, theta, target):
    traj, sim, _ = problem.forward(theta, checkpoints=False)
    sim.close()
    return float(((traj - target) ** 2).sum())


def _oracle_traj(w, theta):
    sD, sL, om = theta
    lat = O.Lattice(*w.shape, om, w.bc)
    bub = O.Bubbles(pos=w.pos.copy(), d=w.d.copy())
    p = dict(w.params)
    p.update(drag_scale=sD, lift_scale=sL)
    return O.run(lat, O.bubble_params(**p), bub, w.steps, record=True)


def _adjoint_grad(problem, theta0, target):
    theta = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
    loss = A.trajectory_loss(problem, theta, target)
    loss.backward()
    return loss.item(), theta.grad.numpy()


@pytest.mark.gpu
def test_adjoint_matches_finite_differences_fp64():
    w = _small()
    prob = _problem(w, "f64", K=50)
    target, sim, _ = prob.forward(w.meta["target"], checkpoints=False)
    sim.close()
    L0, g = _adjoint_grad(prob, w.meta["theta0"], target)
    fd = np.zeros(3)
    for i in range(3):
        e = np.zeros(3)
        e[i] = H
        th = np.array(w.meta["theta0"])
        fd[i] = (_gpu_loss(prob, th + e, target) - _gpu_loss(prob, th - e, target)) / (2 * H)
    print(f"L = {L0:.6e}, adjoint {g}, FD {fd}", flush=True)
    scale = np.abs(fd).max()
    assert np.allclose(g, fd, rtol=1e-4, atol=1e-5 * scale)


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_adjoint_matches_oracle_gradient(precision):
    w = _small()
    th0 = np.array(w.meta["theta0"])
    target_o = _oracle_traj(w, w.meta["target"])
    lo = lambda th: float(np.sum((_oracle_traj(w, th) - target_o) ** 2))
    fd = np.zeros(3)
    for i in range(3):
        e = np.zeros(3)
        e[i] = H
        fd[i] = (lo(th0 + e) - lo(th0 - e)) / (2 * H)
    prob = _problem(w, precision, K=40)
    target = torch.tensor(target_o, device="cuda")
    L0, g = _adjoint_grad(prob, w.meta["theta0"], target)
    print(f"{precision}: L = {L0:.6e}, adjoint {g}, oracle FD {fd}", flush=True)
    scale = np.abs(fd).max()
    tol = 1e-4 if precision == "f64" else 2e-2
    assert np.allclose(g, fd, rtol=tol, atol=tol * scale)


def _shear(steps=150, u0=0.08):
    """Two bubbles in a decaying shear flow u_x = u0 sin(pi (z + 1/2) / n_z) between bounce-back
    plates, periodic sides, omega 1.9: the vorticity at the bubbles is large enough for the lift
    force to move them measurably (dL/d lift_scale is about 2 % of dL/d drag_scale), so each
    gradient component can be checked on its own. Returns the workload, the initial post-collision
    populations (the equilibrium of the flow, from the oracle's eq. (6)) and velocity field."""
    nx, ny, nz = 24, 24, 48
    pos = np.array([[8.0, 15.0], [10.0, 13.0], [7.0, 10.0]])
    w = W.Workload("adjoint_shear_24x24x48_2b", (nx, ny, nz), 1.9, (W.PER,) * 4 + (W.BB,) * 2, pos,
                   np.array([3.0, 3.0]), W.params(g=1e-4, sigma=1e-4), steps, "f64",
                   meta=dict(target=(1.1, 0.6, 1.88), theta0=(1.0, 1.0, 1.9)))
    ux = u0 * np.sin(np.pi * (np.arange(nz) + 0.5) / nz)
    _, wq, _ = O.lattice()
    R = np.empty((19, nz, ny, nx))
    for k in range(nz):
        R[:, k] = (O.equilibrium(1.0, [ux[k], 0.0, 0.0]) - wq)[:, None, None]
    U = np.zeros((3, nz, ny, nx))
    U[0] = ux[:, None, None]
    return w, R, U


def _oracle_traj_from(w, theta, R, U):
    sD, sL, om = theta
    lat = O.Lattice(*w.shape, om, w.bc)
    lat.g = O.stream(R, w.bc)  # the pre-collision state the post-collision buffer R streams into
    lat.U = U.copy()
    bub = O.Bubbles(pos=w.pos.copy(), d=w.d.copy())
    p = dict(w.params)
    p.update(drag_scale=sD, lift_scale=sL)
    return O.run(lat, O.bubble_params(**p), bub, w.steps, record=True)


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_adjoint_in_shear_flow_each_component_matches_oracle(precision):
    """Every component of the gradient, lift included, against the oracle's central differences
    (h = 1e-4: the omega component's O(h^2) error is 3.5e-4 relative at h = 1e-3) with a relative
    bound of its own: 1e-4 in FP64, 2e-3 in FP32."""
    w, R, U = _shear()
    print(f"[case] {w.name} {precision}", flush=True)
    h = 1e-4
    th0 = np.array(w.meta["theta0"])
    target_o = _oracle_traj_from(w, w.meta["target"], R, U)
    lo = lambda th: float(np.sum((_oracle_traj_from(w, th, R, U) - target_o) ** 2))
    fd = np.zeros(3)
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        fd[i] = (lo(th0 + e) - lo(th0 - e)) / (2 * h)
    prob = A.TrajectoryProblem(w.shape, w.bc, w.pos, w.d, w.params, w.steps, precision=precision,
                               checkpoint=40, init_state=R, init_vel=U)
    L0, g = _adjoint_grad(prob, th0, torch.tensor(target_o, device="cuda"))
    rel = np.abs(g - fd) / np.abs(fd)
    print(f"{precision}: L = {L0:.6e} (oracle {lo(th0):.6e}), adjoint {g}, oracle FD {fd}, "
          f"relative error per component {rel}", flush=True)
    assert abs(fd[1]) > 1e-3 * np.abs(fd).max()  # lift carries weight here
    assert np.all(rel <= (1e-4 if precision == "f64" else 2e-3)), rel


@pytest.mark.gpu
def test_adjoint_checkpoint_interval_does_not_change_the_gradient():
    w = _small(steps=90)
    target, sim, _ = _problem(w, "f64", 30).forward(w.meta["target"], checkpoints=False)
    sim.close()
    grads = [_adjoint_grad(_problem(w, "f64", K), w.meta["theta0"], target)[1] for K in (90, 30, 7)]
    assert np.allclose(grads[0], grads[1], rtol=1e-11) and np.allclose(grads[0], grads[2], rtol=1e-11)


@pytest.mark.gpu
@pytest.mark.skipif(not os.path.exists(GOLDEN), reason="oracle gradient file not generated")
def test_adjoint_full_column_against_oracle_gradient():
    """64 x 64 x 192 FP32 column, 4 bubbles, 2000 steps, checkpoints every 100 steps."""
    ref = json.load(open(GOLDEN))
    w = W.adjoint(steps=ref["steps"])
    prob = _problem(w, "f32", K=w.meta["checkpoint"])
    target, sim, _ = prob.forward(w.meta["target"], checkpoints=False)
    sim.close()
    L0, g = _adjoint_grad(prob, w.meta["theta0"], target)
    fd = np.array(ref["gradient"])
    print(f"L = {L0:.6e} (oracle {ref['loss']:.6e}), adjoint {g}, oracle FD {fd}", flush=True)
    assert L0 == pytest.approx(ref["loss"], rel=1e-2)
    scale = np.abs(fd).max()
    # drag and omega components to 2 %, the lift component (orders of magnitude smaller at these
    # Reynolds numbers) to 2 % of the largest component
    assert np.allclose(g, fd, rtol=2e-2, atol=2e-2 * scale)


@pytest.mark.gpu
def test_timed_segment_gives_the_same_gradient():
    """The benchmark times the adjoint liquid launches of the first segment the backward pass
    processes (a partial one here: 130 steps, K = 20) with events: one event pair per step of
    that segment, and the same gradient up to the order of the atomic additions into it."""
    w = _small(steps=130)
    th0 = w.meta["theta0"]
    prob = _problem(w, "f32", K=20)
    target, sim, _ = prob.forward(w.meta["target"], checkpoints=False)
    sim.close()
    L0, g0 = _adjoint_grad(prob, th0, target)
    prob.liquid_events = []
    L1, g1 = _adjoint_grad(prob, th0, target)
    print(f"untimed {g0}, timed {g1}", flush=True)
    assert L0 == L1
    assert len(prob.liquid_events) == 10
    assert all(a.elapsed_time(b) > 0.0 for a, b in prob.liquid_events)
    assert np.allclose(g1, g0, rtol=1e-12, atol=1e-13 * np.abs(g0).max())


def _recorded_step(w, armed, warm=6):
    """A simulation after warm steps, then one bubble half with its step record (armed: filled by
    the bubble update; else the two stages of lbm_bubble_record) and the velocity field it read."""
    from paper_1710_07073_amd import lbm as L
    from gpu_common import gpu_sim
    sim = gpu_sim(w)
    sim.step(warm)
    nb = sim.bubbles.nb
    rec = torch.full((nb, L.LBM_BUBBLE_RECORD), -7.0, dtype=torch.float64, device="cuda")
    vel_prev = sim.vel.clone()
    ub_before = sim.bubbles.velocities()
    p = ctypes_ptr(rec)
    if armed:
        L.lbm_record_next_bubble_half(sim.ctx, p)
        L.bubbles_step(sim.ctx, sim.params, sim.bubbles.soa, nb)
    else:
        L.lbm_bubble_record(sim.ctx, sim.bubbles.soa, nb, 0, p)
        L.bubbles_step(sim.ctx, sim.params, sim.bubbles.soa, nb)
        L.lbm_bubble_record(sim.ctx, sim.bubbles.soa, nb, 1, p)
    L.lbm_step(sim.ctx, 1)
    torch.cuda.synchronize()
    return sim, rec, vel_prev, ub_before


def ctypes_ptr(t):
    import ctypes as ct
    return ct.c_void_p(t.data_ptr())


@pytest.mark.gpu
@pytest.mark.parametrize("nb", [3, 300, "wall"])
def test_armed_record_equals_staged_record(nb):
    """The step record the bubble update fills when armed (3 bubbles: inside k_interp; 300: in
    k_ode) holds the values of the two lbm_bubble_record stages bit for bit, plus sub-step
    velocities that start at the velocity before the step and end at the velocity after it; the
    bubble half's adjoint gives the same result from either record (the staged one makes the
    kernel run the sub-steps again)."""
    from paper_1710_07073_amd import lbm as L
    rng = np.random.default_rng(21)
    shape = (48, 48, 64)
    wall = nb == "wall"  # one bubble thrown at the x = 0 wall: its x velocity is clamped
    nb = 1 if wall else nb
    d = rng.uniform(2.0, 3.0, nb)
    pos = np.stack([rng.uniform(5.0, 42.0, nb), rng.uniform(5.0, 42.0, nb), rng.uniform(5.0, 30.0, nb)])
    vel = None
    if wall:
        pos = np.array([[0.05], [24.0], [20.0]])
        vel = np.array([[-1.0], [0.0], [0.0]])
    w = W.Workload(f"record_{nb}b{'_wall' if wall else ''}", shape, 1.3, (0,) * 6, pos, d,
                   W.params(g=1e-4, sigma=1e-4), 0, "f64", vel=vel)
    print(f"[case] {w.name}", flush=True)
    warm = 0 if wall else 6
    sa, ra, vel, ub0 = _recorded_step(w, True, warm)
    sb, rb, _, _ = _recorded_step(w, False, warm)
    ra_h, rb_h = ra.cpu().numpy(), rb.cpu().numpy()
    assert np.array_equal(ra_h[:, :21], rb_h[:, :21])
    assert np.all(ra_h[:, 21] == 1.0) and np.all(rb_h[:, 21] == 0.0)
    n_sub = W.params()["n_sub"]
    ubs = ra_h[:, 24:24 + 3 * (n_sub + 1)].reshape(nb, n_sub + 1, 3)
    assert np.array_equal(ubs[:, 0, :], ub0.T)
    assert np.array_equal(ubs[:, n_sub, :], sa.bubbles.velocities().T)
    if wall:  # the x component (a = 0) clamped in some sub-step k: bit 3 k
        word = int(ra_h[0, 123]) | (int(ra_h[0, 124]) << 32) | (int(ra_h[0, 125]) << 64)
        assert any((word >> (3 * k)) & 1 for k in range(n_sub))
    else:
        assert np.array_equal(ra_h[:, 123:126], np.zeros((nb, 3)))  # no wall contact
    # the bubble half's adjoint from either record
    outs = []
    for sim, rec in ((sa, ra), (sb, rb)):
        g = torch.Generator(device="cuda").manual_seed(5)
        lam_f = torch.randn(sim.vel.shape, generator=g, device="cuda", dtype=sim.vel.dtype) * 1e-3
        lam_u = torch.zeros_like(sim.vel)
        lam = torch.randn((nb, L.LBM_BUBBLE_ADJ), generator=g, device="cuda", dtype=torch.float64)
        grad = torch.zeros(4, dtype=torch.float64, device="cuda")
        L.lbm_adjoint_bubbles(sim.ctx, sim.params, ctypes_ptr(rec), ctypes_ptr(vel), ctypes_ptr(lam_f),
                              ctypes_ptr(lam_u), ctypes_ptr(lam), None, nb, ctypes_ptr(grad))
        torch.cuda.synchronize()
        outs.append((lam.cpu().numpy(), lam_u.cpu().numpy(), grad.cpu().numpy()))
        sim.check()
        sim.close()
    for a, b in zip(outs[0], outs[1]):
        scale = np.abs(b).max()
        assert np.allclose(a, b, rtol=1e-11, atol=1e-12 * scale)


@pytest.mark.gpu
def test_armed_record_blocks_lbm_run_until_disarmed():
    from paper_1710_07073_amd import lbm as L
    from gpu_common import gpu_sim
    w = W.Workload("arm_run", (24, 24, 32), 1.3, (0,) * 6, np.array([[12.0], [12.0], [8.0]]),
                   np.array([3.0]), W.params(g=1e-4, sigma=1e-4), 0, "f64")
    print(f"[case] {w.name}", flush=True)
    sim = gpu_sim(w)
    rec = torch.zeros((1, L.LBM_BUBBLE_RECORD), dtype=torch.float64, device="cuda")
    L.lbm_record_next_bubble_half(sim.ctx, ctypes_ptr(rec))
    with pytest.raises(L.LbmError) as e:
        sim.run(2)
    assert e.value.code == L.LBM_EINVAL
    L.lbm_record_next_bubble_half(sim.ctx, None)
    sim.run(2)
    sim.check()
    assert torch.count_nonzero(rec).item() == 0  # disarmed before any bubble half ran
    sim.close()


@pytest.mark.gpu
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_tile_mask_gives_the_same_gradient(precision):
    """lbm_adjoint_liquid_tiles with each step's tile mask (lbm_step_tiles) reads the force and the
    velocity adjoint only in the tiles the step flagged and takes them as zero elsewhere: the same
    gradient as lbm_adjoint_liquid reading every cell, up to the order of the atomic additions into
    dL/domega."""
    w = _small(steps=120)
    th0 = w.meta["theta0"]
    target, sim, _ = _problem(w, precision, 40).forward(w.meta["target"], checkpoints=False)
    sim.close()
    grads = []
    for use in (False, True):
        prob = _problem(w, precision, 40)
        prob.use_tiles = use
        grads.append(_adjoint_grad(prob, th0, target)[1])
    print(f"every cell {grads[0]}, tile mask {grads[1]}", flush=True)
    assert np.allclose(grads[1], grads[0], rtol=1e-12, atol=1e-13 * np.abs(grads[0]).max())


@pytest.mark.gpu
def test_step_tiles_flags_the_bubble_windows():
    """The mask lbm_step_tiles copies after a bubble half flags the tiles of each bubble's force
    window and nothing far from the bubbles."""
    from paper_1710_07073_amd import lbm as L
    from paper_1710_07073_amd import sim as S
    w = _small()
    sim = S.Simulation(w.shape, w.omega, precision="f64", bc=w.bc)
    sim.add_bubbles(w.pos, w.d, S.bubble_params(**w.params))
    n = L.lbm_step_tiles(sim.ctx)
    nx, ny, nz = w.shape
    assert n == -(-nx // 8) * -(-ny // 8) * -(-nz // 8)
    mask = torch.zeros(n, dtype=torch.uint8, device="cuda")
    L.bubbles_step(sim.ctx, sim.params, sim.bubbles.soa, sim.bubbles.nb)
    L.lbm_step_tiles(sim.ctx, A._p(mask))
    L.lbm_step(sim.ctx, 1)
    m = mask.cpu().numpy().reshape(-(-nz // 8), -(-ny // 8), -(-nx // 8))
    for b in range(w.pos.shape[1]):
        x, y, z = (int(v) // 8 for v in w.pos[:, b])
        assert m[z, y, x] != 0
    assert m[-1].sum() == 0  # the top tiles are far from every bubble
    sim.close()
