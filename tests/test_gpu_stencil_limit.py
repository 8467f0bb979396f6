"""Bubbles at the stencil limit: a kernel half-width of 1.5 d = 31.4 cells gives windows of 63 or
64 cells per axis wherever the bubble is (64 = LBM_MAX_STENCIL, the widest accepted), so the
weight arrays are used up to their last entry (cell lo - 1 + 65). The forward step against the
oracle in FP64, with the window inside the lattice and clipped by a wall (renormalised weights),
and the adjoint of the same configuration against central finite differences of the GPU forward."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as W
from gpu_common import gpu_sim, gpu_u, oracle_state, rel_l2
from paper_1710_07073_amd import adjoint as A

BB = O.BC_BOUNCE_BACK
SHAPE = (72, 72, 80)
N_HALF = 31.4
D = N_HALF / 1.5
PARAMS = W.params(g=1e-3, sigma=W.sigma_for(1e-3, D))


def _window(x, n):
    lo = np.floor(x - n - 0.5) + 1.0
    hi = np.ceil(x + n + 0.5) - 1.0
    return int(lo), int(hi)


@pytest.mark.gpu
@pytest.mark.parametrize("x0", [36.3, 10.3])
def test_widest_window_matches_oracle(x0):
    pos = np.array([[x0], [36.3], [30.3]])
    lo, hi = _window(x0, N_HALF)
    assert hi - lo + 1 == 64
    w = W.Workload(f"stencil_limit_x{x0}", SHAPE, 1.2, (BB,) * 6, pos, np.array([D]), PARAMS, 6, "f64")
    print(f"[case] {w.name}: window [{lo}, {hi}] along x", flush=True)
    sim = gpu_sim(w)
    lat, bub, P = oracle_state(w)
    for _ in range(w.steps):
        sim.step(1)
        O.method_step(lat, P, bub)
    sim.check()
    u, sums = gpu_u(sim)
    _, u_o, sums_o = lat.moments()
    err = rel_l2(u, u_o)
    dx = np.abs(sim.bubbles.positions() - bub.pos).max()
    print(f"rel-L2(u) = {err:.3e}, max |dx_b| = {dx:.3e}", flush=True)
    assert err <= 1e-12
    assert dx <= 1e-12
    assert np.abs(sim.bubbles.velocities() - bub.vel).max() <= 1e-12 * np.abs(bub.vel).max()
    sim.close()


@pytest.mark.gpu
@pytest.mark.parametrize("x0", [36.3, 10.3])
def test_widest_window_adjoint_matches_finite_differences(x0):
    pos = np.array([[x0], [36.3], [30.3]])
    steps, K, h = 24, 8, 1e-3
    print(f"[case] adjoint at the stencil limit, x0 = {x0}, {steps} steps", flush=True)
    prob = A.TrajectoryProblem(SHAPE, (BB,) * 6, pos, [D], PARAMS, steps, precision="f64",
                               checkpoint=K)
    target, sim, _ = prob.forward((1.15, 0.8, 1.5), checkpoints=False)
    sim.close()

    def loss(theta):
        traj, s, _ = prob.forward(theta, checkpoints=False)
        s.close()
        return float(((traj - target) ** 2).sum())

    th0 = np.array([1.0, 1.0, 1.4])
    theta = torch.tensor(th0, dtype=torch.float64, requires_grad=True)
    L0 = A.trajectory_loss(prob, theta, target)
    L0.backward()
    g = theta.grad.numpy()
    fd = np.zeros(3)
    for i in range(3):
        e = np.zeros(3)
        e[i] = h
        fd[i] = (loss(th0 + e) - loss(th0 - e)) / (2 * h)
    print(f"L = {L0.item():.6e}, adjoint {g}, FD {fd}", flush=True)
    scale = np.abs(fd).max()
    assert scale > 0.0
    assert np.allclose(g, fd, rtol=1e-4, atol=1e-5 * scale)
