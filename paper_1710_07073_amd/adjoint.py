"""Gradients of a bubble-trajectory loss with respect to (drag_scale, lift_scale, omega) through the
hand-written adjoint of the coupled step (lbm_adjoint_liquid, lbm_adjoint_bubbles in
include/lbm.h), exposed as a torch.autograd.Function.

The forward pass runs the column and records the bubble positions after every step, keeping a
checkpoint (population buffer, velocity field, bubble state) every `checkpoint` steps. The
backward pass walks the segments newest first: it restores the segment's checkpoint, re-runs the
segment forward while storing each step's inputs (population buffer, velocity field, force field,
bubble record), then applies the adjoint steps in reverse order. Every step of the method and of
its adjoint runs in the library's kernels; PyTorch holds the buffers.
"""
from __future__ import annotations

import ctypes as ct

import numpy as np
import torch

from . import lbm as L
from . import sim as S

_PRE = ("x", "y", "z", "ux", "uy", "uz", "ulx", "uly", "ulz")


def _p(t):
    return ct.c_void_p(t.data_ptr())


class TrajectoryProblem:
    """One column with bubbles and a trajectory loss to differentiate."""

    def __init__(self, shape, bc, pos, d, params, steps, precision="f32", checkpoint=100,
                 device="cuda", stream=None):
        self.shape = tuple(shape)
        self.bc = tuple(bc)
        self.pos = np.asarray(pos, np.float64).reshape(3, -1)
        self.d = np.asarray(d, np.float64).reshape(-1)
        self.nb = self.d.size
        self.params = dict(params)
        self.steps = int(steps)
        self.precision = precision
        self.K = int(checkpoint)
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        # when a list, backward appends a (start, end) event pair around every adjoint liquid step
        self.liquid_events = None

    # ---- forward ----
    def make_sim(self, theta):
        sD, sL, omega = (float(v) for v in theta)
        p = dict(self.params)
        p.update(drag_scale=sD, lift_scale=sL)
        sim = S.Simulation(self.shape, omega, precision=self.precision, bc=self.bc,
                           device=self.device, stream=self.stream)
        sim.add_bubbles(self.pos, self.d, S.bubble_params(**p))
        return sim

    @staticmethod
    def state_tensor(sim):
        ptr = L.lbm_state_buffer(sim.ctx)
        return sim.pops[0] if sim.pops[0].data_ptr() == ptr else sim.pops[1]

    def _save(self, sim):
        return dict(state=self.state_tensor(sim).clone(), vel=sim.vel.clone(),
                    bub={k: sim.bubbles.t[k].clone() for k in _PRE + ("state",)})

    def _restore(self, sim, ck):
        self.state_tensor(sim).copy_(ck["state"])
        sim.vel.copy_(ck["vel"])
        sim.force.zero_()
        for k, v in ck["bub"].items():
            sim.bubbles.t[k].copy_(v)

    def _positions(self, sim):
        t = sim.bubbles.t
        return torch.stack([t["x"], t["y"], t["z"]])

    def forward(self, theta, checkpoints=True):
        """Trajectory (steps, 3, nb) on the device, the simulation, and the checkpoints."""
        sim = self.make_sim(theta)
        traj = torch.empty((self.steps, 3, self.nb), dtype=torch.float64, device=self.device)
        ckpts = []
        for k in range(self.steps):
            if checkpoints and k % self.K == 0:
                ckpts.append(self._save(sim))
            sim.step(1)
            traj[k] = self._positions(sim)
        return traj, sim, ckpts

    # ---- backward ----
    def _record_pre(self, sim, rec):
        t = sim.bubbles.t
        for i, k in enumerate(_PRE):
            rec[:, i] = t[k]
        rec[:, 9] = t["state"].double()
        rec[:, 20] = t["d"]

    def _record_post(self, sim, rec):
        w = sim.bubbles.t["work"][: self.nb * L.LBM_BUBBLE_WORK].view(self.nb, L.LBM_BUBBLE_WORK)
        rec[:, 10:16] = w[:, 0:6]     # interpolated u_l and curl u_l
        rec[:, 16:19] = w[:, 9:12]    # reaction psi
        rec[:, 19] = w[:, 12]         # window valid

    def backward(self, theta, sim, ckpts, grad_traj):
        """dL/dtheta given dL/d(trajectory)."""
        omega = float(theta[2])
        nb, K = self.nb, self.K
        pops = sim.pops[0]
        lam = [torch.zeros_like(pops), torch.zeros_like(pops)]
        lam_u = torch.zeros_like(sim.vel)
        lam_f = torch.empty_like(sim.vel)
        lam_b = torch.zeros((nb, L.LBM_BUBBLE_ADJ), dtype=torch.float64, device=self.device)
        scr = torch.empty((nb, L.LBM_BUBBLE_WORK), dtype=torch.float64, device=self.device)
        grad = torch.zeros(4, dtype=torch.float64, device=self.device)
        H = torch.empty((K,) + tuple(pops.shape), dtype=pops.dtype, device=self.device)
        Up = torch.empty((K,) + tuple(sim.vel.shape), dtype=pops.dtype, device=self.device)
        Fk = torch.empty_like(Up)
        rec = torch.zeros((K, nb, L.LBM_BUBBLE_RECORD), dtype=torch.float64, device=self.device)
        gt = grad_traj.to(self.device, torch.float64)
        cur = 0
        bub = sim.bubbles
        for s in reversed(range(len(ckpts))):
            k0 = s * K
            k1 = min(k0 + K, self.steps)
            self._restore(sim, ckpts[s])
            for k in range(k0, k1):
                i = k - k0
                H[i].copy_(self.state_tensor(sim))
                Up[i].copy_(sim.vel)
                self._record_pre(sim, rec[i])
                L.bubbles_step(sim.ctx, sim.params, bub.soa, nb)
                self._record_post(sim, rec[i])
                Fk[i].copy_(sim.force)
                L.lbm_step(sim.ctx, 1)
            for k in reversed(range(k0, k1)):
                i = k - k0
                lam_b[:, 0:3] += gt[k].t()
                ev = None
                if self.liquid_events is not None:
                    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                    ev[0].record(self.stream)
                L.lbm_adjoint_liquid(sim.ctx, _p(H[i]), _p(Fk[i]), _p(lam[cur]), _p(lam[1 - cur]),
                                     _p(lam_u), _p(lam_f), _p(grad))
                if ev is not None:
                    ev[1].record(self.stream)
                    self.liquid_events.append(ev)
                cur = 1 - cur
                L.lbm_adjoint_bubbles(sim.ctx, sim.params, _p(rec[i]), _p(Up[i]), _p(lam_f),
                                      _p(lam_u), _p(lam_b), _p(scr), nb, _p(grad))
        g = grad.cpu().numpy()
        # omega enters the collision directly and the bubble closures through nu = (1/omega - 1/2)/3
        return np.array([g[1], g[2], g[0] + g[3] * (-1.0 / (3.0 * omega * omega))])


class BubbleTrajectory(torch.autograd.Function):
    """theta (3, float64: drag_scale, lift_scale, omega) -> bubble positions after every step,
    (steps, 3, nb). Backward runs the checkpointed adjoint."""

    @staticmethod
    def forward(ctx, theta, problem):
        th = theta.detach().cpu().double().numpy().copy()
        traj, sim, ckpts = problem.forward(th)
        ctx.problem = problem
        ctx.state = (th, sim, ckpts)
        ctx.theta_device = theta.device
        return traj

    @staticmethod
    def backward(ctx, grad_traj):
        th, sim, ckpts = ctx.state
        g = ctx.problem.backward(th, sim, ckpts, grad_traj.contiguous())
        sim.close()
        ctx.state = None
        return torch.tensor(g, dtype=torch.float64, device=ctx.theta_device), None


def trajectory_loss(problem, theta, target):
    """Sum over steps and bubbles of |x - x_target|^2 (the adjoint workload's loss)."""
    traj = BubbleTrajectory.apply(theta, problem)
    return ((traj - target) ** 2).sum()
