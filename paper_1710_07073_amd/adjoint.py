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
                 device="cuda", stream=None, init_state=None, init_vel=None):
        """init_state (19, nz, ny, nx), init_vel (3, nz, ny, nx): optional initial liquid, the
        post-collision shifted populations awaiting streaming and the velocity field the first bubble
        half interpolates (default: liquid at rest). The gradient does not flow into them."""
        self.init_state = None if init_state is None else np.asarray(init_state, np.float64)
        self.init_vel = None if init_vel is None else np.asarray(init_vel, np.float64)
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
        # when a list, backward appends a (start, end) event pair around the adjoint liquid kernel
        # of every step of the first segment it processes (the last in time)
        self.liquid_events = None
        # pass each step's tile mask to the adjoint liquid step (False: every cell reads the force
        # and the velocity adjoint; the gradient is the same)
        self.use_tiles = True

    # ---- forward ----
    def make_sim(self, theta):
        sD, sL, omega = (float(v) for v in theta)
        p = dict(self.params)
        p.update(drag_scale=sD, lift_scale=sL)
        sim = S.Simulation(self.shape, omega, precision=self.precision, bc=self.bc,
                           device=self.device, stream=self.stream)
        sim.add_bubbles(self.pos, self.d, S.bubble_params(**p))
        if self.init_state is not None:
            st = torch.from_numpy(self.init_state).to(self.device, sim.dtype)
            if not (sim.flags & L.LBM_FLAG_PLAIN_SOA):
                st = st.permute(1, 0, 2, 3)  # plane-blocked buffer (nz, 19, ny, nx)
            self.state_tensor(sim).copy_(st)
        if self.init_vel is not None:
            sim.vel.copy_(torch.from_numpy(self.init_vel).to(self.device, sim.dtype))
        return sim

    @staticmethod
    def state_tensor(sim):
        ptr = L.lbm_state_buffer(sim.ctx)
        return sim.pops[0] if sim.pops[0].data_ptr() == ptr else sim.pops[1]

    def _save(self, sim):
        return dict(state=self.state_tensor(sim).clone(), vel=sim.vel.clone(),
                    bub={k: sim.bubbles.t[k].clone() for k in _PRE + ("state",)})

    def forward(self, theta, checkpoints=True):
        """Trajectory (steps, 3, nb) on the device, the simulation, and the checkpoints. The steps
        of each checkpoint segment run as one library call (lbm_run, replaying one HIP graph of a
        whole segment when the segment length is even); the bubble update writes the positions
        after every step into the trajectory itself (lbm_record_positions), at the row a device
        counter holds, so the replays fill successive rows."""
        caller = torch.cuda.current_stream(self.device)
        sim = self.make_sim(theta)
        traj = torch.empty((self.steps, 3, self.nb), dtype=torch.float64, device=self.device)
        ckpts = []
        self.stream.wait_stream(caller)
        with torch.cuda.stream(self.stream):
            L.lbm_record_positions(sim.ctx, _p(traj), self.steps)
            bub = sim.bubbles
            for k0 in range(0, self.steps, self.K):
                if checkpoints:
                    ckpts.append(self._save(sim))
                L.lbm_run(sim.ctx, sim.params, bub.soa, bub.nb, min(self.K, self.steps - k0),
                          self.K if self.K % 2 == 0 else 0)
            L.lbm_record_positions(sim.ctx, None, 0)
        caller.wait_stream(self.stream)
        return traj, sim, ckpts

    # ---- backward ----
    def backward(self, theta, sim, ckpts, grad_traj):
        """dL/dtheta given dL/d(trajectory)."""
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        with torch.cuda.stream(self.stream):
            return self._backward(theta, sim, ckpts, grad_traj)

    def _backward(self, theta, sim, ckpts, grad_traj):
        nb, K = self.nb, self.K
        pops = self.state_tensor(sim)
        dev = self.device
        lam = [torch.zeros_like(pops), torch.zeros_like(pops)]
        lam_u = torch.zeros_like(sim.vel)
        lam_f = torch.empty_like(sim.vel)
        lam_b = torch.zeros((nb, L.LBM_BUBBLE_ADJ), dtype=torch.float64, device=dev)
        grad = torch.zeros(4, dtype=torch.float64, device=dev)
        # per step of a segment: the state entering it (H[i], the recompute writes H[i + 1]
        # directly), the velocity field its bubble half reads (Up[i], its collision writes
        # Up[i + 1]), its force field and its bubble record
        H = torch.empty((K + 1,) + tuple(pops.shape), dtype=pops.dtype, device=dev)
        Up = torch.empty((K + 1,) + tuple(sim.vel.shape), dtype=pops.dtype, device=dev)
        Fk = torch.empty((K,) + tuple(sim.vel.shape), dtype=pops.dtype, device=dev)
        rec = torch.zeros((K, nb, L.LBM_BUBBLE_RECORD), dtype=torch.float64, device=dev)
        # the tile mask of each step: the adjoint liquid step reads the force and the velocity
        # adjoint only in its flagged tiles
        Tk = None
        if self.use_tiles:
            Tk = torch.empty((K, L.lbm_step_tiles(sim.ctx)), dtype=torch.uint8, device=dev)
        gt = grad_traj.to(dev, torch.float64).contiguous()
        # buffers are rebound between the bubble half and the liquid step: no overlapped steps
        L.lbm_set_overlap(sim.ctx, False)
        bub = sim.bubbles
        cur = 0  # lam[cur] holds the adjoint state entering the next (earlier) step

        def segment(k0, n, events=None):
            """Recompute of the n steps from step k0 on from H[0], Up[0] and the bubble state,
            then their adjoint steps newest first."""
            nonlocal cur
            for i in range(n):
                L.lbm_bind_buffers(sim.ctx, _p(H[i]), _p(H[i + 1]), _p(Up[i]))
                # the bubble update fills the step record itself, sub-step velocities included
                L.lbm_record_next_bubble_half(sim.ctx, _p(rec[i]))
                L.bubbles_step(sim.ctx, sim.params, bub.soa, nb)
                Fk[i].copy_(sim.force)
                if Tk is not None:
                    L.lbm_step_tiles(sim.ctx, _p(Tk[i]))
                L.lbm_bind_buffers(sim.ctx, None, None, _p(Up[i + 1]))
                L.lbm_step(sim.ctx, 1)
            for i in reversed(range(n)):
                if events is not None:
                    # recorded by the library around the adjoint liquid kernel's launch alone
                    ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                    for e in ev:
                        e.record(self.stream)  # creates the underlying event
                    L.lbm_time_next_adjoint_liquid(sim.ctx, ev[0], ev[1])
                    events.append(ev)
                L.lbm_adjoint_liquid_tiles(sim.ctx, _p(H[i]), _p(Fk[i]), _p(lam[cur]),
                                           _p(lam[1 - cur]), _p(lam_u), _p(lam_f),
                                           _p(Tk[i]) if Tk is not None else None, _p(grad))
                cur = 1 - cur
                # the loss's term in this step's positions is added by the kernel
                L.lbm_adjoint_bubbles(sim.ctx, sim.params, _p(rec[i]), _p(Up[i]), _p(lam_f),
                                      _p(lam_u), _p(lam_b), _p(gt[k0 + i]), nb, _p(grad))

        for s in reversed(range(len(ckpts))):
            k0 = s * K
            k1 = min(k0 + K, self.steps)
            ck = ckpts[s]
            H[0].copy_(ck["state"])
            Up[0].copy_(ck["vel"])
            sim.force.zero_()
            for key, v in ck["bub"].items():
                bub.t[key].copy_(v)
            timed = self.liquid_events is not None and s == len(ckpts) - 1
            segment(k0, k1 - k0, self.liquid_events if timed else None)
        # back to the simulation's own buffers before the segment buffers go away
        L.lbm_bind_buffers(sim.ctx, _p(sim.pops[0]), _p(sim.pops[1]), _p(sim.vel))
        g = grad.cpu().numpy()
        # grad[0] holds dL/domega through the collision and, added by the library, through the
        # bubble closures' nu
        return np.array([g[1], g[2], g[0]])


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
